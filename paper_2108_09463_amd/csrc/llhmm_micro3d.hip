// d = 3 micro boxes (the problem allows d <= 3, Section 2.1), FP64, second-
// order stencil: set-up, time stepping and field evaluation.
//
// A 3-D box does not fit on one compute unit (a 32^3 box holds 0.8 MB of
// FP64 state per stage buffer), so one block per box streams its arrays
// through the caches: the stage input with one ghost layer (two buffers, read
// one and write the other), the state m and the running Runge-Kutta sum live
// in HBM; each thread walks x3 columns (consecutive threads on consecutive x1
// points, so loads coalesce) and one block barrier ends each stage.  The time
// loop is HBM-bound.
//
// Per box (doubles, at plan.tab_offset in the 3-D work buffer), E = n + 2,
// X = E^3 (one ghost layer per side), C = n^3, storage index
// ((i2 + 1) E + (i1 + 1)) E + (i0 + 1) (interior: ((i2 n) + i1) n + i0):
//   A   [3][X]  a^eps on the face between point idx and idx + e_axis, times
//               1/dx^2 (read by the field evaluation; the time loop forms the
//               same values from per-axis factor tables)
//   G   [3][X]  ghost data: m_init (Dirichlet) or m_init(ghost) - m_init(wrapped
//               interior point) (periodic m - m_init), on the face ghost points
//   y0, y1 [3][X]  stage inputs with their ghosts (ping-pong)
//   m   [3][C]  state;  acc [3][C] running sum of b_s k_s
#include "llhmm_micro3d.h"

namespace llhmm {

#pragma clang fp contract(off)
namespace {

constexpr int kThreads3d = 512;

__device__ __forceinline__ double xi_of(const BoxPlan &P, int idx) { return -P.mu_box + (double)idx * P.dx; }

// The factor of term t along axis ax at coordinate x: sin(2 pi f x + phase),
// or exactly 1 where the term does not vary along that axis.
__device__ __forceinline__ double axis_factor(const CoefDev &c, int t, int ax, double x) {
    const double two_pi = 6.283185307179586;
    if (ax >= c.dim || c.freq[t][ax] == 0.0) return 1.0;
    return sin(two_pi * c.freq[t][ax] * x + c.phase[t][ax]);
}

// a^eps at absolute (x0, x1, x2): c0 + sum_t amp_t prod_axis s_{t,axis}
// (a factor of exactly 1 leaves the product's bits unchanged)
__device__ double coef3(const CoefDev &c, double x0, double x1, double x2) {
    const double x[3] = {x0, x1, x2};
    double a = c.c0;
    for (int t = 0; t < c.n_terms; ++t) {
        double p = c.amp[t];
        for (int ax = 0; ax < 3; ++ax) p = p * axis_factor(c, t, ax, x[ax]);
        a = a + p;
    }
    return a;
}

// Coordinates along one axis as the set-up kernel forms them: grid point i,
// and the face between points f and f + 1.
__device__ __forceinline__ double point_pos(const BoxPlan &P, double centre, int i) {
    return centre + xi_of(P, i);
}
__device__ __forceinline__ double face_pos(const BoxPlan &P, double centre, int f) {
    const double x = centre + xi_of(P, f);
    return x + 0.5 * P.dx;
}

// A face coefficient a^eps / dx^2 from the per-axis factor tables: the
// products and sums of coef3 in its order, so the same bits as the set-up
// kernel's stored faces.  t0, t1, t2: term 0's entries along each axis (term t
// at + t * ts); the axis-0 tables hold amp_t times the factor, the first
// product coef3 forms.
__device__ __forceinline__ double face_from_factors(double c0, int nterms, const double *t0, const double *t1,
                                                    const double *t2, int ts, double sc) {
    double a = c0;
    for (int t = 0; t < nterms; ++t) {
        double p = t0[t * ts] * t1[t * ts];
        p = p * t2[t * ts];
        a = a + p;
    }
    return a * sc;
}

__device__ double kernel_space3(const Micro3dArgs &A, double x) {
    if (!(x > -1.0 && x < 1.0)) return 0.0;
    double poly = 0.0, xp = 1.0;
    for (int i = 0; i <= A.kp; ++i) {
        poly = poly + A.kc[i] * xp;
        xp = xp * x;
    }
    double b = 1.0 - x * x, bp = 1.0;
    for (int i = 0; i < A.kq + 1; ++i) bp = bp * b;
    return bp * poly;
}

__device__ void lagrange5_3(double s, double Lb[5]) {
    for (int l = 0; l < 5; ++l) {
        double v = 1.0;
        for (int mm = 0; mm < 5; ++mm)
            if (mm != l) v = v * (s - (double)(mm - 2)) / (double)(l - mm);
        Lb[l] = v;
    }
}

__device__ double node_offset3(double centre, double x0, int k, double dX) {
    const double o = centre - (x0 + (double)k * dX);
    return (fabs(o) <= 1e-9 * dX) ? 0.0 : o;
}

struct Box3 {
    int n, gw, E;   // gw ghost layers per side: 1 (second order) or 3 (fourth order)
    long C, X;
    double *A, *G, *y, *y1, *m, *acc;
    __device__ Box3(double *base, int n_, int gw_ = 1) : n(n_), gw(gw_), E(n_ + 2 * gw_) {
        C = (long)n * n * n;
        X = (long)E * E * E;
        A = base;
        G = A + 3 * X;
        y = G + 3 * X;
        y1 = y + 3 * X;
        m = y1 + 3 * X;
        acc = m + 3 * C;
    }
    // extended index of grid point (i0, i1, i2), ghosts at -gw..-1 and n..n+gw-1
    __device__ long ext(int i0, int i1, int i2) const {
        return ((long)(i2 + gw) * E + (i1 + gw)) * E + (i0 + gw);
    }
    __device__ long stride(int ax) const { return ax == 0 ? 1 : (ax == 1 ? (long)E : (long)E * E); }
};

// The g-th face ghost point (6 gw n^2 of them: per face of the box, gw layers
// of n^2 points; the 7-point and 13-point stencils reach no edge or corner
// ghost): its extended index and the index of the interior point it wraps to
// (periodic images).
__device__ void ghost_point(const Box3 &B, long g, long &gi, long &wi, int &c0, int &c1, int &c2) {
    const int n = B.n;
    const long nn = (long)n * n;
    const int face = (int)(g / (nn * B.gw));
    const int l = (int)((g / nn) % B.gw) + 1;   // layer 1..gw
    const int a = (int)(g % n), b = (int)((g / n) % n);
    const int ax = face >> 1, side = face & 1;
    const int p = side ? n - 1 + l : -l, w = side ? l - 1 : n - l;
    int q[3], r[3];
    if (ax == 0) { q[0] = p; q[1] = a; q[2] = b; }
    else if (ax == 1) { q[0] = a; q[1] = p; q[2] = b; }
    else { q[0] = a; q[1] = b; q[2] = p; }
    r[0] = q[0]; r[1] = q[1]; r[2] = q[2];
    r[ax] = w;
    gi = B.ext(q[0], q[1], q[2]);
    wi = B.ext(r[0], r[1], r[2]);
    c0 = q[0]; c1 = q[1]; c2 = q[2];
}

// m_init at grid point (i0, i1, i2) (ghosts allowed)
__device__ void minit3(const Micro3dArgs &A, const BoxPlan &P, const double *L, int i0, int i1, int i2,
                       double out[3]) {
    if (P.init_mode == LLHMM_INIT_EXPLICIT) {
        const int E6 = P.n + 2 * kGhost;
        const long cells = (long)E6 * E6 * E6;
        const long idx = ((long)(i2 + kGhost) * E6 + (i1 + kGhost)) * E6 + (i0 + kGhost);
        const double *src = A.m_init + P.init_offset;
        out[0] = src[idx];
        out[1] = src[cells + idx];
        out[2] = src[2 * cells + idx];
        return;
    }
    // Q_[4]: tensor-product Lagrange interpolation along x1, then x2, then x3
    const int gw = (P.order == 4) ? 3 : 1;
    const int EL = P.n + 2 * gw;            // basis rows for grid indices -gw .. n+gw-1
    const double *L0 = L + (i0 + gw) * 5;
    const double *L1 = L + (EL + i1 + gw) * 5;
    const double *L2 = L + (2 * EL + i2 + gw) * 5;
    const double *Mloc = L + 3 * EL * 5;    // [c][l0][l1][l2]
    double p[3] = {0.0, 0.0, 0.0};
    for (int l2 = 0; l2 < 5; ++l2) {
        double q1[3] = {0.0, 0.0, 0.0};
        for (int l1 = 0; l1 < 5; ++l1) {
            double q0[3] = {0.0, 0.0, 0.0};
            for (int l0 = 0; l0 < 5; ++l0)
                for (int c = 0; c < 3; ++c) q0[c] = q0[c] + Mloc[((c * 5 + l0) * 5 + l1) * 5 + l2] * L0[l0];
            for (int c = 0; c < 3; ++c) q1[c] = q1[c] + q0[c] * L1[l1];
        }
        for (int c = 0; c < 3; ++c) p[c] = p[c] + q1[c] * L2[l2];
    }
    const double nr = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    out[0] = p[0] / nr;
    out[1] = p[1] / nr;
    out[2] = p[2] / nr;
}

}  // namespace

// One block per 3-D box: faces, initial state, ghost data, stage input,
// space weights; zeroes the box's reference constant.
__global__ void __launch_bounds__(kThreads3d) k_setup3d(Micro3dArgs A) {
    const int box = A.box_ids[blockIdx.x];
    const BoxPlan P = A.plans[box];
    const int n = P.n, tid = threadIdx.x, nth = blockDim.x;
    const int gw = (P.order == 4) ? 3 : 1;
    Box3 B(A.work + P.tab_offset, n, gw);
    const CoefDev &cf = A.coefs[P.coef_index];
    // Lagrange bases per axis for grid indices -gw..n+gw-1, then the 5^3 x 3 macro values
    __shared__ double s_L[3 * (kLagMax2 - 4) * 5 + 375];
    if (P.init_mode == LLHMM_INIT_MACRO_Q) {
        const int nm = A.macro.n, EL = n + 2 * gw;
        const long npts = (long)nm * nm * nm;
        const double dX = A.macro.dX;
        const double cen[3] = {P.cx, P.cy, P.cz};
        const int mi[3] = {P.mi0, P.mi1, P.mi2};
        for (int t = tid; t < 3 * EL; t += nth) {
            const int ax = t / EL, i = t % EL - gw;
            const double o = node_offset3(cen[ax], A.macro.x0[ax], mi[ax], dX);
            lagrange5_3((xi_of(P, i) + o) / dX, s_L + t * 5);
        }
        double *Mloc = s_L + 3 * EL * 5;
        for (int t = tid; t < 375; t += nth) {
            const int c = t / 125, l0 = (t / 25) % 5, l1 = (t / 5) % 5, l2 = t % 5;
            const int k0 = ((P.mi0 + l0 - 2) % nm + nm) % nm;
            const int k1 = ((P.mi1 + l1 - 2) % nm + nm) % nm;
            const int k2 = ((P.mi2 + l2 - 2) % nm + nm) % nm;
            Mloc[t] = A.M_macro[c * npts + ((long)k0 * nm + k1) * nm + k2];
        }
    }
    __syncthreads();
    // faces: a at the midpoint between (i0,i1,i2) and its +e_axis neighbour, for
    // every point of the extended grid whose face an interior stencil reads
    // scaled by 1/dx^2 (second order) or 1/(24 dx)^2 (fourth order)
    const double sc = (P.order == 4) ? P.a_scale : 1.0 / (P.dx * P.dx);
    const int E = B.E;
    for (long t = tid; t < 3 * B.X; t += nth) {
        const int ax = (int)(t / B.X);
        const long e = t % B.X;
        const int i0 = (int)(e % E) - gw, i1 = (int)((e / E) % E) - gw, i2 = (int)(e / ((long)E * E)) - gw;
        double x0 = P.cx + xi_of(P, i0), x1 = P.cy + xi_of(P, i1), x2 = P.cz + xi_of(P, i2);
        if (P.coef_sampled) {   // the caller's face values, [axis][E6^3] on the grid with 3 ghost layers
            const int E6 = n + 2 * kGhost;
            const long si = (long)ax * E6 * E6 * E6 + ((long)(i2 + kGhost) * E6 + (i1 + kGhost)) * E6 + (i0 + kGhost);
            B.A[t] = A.coef_samples[P.coef_offset + si] * sc;
            continue;
        }
        if (ax == 0) x0 = x0 + 0.5 * P.dx;
        else if (ax == 1) x1 = x1 + 0.5 * P.dx;
        else x2 = x2 + 0.5 * P.dx;
        B.A[t] = coef3(cf, x0, x1, x2) * sc;
    }
    // interior state m = m_init, stage input y = m
    for (long t = tid; t < B.C; t += nth) {
        const int i0 = (int)(t % n), i1 = (int)((t / n) % n), i2 = (int)(t / ((long)n * n));
        double v[3];
        minit3(A, P, s_L, i0, i1, i2, v);
        const long e = B.ext(i0, i1, i2);
        for (int c = 0; c < 3; ++c) {
            B.m[c * B.C + t] = v[c];
            B.y[c * B.X + e] = v[c];
        }
    }
    __syncthreads();
    // ghost data and the ghosts of y (as the periodic / Dirichlet rule fills them)
    const long ng = 6L * gw * n * n;
    for (long g = tid; g < ng; g += nth) {
        long gi, wi;
        int q0, q1, q2;
        ghost_point(B, g, gi, wi, q0, q1, q2);
        double v[3];
        minit3(A, P, s_L, q0, q1, q2, v);
        for (int c = 0; c < 3; ++c) {
            if (P.bc == LLHMM_BC_DIRICHLET) {
                B.G[c * B.X + gi] = v[c];
                B.y[c * B.X + gi] = v[c];
            } else {
                const double d = v[c] - B.y[c * B.X + wi];   // m_init(ghost) - m_init(wrapped point)
                B.G[c * B.X + gi] = d;
                B.y[c * B.X + gi] = B.y[c * B.X + wi] + d;
            }
        }
    }
    // space weights: points, east faces
    double *w = A.wts + P.w_offset;
    for (int i = tid; i < n; i += nth) {
        const double xi = xi_of(P, i);
        w[i] = kernel_space3(A, xi / P.mu) * P.dx / P.mu;
        w[n + i] = kernel_space3(A, (xi + 0.5 * P.dx) / P.mu) * P.dx / P.mu;
    }
    if (tid < kMaxQ) A.box_const[(long)box * kMaxQ + tid] = 0.0;
}

#pragma clang fp contract(on)

// Fourth-order part of H along one axis at extended index e (stride st): the
// staggered fluxes F = a' (27 (y_{i+1} - y_i) - (y_{i+2} - y_{i-1})) on the
// faces between points i and i+1, i = j-2..j+1 (faces pre-scaled by
// 1/(24 dx)^2), combined as 27 (F_{j+1/2} - F_{j-1/2}) - (F_{j+3/2} - F_{j-3/2}).
// f_east: the flux on the east face j+1/2.
// Status bits 4 and 8 of a box from its final state m [3][n^3] (points t =
// (i2 n + i1) n + i0), block-wide: 4 when two x1-neighbouring points differ by
// more than kRoughMax (an unresolved, grid-scale state), 8 when ||m|^2 - 1|
// exceeds 1e-10.  Every thread of the block must call it.
__device__ int final_state_bits(const double *m, long C, int n, int tid, int nth) {
    int bits = 0;
    for (long t = tid; t < C; t += nth) {
        const double a0 = m[t], a1 = m[C + t], a2 = m[2 * C + t];
        const double e = __builtin_fma(a0, a0, __builtin_fma(a1, a1, __builtin_fma(a2, a2, -1.0)));
        if (!(__builtin_fabs(e) <= 1e-10)) bits |= 8;
        if (t % n != n - 1) {
            const double d0 = m[t + 1] - a0, d1 = m[C + t + 1] - a1, d2 = m[2 * C + t + 1] - a2;
            if (!(__builtin_fma(d0, d0, __builtin_fma(d1, d1, d2 * d2)) <= kRoughMax * kRoughMax)) bits |= 4;
        }
    }
    return (__syncthreads_or(bits & 4) ? 4 : 0) | (__syncthreads_or(bits & 8) ? 8 : 0);
}

__device__ __forceinline__ double axis_o4(const double *yc, const double *Aax, long e, long st,
                                          double &f_east) {
    double F[4];
    for (int k = -2; k <= 1; ++k) {
        const long f = e + k * st;
        const double g = 27.0 * (yc[f + st] - yc[f]) - (yc[f + 2 * st] - yc[f - st]);
        F[k + 2] = Aax[f] * g;
    }
    f_east = F[2];
    return 27.0 * (F[2] - F[1]) - (F[3] - F[0]);
}

// One block per 3-D box: H(m_init) = div(a grad m_init) at every point (mode 1,
// the field evaluation), from the stored faces and the stage input with its
// ghosts as the set-up kernel leaves them.
__global__ void __launch_bounds__(kThreads3d) k_field3d(Micro3dArgs A) {
    const int box = A.box_ids[blockIdx.x];
    const BoxPlan P = A.plans[box];
    const int n = P.n, tid = threadIdx.x, nth = blockDim.x;
    const bool o4 = (P.order == 4);
    Box3 B(A.work + P.tab_offset, n, o4 ? 3 : 1);
    const long C = B.C, X = B.X, nn = (long)n * n;
    const long s1 = B.stride(1), s2 = B.stride(2);
    for (long t = tid; t < C; t += nth) {
        const int i0 = (int)(t % n), i1 = (int)((t / n) % n), i2 = (int)(t / nn);
        const long e = B.ext(i0, i1, i2);
        if (o4) {
            for (int c = 0; c < 3; ++c) {
                const double *yc = B.y + c * X;
                double fe, h = 0.0;
                for (int ax = 0; ax < 3; ++ax) h += axis_o4(yc, B.A + ax * X, e, B.stride(ax), fe);
                A.out_field[P.mfinal_offset + c * C + t] = h;
            }
            continue;
        }
        const double ae0 = B.A[e], aw0 = B.A[e - 1];
        const double ae1 = B.A[X + e], aw1 = B.A[X + e - s1];
        const double ae2 = B.A[2 * X + e], aw2 = B.A[2 * X + e - s2];
        for (int c = 0; c < 3; ++c) {
            const double *yc = B.y + c * X;
            const double v = yc[e];
            double h = ae0 * (yc[e + 1] - v) - aw0 * (v - yc[e - 1]);
            h += ae1 * (yc[e + s1] - v) - aw1 * (v - yc[e - s1]);
            h += ae2 * (yc[e + s2] - v) - aw2 * (v - yc[e - s2]);
            A.out_field[P.mfinal_offset + c * C + t] = h;
        }
    }
}

// The time loop of fourth-order boxes (mode 0): each stage reads the stage
// input with three ghost layers and writes the next one, walking x3 columns
// (x3 values and face fluxes roll in registers, the x1/x2 parts of the
// 13-point stencil come through the caches); the ghost layers of the new
// input are filled between two block barriers.
__global__ void __launch_bounds__(kThreads3d) k_micro3d_o4(Micro3dArgs A) {
    __shared__ double s_red[kThreads3d][9];
    const int box = A.box_ids[blockIdx.x];
    const BoxPlan P = A.plans[box];
    if (P.order != 4) return;   // second-order boxes: the column kernel
    const int n = P.n, tid = threadIdx.x, nth = kThreads3d;
    Box3 B(A.work + P.tab_offset, n, 3);
    const long C = B.C, X = B.X, nn = (long)n * n;
    const double *w = A.wts + P.w_offset;
    const double *wt = A.wt + P.wt_offset;
    const double alpha = P.alpha, dt = P.dt;
    const bool rk4 = (P.stages == 4), dirichlet = (P.bc == LLHMM_BC_DIRICHLET);
    const bool flux = (P.quantity == LLHMM_Q_FLUX), torque = (P.quantity == LLHMM_Q_TORQUE);
    const int nst = rk4 ? 4 : 2;
    for (int q = 0; q < 9; ++q) s_red[tid][q] = 0.0;   // this thread's share of the average
    double *ycur = B.y, *ynext = B.y1;
    for (int step = 0; step <= P.M; ++step) {
        const double wn = wt[step];
        const bool last_level = (step == P.M);
        for (int s = 0; s < nst; ++s) {
            const double bs = rk4 ? ((s == 0 || s == 3) ? 1.0 / 6.0 : 1.0 / 3.0) : 0.5;
            const double cnext = rk4 ? ((s < 2) ? 0.5 : 1.0) : 1.0;
            // Column walk: a thread owns the x3 columns (i0, i1) = col and walks
            // them upwards.  The stage input at planes i2 .. i2+3 and the fluxes on
            // the x3 faces i2-2 .. i2 (face j between planes j and j+1) roll along
            // in registers, so each point loads one new value and one new face
            // along x3; the x1/x2 stencils are read through the caches.
            const double *A2 = B.A + 2 * X;
            const long s3 = B.stride(2);
            for (long col = tid; col < nn; col += nth) {
                const int i0 = (int)(col % n), i1 = (int)(col / n);
                const long e0 = B.ext(i0, i1, 0);
                double yw[3][4], F3[3][3];
                for (int c = 0; c < 3; ++c) {
                    const double *yc = ycur + c * X;
                    const double ym3 = yc[e0 - 3 * s3], ym2 = yc[e0 - 2 * s3], ym1 = yc[e0 - s3];
                    for (int k = 0; k < 4; ++k) yw[c][k] = yc[e0 + k * s3];
                    F3[c][0] = A2[e0 - 2 * s3] * (27.0 * (ym1 - ym2) - (yw[c][0] - ym3));
                    F3[c][1] = A2[e0 - s3] * (27.0 * (yw[c][0] - ym1) - (yw[c][1] - ym2));
                    F3[c][2] = A2[e0] * (27.0 * (yw[c][1] - yw[c][0]) - (yw[c][2] - ym1));
                }
#pragma unroll 1
                for (int i2 = 0; i2 < n; ++i2) {
                    // opaque to the optimizer: otherwise every stencil address becomes
                    // its own pointer stepped along x3, and the registers overflow
                    long e = e0 + i2 * s3;
                    asm volatile("" : "+v"(e));
                    const long t = (long)i2 * nn + col;
                    double H[3], Fe[3][3];
                    for (int c = 0; c < 3; ++c) {
                        const double *yc = ycur + c * X;
                        double h = 0.0;
                        for (int ax = 0; ax < 2; ++ax) h += axis_o4(yc, B.A + ax * X, e, B.stride(ax), Fe[ax][c]);
                        const double f1 = A2[e + s3] * (27.0 * (yw[c][2] - yw[c][1]) - (yw[c][3] - yw[c][0]));
                        h += 27.0 * (F3[c][2] - F3[c][1]) - (f1 - F3[c][0]);
                        Fe[2][c] = F3[c][2];
                        F3[c][0] = F3[c][1];
                        F3[c][1] = F3[c][2];
                        F3[c][2] = f1;
                        H[c] = h;
                    }
                    const double yv[3] = {yw[0][0], yw[1][0], yw[2][0]};
                    for (int c = 0; c < 3; ++c) {   // next point's window: planes i2+1 .. i2+4
                        yw[c][0] = yw[c][1];
                        yw[c][1] = yw[c][2];
                        yw[c][2] = yw[c][3];
                        yw[c][3] = (i2 + 1 < n) ? ycur[c * X + e + 4 * s3] : 0.0;
                    }
                    double c1[3], c2[3];
                    c1[0] = yv[1] * H[2] - yv[2] * H[1];
                    c1[1] = yv[2] * H[0] - yv[0] * H[2];
                    c1[2] = yv[0] * H[1] - yv[1] * H[0];
                    if (s == 0) {
                        if (flux) {
                            // a grad m on the east face of each axis: the face weight along
                            // that axis, point weights along the others
                            const double wax[3] = {w[n + i0] * w[i1] * w[i2] * wn, w[i0] * w[n + i1] * w[i2] * wn,
                                                   w[i0] * w[i1] * w[n + i2] * wn};
                            for (int ax = 0; ax < 3; ++ax)
                                for (int c = 0; c < 3; ++c) s_red[tid][ax * 3 + c] += wax[ax] * Fe[ax][c];
                        } else {
                            const double wc = w[i0] * w[i1] * w[i2] * wn;
                            for (int c = 0; c < 3; ++c) s_red[tid][c] += wc * (torque ? c1[c] : H[c]);
                        }
                    }
                    if (last_level) continue;
                    c2[0] = yv[1] * c1[2] - yv[2] * c1[1];
                    c2[1] = yv[2] * c1[0] - yv[0] * c1[2];
                    c2[2] = yv[0] * c1[1] - yv[1] * c1[0];
                    if (s < nst - 1) {
                        for (int c = 0; c < 3; ++c) {
                            const double k = -c1[c] - alpha * c2[c];
                            double *pa = B.acc + c * C + t;
                            __builtin_nontemporal_store((s == 0) ? bs * k : __builtin_nontemporal_load(pa) + bs * k, pa);
                            ynext[c * X + e] = __builtin_nontemporal_load(B.m + c * C + t) + cnext * dt * k;
                        }
                    } else {
                        double v[3];
                        for (int c = 0; c < 3; ++c) {
                            const double k = -c1[c] - alpha * c2[c];
                            v[c] = __builtin_nontemporal_load(B.m + c * C + t) +
                                   dt * (__builtin_nontemporal_load(B.acc + c * C + t) + bs * k);
                        }
                        const double nr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                        for (int c = 0; c < 3; ++c) {
                            __builtin_nontemporal_store(v[c] / nr, B.m + c * C + t);
                            ynext[c * X + e] = v[c] / nr;
                        }
                    }
                }
            }
            if (last_level) break;
            __syncthreads();
            // the three ghost layers of the new stage input
            for (long g = tid; g < 18 * nn; g += nth) {
                long gi, wi;
                int q0, q1, q2;
                ghost_point(B, g, gi, wi, q0, q1, q2);
                for (int c = 0; c < 3; ++c)
                    ynext[c * X + gi] = dirichlet ? B.G[c * X + gi] : ynext[c * X + wi] + B.G[c * X + gi];
            }
            __syncthreads();
            double *tmp = ycur;
            ycur = ynext;
            ynext = tmp;
        }
    }

    // the box's average: fixed-order block reduction into its partial-sum slot
    __syncthreads();
    for (int half = kThreads3d / 2; half > 0; half >>= 1) {
        if (tid < half)
            for (int c = 0; c < 9; ++c) s_red[tid][c] = s_red[tid][c] + s_red[tid + half][c];
        __syncthreads();
    }
    const int hbits = final_state_bits(B.m, C, n, tid, kThreads3d);
    if (tid == 0) {
        double *dst = A.partials + P.part_offset * kMaxQ;
        int bad = hbits;
        for (int q = 0; q < kMaxQ; ++q) {
            const double v = (q < 9) ? s_red[0][q] : 0.0;
            dst[q] = v;
            if (!__builtin_isfinite(v)) bad |= 1;
        }
        A.wave_status[P.part_offset] = bad;
    }
    if (A.out_field) {   // the columns this thread walked
        for (long col = tid; col < nn; col += nth)
            for (int i2 = 0; i2 < n; ++i2) {
                const long t = (long)i2 * nn + col;
                for (int c = 0; c < 3; ++c) A.out_field[P.mfinal_offset + c * C + t] = B.m[c * C + t];
            }
    }
}

// Loads and stores at a byte offset from a block-uniform base: the base stays
// in scalar registers and each address costs one 32-bit vector register.
__device__ __forceinline__ double ldo(const double *base, uint32_t off) {
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + off);
}
__device__ __forceinline__ void sto(double *base, uint32_t off, double v) {
    *reinterpret_cast<double *>(reinterpret_cast<char *>(base) + off) = v;
}
// Streaming loads (data not read again within the stage): non-temporal, so
// they do not push the stage input's reusable lines out of L2.
__device__ __forceinline__ double ldo_nt(const double *base, uint32_t off) {
    return __builtin_nontemporal_load(reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + off));
}
__device__ __forceinline__ void sto_nt(double *base, uint32_t off, double v) {
    __builtin_nontemporal_store(v, reinterpret_cast<double *>(reinterpret_cast<char *>(base) + off));
}

// The time loop (mode 0; boxes with n >= 8), walking columns.  Thread t owns the
// x3 columns (i0, i1) = (q % n, q / n), q = t + j NT, and walks each from
// x3 = 0 to n - 1 in every stage:
//  * the stage input below, at and above the point and the x3 face below stay
//    in registers from one point to the next; the x1 / x2 neighbours come from
//    the caches, where the waves holding the neighbouring columns brought
//    them a moment earlier;
//  * the face coefficients a^eps / dx^2 of a closed-form coefficient are
//    formed from per-axis factor tables in LDS, bit for bit the values the
//    set-up kernel stores, which takes a sixth of the streamed bytes off
//    every stage (STORED, for a batch with a sampled coefficient: the stored
//    faces are read with the point's other operands);
//  * no wave waits for another inside a stage (stage inputs are read-only
//    there and every other array is touched only at the thread's own
//    points), and all loads of a point are issued together;
//  * a point on a box face also writes the face ghosts of the next stage
//    input that wrap to it (periodic image plus offset, or the Dirichlet
//    datum), their ghost data loaded with the point's other operands, so a
//    stage ends with a single barrier.
template <int NT, int NQ, bool STORED>
__global__ void __launch_bounds__(NT, 1) k_micro3d(Micro3dArgs A) {
    __shared__ double s_red[NT][NQ];
    // factor tables [term][axis][TR]: points 0..n-1, faces -1/2..n-1/2 (index f + 1);
    // STORED (a sampled coefficient in the batch): the faces the set-up stored
    constexpr int TR = kMaxN3 + 1;
    __shared__ double s_pt[STORED ? 1 : LLHMM_MAX_TERMS * 3 * TR];
    __shared__ double s_fc[STORED ? 1 : LLHMM_MAX_TERMS * 3 * TR];
    const int box = A.box_ids[blockIdx.x];
    const BoxPlan P = A.plans[box];
    if (P.order != 2) return;   // fourth-order boxes: k_micro3d_o4
    const int n = P.n, tid = threadIdx.x, nn = n * n;
    Box3 B(A.work + P.tab_offset, n);
    const long C = B.C, X = B.X;
    const uint32_t s1b = (uint32_t)B.stride(1) * 8, s2b = (uint32_t)B.stride(2) * 8;
    const int32_t n8 = n * 8, ns1 = n * (int32_t)s1b, ns2 = n * (int32_t)s2b;
    const double *w = A.wts + P.w_offset;
    const double *wt = A.wt + P.wt_offset;
    const double alpha = P.alpha, dt = P.dt;
    const bool rk4 = (P.stages == 4), dirichlet = (P.bc == LLHMM_BC_DIRICHLET);
    const int nst = rk4 ? 4 : 2;
    const CoefDev &cf = A.coefs[P.coef_index];
    const double sc = 1.0 / (P.dx * P.dx);
    const double c0 = cf.c0;
    const int nterms = cf.n_terms;
    if (!STORED) {
        const double cen[3] = {P.cx, P.cy, P.cz};
        for (int k = tid; k < nterms * 3 * (2 * n + 1); k += NT) {
            const int t = k / (3 * (2 * n + 1)), r = k % (3 * (2 * n + 1));
            const int ax = r / (2 * n + 1), i = r % (2 * n + 1);
            const double pre = (ax == 0) ? cf.amp[t] : 1.0;   // amp_t times the axis-0 factor
            if (i < n) {
                s_pt[(t * 3 + ax) * TR + i] = pre * axis_factor(cf, t, ax, point_pos(P, cen[ax], i));
            } else {
                const int f = i - n - 1;   // face between points f and f + 1, f = -1..n-1
                s_fc[(t * 3 + ax) * TR + f + 1] = pre * axis_factor(cf, t, ax, face_pos(P, cen[ax], f));
            }
        }
        __syncthreads();
    }
    constexpr int TS = 3 * TR;   // term stride of both tables
    const double *Ab[3] = {B.A, B.A + X, B.A + 2 * X};
    const double *Gb[3] = {B.G, B.G + X, B.G + 2 * X};
    double *mb[3] = {B.m, B.m + C, B.m + 2 * C};
    double *ab[3] = {B.acc, B.acc + C, B.acc + 2 * C};
    const bool flux = (NQ == 9) && (P.quantity == LLHMM_Q_FLUX);
    // this thread's share of the average: in registers (3 sums), or with nine
    // sums in its row of the reduction buffer (registers would spill)
    constexpr bool SUM_LDS = (NQ == 9);
    double sum[SUM_LDS ? 1 : NQ];
    for (int q = 0; q < NQ; ++q) {
        if (SUM_LDS) s_red[tid][q] = 0.0;
        else sum[SUM_LDS ? 0 : q] = 0.0;
    }
    auto add_sum = [&](int q, double v) {
        if (SUM_LDS) s_red[tid][q] += v;
        else sum[SUM_LDS ? 0 : q] += v;
    };
    double *ycur = B.y, *ynext = B.y1;
    for (int step = 0; step <= P.M; ++step) {
        const double wn = wt[step];
        const bool last_level = (step == P.M);
        for (int s = 0; s < nst; ++s) {
            const double bs = rk4 ? ((s == 0 || s == 3) ? 1.0 / 6.0 : 1.0 / 3.0) : 0.5;
            const double cnext = rk4 ? ((s < 2) ? 0.5 : 1.0) : 1.0;
            const double *yb[3] = {ycur, ycur + X, ycur + 2 * X};
            double *nb[3] = {ynext, ynext + X, ynext + 2 * X};
            // the running sum is not read at the first stage: its load then repeats
            // the state's (same lines, no extra traffic)
            const double *const *accr = (s == 0) ? (const double *const *)mb : (const double *const *)ab;
            for (int q = tid; q < nn; q += NT) {
                const int i0 = q % n, i1 = q / n;
                uint32_t eb = (uint32_t)B.ext(i0, i1, -1) * 8;
                uint32_t tb = (uint32_t)q * 8;
                double ylo[3], yc[3];
                for (int c = 0; c < 3; ++c) {
                    ylo[c] = ldo(yb[c], eb);
                    yc[c] = ldo(yb[c], eb + s2b);
                }
                // factor table rows of this column (term 0)
                const double *p0 = s_pt + i0, *p1 = s_pt + TR + i1, *p2 = s_pt + 2 * TR;
                const double *f0 = s_fc + i0 + 1, *f1 = s_fc + TR + i1 + 1, *f2 = s_fc + 2 * TR;
                double aw2 = STORED ? ldo(Ab[2], eb) : face_from_factors(c0, nterms, p0, p1, f2, TS, sc);
                const double wxy = w[i0] * w[i1];
                // flux: the face weight along the flux axis, point weights along the
                // others (axis 0 first), as products over the axes
                const double wfx = (NQ == 9) ? w[n + i0] * w[i1] : 0.0;
                const double wfy = (NQ == 9) ? w[i0] * w[n + i1] : 0.0;
                // byte offsets from a point of this column to the face ghosts that
                // wrap to it (0: none): x1 (slot a), x2 (slot b; x3 when the column
                // is not on an x2 face)
                const int32_t da = (i0 == n - 1) ? -n8 : ((i0 == 0) ? n8 : 0);
                const int32_t dy = (i1 == n - 1) ? -ns1 : ((i1 == 0) ? ns1 : 0);
                for (int i2 = 0; i2 < n; ++i2, tb += (uint32_t)nn * 8) {
                    eb += s2b;
                    const int32_t dz = (i2 == n - 1) ? -ns2 : ((i2 == 0) ? ns2 : 0);
                    const int32_t db = dy ? dy : dz;
                    const uint32_t ga = da ? eb + da : 0u, gb = db ? eb + db : 0u;
                    // every load of the point first, so they are in flight together
                    double yhi[3], ye[3], yw[3], yn[3], ys[3], mo[3], ao[3], gav[3], gbv[3];
                    for (int c = 0; c < 3; ++c) {
                        const double *yp = yb[c];
                        yhi[c] = ldo(yp, eb + s2b);
                        ye[c] = ldo(yp, eb + 8);
                        yw[c] = ldo(yp, eb - 8);
                        yn[c] = ldo(yp, eb + s1b);
                        ys[c] = ldo(yp, eb - s1b);
                    }
                    for (int c = 0; c < 3; ++c) {
                        mo[c] = ldo_nt(mb[c], tb);
                        ao[c] = ldo_nt(accr[c], tb);
                        gav[c] = ldo(Gb[c], ga);
                        gbv[c] = ldo(Gb[c], gb);
                    }
                    const double wz = w[i2];
                    const double wfz = (NQ == 9) ? w[n + i2] : 0.0;
                    double sae0 = 0.0, saw0 = 0.0, sae1 = 0.0, saw1 = 0.0, sae2 = 0.0;
                    if (STORED) {
                        sae0 = ldo(Ab[0], eb);
                        saw0 = ldo(Ab[0], eb - 8);
                        sae1 = ldo(Ab[1], eb);
                        saw1 = ldo(Ab[1], eb - s1b);
                        sae2 = ldo(Ab[2], eb);
                    }
                    // keep the scheduler from splitting the loads into dependent groups
                    __builtin_amdgcn_sched_barrier(0);
                    const double ae0 = STORED ? sae0 : face_from_factors(c0, nterms, f0, p1, p2 + i2, TS, sc);
                    const double aw0 = STORED ? saw0 : face_from_factors(c0, nterms, f0 - 1, p1, p2 + i2, TS, sc);
                    const double ae1 = STORED ? sae1 : face_from_factors(c0, nterms, p0, f1, p2 + i2, TS, sc);
                    const double aw1 = STORED ? saw1 : face_from_factors(c0, nterms, p0, f1 - 1, p2 + i2, TS, sc);
                    const double ae2 = STORED ? sae2 : face_from_factors(c0, nterms, p0, p1, f2 + i2 + 1, TS, sc);
                    double H[3];
                    for (int c = 0; c < 3; ++c) {
                        const double v = yc[c];
                        double h = ae0 * (ye[c] - v) - aw0 * (v - yw[c]);
                        h += ae1 * (yn[c] - v) - aw1 * (v - ys[c]);
                        h += ae2 * (yhi[c] - v) - aw2 * (v - ylo[c]);
                        H[c] = h;
                    }
                    double c1[3], c2[3];
                    c1[0] = yc[1] * H[2] - yc[2] * H[1];
                    c1[1] = yc[2] * H[0] - yc[0] * H[2];
                    c1[2] = yc[0] * H[1] - yc[1] * H[0];
                    if (s == 0 && flux) {
                        // a grad m on the east face of the point along each axis
                        // ([axis][component]; a / dx^2 here, times dx at the upscale)
                        const double w0 = wfx * wz * wn, w1 = wfy * wz * wn, w2 = wxy * wfz * wn;
                        for (int c = 0; c < 3; ++c) {
                            add_sum(c, w0 * (ae0 * (ye[c] - yc[c])));
                            add_sum(3 + c, w1 * (ae1 * (yn[c] - yc[c])));
                            add_sum(6 + c, w2 * (ae2 * (yhi[c] - yc[c])));
                        }
                    } else if (s == 0) {
                        const double wc = wxy * wz * wn;
                        if (P.quantity == LLHMM_Q_TORQUE)
                            for (int c = 0; c < 3; ++c) add_sum(c, wc * c1[c]);
                        else
                            for (int c = 0; c < 3; ++c) add_sum(c, wc * H[c]);
                    }
                    if (!last_level) {
                        c2[0] = yc[1] * c1[2] - yc[2] * c1[1];
                        c2[1] = yc[2] * c1[0] - yc[0] * c1[2];
                        c2[2] = yc[0] * c1[1] - yc[1] * c1[0];
                        double vn[3];
                        if (s < nst - 1) {
                            for (int c = 0; c < 3; ++c) {
                                const double k = -c1[c] - alpha * c2[c];
                                sto_nt(ab[c], tb, (s == 0) ? bs * k : ao[c] + bs * k);
                                vn[c] = mo[c] + cnext * dt * k;
                            }
                        } else {
                            double v[3];
                            for (int c = 0; c < 3; ++c) {
                                const double k = -c1[c] - alpha * c2[c];
                                v[c] = mo[c] + dt * (ao[c] + bs * k);
                            }
                            const double nr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                            for (int c = 0; c < 3; ++c) {
                                vn[c] = v[c] / nr;
                                sto_nt(mb[c], tb, vn[c]);
                            }
                        }
                        for (int c = 0; c < 3; ++c) sto(nb[c], eb, vn[c]);
                        if (da)
                            for (int c = 0; c < 3; ++c) sto(nb[c], eb + da, dirichlet ? gav[c] : vn[c] + gav[c]);
                        if (db)
                            for (int c = 0; c < 3; ++c) sto(nb[c], eb + db, dirichlet ? gbv[c] : vn[c] + gbv[c]);
                        // the x3 ghost of a point on an edge shared by an x2 face and an
                        // x3 face (slot b holds its x2 ghost)
                        if (dy && dz)
                            for (int c = 0; c < 3; ++c) {
                                const double g = ldo(Gb[c], eb + dz);
                                sto(nb[c], eb + dz, dirichlet ? g : vn[c] + g);
                            }
                    }
                    for (int c = 0; c < 3; ++c) {
                        ylo[c] = yc[c];
                        yc[c] = yhi[c];
                    }
                    aw2 = ae2;
                }
            }
            if (last_level) break;
            __syncthreads();   // the next stage input is complete, ghosts included
            double *tmp = ycur;
            ycur = ynext;
            ynext = tmp;
        }
    }

    // the box's average: fixed-order block reduction into its partial-sum slot
    if (!SUM_LDS)
        for (int c = 0; c < NQ; ++c) s_red[tid][c] = sum[SUM_LDS ? 0 : c];
    __syncthreads();
    for (int half = NT / 2; half > 0; half >>= 1) {
        if (tid < half)
            for (int c = 0; c < NQ; ++c) s_red[tid][c] = s_red[tid][c] + s_red[tid + half][c];
        __syncthreads();
    }
    const int hbits = final_state_bits(B.m, C, n, tid, NT);
    if (tid == 0) {
        double *dst = A.partials + P.part_offset * kMaxQ;
        int bad = hbits;
        for (int q = 0; q < kMaxQ; ++q) {
            const double v = (q < NQ) ? s_red[0][q] : 0.0;
            dst[q] = v;
            if (!__builtin_isfinite(v)) bad |= 1;
        }
        A.wave_status[P.part_offset] = bad;
    }
    if (A.out_field) {
        for (long t = tid; t < C; t += NT)
            for (int c = 0; c < 3; ++c) A.out_field[P.mfinal_offset + c * C + t] = B.m[c * C + t];
    }
}

template <int NT, bool STORED>
static void launch_cols_faces(const Micro3dArgs &a, hipStream_t s) {
    if (a.nq_max > 3)   // a flux box in the batch: nine sums per thread
        hipLaunchKernelGGL((k_micro3d<NT, 9, STORED>), dim3(a.nbox), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_micro3d<NT, 3, STORED>), dim3(a.nbox), dim3(NT), 0, s, a);
}

template <int NT>
static void launch_cols(const Micro3dArgs &a, hipStream_t s) {
    if (a.sampled) launch_cols_faces<NT, true>(a, s);   // a sampled coefficient: the stored faces
    else launch_cols_faces<NT, false>(a, s);
}

hipError_t launch_setup3d(const Micro3dArgs &a, hipStream_t s) {
    if (a.nbox <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_setup3d, dim3(a.nbox), dim3(kThreads3d), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_micro3d(const Micro3dArgs &a, hipStream_t s) {
    if (a.nbox <= 0) return hipSuccess;
    if (a.mode == 1) {
        hipLaunchKernelGGL(k_field3d, dim3(a.nbox), dim3(kThreads3d), 0, s, a);
    } else {
        // second-order boxes: threads per block = the columns of the largest box,
        // rounded up (larger boxes take several passes over their columns)
        if (a.orders & 1) {
            const int cols = a.nmax * a.nmax;
            if (cols <= 256) launch_cols<256>(a, s);
            else if (cols <= 512) launch_cols<512>(a, s);
            else launch_cols<1024>(a, s);
        }
        if (a.orders & 2) hipLaunchKernelGGL(k_micro3d_o4, dim3(a.nbox), dim3(kThreads3d), 0, s, a);
    }
    return hipGetLastError();
}

int64_t work3d_size(int n, int order) {
    const int64_t E = n + ((order == 4) ? 6 : 2);
    return 12 * E * E * E + 6 * (int64_t)n * n * n;
}

}  // namespace llhmm
