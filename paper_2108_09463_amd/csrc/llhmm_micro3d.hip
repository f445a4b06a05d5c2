// d = 3 micro boxes (the problem allows d <= 3, Section 2.1), FP64, second-
// order stencil: set-up and time stepping.
//
// A 3-D box does not fit on one compute unit (a 32^3 box holds 0.8 MB of
// FP64 state per stage buffer), so one block per box streams its arrays
// through the caches: the stage input with one ghost layer (two buffers, read
// one and write the other), the state m and the running Runge-Kutta sum live
// in HBM, the block walks all cells per stage (consecutive threads on
// consecutive x1 points, so loads coalesce) and block barriers separate the
// phases.  The kernel is HBM-bound.
//
// Per box (doubles, at plan.tab_offset in the 3-D work buffer), E = n + 2,
// X = E^3 (one ghost layer per side), C = n^3, storage index
// ((i2 + 1) E + (i1 + 1)) E + (i0 + 1) (interior: ((i2 n) + i1) n + i0):
//   A   [3][X]  a^eps on the face between point idx and idx + e_axis, times 1/dx^2
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

// a^eps at absolute (x0, x1, x2): c0 + sum_t amp_t prod_axis s_{t,axis}
__device__ double coef3(const CoefDev &c, double x0, double x1, double x2) {
    const double two_pi = 6.283185307179586;
    const double x[3] = {x0, x1, x2};
    double a = c.c0;
    for (int t = 0; t < c.n_terms; ++t) {
        double p = c.amp[t];
        for (int ax = 0; ax < c.dim; ++ax)
            if (c.freq[t][ax] != 0.0) p = p * sin(two_pi * c.freq[t][ax] * x[ax] + c.phase[t][ax]);
        a = a + p;
    }
    return a;
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
    int n, E;
    long C, X;
    double *A, *G, *y, *y1, *m, *acc;
    __device__ Box3(double *base, int n_) : n(n_), E(n_ + 2) {
        C = (long)n * n * n;
        X = (long)E * E * E;
        A = base;
        G = A + 3 * X;
        y = G + 3 * X;
        y1 = y + 3 * X;
        m = y1 + 3 * X;
        acc = m + 3 * C;
    }
    // extended index of grid point (i0, i1, i2), ghosts at -1 and n
    __device__ long ext(int i0, int i1, int i2) const { return ((long)(i2 + 1) * E + (i1 + 1)) * E + (i0 + 1); }
    __device__ long stride(int ax) const { return ax == 0 ? 1 : (ax == 1 ? (long)E : (long)E * E); }
};

// The g-th face ghost point (6 n^2 of them): its extended index and the index
// of the interior point it wraps to (periodic images).
__device__ void ghost_point(const Box3 &B, long g, long &gi, long &wi, int &c0, int &c1, int &c2) {
    const int n = B.n;
    const long nn = (long)n * n;
    const int face = (int)(g / nn);
    const int a = (int)(g % n), b = (int)((g / n) % n);
    const int ax = face >> 1, side = face & 1;
    const int p = side ? n : -1, w = side ? 0 : n - 1;
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
    const int EL = P.n + 2;                 // basis rows for grid indices -1 .. n
    const double *L0 = L + (i0 + 1) * 5;
    const double *L1 = L + (EL + i1 + 1) * 5;
    const double *L2 = L + (2 * EL + i2 + 1) * 5;
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
    Box3 B(A.work + P.tab_offset, n);
    const CoefDev &cf = A.coefs[P.coef_index];
    // Lagrange bases per axis for grid indices -1..n, then the 5^3 x 3 macro values
    __shared__ double s_L[3 * (kLagMax2 - 4) * 5 + 375];
    if (P.init_mode == LLHMM_INIT_MACRO_Q) {
        const int nm = A.macro.n, EL = n + 2;
        const long npts = (long)nm * nm * nm;
        const double dX = A.macro.dX;
        const double cen[3] = {P.cx, P.cy, P.cz};
        const int mi[3] = {P.mi0, P.mi1, P.mi2};
        for (int t = tid; t < 3 * EL; t += nth) {
            const int ax = t / EL, i = t % EL - 1;
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
    const double sc = 1.0 / (P.dx * P.dx);
    const int E = B.E;
    for (long t = tid; t < 3 * B.X; t += nth) {
        const int ax = (int)(t / B.X);
        const long e = t % B.X;
        const int i0 = (int)(e % E) - 1, i1 = (int)((e / E) % E) - 1, i2 = (int)(e / ((long)E * E)) - 1;
        double x0 = P.cx + xi_of(P, i0), x1 = P.cy + xi_of(P, i1), x2 = P.cz + xi_of(P, i2);
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
    const long ng = 6L * n * n;
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

// One block per 3-D box, point by point: the whole time loop (HeunP / RK4P with
// projection), the weighted space/time average of the field (or torque) at
// stage 1 of every step, and m_final; mode 1 evaluates H(m_init) once.  Each
// stage reads one stage-input buffer and writes the next stage input into the
// other, so a point's slope never goes through memory.  The solve uses the
// plane-walking kernel below; this one serves the field evaluation.
__global__ void __launch_bounds__(kThreads3d) k_micro3d(Micro3dArgs A) {
    const int box = A.box_ids[blockIdx.x];
    const BoxPlan P = A.plans[box];
    const int n = P.n, tid = threadIdx.x, nth = blockDim.x;
    Box3 B(A.work + P.tab_offset, n);
    const long C = B.C, X = B.X, nn = (long)n * n;
    const double *w = A.wts + P.w_offset;
    const double *wt = A.wt + P.wt_offset;
    const double alpha = P.alpha, dt = P.dt;
    const bool rk4 = (P.stages == 4);
    const long s1 = B.stride(1), s2 = B.stride(2);
    // this thread's points t = tid + k nth, walked with incremental coordinates
    const int d0 = nth % n, d1 = (nth / n) % n, d2 = (int)(nth / nn);
    const int b0 = tid % n, b1 = (tid / n) % n, b2 = (int)(tid / nn);
    auto advance = [&](int &i0, int &i1, int &i2) {
        i0 += d0;
        if (i0 >= n) { i0 -= n; ++i1; }
        i1 += d1;
        if (i1 >= n) { i1 -= n; ++i2; }
        i2 += d2;
    };

    // H = div(a grad y) at the interior point with extended index e
    auto field = [&](const double *y, long e, double H[3]) {
        const double ae0 = B.A[e], aw0 = B.A[e - 1];
        const double ae1 = B.A[X + e], aw1 = B.A[X + e - s1];
        const double ae2 = B.A[2 * X + e], aw2 = B.A[2 * X + e - s2];
        for (int c = 0; c < 3; ++c) {
            const double *yc = y + c * X;
            const double v = yc[e];
            double h = ae0 * (yc[e + 1] - v) - aw0 * (v - yc[e - 1]);
            h += ae1 * (yc[e + s1] - v) - aw1 * (v - yc[e - s1]);
            h += ae2 * (yc[e + s2] - v) - aw2 * (v - yc[e - s2]);
            H[c] = h;
        }
    };

    if (A.mode == 1) {
        int i0 = b0, i1 = b1, i2 = b2;
        for (long t = tid; t < C; t += nth, advance(i0, i1, i2)) {
            double H[3];
            field(B.y, B.ext(i0, i1, i2), H);
            for (int c = 0; c < 3; ++c) A.out_field[P.mfinal_offset + c * C + t] = H[c];
        }
        return;
    }

    double sum[3] = {0.0, 0.0, 0.0};   // this thread's share of the average
    const int nst = rk4 ? 4 : 2;
    double *ycur = B.y, *ynext = B.y1;
    for (int step = 0; step <= P.M; ++step) {
        const double wn = wt[step];
        for (int s = 0; s < nst; ++s) {
            const double bs = rk4 ? ((s == 0 || s == 3) ? 1.0 / 6.0 : 1.0 / 3.0) : 0.5;
            const double cnext = rk4 ? ((s < 2) ? 0.5 : 1.0) : 1.0;
            int i0 = b0, i1 = b1, i2 = b2;
            for (long t = tid; t < C; t += nth, advance(i0, i1, i2)) {
                const long e = B.ext(i0, i1, i2);
                double H[3];
                field(ycur, e, H);
                const double yv[3] = {ycur[e], ycur[X + e], ycur[2 * X + e]};
                double c1[3], c2[3];
                c1[0] = yv[1] * H[2] - yv[2] * H[1];
                c1[1] = yv[2] * H[0] - yv[0] * H[2];
                c1[2] = yv[0] * H[1] - yv[1] * H[0];
                if (s == 0) {
                    const double wc = w[i0] * w[i1] * w[i2] * wn;
                    if (P.quantity == LLHMM_Q_TORQUE)
                        for (int c = 0; c < 3; ++c) sum[c] += wc * c1[c];
                    else
                        for (int c = 0; c < 3; ++c) sum[c] += wc * H[c];
                }
                if (step == P.M) continue;
                c2[0] = yv[1] * c1[2] - yv[2] * c1[1];
                c2[1] = yv[2] * c1[0] - yv[0] * c1[2];
                c2[2] = yv[0] * c1[1] - yv[1] * c1[0];
                if (s < nst - 1) {
                    for (int c = 0; c < 3; ++c) {
                        const double k = -c1[c] - alpha * c2[c];
                        B.acc[c * C + t] = (s == 0) ? bs * k : B.acc[c * C + t] + bs * k;
                        ynext[c * X + e] = B.m[c * C + t] + cnext * dt * k;
                    }
                } else {
                    double v[3];
                    for (int c = 0; c < 3; ++c) {
                        const double k = -c1[c] - alpha * c2[c];
                        v[c] = B.m[c * C + t] + dt * (B.acc[c * C + t] + bs * k);
                    }
                    const double nr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    for (int c = 0; c < 3; ++c) {
                        B.m[c * C + t] = v[c] / nr;
                        ynext[c * X + e] = v[c] / nr;
                    }
                }
            }
            if (step == P.M) break;
            __syncthreads();
            // ghosts of the new stage input
            for (long g = tid; g < 6 * nn; g += nth) {
                long gi, wi;
                int q0, q1, q2;
                ghost_point(B, g, gi, wi, q0, q1, q2);
                for (int c = 0; c < 3; ++c)
                    ynext[c * X + gi] = (P.bc == LLHMM_BC_DIRICHLET) ? B.G[c * X + gi]
                                                                     : ynext[c * X + wi] + B.G[c * X + gi];
            }
            __syncthreads();
            double *tmp = ycur;
            ycur = ynext;
            ynext = tmp;
        }
    }

    // the box's average: fixed-order block reduction into its partial-sum slot
    __shared__ double s_red[kThreads3d][3];
    for (int c = 0; c < 3; ++c) s_red[tid][c] = sum[c];
    __syncthreads();
    for (int half = kThreads3d / 2; half > 0; half >>= 1) {
        if (tid < half)
            for (int c = 0; c < 3; ++c) s_red[tid][c] = s_red[tid][c] + s_red[tid + half][c];
        __syncthreads();
    }
    if (tid == 0) {
        double *dst = A.partials + P.part_offset * kMaxQ;
        int bad = 0;
        for (int q = 0; q < kMaxQ; ++q) {
            const double v = (q < 3) ? s_red[0][q] : 0.0;
            dst[q] = v;
            if (!__builtin_isfinite(v)) bad = 1;
        }
        A.wave_status[P.part_offset] = bad;
    }
    if (A.out_field) {
        for (long t = tid; t < C; t += nth)
            for (int c = 0; c < 3; ++c) A.out_field[P.mfinal_offset + c * C + t] = B.m[c * C + t];
    }
}

// The time loop walking each stage plane by plane (mode 0).  A block owns the
// whole (x1, x2) plane of its box at once (PT points per thread); the stage
// input of the plane below, the plane itself and the x3 face below stay in
// registers from one plane to the next, and the plane with its ghost ring is
// staged in LDS for the x1 / x2 neighbours.  NT threads per block, one point of
// the plane per thread (n <= 22: 512 threads, n <= 32: 1024).  Every array element then crosses
// HBM once per stage: the streamed bytes are the algorithmic ones.
template <int NMAX, int NT>
__global__ void __launch_bounds__(NT, 1) k_micro3d_planes(Micro3dArgs A) {
    constexpr int PT = (NMAX * NMAX + NT - 1) / NT;
    constexpr int PLMAX = (NMAX + 2) * (NMAX + 2);
    __shared__ double s_plane[3 * PLMAX];
    __shared__ double s_red[NT][3];
    const int box = A.box_ids[blockIdx.x];
    const BoxPlan P = A.plans[box];
    const int n = P.n, tid = threadIdx.x;
    Box3 B(A.work + P.tab_offset, n);
    const long C = B.C, X = B.X, nn = (long)n * n;
    const int E = B.E, PL = E * E;
    const long s1 = B.stride(1), s2 = B.stride(2);
    const double *w = A.wts + P.w_offset;
    const double *wt = A.wt + P.wt_offset;
    const double alpha = P.alpha, dt = P.dt;
    const bool rk4 = (P.stages == 4);
    const int nst = rk4 ? 4 : 2;
    // this thread's points of a plane: q = tid + j * threads, (i0, i1) = (q % n, q / n)
    int q0[PT], q1[PT], gside[PT];   // gside: -1 / +1 at the x1 ends of a row, else 0
    bool act[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int q = tid + j * NT;
        act[j] = q < nn;
        q0[j] = act[j] ? q % n : 0;
        q1[j] = act[j] ? q / n : 0;
        gside[j] = (q0[j] == 0) ? -1 : (q0[j] == n - 1 ? 1 : 0);
    }
    double sum[3] = {0.0, 0.0, 0.0};
    double *ycur = B.y, *ynext = B.y1;
    for (int step = 0; step <= P.M; ++step) {
        const double wn = wt[step];
        for (int s = 0; s < nst; ++s) {
            const double bs = rk4 ? ((s == 0 || s == 3) ? 1.0 / 6.0 : 1.0 / 3.0) : 0.5;
            const double cnext = rk4 ? ((s < 2) ? 0.5 : 1.0) : 1.0;
            const bool last_level = (step == P.M);
            // per point: the stage input of the plane below (ylo) and of the
            // plane itself (yc), the x3 face below (aw2) and, for points at the
            // x1 ends of a row, the row's ghost value (gx; it shares the cache
            // line that brings the point itself)
            double ylo[PT][3], yc[PT][3], aw2[PT], gx[PT][3];
#pragma unroll
            for (int j = 0; j < PT; ++j) {
                if (!act[j]) continue;
                const long elo = B.ext(q0[j], q1[j], -1), e0 = B.ext(q0[j], q1[j], 0);
                const long eg = e0 + gside[j];
                for (int c = 0; c < 3; ++c) {
                    ylo[j][c] = ycur[c * X + elo];
                    yc[j][c] = ycur[c * X + e0];
                    gx[j][c] = gside[j] ? ycur[c * X + eg] : 0.0;
                }
                aw2[j] = B.A[2 * X + elo];
            }
            for (int i2 = 0; i2 < n; ++i2) {
                // this plane's loads from memory (the plane above and the faces)
                // are issued before the staging barrier, so they are in flight
                // while the block synchronizes
                double yhi[PT][3], ghi[PT][3], fa[PT][5];
#pragma unroll
                for (int j = 0; j < PT; ++j) {
                    if (!act[j]) continue;
                    const long e = B.ext(q0[j], q1[j], i2);
                    for (int c = 0; c < 3; ++c) {
                        yhi[j][c] = ycur[c * X + e + s2];
                        ghi[j][c] = gside[j] ? ycur[c * X + e + s2 + gside[j]] : 0.0;
                    }
                    fa[j][0] = B.A[e];
                    fa[j][1] = B.A[e - 1];
                    fa[j][2] = B.A[X + e];
                    fa[j][3] = B.A[X + e - s1];
                    fa[j][4] = B.A[2 * X + e];
                }
                // the plane's stage input into LDS: own points and the x1 ghosts
                // from registers, the x2 ghost rows from memory
#pragma unroll
                for (int j = 0; j < PT; ++j) {
                    if (!act[j]) continue;
                    const int l = (q1[j] + 1) * E + (q0[j] + 1);
                    for (int c = 0; c < 3; ++c) s_plane[c * PL + l] = yc[j][c];
                    if (gside[j])
                        for (int c = 0; c < 3; ++c) s_plane[c * PL + l + gside[j]] = gx[j][c];
                }
                for (int g = tid; g < 2 * n; g += NT) {
                    const int i0 = g % n, i1 = (g < n) ? -1 : n;
                    const long e = B.ext(i0, i1, i2);
                    const int l = (i1 + 1) * E + (i0 + 1);
                    for (int c = 0; c < 3; ++c) s_plane[c * PL + l] = ycur[c * X + e];
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < PT; ++j) {
                    if (!act[j]) continue;
                    const int i0 = q0[j], i1 = q1[j];
                    const long e = B.ext(i0, i1, i2);
                    const long t = ((long)i2 * n + i1) * n + i0;
                    const int l = (i1 + 1) * E + (i0 + 1);
                    const double ae0 = fa[j][0], aw0 = fa[j][1];
                    const double ae1 = fa[j][2], aw1 = fa[j][3];
                    const double ae2 = fa[j][4];
                    double H[3];
                    for (int c = 0; c < 3; ++c) {
                        const double *pl = s_plane + c * PL;
                        const double v = yc[j][c];
                        double h = ae0 * (pl[l + 1] - v) - aw0 * (v - pl[l - 1]);
                        h += ae1 * (pl[l + E] - v) - aw1 * (v - pl[l - E]);
                        h += ae2 * (yhi[j][c] - v) - aw2[j] * (v - ylo[j][c]);
                        H[c] = h;
                    }
                    const double yv[3] = {yc[j][0], yc[j][1], yc[j][2]};
                    double c1[3], c2[3];
                    c1[0] = yv[1] * H[2] - yv[2] * H[1];
                    c1[1] = yv[2] * H[0] - yv[0] * H[2];
                    c1[2] = yv[0] * H[1] - yv[1] * H[0];
                    if (s == 0) {
                        const double wc = w[i0] * w[i1] * w[i2] * wn;
                        if (P.quantity == LLHMM_Q_TORQUE)
                            for (int c = 0; c < 3; ++c) sum[c] += wc * c1[c];
                        else
                            for (int c = 0; c < 3; ++c) sum[c] += wc * H[c];
                    }
                    if (!last_level) {
                        c2[0] = yv[1] * c1[2] - yv[2] * c1[1];
                        c2[1] = yv[2] * c1[0] - yv[0] * c1[2];
                        c2[2] = yv[0] * c1[1] - yv[1] * c1[0];
                        if (s == 0) {
                            for (int c = 0; c < 3; ++c) {
                                const double k = -c1[c] - alpha * c2[c];
                                B.acc[c * C + t] = bs * k;
                                ynext[c * X + e] = B.m[c * C + t] + cnext * dt * k;
                            }
                        } else if (s < nst - 1) {
                            for (int c = 0; c < 3; ++c) {
                                const double k = -c1[c] - alpha * c2[c];
                                B.acc[c * C + t] = B.acc[c * C + t] + bs * k;
                                ynext[c * X + e] = B.m[c * C + t] + cnext * dt * k;
                            }
                        } else {
                            double v[3];
                            for (int c = 0; c < 3; ++c) {
                                const double k = -c1[c] - alpha * c2[c];
                                v[c] = B.m[c * C + t] + dt * (B.acc[c * C + t] + bs * k);
                            }
                            const double nr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                            for (int c = 0; c < 3; ++c) {
                                B.m[c * C + t] = v[c] / nr;
                                ynext[c * X + e] = v[c] / nr;
                            }
                        }
                    }
                    // move up one plane
                    for (int c = 0; c < 3; ++c) {
                        ylo[j][c] = yc[j][c];
                        yc[j][c] = yhi[j][c];
                        gx[j][c] = ghi[j][c];
                    }
                    aw2[j] = ae2;
                }
                __syncthreads();  // the plane buffer is rewritten next
            }
            if (last_level) break;
            // ghosts of the new stage input
            for (long g = tid; g < 6 * nn; g += NT) {
                long gi, wi;
                int r0, r1, r2;
                ghost_point(B, g, gi, wi, r0, r1, r2);
                for (int c = 0; c < 3; ++c)
                    ynext[c * X + gi] = (P.bc == LLHMM_BC_DIRICHLET) ? B.G[c * X + gi]
                                                                     : ynext[c * X + wi] + B.G[c * X + gi];
            }
            __syncthreads();
            double *tmp = ycur;
            ycur = ynext;
            ynext = tmp;
        }
    }

    // the box's average: fixed-order block reduction into its partial-sum slot
    for (int c = 0; c < 3; ++c) s_red[tid][c] = sum[c];
    __syncthreads();
    for (int half = NT / 2; half > 0; half >>= 1) {
        if (tid < half)
            for (int c = 0; c < 3; ++c) s_red[tid][c] = s_red[tid][c] + s_red[tid + half][c];
        __syncthreads();
    }
    if (tid == 0) {
        double *dst = A.partials + P.part_offset * kMaxQ;
        int bad = 0;
        for (int q = 0; q < kMaxQ; ++q) {
            const double v = (q < 3) ? s_red[0][q] : 0.0;
            dst[q] = v;
            if (!__builtin_isfinite(v)) bad = 1;
        }
        A.wave_status[P.part_offset] = bad;
    }
    if (A.out_field) {
        for (long t = tid; t < C; t += NT)
            for (int c = 0; c < 3; ++c) A.out_field[P.mfinal_offset + c * C + t] = B.m[c * C + t];
    }
}

hipError_t launch_setup3d(const Micro3dArgs &a, hipStream_t s) {
    if (a.nbox <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_setup3d, dim3(a.nbox), dim3(kThreads3d), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_micro3d(const Micro3dArgs &a, hipStream_t s) {
    if (a.nbox <= 0) return hipSuccess;
    // field evaluation, and boxes above 32 points per axis (whose plane would take
    // 4 or more points per thread and spill): the point-by-point kernel
    if (a.mode == 1 || a.nmax > 32) {
        hipLaunchKernelGGL(k_micro3d, dim3(a.nbox), dim3(kThreads3d), 0, s, a);
    } else if (a.nmax <= 22) {
        hipLaunchKernelGGL((k_micro3d_planes<22, 512>), dim3(a.nbox), dim3(512), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_micro3d_planes<32, 1024>), dim3(a.nbox), dim3(1024), 0, s, a);
    }
    return hipGetLastError();
}

int64_t work3d_size(int n) {
    const int64_t E = n + 2;
    return 12 * E * E * E + 6 * (int64_t)n * n * n;
}

}  // namespace llhmm
