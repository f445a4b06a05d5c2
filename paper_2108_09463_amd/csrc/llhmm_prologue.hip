// Prologue kernel: builds the per-box tables the time-stepping kernel reads.
// All arithmetic in FP64; stored in the precision of the batch.
//
//   * micro grid xi_j = -mu' + j dx, dx = 2 mu' / n (micro domain of eq. (micro));
//   * face coefficients a^eps(x_b + xi + dx/2 e_axis), pre-multiplied by
//     1/dx^2 (second order) or 1/(24 dx)^2 (fourth order);
//   * micro initial data: sampled m_init, or the normalized fourth-order
//     interpolant Q_[4] = P_[4]/|P_[4]| of the macro field around the box's
//     macro node (Section 4.1, eq. (Q_k)): 5-node Lagrange basis in
//     s = xi/dX, along x1 then x2, periodic macro indices;
//   * boundary flux offsets tau_f = a'_f G_f(delta) for the faces whose
//     stencil reaches a ghost point, with delta = m_init(ghost) -
//     m_init(wrapped) for periodic m - m_init and delta = m_init(ghost) for
//     Dirichlet (Section 4.2);
//   * space weights K(xi/mu) dx/mu of the scaled kernel K_mu (Definition 2.3)
//     at points and at east faces.
#include "llhmm_internal.h"

namespace llhmm {

#pragma clang fp contract(off)
namespace {

__device__ __forceinline__ double grid_xi(const BoxPlan &P, int idx) {
    return -P.mu_box + (double)idx * P.dx;
}

__device__ double coef_closed(const CoefDev &c, double x0, double x1) {
    const double two_pi = 6.283185307179586;
    double a = c.c0;
    for (int t = 0; t < c.n_terms; ++t) {
        double p = c.amp[t];
        if (c.freq[t][0] != 0.0) p = p * sin(two_pi * c.freq[t][0] * x0 + c.phase[t][0]);
        if (c.dim == 2 && c.freq[t][1] != 0.0)
            p = p * sin(two_pi * c.freq[t][1] * x1 + c.phase[t][1]);
        a = a + p;
    }
    return a;
}

// Sine factors of a closed-form coefficient, tabulated once per box: for term
// t, S[(t * K + k) * len + idx] (K = 4 row kinds in 2-D, 2 in 1-D; len = n + 3)
// with k = 0: x1 factor at x1 faces f
// (idx f + 2), 1: x1 factor at points, 2: x2 factor at x2 faces, 3: x2 factor
// at points.  Each entry is the same expression coef_closed evaluates, so a
// coefficient built from the table is bit-identical to the direct one.
constexpr int kCoefTabTerms = 4;
// 2-D boxes have n <= 128 and four row kinds, 1-D boxes n <= 256 and two: one
// size fits both, small enough for four set-up blocks per CU
constexpr int kCoefTabSize = kCoefTabTerms * 4 * (128 + 3);
static_assert(kCoefTabTerms * 2 * (256 + 3) <= kCoefTabSize, "1-D sine tables");
struct CoefTables {
    const double *S;  // nullptr: evaluate directly
    int kinds, len;   // row kinds per term, entries per row
};

// a^eps on the face between point (i0, i1) and (i0, i1) + e_axis (unscaled).
__device__ double face_coef(const PrologueArgs &A, const BoxPlan &P, const CoefTables &CT, int axis, int i0,
                            int i1) {
    const int D = P.dim;
    if (P.coef_sampled) {
        const int E = P.n + 2 * kGhost;
        long idx = (D == 1) ? (long)(i0 + kGhost)
                            : (long)axis * E * E + (long)(i1 + kGhost) * E + (i0 + kGhost);
        return A.coef_samples[P.coef_offset + idx];
    }
    const CoefDev &c = A.coefs[P.coef_index];
    if (CT.S) {
        double a = c.c0;
        for (int t = 0; t < c.n_terms; ++t) {
            double p = c.amp[t];
            const double *St = CT.S + t * CT.kinds * CT.len;
            if (c.freq[t][0] != 0.0) p = p * (axis == 0 ? St[i0 + 2] : St[CT.len + i0]);
            if (c.dim == 2 && c.freq[t][1] != 0.0)
                p = p * (axis == 1 ? St[2 * CT.len + i1 + 2] : St[3 * CT.len + i1]);
            a = a + p;
        }
        return a;
    }
    double x0 = P.cx + grid_xi(P, i0);
    double x1 = (D == 2) ? P.cy + grid_xi(P, i1) : 0.0;
    if (axis == 0) x0 = x0 + 0.5 * P.dx;
    else x1 = x1 + 0.5 * P.dx;
    return coef_closed(c, x0, x1);
}

__device__ void lagrange5(double s, double Lb[5]) {
    for (int l = 0; l < 5; ++l) {
        double v = 1.0;
        for (int mm = 0; mm < 5; ++mm)
            if (mm != l) v = v * (s - (double)(mm - 2)) / (double)(l - mm);
        Lb[l] = v;
    }
}

// Per-block tables for Q_[4]: the 5^dim x 3 macro values around the box's
// macro node ([c][l0][l1] in 2-D, [c][l0] in 1-D) and the Lagrange basis at
// every grid index i = -3 .. n+2 ([(i + 3) * 5 + l]; the same grid along x1
// and x2).  Built once per box in LDS by init_tables.
struct InitTables {
    const double *Mloc;
    const double *Lb;   // basis along x1
    const double *Lb1;  // basis along x2 (2-D)
};

// Offset of the box centre from its macro node x_k = x0 + k dX along one axis.
// Q_[4] is evaluated at absolute positions, so a centre between nodes (the
// staggered flux points) shifts the Lagrange arguments; offsets within
// 1e-9 dX of zero are taken as zero (a centre given as i / n is the node).
__device__ double node_offset(double centre, double x0, int k, double dX) {
    const double o = centre - (x0 + (double)k * dX);
    return (fabs(o) <= 1e-9 * dX) ? 0.0 : o;
}

// m_init at grid point (i0, i1); ghost points allowed.
__device__ void minit_at(const PrologueArgs &A, const BoxPlan &P, const InitTables &T, int i0, int i1,
                         double out[3]) {
    const int D = P.dim;
    if (P.init_mode == LLHMM_INIT_EXPLICIT) {
        const int E = P.n + 2 * kGhost;
        const long cells = (D == 1) ? (long)E : (long)E * E;
        long idx = (D == 1) ? (long)(i0 + kGhost) : (long)(i1 + kGhost) * E + (i0 + kGhost);
        const double *src = A.m_init + P.init_offset;
        out[0] = src[idx];
        out[1] = src[cells + idx];
        out[2] = src[2 * cells + idx];
        return;
    }
    const double *L0 = T.Lb + (i0 + kGhost) * 5;
    double p[3] = {0.0, 0.0, 0.0};
    if (D == 1) {
        for (int l0 = 0; l0 < 5; ++l0)
            for (int c = 0; c < 3; ++c) p[c] = p[c] + T.Mloc[c * 5 + l0] * L0[l0];
    } else {
        const double *L1 = T.Lb1 + (i1 + kGhost) * 5;
        // kept rolled: unrolled, the 75 macro values and the basis stay live at
        // once and the kernel needs 300-400 VGPRs (one block per CU instead of three)
#pragma unroll 1
        for (int l1 = 0; l1 < 5; ++l1) {
            double q[3] = {0.0, 0.0, 0.0};
            for (int l0 = 0; l0 < 5; ++l0)  // along x1 first
                for (int c = 0; c < 3; ++c) q[c] = q[c] + T.Mloc[(c * 5 + l0) * 5 + l1] * L0[l0];
            for (int c = 0; c < 3; ++c) p[c] = p[c] + q[c] * L1[l1];
        }
    }
    double nr = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    out[0] = p[0] / nr;
    out[1] = p[1] / nr;
    out[2] = p[2] / nr;
}

// Ghost offset delta at point p along `axis` (other coordinate o); zero inside.
__device__ void ghost_delta(const PrologueArgs &A, const BoxPlan &P, const InitTables &T, int axis, int p,
                            int o, double out[3]) {
    const int N = P.n;
    if (p >= 0 && p < N) {
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    double g[3];
    if (axis == 0) minit_at(A, P, T, p, o, g);
    else minit_at(A, P, T, o, p, g);
    if (P.bc == LLHMM_BC_DIRICHLET) {
        out[0] = g[0]; out[1] = g[1]; out[2] = g[2];
        return;
    }
    int w = ((p % N) + N) % N;
    double h[3];
    if (axis == 0) minit_at(A, P, T, w, o, h);
    else minit_at(A, P, T, o, w, h);
    out[0] = g[0] - h[0];
    out[1] = g[1] - h[1];
    out[2] = g[2] - h[2];
}

// tau on face f (between points f and f+1 along `axis`) as a double word
// hi + lo = a' * G(delta) (lo is the rounding error of the product, exact by
// FMA): with Dirichlet data delta is O(1) and a' = O(dx^-2), so hi alone would
// carry an absolute error far above the flux's own rounding.
__device__ void face_tau(const PrologueArgs &A, const BoxPlan &P, const InitTables &T, const CoefTables &CT,
                         int axis, int f, int o, double hi[3], double lo[3]) {
    double a = face_coef(A, P, CT, axis, axis == 0 ? f : o, axis == 0 ? o : f) * P.a_scale;
    double dp1[3], d0[3], g[3];
    ghost_delta(A, P, T, axis, f + 1, o, dp1);
    ghost_delta(A, P, T, axis, f, o, d0);
    if (P.order == 2) {
        for (int c = 0; c < 3; ++c) g[c] = dp1[c] - d0[c];
    } else {
        double dp2[3], dm1[3];
        ghost_delta(A, P, T, axis, f + 2, o, dp2);
        ghost_delta(A, P, T, axis, f - 1, o, dm1);
        for (int c = 0; c < 3; ++c) g[c] = 27.0 * (dp1[c] - d0[c]) - (dp2[c] - dm1[c]);
    }
    for (int c = 0; c < 3; ++c) {
        hi[c] = a * g[c];
        lo[c] = __builtin_fma(a, g[c], -hi[c]);
    }
}

__device__ double kernel_space(const PrologueArgs &A, double x) {
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

}  // namespace

// Form-1 set-up scratch views (see scratch64_size).
struct Scratch64 {
    double *ax, *ay, *gx, *gy;
    int n, lines;
    __device__ Scratch64(double *base, int d, int n_) : n(n_) {
        lines = (d == 1) ? 1 : n;
        ax = base;
        ay = ax + (long)lines * (n + 3);
        gx = ay + (d == 2 ? (long)n * (n + 3) : 0);
        gy = gx + (long)lines * 18;
    }
};

// Reference value r at a ghost point (i0, i1), form 1.  Periodic m - m_init:
// r_g = r_w + m_init(g) - m_init(w), so that u = m - r is periodic with r_w the
// stored reference of the wrapped point w.  Dirichlet: r_g = m_init(g), so
// that u vanishes on the ghosts.
__device__ void ref_ghost(const PrologueArgs &A, const BoxPlan &P, const InitTables &T, int i0, int i1,
                          double out[3]) {
    const int N = P.n, D = P.dim;
    double g[3];
    minit_at(A, P, T, i0, i1, g);
    if (P.bc == LLHMM_BC_DIRICHLET) {
        for (int c = 0; c < 3; ++c) out[c] = g[c];
        return;
    }
    const int w0 = ((i0 % N) + N) % N, w1 = (D == 1) ? 0 : ((i1 % N) + N) % N;
    double h[3];
    minit_at(A, P, T, w0, w1, h);
    for (int c = 0; c < 3; ++c) {
        // stored reference of w: m_init(w) rounded to the batch precision
        const double rw = (P.prec == LLHMM_FP32) ? (double)(float)h[c] : h[c];
        out[c] = rw + (g[c] - h[c]);
    }
}

template <typename T>
__device__ __forceinline__ double ref_at(const BoxPlan &P, const T *tab, const TabLayout &L,
                                         const Scratch64 &S, int i0, int i1, int c) {
    const int N = P.n, D = P.dim;
    const long C = (D == 1) ? (long)N : (long)N * N;
    if (i0 < 0 || i0 >= N) {  // x1 ghost
        const int side = (i0 < 0) ? 0 : 1, layer = (i0 < 0) ? i0 + 3 : i0 - N;
        return S.gx[(((long)(D == 1 ? 0 : i1) * 2 + side) * 3 + layer) * 3 + c];
    }
    if (D == 2 && (i1 < 0 || i1 >= N)) {  // x2 ghost
        const int side = (i1 < 0) ? 0 : 1, layer = (i1 < 0) ? i1 + 3 : i1 - N;
        return S.gy[(((long)i0 * 2 + side) * 3 + layer) * 3 + c];
    }
    return (double)tab[L.ref + c * C + (long)(D == 1 ? 0 : i1) * N + i0];
}

// Flux a' G(r) on the face between (i0, i1) and (i0, i1) + e_axis, FP64.
template <typename T>
__device__ double ref_flux(const BoxPlan &P, const T *tab, const TabLayout &L, const Scratch64 &S,
                           int axis, int i0, int i1, int c) {
    const int s0 = (axis == 0), s1 = (axis == 1);
    const double a = (axis == 0) ? S.ax[(long)(P.dim == 1 ? 0 : i1) * (P.n + 3) + i0 + 2]
                                 : S.ay[(long)i0 * (P.n + 3) + i1 + 2];
    const double r0 = ref_at(P, tab, L, S, i0, i1, c);
    const double rp = ref_at(P, tab, L, S, i0 + s0, i1 + s1, c);
    if (P.order == 2) return a * (rp - r0);
    const double rpp = ref_at(P, tab, L, S, i0 + 2 * s0, i1 + 2 * s1, c);
    const double rm = ref_at(P, tab, L, S, i0 - s0, i1 - s1, c);
    return a * (27.0 * (rp - r0) - (rpp - rm));
}

template <typename T>
__global__ void __launch_bounds__(256, 4) k_prologue(PrologueArgs A) {
    const int box = blockIdx.x;
    const BoxPlan P = A.plans[box];
    if (P.dim == 3) return;  // d = 3 boxes have their own set-up kernel (k_setup3d)
    const int D = P.dim, N = P.n;
    const int lines = (D == 1) ? 1 : N;
    const long cells = (long)N * lines;
    const int GF = (P.order == 2) ? 1 : 3;
    const int FW = (P.order == 2) ? 1 : 2;
    const int FE = (P.order == 2) ? 0 : 1;
    const TabLayout L = tab_layout(D, N, P.form);
    T *tab = (T *)A.tabs + P.tab_offset;
    const int nth = blockDim.x, tid = threadIdx.x;
    __shared__ double s_red[4][kMaxQ];
    __shared__ double s_Mloc[75];
    __shared__ double s_Lb[kLagMax * 5];
    __shared__ double s_Lb1[kLagMax2 * 5];
    __shared__ double s_sin[kCoefTabSize];
    InitTables IT{s_Mloc, s_Lb, s_Lb1};
    CoefTables CT{nullptr, (D == 2) ? 4 : 2, N + 3};
    {
        const CoefDev &c = A.coefs[P.coef_index];
        if (!P.coef_sampled && c.n_terms <= kCoefTabTerms && c.n_terms * CT.kinds * CT.len <= kCoefTabSize) {
            // sine factors at every face and point position, once per box
            const double two_pi = 6.283185307179586;
            const int len = CT.len, kinds = CT.kinds;
            for (int t2 = tid; t2 < c.n_terms * kinds * len; t2 += nth) {
                const int t = t2 / (kinds * len), k = (t2 / len) % kinds, idx = t2 % len;
                const int ax = k / 2;
                const bool face = (k % 2) == 0;
                if (face ? idx > N + 2 : idx >= N) continue;
                const int gi = face ? idx - 2 : idx;
                if (ax == 1 && (c.dim != 2 || D != 2)) continue;
                double x = (ax == 0 ? P.cx : P.cy) + grid_xi(P, gi);
                if (face) x = x + 0.5 * P.dx;
                s_sin[(t * kinds + k) * len + idx] = sin(two_pi * c.freq[t][ax] * x + c.phase[t][ax]);
            }
            CT.S = s_sin;
        }
    }
    if (P.init_mode == LLHMM_INIT_MACRO_Q) {
        // the macro values around the node and the basis at every grid index, once per box
        const int nm = A.macro.n;
        const long npts = (D == 1) ? (long)nm : (long)nm * nm;
        const int nv = (D == 1) ? 15 : 75;
        for (int t = tid; t < nv; t += nth) {
            if (D == 1) {
                const int c = t / 5, l0 = t % 5;
                const int k0 = ((P.mi0 + l0 - 2) % nm + nm) % nm;
                s_Mloc[t] = A.M_macro[c * npts + k0];
            } else {
                const int c = t / 25, l0 = (t / 5) % 5, l1 = t % 5;
                const int k0 = ((P.mi0 + l0 - 2) % nm + nm) % nm, k1 = ((P.mi1 + l1 - 2) % nm + nm) % nm;
                s_Mloc[t] = A.M_macro[c * npts + (long)k0 * nm + k1];
            }
        }
        const double dX = A.macro.dX;
        const double o0 = node_offset(P.cx, A.macro.x0[0], P.mi0, dX);
        for (int i = tid; i < N + 2 * kGhost; i += nth) lagrange5((grid_xi(P, i - kGhost) + o0) / dX, s_Lb + i * 5);
        if (D == 2) {
            const double o1 = node_offset(P.cy, A.macro.x0[1], P.mi1, dX);
            for (int i = tid; i < N + 2 * kGhost; i += nth)
                lagrange5((grid_xi(P, i - kGhost) + o1) / dX, s_Lb1 + i * 5);
        }
    }
    __syncthreads();  // per-box tables written

    // initial state (form 0) or reference + residual (form 1)
    for (long p = tid; p < cells; p += nth) {
        double v[3];
        minit_at(A, P, IT, (int)(p % N), (int)(p / N), v);
        if (P.form == 0) {
            for (int c = 0; c < 3; ++c) tab[L.m0 + c * cells + p] = (T)v[c];
        } else {
            double n2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const T r = (T)v[c];
                tab[L.ref + c * cells + p] = r;
                tab[L.m0 + c * cells + p] = (T)(v[c] - (double)r);
                n2 = n2 + (double)r * (double)r;
            }
            tab[L.dm + p] = (T)(n2 - 1.0);
        }
    }
    // face coefficients: x1 faces of every line, x2 faces of every column
    const int nf = N + kFaceHalo;
    Scratch64 S64(A.scratch64 + (P.form == 1 ? P.s64_offset : 0), D, N);
    for (long t = tid; t < (long)lines * nf; t += nth) {
        int line = (int)(t / nf), f = (int)(t % nf) - 2;
        const double a = face_coef(A, P, CT, 0, f, line) * P.a_scale;
        tab[L.ax + t] = (T)a;
        if (P.form == 1) S64.ax[t] = a;
    }
    if (D == 2) {
        for (long t = tid; t < (long)N * nf; t += nth) {
            int col = (int)(t / nf), f = (int)(t % nf) - 2;
            const double a = face_coef(A, P, CT, 1, col, f) * P.a_scale;
            tab[L.ay + t] = (T)a;
            if (P.form == 1) S64.ay[t] = a;
        }
    }
    // space weights of the scaled kernel at points and east faces
    double *w = A.wts + P.w_offset;
    for (int i = tid; i < N; i += nth) {
        double xi = grid_xi(P, i);
        w[i] = kernel_space(A, xi / P.mu) * P.dx / P.mu;
        w[N + i] = kernel_space(A, (xi + 0.5 * P.dx) / P.mu) * P.dx / P.mu;
    }
    if (P.form == 0) {
        // boundary flux offsets, x1 then x2
        for (int axis = 0; axis < D; ++axis) {
            const int nl = (axis == 0) ? lines : N;
            for (long t = tid; t < (long)nl * 2 * 3; t += nth) {
                int line = (int)(t / 6), side = (int)((t / 3) % 2), q = (int)(t % 3);
                double hi[3] = {0.0, 0.0, 0.0}, lo[3] = {0.0, 0.0, 0.0};
                if (q < GF) {
                    int f = (side == 0) ? (-FW + q) : (N - GF + FE + q);
                    face_tau(A, P, IT, CT, axis, f, line, hi, lo);
                }
                T *dst = tab + (axis == 0 ? L.tau1 : L.tau2) + t * 8;
                for (int c = 0; c < 3; ++c) {
                    dst[c] = (T)hi[c];
                    dst[4 + c] = (T)lo[c];
                }
                dst[3] = (T)0;
                dst[7] = (T)0;
            }
        }
        if (tid < kMaxQ) A.box_const[(long)box * kMaxQ + tid] = 0.0;
        return;
    }
    // ghost references: x1 ghosts of every line, x2 ghosts of every column (3 components each)
    for (long t = tid; t < (long)lines * 6; t += nth) {
        const int line = (int)(t / 6), side = (int)((t / 3) % 2), layer = (int)(t % 3);
        const int i0 = (side == 0) ? layer - 3 : N + layer;
        ref_ghost(A, P, IT, i0, line, S64.gx + t * 3);
    }
    if (D == 2) {
        for (long t = tid; t < (long)N * 6; t += nth) {
            const int col = (int)(t / 6), side = (int)((t / 3) % 2), layer = (int)(t % 3);
            const int i1 = (side == 0) ? layer - 3 : N + layer;
            ref_ghost(A, P, IT, col, i1, S64.gy + t * 3);
        }
    }
    __syncthreads();  // reference values, scratch and weights written (form 1)
    // H0 = H(r) in FP64 and the time-independent part of the average:
    //   field: sum_j w_j H0_j; flux: sum_f w_f a'_f G_f(r); torque: 0 (accumulated whole)
    double acc[kMaxQ] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long p = tid; p < cells; p += nth) {
        const int i0 = (int)(p % N), i1 = (int)(p / N);
        const double wy = (D == 2) ? w[i1] : 1.0, wfy = (D == 2) ? w[N + i1] : 1.0;
        for (int c = 0; c < 3; ++c) {
            double h = 0.0;
            for (int ax = 0; ax < D; ++ax) {
                const int s0 = (ax == 0), s1 = (ax == 1);
                if (P.order == 2) {
                    h += ref_flux(P, tab, L, S64, ax, i0, i1, c) -
                         ref_flux(P, tab, L, S64, ax, i0 - s0, i1 - s1, c);
                } else {
                    const double f0 = ref_flux(P, tab, L, S64, ax, i0, i1, c);
                    const double fm1 = ref_flux(P, tab, L, S64, ax, i0 - s0, i1 - s1, c);
                    const double fp1 = ref_flux(P, tab, L, S64, ax, i0 + s0, i1 + s1, c);
                    const double fm2 = ref_flux(P, tab, L, S64, ax, i0 - 2 * s0, i1 - 2 * s1, c);
                    h += 27.0 * (f0 - fm1) - (fp1 - fm2);
                }
                if (P.quantity == LLHMM_Q_FLUX) {
                    const double wf = (ax == 0) ? w[N + i0] * wy : w[i0] * wfy;
                    acc[3 * ax + c] += wf * ref_flux(P, tab, L, S64, ax, i0, i1, c);
                }
            }
            tab[L.H0 + c * cells + p] = (T)h;
            if (P.quantity == LLHMM_Q_FIELD) acc[c] += w[i0] * wy * h;
        }
    }
    // fixed-order reduction: wavefront shuffles, then the four wave sums
    for (int q = 0; q < kMaxQ; ++q) {
        double v = acc[q];
        for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) == 0) s_red[tid >> 6][q] = v;
    }
    __syncthreads();
    if (tid < kMaxQ) A.box_const[(long)box * kMaxQ + tid] = (s_red[0][tid] + s_red[1][tid]) + (s_red[2][tid] + s_red[3][tid]);
}
#pragma clang fp contract(on)

hipError_t launch_prologue(int prec, const PrologueArgs &a, hipStream_t s) {
    if (a.nboxes <= 0) return hipSuccess;
    if (prec == LLHMM_FP32)
        hipLaunchKernelGGL(k_prologue<float>, dim3(a.nboxes), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_prologue<double>, dim3(a.nboxes), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace llhmm
