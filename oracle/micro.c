/*
 * FP64 CPU oracle: time stepping and averaging of ONE micro problem.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain loops, no blocking,
 * no fusion, no reordering beyond what the paper's definitions state.
 *
 * Paper passages followed (Leitenmaier & Runborg, HMM for the LL equation):
 *   - micro problem eq. (micro), Section 2.2: dm/dt = -m x H - alpha m x (m x H),
 *     H = div(a grad m), on [-mu', mu']^d x [0, eta];
 *   - second-order central difference for div(a grad m) (Section 2.3 and the
 *     opening of Section 4); an optional fourth-order conservative variant;
 *   - boundary conditions of Section 4.2: periodic m - m_init, or Dirichlet
 *     m = m_init on the ghost points;
 *   - HeunP and RK4P (Section 3.1): Runge-Kutta stages, then projection
 *     m <- m / |m| every step.  Readings: HeunP's second stage uses the full
 *     step m + dt k1 (the printed half step would make the method first
 *     order, contradicting its stated second order); RK4's third stage is
 *     k3 = f(m + dt/2 k2) (the printed "k_2" there is a typo);
 *   - upscaling eq. (upscaling), Section 2.3: H_avg = sum_n w^n sum_j w_j Q_j(m^n)
 *     with Q the discrete field H (field model), the face flux a grad m (flux
 *     model) or m x H (torque model), accumulated in index order.
 *
 * Grid (extended with G ghost layers per side): interior index i in [0, N),
 * extended side E = N + 2G, storage index ((i2+G)*E + (i1+G))*E + (i0+G)
 * (fewer terms for d < 3) with axis 0 fastest.  A[ax][idx] is the coefficient
 * on the face between cell idx and idx + e_ax.  m_init is given on the whole
 * extended grid.  d = 1, 2, 3 (the problem allows d <= 3, Section 2.1).
 *
 * Arithmetic type.  The oracle computes in `real`: FP64 by default.  Built with
 * -DORACLE_LONG_DOUBLE (x87 extended, 64-bit significand, unit roundoff 5.4e-20)
 * or -DORACLE_QUAD (binary128 via libquadmath, unit roundoff 9.6e-35) the same
 * algorithm runs in higher precision on the same FP64 inputs (faces, initial
 * data, weights, dx, dt, alpha) and returns FP64 outputs.  Those builds are the
 * higher-precision answers the FP64 parity bars are measured against: their
 * rounding is 2048 times (extended) or 1e18 times (binary128) smaller than any
 * FP64 implementation's.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#if defined(ORACLE_QUAD)
#include <quadmath.h>
typedef __float128 real;
#define R_SQRT sqrtq
#define R_FABS fabsq
#define R_POW powq
#define R_FINITE(x) finiteq(x)
#elif defined(ORACLE_LONG_DOUBLE)
typedef long double real;
#define R_SQRT sqrtl
#define R_FABS fabsl
#define R_POW powl
#define R_FINITE(x) isfinite(x)
#else
typedef double real;
#define R_SQRT sqrt
#define R_FABS fabs
#define R_POW pow
#define R_FINITE(x) isfinite(x)
#endif

#define GW 3 /* ghost width: the fourth-order stencil reaches 3 cells */

typedef struct {
    int d, N, E, order, bc;
    long cells_ext;
    real dx;
    const double *A;     /* [d][E^d] */
    const double *minit; /* [3][E^d] */
} grid_t;

static long ext_index3(const grid_t *g, int i0, int i1, int i2) {
    if (g->d == 1) return (long)(i0 + GW);
    if (g->d == 2) return (long)(i1 + GW) * g->E + (i0 + GW);
    return ((long)(i2 + GW) * g->E + (i1 + GW)) * g->E + (i0 + GW);
}

static long axis_stride(const grid_t *g, int ax) {
    return ax == 0 ? 1 : (ax == 1 ? g->E : (long)g->E * g->E);
}

/* interior extents along axes 1 and 2 (1 when the axis does not exist) */
static int ext_n1(const grid_t *g) { return g->d >= 2 ? g->N : 1; }
static int ext_n2(const grid_t *g) { return g->d >= 3 ? g->N : 1; }

/* Fill the ghost layers of y (3 components, extended storage) from its interior:
 * for each axis, the ghost points whose other coordinates are interior. */
static void fill_ghosts(const grid_t *g, real *y) {
    const int N = g->N;
    for (int ax = 0; ax < g->d; ++ax) {
        int na = (g->d >= 2) ? N : 1; /* first other axis */
        int nb = (g->d >= 3) ? N : 1; /* second other axis */
        for (int ob = 0; ob < nb; ++ob)
            for (int oa = 0; oa < na; ++oa) {
                for (int gi = -GW; gi < N + GW; ++gi) {
                    if (gi >= 0 && gi < N) continue;
                    int wrap = ((gi % N) + N) % N;
                    long gidx, widx;
                    if (ax == 0) {
                        gidx = ext_index3(g, gi, oa, ob);
                        widx = ext_index3(g, wrap, oa, ob);
                    } else if (ax == 1) {
                        gidx = ext_index3(g, oa, gi, ob);
                        widx = ext_index3(g, oa, wrap, ob);
                    } else {
                        gidx = ext_index3(g, oa, ob, gi);
                        widx = ext_index3(g, oa, ob, wrap);
                    }
                    for (int c = 0; c < 3; ++c) {
                        const double *mi = g->minit + c * g->cells_ext;
                        real *yc = y + c * g->cells_ext;
                        if (g->bc == 0) /* periodic perturbation m - m_init */
                            yc[gidx] = yc[widx] + ((real)mi[gidx] - (real)mi[widx]);
                        else            /* Dirichlet: m = m_init on ghosts */
                            yc[gidx] = mi[gidx];
                    }
                }
            }
    }
}

/* Discrete gradient of component array yc on face idx (between idx and idx+s), times a. */
static real face_flux(const grid_t *g, const real *yc, long idx, int ax) {
    long s = axis_stride(g, ax);
    real a = g->A[ax * g->cells_ext + idx];
    if (g->order == 2) {
        return a * (yc[idx + s] - yc[idx]) / g->dx;
    }
    real gp = 27.0 * (yc[idx + s] - yc[idx]) - (yc[idx + 2 * s] - yc[idx - s]);
    return a * gp / (24.0 * g->dx);
}

/* H = div(a grad y) at interior cell idx (ghosts of y must be filled). */
static real field_at(const grid_t *g, const real *yc, long idx) {
    real h = 0.0;
    for (int ax = 0; ax < g->d; ++ax) {
        long s = axis_stride(g, ax);
        if (g->order == 2) {
            real fp = face_flux(g, yc, idx, ax);
            real fm = face_flux(g, yc, idx - s, ax);
            h += (fp - fm) / g->dx;
        } else {
            real f0 = face_flux(g, yc, idx, ax);
            real fm1 = face_flux(g, yc, idx - s, ax);
            real fp1 = face_flux(g, yc, idx + s, ax);
            real fm2 = face_flux(g, yc, idx - 2 * s, ax);
            h += (27.0 * (f0 - fm1) - (fp1 - fm2)) / (24.0 * g->dx);
        }
    }
    return h;
}

static void cross(const real *a, const real *b, real *out) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* H for every interior cell: H[c][ext idx].  y gets its ghosts filled first. */
static void field_all(const grid_t *g, real *y, real *H) {
    fill_ghosts(g, y);
    int n1 = ext_n1(g), n2 = ext_n2(g);
    for (int c = 0; c < 3; ++c)
        for (int i2 = 0; i2 < n2; ++i2)
            for (int i1 = 0; i1 < n1; ++i1)
                for (int i0 = 0; i0 < g->N; ++i0) {
                    long idx = ext_index3(g, i0, i1, i2);
                    H[c * g->cells_ext + idx] = field_at(g, y + c * g->cells_ext, idx);
                }
}

/* f(y) = -y x H - alpha y x (y x H) for every interior cell; also returns H. */
static void rhs_all(const grid_t *g, real alpha, real *y, real *H, real *f) {
    field_all(g, y, H);
    int n1 = ext_n1(g), n2 = ext_n2(g);
    long ce = g->cells_ext;
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1)
            for (int i0 = 0; i0 < g->N; ++i0) {
                long idx = ext_index3(g, i0, i1, i2);
                real m[3] = {y[idx], y[ce + idx], y[2 * ce + idx]};
                real h[3] = {H[idx], H[ce + idx], H[2 * ce + idx]};
                real mxh[3], mxmxh[3];
                cross(m, h, mxh);
                cross(m, mxh, mxmxh);
                for (int c = 0; c < 3; ++c) f[c * ce + idx] = -mxh[c] - alpha * mxmxh[c];
            }
}

/* Product weight of cell (i0, i1, i2): w_c along every axis except `face_ax`,
 * where the east-face weight w_f is used (face_ax = -1: cell weight everywhere). */
static real weight(const grid_t *g, const double *wc, const double *wf, int face_ax,
                   int i0, int i1, int i2) {
    const int idx[3] = {i0, i1, i2};
    real w = 1.0;
    for (int ax = 0; ax < g->d; ++ax) {
        real f = (ax == face_ax) ? wf[idx[ax]] : wc[idx[ax]];
        w = (ax == 0) ? f : w * f;
    }
    return w;
}

/* Quantity sum at one time level: out3d[...] += wt * sum_j w_j Q_j.  The boxes
 * are cubes, so every axis uses the same cell weights wc and face weights wf. */
static void accumulate(const grid_t *g, int quantity, real wt, real *y, real *H,
                       const double *wc, const double *wf, real *out) {
    field_all(g, y, H);
    int n1 = ext_n1(g), n2 = ext_n2(g);
    long ce = g->cells_ext;
    if (quantity == 1) { /* flux model: a grad m on the east face of each cell */
        for (int ax = 0; ax < g->d; ++ax)
            for (int c = 0; c < 3; ++c) {
                real s = 0.0;
                for (int i2 = 0; i2 < n2; ++i2)
                    for (int i1 = 0; i1 < n1; ++i1)
                        for (int i0 = 0; i0 < g->N; ++i0) {
                            long idx = ext_index3(g, i0, i1, i2);
                            real w = weight(g, wc, wf, ax, i0, i1, i2);
                            s += w * face_flux(g, y + c * ce, idx, ax);
                        }
                out[ax * 3 + c] += wt * s;
            }
        return;
    }
    for (int c = 0; c < 3; ++c) {
        real s = 0.0;
        for (int i2 = 0; i2 < n2; ++i2)
            for (int i1 = 0; i1 < n1; ++i1)
                for (int i0 = 0; i0 < g->N; ++i0) {
                    long idx = ext_index3(g, i0, i1, i2);
                    real w = weight(g, wc, wf, -1, i0, i1, i2);
                    real q;
                    if (quantity == 0) {
                        q = H[c * ce + idx];
                    } else { /* torque m x H */
                        real m[3] = {y[idx], y[ce + idx], y[2 * ce + idx]};
                        real h[3] = {H[idx], H[ce + idx], H[2 * ce + idx]};
                        real t[3];
                        cross(m, h, t);
                        q = t[c];
                    }
                    s += w * q;
                }
        out[c] += wt * s;
    }
}

static double energy(const grid_t *g, real *y) {
    fill_ghosts(g, y);
    int n1 = ext_n1(g), n2 = ext_n2(g);
    long ce = g->cells_ext;
    real e = 0.0;
    for (int ax = 0; ax < g->d; ++ax)
        for (int i2 = 0; i2 < n2; ++i2)
            for (int i1 = 0; i1 < n1; ++i1)
                for (int i0 = 0; i0 < g->N; ++i0) {
                    long idx = ext_index3(g, i0, i1, i2);
                    real a = g->A[ax * ce + idx];
                    for (int c = 0; c < 3; ++c) {
                        real fl = face_flux(g, y + c * ce, idx, ax);
                        /* fl = a * grad; energy density a |grad|^2 / 2 = fl^2 / (2a) */
                        e += 0.5 * fl * fl / a;
                    }
                }
    return (double)(e * R_POW(g->dx, g->d));
}

static double norm_dev(const grid_t *g, const real *y) {
    int n1 = ext_n1(g), n2 = ext_n2(g);
    long ce = g->cells_ext;
    real dev = 0.0;
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1)
            for (int i0 = 0; i0 < g->N; ++i0) {
                long idx = ext_index3(g, i0, i1, i2);
                real n = R_SQRT(y[idx] * y[idx] + y[ce + idx] * y[ce + idx] + y[2 * ce + idx] * y[2 * ce + idx]);
                real d = R_FABS(n - 1.0);
                if (d > dev) dev = d;
            }
    return (double)dev;
}

static long cells_ext_of(int d, int E) {
    return (d == 1) ? (long)E : (d == 2 ? (long)E * E : (long)E * E * E);
}

/* Copy the interior of an extended [3][E^d] array into a packed [3][N^d] one. */
static void pack_interior(const grid_t *g, const real *src, double *dst) {
    int n1 = ext_n1(g), n2 = ext_n2(g);
    long nc = (long)g->N * n1 * n2;
    for (int c = 0; c < 3; ++c)
        for (int i2 = 0; i2 < n2; ++i2)
            for (int i1 = 0; i1 < n1; ++i1)
                for (int i0 = 0; i0 < g->N; ++i0)
                    dst[c * nc + ((long)i2 * n1 + i1) * g->N + i0] =
                        (double)src[c * g->cells_ext + ext_index3(g, i0, i1, i2)];
}

/* Evaluate H(y) once; y_ext [3][E^d] (interior used, ghosts refilled), H_out [3][N^d]. */
int oracle_eval_field(int d, int N, int order, int bc, double dx, const double *A,
                      const double *minit, const double *y_ext, double *H_out) {
    grid_t g = {d, N, N + 2 * GW, order, bc, 0, (real)dx, A, minit};
    g.cells_ext = cells_ext_of(d, g.E);
    real *y = malloc(sizeof(real) * 3 * g.cells_ext);
    real *H = calloc(3 * g.cells_ext, sizeof(real));
    for (long t = 0; t < 3 * g.cells_ext; ++t) y[t] = y_ext[t];
    field_all(&g, y, H);
    pack_interior(&g, H, H_out);
    free(y);
    free(H);
    return 0;
}

/*
 * Solve one micro problem.
 *   integ: 1 = HeunP, 2 = RK4P; bc: 0 periodic m - m_init, 1 Dirichlet;
 *   quantity: 0 field, 1 flux, 2 torque; project: 1 normal, 0 off (tests only)
 *   wc: cell weights [N]; wf: east-face weights [N] (the same on every axis)
 *   wt: time weights [M+1]
 *   out: [3] or [3d] (flux: [axis][component]); mfinal [3][N^d] (nullable);
 *   energy_out, normdev_out: [M+1] (nullable)
 */
int oracle_solve_box(int d, int N, int order, int integ, int bc, int quantity, int project,
                     double dx, double alpha, double dt, int M,
                     const double *A, const double *minit, const double *wc, const double *wf,
                     const double *wt, double *out, double *mfinal,
                     double *energy_out, double *normdev_out) {
    grid_t g = {d, N, N + 2 * GW, order, bc, 0, (real)dx, A, minit};
    g.cells_ext = cells_ext_of(d, g.E);
    long ce = g.cells_ext;
    size_t bytes = sizeof(real) * 3 * ce;
    real *m = malloc(bytes), *y = malloc(bytes), *H = calloc(3 * ce, sizeof(real));
    real *k1 = calloc(3 * ce, sizeof(real)), *k2 = calloc(3 * ce, sizeof(real));
    real *k3 = calloc(3 * ce, sizeof(real)), *k4 = calloc(3 * ce, sizeof(real));
    for (long t = 0; t < 3 * ce; ++t) m[t] = minit[t]; /* interior = m_init; ghosts are refilled before use */
    int nq = (quantity == 1) ? 3 * d : 3;
    real acc[9];
    for (int q = 0; q < nq; ++q) acc[q] = 0.0;
    const real rdt = dt, ralpha = alpha;
    int n1 = ext_n1(&g), n2 = ext_n2(&g);

    for (int n = 0; n <= M; ++n) {
        accumulate(&g, quantity, wt[n], m, H, wc, wf, acc);
        if (energy_out) energy_out[n] = energy(&g, m);
        if (normdev_out) normdev_out[n] = norm_dev(&g, m);
        if (n == M) break;

        rhs_all(&g, ralpha, m, H, k1);
        if (integ == 1) { /* HeunP */
            for (long t = 0; t < 3 * ce; ++t) y[t] = m[t] + rdt * k1[t];
            rhs_all(&g, ralpha, y, H, k2);
            for (long t = 0; t < 3 * ce; ++t) m[t] = m[t] + 0.5 * rdt * (k1[t] + k2[t]);
        } else { /* RK4P */
            for (long t = 0; t < 3 * ce; ++t) y[t] = m[t] + 0.5 * rdt * k1[t];
            rhs_all(&g, ralpha, y, H, k2);
            for (long t = 0; t < 3 * ce; ++t) y[t] = m[t] + 0.5 * rdt * k2[t];
            rhs_all(&g, ralpha, y, H, k3);
            for (long t = 0; t < 3 * ce; ++t) y[t] = m[t] + rdt * k3[t];
            rhs_all(&g, ralpha, y, H, k4);
            for (long t = 0; t < 3 * ce; ++t)
                m[t] = m[t] + rdt / 6.0 * (k1[t] + 2.0 * k2[t] + 2.0 * k3[t] + k4[t]);
        }
        if (project) {
            for (int i2 = 0; i2 < n2; ++i2)
                for (int i1 = 0; i1 < n1; ++i1)
                    for (int i0 = 0; i0 < N; ++i0) {
                        long idx = ext_index3(&g, i0, i1, i2);
                        real nr = R_SQRT(m[idx] * m[idx] + m[ce + idx] * m[ce + idx] +
                                         m[2 * ce + idx] * m[2 * ce + idx]);
                        for (int c = 0; c < 3; ++c) m[c * ce + idx] /= nr;
                    }
        }
    }
    if (mfinal) pack_interior(&g, m, mfinal);
    free(m); free(y); free(H); free(k1); free(k2); free(k3); free(k4);
    int bad = 0;
    for (int q = 0; q < nq; ++q) {
        out[q] = (double)acc[q];
        if (!R_FINITE(acc[q])) bad = 1;
    }
    return bad ? 1 : 0;
}
