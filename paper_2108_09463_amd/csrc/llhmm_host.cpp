// Host side of libllhmm: validation, the stability rule, kernel coefficients,
// batch planning (tile class per box, table offsets, time weights) and the
// launches.  See include/llhmm.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "llhmm_internal.h"
#include "llhmm_micro3d.h"

using namespace llhmm;

namespace {

thread_local std::string g_err;

llhmm_status fail(llhmm_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(LLHMM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

// ------------------------------------------------------------- stability rule
// |R(z)|^2 - 1 at z = s(-alpha + i); R = Heun (RK2) or RK4 stability polynomial.
double growth(double s, double alpha, int integ) {
    const double zr = -alpha * s, zi = s;
    // powers of z
    const double z2r = zr * zr - zi * zi, z2i = 2.0 * zr * zi;
    double rr = 1.0 + zr + 0.5 * z2r, ri = zi + 0.5 * z2i;
    if (integ == LLHMM_RK4P) {
        const double z3r = z2r * zr - z2i * zi, z3i = z2r * zi + z2i * zr;
        const double z4r = z3r * zr - z3i * zi, z4i = z3r * zi + z3i * zr;
        rr += z3r / 6.0 + z4r / 24.0;
        ri += z3i / 6.0 + z4i / 24.0;
    }
    return rr * rr + ri * ri - 1.0;
}

// Largest r with |R(s(-alpha+i))| <= 1 for all s in [0, r]: scan (step 1e-3), then bisection.
double stability_radius(double alpha, int integ) {
    const double h = 1e-3;
    long k = 1;
    for (;; ++k) {
        if (growth(k * h, alpha, integ) > 0.0) break;
        if (k * h > 20.0) return -1.0;
    }
    double lo = (k - 1) * h, hi = k * h;
    for (int it = 0; it < 80; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (growth(mid, alpha, integ) > 0.0) hi = mid;
        else lo = mid;
    }
    return lo;
}

int resolve_integrator(int integ, double alpha) {
    if (integ == LLHMM_HEUNP || integ == LLHMM_RK4P) return integ;
    return alpha > 0.2 ? LLHMM_HEUNP : LLHMM_RK4P;
}

llhmm_status validate_box(const llhmm_box &b, int i, int ncoefs) {
    auto finite = [](double v) { return std::isfinite(v); };
    if (b.dim < 1 || b.dim > 3) return fail(LLHMM_E_INVALID, "box %d: dim must be 1, 2 or 3", i);
    if (b.n < 8 || (b.n & 1)) return fail(LLHMM_E_INVALID, "box %d: n must be even and >= 8", i);
    if (b.order != 2 && b.order != 4) return fail(LLHMM_E_INVALID, "box %d: order must be 2 or 4", i);
    if (b.integrator < 0 || b.integrator > 2) return fail(LLHMM_E_INVALID, "box %d: bad integrator", i);
    if (b.bc != 0 && b.bc != 1) return fail(LLHMM_E_INVALID, "box %d: bad bc", i);
    if (b.quantity < 0 || b.quantity > 2) return fail(LLHMM_E_INVALID, "box %d: bad quantity", i);
    if (b.init_mode != 0 && b.init_mode != 1) return fail(LLHMM_E_INVALID, "box %d: bad init_mode", i);
    if (b.n_steps < 0) return fail(LLHMM_E_INVALID, "box %d: n_steps < 0", i);
    if (b.coef_index < 0 || b.coef_index >= ncoefs)
        return fail(LLHMM_E_INVALID, "box %d: coef_index out of range", i);
    if (!(finite(b.eps) && b.eps > 0.0 && b.eps < 1.0))
        return fail(LLHMM_E_INVALID, "box %d: need 0 < eps < 1 (assumption A2)", i);
    if (!(finite(b.alpha) && b.alpha > 0.0))
        return fail(LLHMM_E_INVALID, "box %d: need alpha > 0 (damping)", i);
    if (!(finite(b.mu_box) && b.mu_box > 0.0)) return fail(LLHMM_E_INVALID, "box %d: need mu' > 0", i);
    if (!(finite(b.mu) && b.mu > 0.0 && b.mu <= b.mu_box))
        return fail(LLHMM_E_INVALID, "box %d: need 0 < mu <= mu'", i);
    if (!(finite(b.eta) && b.eta > 0.0)) return fail(LLHMM_E_INVALID, "box %d: need eta > 0", i);
    if (!(finite(b.a_max) && b.a_max > 0.0))
        return fail(LLHMM_E_INVALID, "box %d: need a_max > 0 (assumption A1)", i);
    if (!finite(b.center[0]) || !finite(b.center[1]) || !finite(b.center[2]))
        return fail(LLHMM_E_INVALID, "box %d: non-finite centre", i);
    if (b.init_mode == LLHMM_INIT_EXPLICIT && b.init_offset < 0)
        return fail(LLHMM_E_INVALID, "box %d: negative init_offset", i);
    if (b.init_mode == LLHMM_INIT_MACRO_Q && b.n + 2 * kGhost > (b.dim == 1 ? kLagMax : kLagMax2))
        return fail(LLHMM_E_INVALID, "box %d: macro-interpolated data needs n <= %d", i, b.dim == 1 ? 256 : 128);
    if (b.dim == 3 && b.n > kMaxN3)
        return fail(LLHMM_E_INVALID, "box %d: d = 3 boxes need n <= %d", i, kMaxN3);
    return LLHMM_OK;
}

// FP32 domain.  The FP32 path rounds its state, stencil, right-hand side and
// stored tables to FP32.  The upscaled average sums these roundings over the
// averaging region and the time steps; on wide, weakly damped boxes the average
// cancels so many digits that each rounding alone moves it by about 1e-5
// relative, and with an averaging radius below 2 eps too few points enter it
// for the rounding noise to average out (CPU emulation of the kernel's
// arithmetic).  No FP32 arrangement of the scheme holds the 1e-5 bar there, so
// such boxes are refused in FP32 (they are solved in FP64).
llhmm_status check_fp32_domain(const llhmm_box &b, int i, int precision) {
    if (precision != LLHMM_FP32) return LLHMM_OK;
    if (b.mu_box > LLHMM_FP32_MAX_WIDTH_EPS * b.eps * (1.0 + 1e-12) && b.alpha < LLHMM_FP32_MIN_ALPHA_WIDE)
        return fail(LLHMM_E_NOTSUP,
                    "box %d: FP32 cannot hold the 1e-5 bar on a weakly damped wide box (mu' = %.4g eps > %g eps "
                    "with alpha = %.3g < %g); solve it in FP64",
                    i, b.mu_box / b.eps, (double)LLHMM_FP32_MAX_WIDTH_EPS, b.alpha, (double)LLHMM_FP32_MIN_ALPHA_WIDE);
    if (b.mu < LLHMM_FP32_MIN_MU_EPS * b.eps * (1.0 - 1e-12))
        return fail(LLHMM_E_NOTSUP,
                    "box %d: FP32 cannot hold the 1e-5 bar with an averaging radius mu = %.4g eps < %g eps; "
                    "solve it in FP64",
                    i, b.mu / b.eps, (double)LLHMM_FP32_MIN_MU_EPS);
    if (b.order == 4 && b.eps * b.n < LLHMM_FP32_MIN_PPE_O4 * 2.0 * b.mu_box * (1.0 - 1e-12))
        return fail(LLHMM_E_NOTSUP,
                    "box %d: the fourth-order stencil in FP32 needs at least %g grid points per eps (here %.4g); "
                    "solve it in FP64",
                    i, (double)LLHMM_FP32_MIN_PPE_O4, b.eps * b.n / (2.0 * b.mu_box));
    return LLHMM_OK;
}

struct Planned {
    int integ, M;
    double dt;
};

llhmm_status plan_one(const llhmm_box &b, int i, Planned &out) {
    out.integ = resolve_integrator(b.integrator, b.alpha);
    if (b.n_steps > 0) {
        out.M = b.n_steps;
    } else {
        const double dx = 2.0 * b.mu_box / b.n;
        const double sigma = (b.order == 2) ? 4.0 : (7.0 / 3.0) * (7.0 / 3.0);
        const double omega = sigma * b.dim * b.a_max / (dx * dx);
        const double r = stability_radius(b.alpha, out.integ);
        if (!(r > 0.0)) return fail(LLHMM_E_INVALID, "box %d: no stability limit found", i);
        const double dt_max = 0.9 * r / omega;
        const double Md = std::ceil(b.eta / dt_max);
        if (!(Md >= 1.0 && Md < 2.0e9)) return fail(LLHMM_E_INVALID, "box %d: step count out of range", i);
        out.M = (int)Md;
    }
    out.dt = b.eta / out.M;
    return LLHMM_OK;
}

// ------------------------------------------------------------- kernel coefficients
// Moment conditions solved in binary128 (113-bit significand, Gaussian elimination
// with pivoting): the one-sided system is ill-conditioned (coefficients of size
// 1e9 for p = 3, q = 7), so double or x87 long double would lose the last digits.
typedef __float128 qreal;
qreal qabs(qreal v) { return v < 0 ? -v : v; }

llhmm_status kernel_coeffs(int p, int q, bool one_sided, double *out) {
    if (p < 0 || p > 7 || q < 0 || q > 30) return fail(LLHMM_E_INVALID, "kernel p in [0,7], q in [0,30]");
    const int n = p + 1;
    qreal A[8][9];
    // moment m of the weight: symmetric (1-x^2)^(q+1) on [-1,1]; one-sided t^(q+1)(1-t)^(q+1) on [0,1]
    auto moment = [&](int m) -> qreal {
        if (!one_sided) {
            if (m & 1) return 0;
            qreal s = 0, c = 1;  // sum_k C(q+1,k) (-1)^k 2/(2k+m+1)
            for (int k = 0; k <= q + 1; ++k) {
                s += c * 2 / (qreal)(2 * k + m + 1);
                c = -c * (qreal)(q + 1 - k) / (qreal)(k + 1);
            }
            return s;
        }
        // Beta(q+2+m, q+2) = (q+1+m)! (q+1)! / (2q+3+m)!
        qreal v = 1;
        const int a = q + 1 + m, b = q + 1;
        for (int k = 1; k <= b; ++k) v = v * (qreal)k / (qreal)(a + k);
        return v / (qreal)(a + b + 1);
    };
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) A[r][c] = moment(r + c);
        A[r][n] = (r == 0) ? 1 : 0;
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (qabs(A[r][c]) > qabs(A[piv][c])) piv = r;
        for (int k = 0; k <= n; ++k) std::swap(A[c][k], A[piv][k]);
        for (int r = 0; r < n; ++r) {
            if (r == c || A[r][c] == 0) continue;
            const qreal f = A[r][c] / A[c][c];
            for (int k = c; k <= n; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int r = 0; r < n; ++r) {
        qreal v = A[r][n] / A[r][r];
        if (!one_sided && (r & 1)) v = 0;  // odd coefficients vanish by symmetry
        out[r] = (double)v;
    }
    return LLHMM_OK;
}

double time_kernel(double t, const double *d, int p, int q) {
    if (!(t > 0.0 && t < 1.0)) return 0.0;
    double poly = 0.0, tp = 1.0;
    for (int i = 0; i <= p; ++i) {
        poly += d[i] * tp;
        tp *= t;
    }
    double f = 1.0;
    for (int i = 0; i < q + 1; ++i) f *= t * (1.0 - t);
    return f * poly;
}

// ------------------------------------------------------------- tile registry
struct TileKey {
    int prec, dim, n, order, bc, qty;
    bool operator<(const TileKey &o) const {
        return std::tie(prec, dim, n, order, bc, qty) < std::tie(o.prec, o.dim, o.n, o.order, o.bc, o.qty);
    }
};

const std::map<TileKey, const TileInfo *> &registry() {
    static std::map<TileKey, const TileInfo *> reg = [] {
        std::map<TileKey, const TileInfo *> r;
        const TileInfo *(*fns[])(int *) = {tiles_f32_2d, tiles_f64_2d, tiles_f32_1d, tiles_f64_1d};
        for (auto fn : fns) {
            int cnt = 0;
            const TileInfo *t = fn(&cnt);
            for (int i = 0; i < cnt; ++i) {
                TileKey k{t[i].prec, t[i].dim, t[i].n, t[i].order, t[i].bc, t[i].qty};
                if (!r.count(k)) r[k] = &t[i];
            }
        }
        return r;
    }();
    return reg;
}

struct SlabKey {
    int prec, n, order, bc, qty;
    bool operator<(const SlabKey &o) const {
        return std::tie(prec, n, order, bc, qty) < std::tie(o.prec, o.n, o.order, o.bc, o.qty);
    }
};

// Slab tile variants per class, in registration order (the first is the default).
const std::map<SlabKey, std::vector<const SlabTileInfo *>> &slab_registry() {
    static std::map<SlabKey, std::vector<const SlabTileInfo *>> reg = [] {
        std::map<SlabKey, std::vector<const SlabTileInfo *>> r;
        int cnt = 0;
        const SlabTileInfo *t = tiles_slab(&cnt);
        for (int i = 0; i < cnt; ++i) r[SlabKey{t[i].prec, t[i].n, t[i].order, t[i].bc, t[i].qty}].push_back(&t[i]);
        return r;
    }();
    return reg;
}

// Slab geometry of an n x n box for a tile whose window holds WR = R * NG rows,
// with `stages` Runge-Kutta stages per step and an exchange every `spe` steps:
// h halo rows on each side (each stage moves the error of the zeros beyond the
// window inwards by the stencil's reach, one row at second order and three at
// fourth, so h >= reach * spe * stages, rounded up to whole row groups), at most WR - 2h own rows per slab, the box's row groups split as
// evenly as possible over ns >= 2 slabs.  Every slab keeps h halo rows on each
// side (window rows beyond them stay unused) and publishes xd = h rows at each
// edge, which it must own.  ns = 0: invalid.
struct SlabGeom {
    int spe = 0, h = 0, ns = 0, xd = 0;
};

// exchange intervals in steps, each dividing kRerefSteps; 0: at every stage
constexpr int kSlabSpe[] = {0, 1, 2, 4, 8};
constexpr int kNumSpe = (int)(sizeof(kSlabSpe) / sizeof(kSlabSpe[0]));

SlabGeom slab_geom(const SlabTileInfo &t, int n, int stages, int spe) {
    SlabGeom g;
    const int WR = t.R * t.NG;
    if (n % t.R != 0 || spe < 0 || (spe > 0 && kRerefSteps % spe != 0)) return g;
    const int reach = (t.order == 2) ? 1 : 3;
    if (spe == 0) {
        // every stage (second order): no halo rows in the window; the slab's
        // first and last rows go to the neighbours after each stage
        if (t.order != 2) return g;
        const int groups = n / t.R;
        const int ns = (groups + t.NG - 1) / t.NG;
        if (ns < 2 || groups / ns * t.R < reach) return g;
        g.spe = 0;
        g.h = 0;
        g.ns = ns;
        g.xd = reach;
        return g;
    }
    const int h = (reach * spe * stages + t.R - 1) / t.R * t.R;
    const int capg = (WR - 2 * h) / t.R;  // own row groups per slab at most
    if (capg < 1) return g;
    const int groups = n / t.R;
    const int ns = (groups + capg - 1) / capg;
    const int own_min = groups / ns * t.R;
    const int xd = h;
    if (ns < 2 || own_min < xd) return g;
    g.spe = spe;
    g.h = h;
    g.ns = ns;
    g.xd = xd;
    return g;
}

// Own rows of slab s: the first (groups % ns) slabs take one row group more.
void slab_rows(const SlabTileInfo &t, int n, int ns, int s, int *o0, int *rows) {
    const int groups = n / t.R, base = groups / ns, extra = groups % ns;
    *o0 = (s * base + std::min(s, extra)) * t.R;
    *rows = (base + (s < extra ? 1 : 0)) * t.R;
}

// Exchange interval without tuning: fewest window rows computed per box, an
// exchange weighted as half a step of the window.  An exchange at every stage
// weighs a fifth of a step when interior rows (R >= 3) overlap its wait.
// Without them the wait is exposed: it weighs a step in FP64 and 1.2 steps in
// FP32, whose stages are cheaper.  Measured, the 32-row FP32 windows then keep
// one exchange per step (a quarter of their rows are halo), while the 16-row
// windows, half halo at one exchange per step, run up to twice as fast with
// the exchange at every stage (all FP64 classes; FP32 n = 112 with RK4P, not
// with HeunP, whose halo is half as deep).  -1: none fits.
int slab_default_spe(const SlabTileInfo &t, int n, int stages) {
    int best = -1;
    double best_cost = 0.0;
    for (int spe : kSlabSpe) {
        const SlabGeom g = slab_geom(t, n, stages, spe);
        if (g.ns == 0) continue;
        const double wait = (t.R >= 3) ? 0.2 : (t.prec == LLHMM_FP64 ? 1.0 : 1.2);
        const double cost = g.ns * (1.0 + (spe == 0 ? wait : 0.5 / spe));
        if (best < 0 || cost < best_cost) {
            best = spe;
            best_cost = cost;
        }
    }
    return best;
}

// 64-bit exchange words of a box: [slabs][2 edges][2 parities][xd rows][3][n],
// two words per value in FP64.
int64_t slab_xwords(const SlabTileInfo &t, int n, const SlabGeom &g) {
    return (int64_t)g.ns * 2 * 2 * g.xd * 3 * n * (t.prec == LLHMM_FP64 ? 2 : 1);
}

// Per-box reservations that fit every variant and exchange interval of the
// class (tuning swaps them without reallocating): partial-sum slots, exchange
// words and work items.
struct SlabReserve {
    int64_t slots = 0, xwords = 0, items = 0;
};

SlabReserve slab_reserve(const std::vector<const SlabTileInfo *> &variants, int n, int stages) {
    SlabReserve r;
    for (const SlabTileInfo *t : variants)
        for (int spe : kSlabSpe) {
            const SlabGeom g = slab_geom(*t, n, stages, spe);
            if (g.ns == 0) continue;
            r.slots = std::max<int64_t>(r.slots, (int64_t)g.ns * (t->threads / 64));
            r.xwords = std::max<int64_t>(r.xwords, slab_xwords(*t, n, g));
            r.items = std::max<int64_t>(r.items, g.ns);
        }
    return r;
}

template <typename T>
hipError_t dev_upload(T **dst, const T *src, size_t count) {
    *dst = nullptr;
    if (count == 0) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * count);
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice);
}

}  // namespace

using TuneKey = std::tuple<int, int, int, int, int>;  // precision, n, bc, quantity, stages
using TuneVal = std::pair<int, int>;                   // slab tile variant, steps per exchange

// Device memory reserved once and handed out in 256-byte aligned pieces
// (first fit, neighbouring free pieces merged on release).  The serving loop
// allocates its micro-batches here, so admitting work never calls hipMalloc.
struct Arena {
    static constexpr size_t kAlign = 256;
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_, taken_;  // offset -> bytes
    hipError_t init(size_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        hipError_t e = hipMalloc((void **)&base, bytes);
        if (e != hipSuccess) return e;
        size = bytes;
        free_[0] = bytes;
        return hipSuccess;
    }
    // Hands out memory the caller already owns (base must be kAlign-aligned).
    void init_external(char *mem, size_t bytes) {
        base = mem;
        size = bytes / kAlign * kAlign;
        used = 0;
        free_.clear();
        taken_.clear();
        free_[0] = size;
    }
    void *alloc(size_t bytes) {
        bytes = std::max<size_t>(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, left = it->second - bytes;
            free_.erase(it);
            if (left) free_[off + bytes] = left;
            taken_[off] = bytes;
            used += bytes;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p) {
        auto t = taken_.find((size_t)((char *)p - base));
        if (t == taken_.end()) return;
        size_t off = t->first, bytes = t->second;
        taken_.erase(t);
        used -= bytes;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + bytes) {
            bytes += nx->second;
            free_.erase(nx);
        }
        auto pv = free_.lower_bound(off);
        if (pv != free_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                off = pv->first;
                bytes += pv->second;
                free_.erase(pv);
            }
        }
        free_[off] = bytes;
    }
};

struct llhmm_ctx {
    int device;
    char *scratch = nullptr;           // this device's copy of the allocation-free solve's scratch array
    std::map<TuneKey, TuneVal> tuned;  // slab classes: tile variant from llhmm_batch_tune
};

struct ClassLaunch {
    const TileInfo *tile;
    int first, count, nblocks;  // range in the concatenated box-id list
    double cost;                // cell-stage estimate, for spreading classes over streams
};

struct SlabClass {
    const SlabTileInfo *tile;
    SlabGeom geom;                // shared by the class's boxes (same n, stages and interval)
    int stages;
    int first, count;             // range of (box, slab) items in the concatenated job list
    int nq;                       // work queues, one per XCD
    int qoff[kMaxXcc + 1];        // queue q: items [first + qoff[q], first + qoff[q + 1])
    int index;                    // class index: its counters and abort word in slab_sync
    double cost;
};

constexpr int kSlabSyncInts = 16;  // per class in slab_sync: kMaxXcc queue counters, abort word, padding

// Polls before a wait for a neighbouring slab gives up (about a minute at the
// poll interval); LLHMM_SLAB_SPIN_MAX overrides it (tests of the give-up path).
long long slab_spin_max() {
    const char *e = getenv("LLHMM_SLAB_SPIN_MAX");
    return e ? std::max(0LL, atoll(e)) : (1LL << 26);
}

constexpr int kSideStreams = 3;   // extra streams a batch spreads its classes over

// Arguments a captured graph was built with; a call with other arguments captures again.
struct GraphArgs {
    const double *m_init, *M_macro, *coef;
    double *m_final, *H;
    int32_t *status;
    int32_t ld, has_macro;
    llhmm_macro macro;
    bool operator==(const GraphArgs &o) const { return memcmp(this, &o, sizeof *this) == 0; }
};

struct llhmm_batch {
    int nboxes, prec, dim_max, nmax;
    int ncu = 1;                                  // compute units of the device (slab grid size)
    int nxcc = 1;                                 // XCDs of the device (slab work queues)
    int64_t cell_steps;
    bool any_explicit, any_macro, any_sampled;
    std::vector<BoxPlan> plans_h;
    std::vector<ClassLaunch> classes;
    std::vector<SlabClass> slabs;
    std::vector<const SlabTileInfo *> slab_tile;  // per box; nullptr for resident boxes
    std::vector<int> slab_spe;                    // per slab box: steps between exchanges
    std::vector<int64_t> xoff_h;                  // per slab box: first exchange word
    BoxPlan *plans = nullptr;
    SlabJob *jobs = nullptr;
    uint64_t *xbuf = nullptr;                     // slab boxes' exchanged edge rows (tagged words)
    int64_t nxwords = 0;
    int32_t *slab_sync = nullptr;                 // per class: work counter, abort word
    int64_t nsync = 0;                            // int32 entries of slab_sync
    int nslab_boxes = 0;
    int32_t *box_ids = nullptr;
    int32_t *box3_ids = nullptr;                  // the d = 3 boxes
    int nbox3 = 0, nmax3 = 0;
    int nq3 = 3;                                  // largest number of outputs of a d = 3 box
    int orders3 = 0;                              // stencil orders of the d = 3 boxes (bit 0: 2, bit 1: 4)
    int sampled3 = 0;                             // a d = 3 box's coefficient is sampled
    double cost3 = 0.0;
    double *work3d = nullptr;                     // their work areas (work3d_size doubles each)
    CoefDev *coefs = nullptr;
    void *tabs = nullptr;
    double *wts = nullptr, *wt = nullptr, *partials = nullptr, *box_const = nullptr, *scratch64 = nullptr;
    int32_t *wave_status = nullptr, *status = nullptr;
    hipEvent_t ev[LLHMM_TIMING_SLOTS][3] = {};
    hipStream_t side[kSideStreams] = {};          // created on first use, default priority
    hipEvent_t fork = nullptr, join[kSideStreams] = {};
    Arena *arena = nullptr;                       // device memory source (nullptr: hipMalloc)
    bool async_upload = false;                    // host tables go up with hipMemcpyAsync on upload_stream
    hipStream_t upload_stream = nullptr;
    int max_lanes = 1 + kSideStreams;             // streams the classes may spread over
    hipStream_t cap_stream = nullptr;             // capture stream of llhmm_batch_run_graph
    hipGraphExec_t exec = nullptr;
    GraphArgs gargs{};
    bool capturing = false;
    bool timing = false;
    int64_t timed = 0;  // timed calls since timing was enabled
    double kc[8];
    int kp, kq;
};

static hipError_t balloc(llhmm_batch *b, void **p, size_t bytes) {
    if (b->arena) {
        *p = b->arena->alloc(bytes);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

// Host -> device copy of batch tables: synchronous, or ordered on the batch's
// upload stream (pageable source: consumed before the call returns).
static hipError_t bcopy_h2d(llhmm_batch *b, void *dst, const void *src, size_t bytes) {
    if (b->async_upload) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->upload_stream);
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
}

static void bfree(llhmm_batch *b, void *p) {
    if (!p) return;
    if (b->arena) b->arena->release(p);
    else (void)hipFree(p);
}

template <typename T>
static hipError_t bupload(llhmm_batch *b, T **dst, const T *src, size_t count) {
    *dst = nullptr;
    if (count == 0) return hipSuccess;
    hipError_t e = balloc(b, (void **)dst, sizeof(T) * count);
    if (e != hipSuccess) return e;
    return bcopy_h2d(b, *dst, src, sizeof(T) * count);
}

// Slab boxes: classes by tile; per class the (box, slab) items, the slabs of
// a box consecutive and the longest boxes first (LPT order), uploaded with the
// plans into the job buffer reserved at creation.  Drops a captured graph (its
// launches change).
static llhmm_status rebuild_slabs(llhmm_batch *b) {
    std::map<std::tuple<const SlabTileInfo *, int, int>, std::vector<int>> groups;  // tile, stages, interval
    for (int i = 0; i < b->nboxes; ++i) {
        const SlabTileInfo *t = b->slab_tile[i];
        if (!t) continue;
        BoxPlan &P = b->plans_h[i];
        const SlabGeom g = slab_geom(*t, P.n, P.stages, b->slab_spe[i]);
        if (g.ns == 0)
            return fail(LLHMM_E_INVALID, "box %d: n = %d has no slab geometry for %s every %d steps", i, P.n,
                        t->name, b->slab_spe[i]);
        P.strips = g.ns;
        P.nwaves = g.ns * (t->threads / 64);
        groups[std::make_tuple(t, P.stages, g.spe)].push_back(i);
    }
    b->slabs.clear();
    std::vector<SlabJob> jobs_h;
    for (auto &kv : groups) {
        auto &v = kv.second;
        std::stable_sort(v.begin(), v.end(), [&](int a, int c) {
            return (int64_t)b->plans_h[a].M * b->plans_h[a].stages > (int64_t)b->plans_h[c].M * b->plans_h[c].stages;
        });
        SlabClass sc;
        sc.tile = std::get<0>(kv.first);
        sc.stages = std::get<1>(kv.first);
        sc.geom = slab_geom(*sc.tile, b->plans_h[v[0]].n, sc.stages, std::get<2>(kv.first));
        sc.first = (int)jobs_h.size();
        sc.index = (int)b->slabs.size();
        sc.cost = 0.0;
        sc.nq = b->nxcc;
        const int WR = sc.tile->R * sc.tile->NG;
        // boxes onto the XCD queues, longest first onto the least loaded
        std::vector<std::vector<int>> q(sc.nq);
        std::vector<double> qload(sc.nq, 0.0);
        for (int i : v) {
            const int k = (int)(std::min_element(qload.begin(), qload.end()) - qload.begin());
            qload[k] += (double)b->plans_h[i].M * b->plans_h[i].stages;
            q[k].push_back(i);
        }
        for (int k = 0; k < sc.nq; ++k) {
            sc.qoff[k] = (int)jobs_h.size() - sc.first;
            for (int i : q[k]) {
                const BoxPlan &P = b->plans_h[i];
                for (int s = 0; s < sc.geom.ns; ++s) {
                    SlabJob J{};
                    J.box = i;
                    J.slab = s;
                    J.nslabs = sc.geom.ns;
                    slab_rows(*sc.tile, P.n, sc.geom.ns, s, &J.o0, &J.rows);
                    J.xoff = b->xoff_h[i];
                    jobs_h.push_back(J);
                }
                sc.cost += (double)P.M * P.stages * sc.geom.ns * WR * P.n;  // window rows computed
            }
        }
        sc.count = (int)jobs_h.size() - sc.first;
        for (int k = sc.nq; k <= kMaxXcc; ++k) sc.qoff[k] = sc.count;
        b->slabs.push_back(sc);
    }
    if (!jobs_h.empty()) HIP_TRY(bcopy_h2d(b, b->jobs, jobs_h.data(), sizeof(SlabJob) * jobs_h.size()));
    HIP_TRY(bcopy_h2d(b, b->plans, b->plans_h.data(), sizeof(BoxPlan) * b->plans_h.size()));
    if (b->exec) {
        HIP_TRY(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    return LLHMM_OK;
}

static llhmm_status scratch_address(int device, char **out);

extern "C" {

int32_t llhmm_abi_version(void) { return LLHMM_ABI_VERSION; }

const char *llhmm_last_error(void) { return g_err.c_str(); }

llhmm_status llhmm_create(llhmm_ctx **ctx, int32_t device) {
    if (!ctx) return fail(LLHMM_E_INVALID, "ctx is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(LLHMM_E_INVALID, "device %d out of range (%d)", device, n);
    HIP_TRY(hipSetDevice(device));
    char *scratch_dev = nullptr;
    const llhmm_status st = scratch_address(device, &scratch_dev);
    if (st != LLHMM_OK) return st;
    *ctx = new llhmm_ctx();
    (*ctx)->device = device;
    (*ctx)->scratch = scratch_dev;
    return LLHMM_OK;
}

llhmm_status llhmm_destroy(llhmm_ctx *ctx) {
    delete ctx;
    return LLHMM_OK;
}

llhmm_status llhmm_plan(const llhmm_box *boxes, int32_t nboxes, int32_t *n_steps_out,
                        double *dt_out, int32_t *integrator_out) {
    if (nboxes < 0 || (nboxes > 0 && !boxes)) return fail(LLHMM_E_INVALID, "bad box array");
    for (int i = 0; i < nboxes; ++i) {
        llhmm_status s = validate_box(boxes[i], i, 1 << 30);
        if (s != LLHMM_OK) return s;
        Planned p;
        s = plan_one(boxes[i], i, p);
        if (s != LLHMM_OK) return s;
        if (n_steps_out) n_steps_out[i] = p.M;
        if (dt_out) dt_out[i] = p.dt;
        if (integrator_out) integrator_out[i] = p.integ;
    }
    return LLHMM_OK;
}

llhmm_status llhmm_check_boxes(const llhmm_box *boxes, int32_t nboxes, int32_t ncoefs, int32_t precision,
                               int32_t *first_bad) {
    if (first_bad) *first_bad = -1;
    if (nboxes <= 0 || !boxes) return fail(LLHMM_E_INVALID, "empty batch");
    if (precision != LLHMM_FP64 && precision != LLHMM_FP32) return fail(LLHMM_E_INVALID, "bad precision");
    for (int i = 0; i < nboxes; ++i) {
        const llhmm_box &bx = boxes[i];
        llhmm_status s = validate_box(bx, i, ncoefs);
        Planned p;
        if (s == LLHMM_OK) s = plan_one(bx, i, p);
        if (s == LLHMM_OK && bx.dim == 3 && precision != LLHMM_FP64)
            s = fail(LLHMM_E_NOTSUP, "box %d: d = 3 boxes need FP64", i);
        if (s == LLHMM_OK) s = check_fp32_domain(bx, i, precision);
        if (s == LLHMM_OK && bx.dim != 3 &&
            registry().find(TileKey{precision, bx.dim, bx.n, bx.order, bx.bc, bx.quantity}) == registry().end() &&
            !(bx.dim == 2 && slab_registry().count(SlabKey{precision, bx.n, bx.order, bx.bc, bx.quantity})))
            s = fail(LLHMM_E_NOTSUP, "box %d: no kernel for precision %s, dim %d, n %d, order %d, bc %d, quantity %d",
                     i, precision == LLHMM_FP32 ? "fp32" : "fp64", bx.dim, bx.n, bx.order, bx.bc, bx.quantity);
        if (s != LLHMM_OK) {
            if (first_bad) *first_bad = i;
            return s;
        }
    }
    return LLHMM_OK;
}

llhmm_status llhmm_kernel_coeffs(const llhmm_kernel *K, double *c_space, double *d_time) {
    if (!K) return fail(LLHMM_E_INVALID, "kernel is NULL");
    llhmm_status s = LLHMM_OK;
    if (c_space) s = kernel_coeffs(K->p_x, K->q_x, false, c_space);
    if (s == LLHMM_OK && d_time) s = kernel_coeffs(K->p_t, K->q_t, true, d_time);
    return s;
}

static void batch_free(llhmm_batch *b) {
    if (!b) return;
    void *ptrs[] = {b->plans, b->box_ids, b->coefs, b->tabs, b->wts, b->wt, b->partials,
                    b->wave_status, b->status, b->box_const, b->scratch64, b->jobs,
                    b->xbuf, b->slab_sync, b->box3_ids, b->work3d};
    for (void *p : ptrs) bfree(b, p);
    for (auto &slot : b->ev)
        for (hipEvent_t e : slot)
            if (e) (void)hipEventDestroy(e);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    for (int i = 0; i < kSideStreams; ++i) {
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
        if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

static llhmm_status batch_create_impl(llhmm_ctx *ctx, const llhmm_box *boxes, int32_t nboxes,
                                      const llhmm_kernel *K, const llhmm_coef *coefs, int32_t ncoefs,
                                      int32_t precision, Arena *arena, int max_lanes, llhmm_batch **out,
                                      hipStream_t upload_stream = nullptr, bool async_upload = false);

llhmm_status llhmm_batch_create(llhmm_ctx *ctx, const llhmm_box *boxes, int32_t nboxes,
                                const llhmm_kernel *K, const llhmm_coef *coefs, int32_t ncoefs,
                                int32_t precision, llhmm_batch **out) {
    return batch_create_impl(ctx, boxes, nboxes, K, coefs, ncoefs, precision, nullptr, 1 + kSideStreams, out);
}

}  // extern "C"

static llhmm_status batch_create_impl(llhmm_ctx *ctx, const llhmm_box *boxes, int32_t nboxes,
                                      const llhmm_kernel *K, const llhmm_coef *coefs, int32_t ncoefs,
                                      int32_t precision, Arena *arena, int max_lanes, llhmm_batch **out,
                                      hipStream_t upload_stream, bool async_upload) {
    if (!ctx || !out) return fail(LLHMM_E_INVALID, "ctx/out is NULL");
    *out = nullptr;
    if (nboxes <= 0 || !boxes) return fail(LLHMM_E_INVALID, "empty batch");
    if (!K || !coefs || ncoefs <= 0) return fail(LLHMM_E_INVALID, "kernel/coefficients missing");
    if (precision != LLHMM_FP64 && precision != LLHMM_FP32) return fail(LLHMM_E_INVALID, "bad precision");
    if (K->p_x > 7 || K->p_t > 7) return fail(LLHMM_E_INVALID, "kernel order p must be <= 7");
    for (int c = 0; c < ncoefs; ++c) {
        const llhmm_coef &cf = coefs[c];
        if (cf.n_terms < 0 || cf.n_terms > LLHMM_MAX_TERMS || cf.dim < 1 || cf.dim > 3)
            return fail(LLHMM_E_INVALID, "coef %d: bad dim / n_terms", c);
    }
    HIP_TRY(hipSetDevice(ctx->device));
    double dcoef[8] = {0};
    int ncu = 0, nxcc = 1;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, ctx->device) != hipSuccess) nxcc = 1;
    llhmm_batch *b = new llhmm_batch();
    b->arena = arena;
    b->nxcc = std::min(std::max(1, nxcc), kMaxXcc);
    b->ncu = std::max(1, ncu);
    b->upload_stream = upload_stream;
    b->async_upload = async_upload;
    b->max_lanes = std::max(1, std::min(max_lanes, 1 + kSideStreams));
    b->nboxes = nboxes;
    b->prec = precision;
    llhmm_status st = kernel_coeffs(K->p_x, K->q_x, false, b->kc);
    if (st == LLHMM_OK) st = kernel_coeffs(K->p_t, K->q_t, true, dcoef);
    if (st != LLHMM_OK) {
        delete b;
        return st;
    }
    b->kp = K->p_x;
    b->kq = K->q_x;

    const auto &reg = registry();
    const auto &sregistry = slab_registry();
    const size_t tsize = (precision == LLHMM_FP32) ? sizeof(float) : sizeof(double);
    b->plans_h.resize(nboxes);
    std::vector<const TileInfo *> tile_of(nboxes);
    b->slab_tile.assign(nboxes, nullptr);
    b->slab_spe.assign(nboxes, 0);
    b->xoff_h.assign(nboxes, 0);
    int dim_max = 1, nmax = 0;
    for (int i = 0; i < nboxes; ++i) {
        dim_max = std::max(dim_max, boxes[i].dim);
        nmax = std::max(nmax, boxes[i].n);
    }
    b->dim_max = dim_max;
    b->nmax = nmax;
    int64_t tab_off = 0, w_off = 0, s64_off = 0, part_off = 0, work3_off = 0;
    int64_t xbuf_off = 0, max_items = 0;
    std::vector<int32_t> ids3;
    std::map<int, int64_t> wt_off_of_M;
    std::vector<double> wt_h;
    int64_t cell_steps = 0;
    for (int i = 0; i < nboxes; ++i) {
        const llhmm_box &bx = boxes[i];
        st = validate_box(bx, i, ncoefs);
        if (st == LLHMM_OK && coefs[bx.coef_index].dim != bx.dim)
            st = fail(LLHMM_E_INVALID, "box %d: coefficient dimension differs from box", i);
        Planned pl{};
        if (st == LLHMM_OK) st = plan_one(bx, i, pl);
        if (st != LLHMM_OK) {
            delete b;
            return st;
        }
        if (bx.dim == 3 && precision != LLHMM_FP64) {
            delete b;
            return fail(LLHMM_E_NOTSUP, "box %d: d = 3 boxes need FP64", i);
        }
        st = check_fp32_domain(bx, i, precision);
        if (st != LLHMM_OK) {
            delete b;
            return st;
        }
        auto it = reg.find(TileKey{precision, bx.dim, bx.n, bx.order, bx.bc, bx.quantity});
        const SlabTileInfo *bt = nullptr;
        SlabReserve sres;
        if (it == reg.end() && bx.dim == 2) {
            auto bit = sregistry.find(SlabKey{precision, bx.n, bx.order, bx.bc, bx.quantity});
            const int stages = (pl.integ == LLHMM_RK4P) ? 4 : 2;
            if (bit != sregistry.end()) {
                // the tuned variant and interval for this class, else the first
                // variant with its default interval
                int v = 0, spe = 0;
                auto tit = ctx->tuned.find(TuneKey{precision, bx.n, bx.bc, bx.quantity, stages});
                if (tit != ctx->tuned.end() && tit->second.first < (int)bit->second.size() &&
                    slab_geom(*bit->second[tit->second.first], bx.n, stages, tit->second.second).ns > 0) {
                    v = tit->second.first;
                    spe = tit->second.second;
                } else {
                    spe = slab_default_spe(*bit->second[0], bx.n, stages);
                }
                if (spe >= 0) {
                    bt = bit->second[v];
                    b->slab_spe[i] = spe;
                }
                sres = slab_reserve(bit->second, bx.n, stages);
            }
        }
        if (it == reg.end() && !bt && bx.dim != 3) {
            delete b;
            return fail(LLHMM_E_NOTSUP,
                        "box %d: no kernel for precision %s, dim %d, n %d, order %d, bc %d, quantity %d",
                        i, precision == LLHMM_FP32 ? "fp32" : "fp64", bx.dim, bx.n, bx.order, bx.bc,
                        bx.quantity);
        }
        tile_of[i] = (bt || bx.dim == 3) ? nullptr : it->second;
        b->slab_tile[i] = bt;
        BoxPlan &P = b->plans_h[i];
        memset(&P, 0, sizeof P);
        P.dim = bx.dim;
        P.n = bx.n;
        P.order = bx.order;
        P.stages = (pl.integ == LLHMM_RK4P) ? 4 : 2;
        P.bc = bx.bc;
        P.quantity = bx.quantity;
        P.init_mode = bx.init_mode;
        P.M = pl.M;
        P.coef_index = bx.coef_index;
        P.mi0 = bx.macro_index[0];
        P.mi1 = bx.macro_index[1];
        P.mi2 = bx.macro_index[2];
        P.nq = (bx.quantity == LLHMM_Q_FLUX) ? 3 * bx.dim : 3;
        P.coef_sampled = coefs[bx.coef_index].sampled ? 1 : 0;
        int64_t slots;
        if (bt) {
            // slabs and partial-sum slots follow the variant; reserve for the
            // largest slab count any variant gives
            P.slab = 1;
            slots = sres.slots;
        } else if (bx.dim == 3) {
            P.nwaves = 1;
            slots = 1;
        } else {
            P.nwaves = (bx.dim == 2) ? it->second->threads / 64 : 1;
            slots = P.nwaves;
        }
        P.part_offset = part_off;
        part_off += slots;
        if (bt) {
            b->xoff_h[i] = xbuf_off;
            xbuf_off += sres.xwords;
            max_items += sres.items;
            ++b->nslab_boxes;
        }
        P.prec = precision;
        P.form = (precision == LLHMM_FP32 || P.slab || (tile_of[i] && (tile_of[i]->opt & kOptForm1))) ? 1 : 0;
        if (bx.dim == 3) P.form = 0;
        P.dt = pl.dt;
        P.alpha = bx.alpha;
        P.dx = 2.0 * bx.mu_box / bx.n;
        P.mu = bx.mu;
        P.mu_box = bx.mu_box;
        P.a_scale = (bx.order == 2) ? 1.0 / (P.dx * P.dx) : 1.0 / (576.0 * P.dx * P.dx);
        P.out_scale = (bx.quantity == LLHMM_Q_FLUX) ? ((bx.order == 2) ? P.dx : 24.0 * P.dx) : 1.0;
        P.cx = bx.center[0];
        P.cy = bx.center[1];
        P.cz = bx.center[2];
        P.init_offset = bx.init_offset;
        P.coef_offset = bx.coef_offset;
        // per-box stride 3 nmax^dim_max (largest n and d of the batch)
        P.mfinal_offset = (int64_t)i * 3 *
                          (dim_max == 1 ? (int64_t)nmax : (dim_max == 2 ? (int64_t)nmax * nmax : (int64_t)nmax * nmax * nmax));
        if (bx.dim == 3) {
            P.tab_offset = work3_off;  // in the 3-D work buffer
            work3_off += work3d_size(bx.n, bx.order);
            b->orders3 |= (bx.order == 4) ? 2 : 1;
            b->sampled3 |= P.coef_sampled;
            ids3.push_back(i);
            b->nmax3 = std::max(b->nmax3, bx.n);
            b->nq3 = std::max(b->nq3, P.nq);
            b->cost3 += (double)pl.M * P.stages * bx.n * bx.n * bx.n;
        } else {
            P.tab_offset = tab_off;
            tab_off += tab_layout(bx.dim, bx.n, P.form).size;
        }
        P.w_offset = w_off;
        w_off += 2 * bx.n;
        P.s64_offset = s64_off;
        if (P.form == 1) s64_off += scratch64_size(bx.dim, bx.n);
        auto wit = wt_off_of_M.find(pl.M);
        if (wit == wt_off_of_M.end()) {
            const int64_t o = (int64_t)wt_h.size();
            // w^n = K0(n/M)/M, n = 0..M, then the tails sum_{n' >= n} w^n'
            for (int n = 0; n <= pl.M; ++n)
                wt_h.push_back(time_kernel((double)n / pl.M, dcoef, K->p_t, K->q_t) / pl.M);
            std::vector<double> tail(pl.M + 1);
            double acc = 0.0;
            for (int n = pl.M; n >= 0; --n) {
                acc += wt_h[o + n];
                tail[n] = acc;
            }
            wt_h.insert(wt_h.end(), tail.begin(), tail.end());
            wit = wt_off_of_M.emplace(pl.M, o).first;
        }
        P.wt_offset = wit->second;
        double ws = 0.0;
        for (int n = 0; n <= pl.M; ++n) ws += wt_h[P.wt_offset + n];
        P.wsum = ws;
        cell_steps += (int64_t)pl.M * (bx.dim == 1 ? bx.n : (bx.dim == 2 ? (int64_t)bx.n * bx.n
                                                                          : (int64_t)bx.n * bx.n * bx.n));
        b->any_explicit |= (bx.init_mode == LLHMM_INIT_EXPLICIT);
        b->any_macro |= (bx.init_mode == LLHMM_INIT_MACRO_Q);
        b->any_sampled |= (P.coef_sampled != 0);
    }
    b->cell_steps = cell_steps;

    // group boxes by tile class; 1-D classes further by (M, stages) so that a
    // block's boxes share the time loop; longest boxes first (LPT order)
    std::map<std::tuple<const TileInfo *, int, int>, std::vector<int>> groups;
    for (int i = 0; i < nboxes; ++i) {
        const TileInfo *t = tile_of[i];
        if (!t) continue;  // slab box
        const int key_m = (t->dim == 1) ? b->plans_h[i].M : 0;
        const int key_s = (t->dim == 1) ? b->plans_h[i].stages : 0;
        groups[std::make_tuple(t, key_m, key_s)].push_back(i);
    }
    std::vector<int32_t> ids;
    for (auto &kv : groups) {
        const TileInfo *t = std::get<0>(kv.first);
        auto &v = kv.second;
        std::stable_sort(v.begin(), v.end(), [&](int a, int c) {
            return (int64_t)b->plans_h[a].M * b->plans_h[a].stages > (int64_t)b->plans_h[c].M * b->plans_h[c].stages;
        });
        ClassLaunch cl;
        cl.tile = t;
        cl.first = (int)ids.size();
        cl.cost = 0.0;
        for (int i : v)
            cl.cost += (double)b->plans_h[i].M * b->plans_h[i].stages *
                       (b->plans_h[i].dim == 1 ? b->plans_h[i].n : b->plans_h[i].n * b->plans_h[i].n);
        for (int i : v) ids.push_back(i);
        if (t->dim == 1) {
            while ((ids.size() - cl.first) % t->boxes_per_block) ids.push_back(-1);
        }
        cl.count = (int)ids.size() - cl.first;
        cl.nblocks = cl.count / t->boxes_per_block;
        b->classes.push_back(cl);
    }

    hipError_t e = hipSuccess;
    std::vector<CoefDev> cdev(ncoefs);
    memcpy(cdev.data(), coefs, sizeof(CoefDev) * ncoefs);
    if (e == hipSuccess) e = bupload(b, &b->plans, b->plans_h.data(), b->plans_h.size());
    if (e == hipSuccess) e = bupload(b, &b->box_ids, ids.data(), ids.size());
    if (e == hipSuccess) e = bupload(b, &b->coefs, cdev.data(), cdev.size());
    if (e == hipSuccess) e = bupload(b, &b->wt, wt_h.data(), wt_h.size());
    if (e == hipSuccess) e = balloc(b, &b->tabs, tsize * std::max<int64_t>(tab_off, 1));
    if (e == hipSuccess) e = balloc(b, (void **)&b->wts, sizeof(double) * std::max<int64_t>(w_off, 1));
    if (e == hipSuccess) e = balloc(b, (void **)&b->partials, sizeof(double) * (size_t)part_off * kMaxQ);
    if (e == hipSuccess) e = balloc(b, (void **)&b->wave_status, sizeof(int32_t) * (size_t)part_off);
    if (b->nslab_boxes > 0) {
        // slab_sync: per class (at most one class per slab box) its queue counters
        // and abort word
        b->nsync = kSlabSyncInts * (int64_t)b->nslab_boxes;
        b->nxwords = xbuf_off;
        if (e == hipSuccess) e = balloc(b, (void **)&b->slab_sync, sizeof(int32_t) * b->nsync);
        if (e == hipSuccess) e = balloc(b, (void **)&b->xbuf, sizeof(uint64_t) * xbuf_off);
        if (e == hipSuccess) e = balloc(b, (void **)&b->jobs, sizeof(SlabJob) * max_items);
    }
    if (e == hipSuccess) e = balloc(b, (void **)&b->status, sizeof(int32_t) * (size_t)nboxes);
    if (e == hipSuccess) e = balloc(b, (void **)&b->box_const, sizeof(double) * (size_t)nboxes * kMaxQ);
    if (e == hipSuccess) e = balloc(b, (void **)&b->scratch64, sizeof(double) * std::max<int64_t>(s64_off, 1));
    b->nbox3 = (int)ids3.size();
    if (e == hipSuccess && b->nbox3 > 0) e = bupload(b, &b->box3_ids, ids3.data(), ids3.size());
    if (e == hipSuccess && work3_off > 0) e = balloc(b, (void **)&b->work3d, sizeof(double) * work3_off);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(e == hipErrorOutOfMemory ? LLHMM_E_NOMEM : LLHMM_E_HIP, "batch allocation: %s",
                    hipGetErrorString(e));
    }
    st = rebuild_slabs(b);
    if (st != LLHMM_OK) {
        batch_free(b);
        return st;
    }
    *out = b;
    return LLHMM_OK;
}

extern "C" {

llhmm_status llhmm_batch_destroy(llhmm_ctx *, llhmm_batch *batch) {
    batch_free(batch);
    return LLHMM_OK;
}

int64_t llhmm_batch_cell_steps(const llhmm_batch *batch) { return batch ? batch->cell_steps : -1; }

// Checks the inputs of a solve / evaluation and fills the set-up kernel's arguments.
static llhmm_status prologue_args(llhmm_batch *b, const double *m_init_dev, const llhmm_macro *macro,
                                  const double *M_macro_dev, const double *coef_dev, PrologueArgs &pa) {
    if (b->any_explicit && !m_init_dev) return fail(LLHMM_E_INVALID, "explicit init needs m_init_dev");
    if (b->any_macro && (!macro || !M_macro_dev))
        return fail(LLHMM_E_INVALID, "macro-interpolated init needs macro and M_macro_dev");
    if (b->any_sampled && !coef_dev) return fail(LLHMM_E_INVALID, "sampled coefficient needs coef_dev");
    MacroDev md{};
    if (b->any_macro) {
        if (macro->n < 5 || !(macro->dX > 0.0)) return fail(LLHMM_E_INVALID, "macro grid: n >= 5, dX > 0");
        md.dim = macro->dim;
        md.n = macro->n;
        md.dX = macro->dX;
        md.x0[0] = macro->x0[0];
        md.x0[1] = macro->x0[1];
        md.x0[2] = macro->x0[2];
        for (int i = 0; i < b->nboxes; ++i) {
            const BoxPlan &P = b->plans_h[i];
            if (P.init_mode != LLHMM_INIT_MACRO_Q) continue;
            if (macro->dim != P.dim) return fail(LLHMM_E_INVALID, "box %d: macro dim differs", i);
            if (P.mi0 < 0 || P.mi0 >= macro->n || (P.dim >= 2 && (P.mi1 < 0 || P.mi1 >= macro->n)) ||
                (P.dim == 3 && (P.mi2 < 0 || P.mi2 >= macro->n)))
                return fail(LLHMM_E_INVALID, "box %d: macro_index out of range", i);
            // Q_[4] around node k is evaluated at the box's absolute positions; a
            // centre off the node (staggered flux points) must stay within one
            // macro cell of it
            const double tol = (1.0 + 1e-9) * macro->dX;
            if (std::fabs(P.cx - (macro->x0[0] + P.mi0 * macro->dX)) > tol ||
                (P.dim >= 2 && std::fabs(P.cy - (macro->x0[1] + P.mi1 * macro->dX)) > tol) ||
                (P.dim == 3 && std::fabs(P.cz - (macro->x0[2] + P.mi2 * macro->dX)) > tol))
                return fail(LLHMM_E_INVALID, "box %d: centre more than one macro cell from its node", i);
        }
    }
    pa = PrologueArgs{};
    pa.plans = b->plans;
    pa.nboxes = b->nboxes;
    pa.coefs = b->coefs;
    pa.m_init = m_init_dev;
    pa.M_macro = M_macro_dev;
    pa.macro = md;
    pa.coef_samples = coef_dev;
    pa.tabs = b->tabs;
    pa.wts = b->wts;
    pa.box_const = b->box_const;
    pa.scratch64 = b->scratch64;
    memcpy(pa.kc, b->kc, sizeof pa.kc);
    pa.kp = b->kp;
    pa.kq = b->kq;
    return LLHMM_OK;
}

static llhmm_status launch_resident(llhmm_batch *b, const ClassLaunch &cl, int mode, double *field_dev,
                                    hipStream_t stream) {
    MicroArgs a{};
    a.plans = b->plans;
    a.box_ids = b->box_ids + cl.first;
    a.nbox_class = cl.count;
    a.mode = mode;
    a.tabs = b->tabs;
    a.wts = b->wts;
    a.wt = b->wt;
    a.partials = b->partials;
    a.wave_status = b->wave_status;
    a.out_field = field_dev;
    HIP_TRY(cl.tile->launch(a, cl.nblocks, stream));
    return LLHMM_OK;
}

// Zeroes the slab classes' counters, abort words and exchange words.
static hipError_t clear_slab_sync(llhmm_batch *b, hipStream_t stream) {
    if (b->nsync == 0) return hipSuccess;
    hipError_t e = launch_fill_i32(b->slab_sync, b->nsync, 0, stream);
    if (e == hipSuccess) e = launch_fill_i32((int32_t *)b->xbuf, 2 * b->nxwords, 0, stream);
    return e;
}

// Workgroups of a slab tile that fit one CU at once (cached per tile).
static llhmm_status slab_blocks_per_cu(const SlabTileInfo *t, int *out) {
    static std::mutex mu;
    static std::map<const SlabTileInfo *, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(t);
    if (it == cache.end()) {
        int bpc = 0;
        HIP_TRY(t->occupancy(&bpc));
        if (bpc < 1) return fail(LLHMM_E_HIP, "%s: no workgroup fits a CU", t->name);
        it = cache.emplace(t, bpc).first;
    }
    *out = it->second;
    return LLHMM_OK;
}

// One persistent launch of a slab class: as many workgroups as fit the GPU at
// once (at most one per item); they take the class's items in order.
static llhmm_status launch_slab_class(llhmm_batch *b, const SlabClass &sc, int mode, double *field_dev,
                                      hipStream_t stream) {
    int bpc = 0;
    llhmm_status st = slab_blocks_per_cu(sc.tile, &bpc);
    if (st != LLHMM_OK) return st;
    SlabArgs a{};
    a.plans = b->plans;
    a.jobs = b->jobs + sc.first;
    a.nqueues = sc.nq;
    for (int k = 0; k <= kMaxXcc; ++k) a.qoff[k] = sc.qoff[k];
    a.mode = mode;
    a.counter = b->slab_sync + kSlabSyncInts * sc.index;
    a.abort_word = b->slab_sync + kSlabSyncInts * sc.index + kMaxXcc;
    a.spin_max = slab_spin_max();
    a.h = sc.geom.h;
    a.spe = sc.geom.spe;
    a.xdepth = sc.geom.xd;
    a.tabs = b->tabs;
    a.wts = b->wts;
    a.wt = b->wt;
    a.partials = b->partials;
    a.wave_status = b->wave_status;
    a.xbuf = b->xbuf;
    a.out_field = field_dev;
    // every XCD gets its share of the resident workgroups (dispatch is round robin
    // over the XCDs); workgroups whose queue is empty end at once
    const int grid = bpc * b->ncu;
    HIP_TRY(sc.tile->launch(a, grid, stream));
    return LLHMM_OK;
}

static llhmm_status ensure_side_streams(llhmm_batch *b) {
    if (b->fork) return LLHMM_OK;
    HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    for (int i = 0; i < kSideStreams; ++i) {
        HIP_TRY(hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming));
    }
    return LLHMM_OK;
}

// The whole solve (mode 0) or field evaluation (mode 1) of a batch on `stream`:
// set-up kernel, then the tile classes.  Classes are independent, so with more
// than one they are spread over the caller's stream and up to kSideStreams
// side streams (longest first onto the least loaded stream), forked after the
// set-up and joined back into the caller's stream before returning.
static llhmm_status run_batch(llhmm_ctx *ctx, llhmm_batch *b, const double *m_init_dev,
                              const llhmm_macro *macro, const double *M_macro_dev,
                              const double *coef_dev, double *field_dev, int mode,
                              hipStream_t stream) {
    if (!ctx || !b) return fail(LLHMM_E_INVALID, "ctx/batch is NULL");
    PrologueArgs pa;
    llhmm_status st = prologue_args(b, m_init_dev, macro, M_macro_dev, coef_dev, pa);
    if (st != LLHMM_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    const bool timed = b->timing && !b->capturing;
    hipEvent_t *ev = b->ev[b->timed % LLHMM_TIMING_SLOTS];
    if (timed) HIP_TRY(hipEventRecord(ev[0], stream));
    HIP_TRY(launch_prologue(b->prec, pa, stream));
    Micro3dArgs a3{};
    if (b->nbox3 > 0) {
        a3.plans = b->plans;
        a3.box_ids = b->box3_ids;
        a3.nbox = b->nbox3;
        a3.nmax = b->nmax3;
        a3.nq_max = b->nq3;
        a3.orders = b->orders3;
        a3.sampled = b->sampled3;
        a3.coef_samples = pa.coef_samples;
        a3.mode = mode;
        a3.coefs = b->coefs;
        a3.m_init = m_init_dev;
        a3.M_macro = M_macro_dev;
        a3.macro = pa.macro;
        a3.work = b->work3d;
        a3.wts = b->wts;
        a3.wt = b->wt;
        a3.partials = b->partials;
        a3.wave_status = b->wave_status;
        a3.box_const = b->box_const;
        a3.out_field = field_dev;
        memcpy(a3.kc, b->kc, sizeof a3.kc);
        a3.kp = b->kp;
        a3.kq = b->kq;
        HIP_TRY(launch_setup3d(a3, stream));
    }
    // slab classes: work counters, abort words and the exchange words' tags
    // start at zero (a kernel, not a memset, so that a captured graph resets
    // them on replay)
    HIP_TRY(clear_slab_sync(b, stream));
    if (timed) HIP_TRY(hipEventRecord(ev[1], stream));

    // work items: resident classes (index >= 0) and slab classes (~index)
    struct Item { double cost; int idx; };
    std::vector<Item> items;
    for (size_t i = 0; i < b->classes.size(); ++i) items.push_back({b->classes[i].cost, (int)i});
    for (size_t i = 0; i < b->slabs.size(); ++i) items.push_back({b->slabs[i].cost, ~(int)i});
    constexpr int kItem3d = std::numeric_limits<int>::max();
    if (b->nbox3 > 0) items.push_back({b->cost3, kItem3d});
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    const int lanes = std::min<int>((int)items.size(), b->max_lanes);
    if (lanes > 1) {
        st = ensure_side_streams(b);
        if (st != LLHMM_OK) return st;
        HIP_TRY(hipEventRecord(b->fork, stream));
        for (int l = 1; l < lanes; ++l) HIP_TRY(hipStreamWaitEvent(b->side[l - 1], b->fork, 0));
    }
    std::vector<double> load(std::max(lanes, 1), 0.0);
    for (const Item &it : items) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[l] += it.cost;
        hipStream_t s = (l == 0) ? stream : b->side[l - 1];
        if (it.idx == kItem3d) {
            HIP_TRY(launch_micro3d(a3, s));
            continue;
        }
        st = (it.idx >= 0) ? launch_resident(b, b->classes[it.idx], mode, field_dev, s)
                           : launch_slab_class(b, b->slabs[~it.idx], mode, field_dev, s);
        if (st != LLHMM_OK) return st;
    }
    for (int l = 1; l < lanes; ++l) {
        HIP_TRY(hipEventRecord(b->join[l - 1], b->side[l - 1]));
        HIP_TRY(hipStreamWaitEvent(stream, b->join[l - 1], 0));
    }
    if (timed) {
        HIP_TRY(hipEventRecord(ev[2], stream));
        ++b->timed;
    }
    return LLHMM_OK;
}

llhmm_status llhmm_batch_set_timing(llhmm_batch *b, int32_t enable) {
    if (!b) return fail(LLHMM_E_INVALID, "batch is NULL");
    if (enable)
        for (auto &slot : b->ev)
            for (hipEvent_t &e : slot)
                if (!e) HIP_TRY(hipEventCreate(&e));
    b->timing = enable != 0;
    b->timed = 0;
    return LLHMM_OK;
}

llhmm_status llhmm_batch_timing(llhmm_batch *b, int32_t back, float *setup_ms, float *step_ms) {
    if (!b) return fail(LLHMM_E_INVALID, "batch is NULL");
    if (!b->timing) return fail(LLHMM_E_INVALID, "timing is off");
    if (back < 0 || back >= LLHMM_TIMING_SLOTS || back >= b->timed)
        return fail(LLHMM_E_INVALID, "timed call %d back is not kept (%lld timed calls)", back,
                    (long long)b->timed);
    hipEvent_t *ev = b->ev[(b->timed - 1 - back) % LLHMM_TIMING_SLOTS];
    HIP_TRY(hipEventSynchronize(ev[2]));
    float s = 0.f, t = 0.f;
    HIP_TRY(hipEventElapsedTime(&s, ev[0], ev[1]));
    HIP_TRY(hipEventElapsedTime(&t, ev[1], ev[2]));
    if (setup_ms) *setup_ms = s;
    if (step_ms) *step_ms = t;
    return LLHMM_OK;
}

llhmm_status llhmm_micro_batch(llhmm_ctx *ctx, llhmm_batch *batch, const double *m_init_dev,
                               const llhmm_macro *macro, const double *M_macro_dev,
                               const double *coef_dev, double *m_final_dev, hipStream_t stream) {
    return run_batch(ctx, batch, m_init_dev, macro, M_macro_dev, coef_dev, m_final_dev, 0, stream);
}

llhmm_status llhmm_eval_field(llhmm_ctx *ctx, llhmm_batch *batch, const double *m_init_dev,
                              const llhmm_macro *macro, const double *M_macro_dev,
                              const double *coef_dev, double *H_dev, hipStream_t stream) {
    if (!H_dev) return fail(LLHMM_E_INVALID, "H_dev is NULL");
    return run_batch(ctx, batch, m_init_dev, macro, M_macro_dev, coef_dev, H_dev, 1, stream);
}

llhmm_status llhmm_upscale(llhmm_ctx *ctx, llhmm_batch *b, double *H_avg_dev, int32_t ld,
                           int32_t *status_dev, int32_t check, hipStream_t stream) {
    if (!ctx || !b) return fail(LLHMM_E_INVALID, "ctx/batch is NULL");
    if (H_avg_dev && ld < 3 * b->dim_max) {
        bool flux2d = false;
        for (const BoxPlan &P : b->plans_h) flux2d |= (P.nq > ld);
        if (flux2d) return fail(LLHMM_E_INVALID, "ld %d smaller than the outputs per box", ld);
    }
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_upscale(b->partials, b->wave_status, b->box_const, b->plans, b->nboxes, H_avg_dev, ld,
                           b->status, status_dev, stream));
    if (check) {
        std::vector<int32_t> st(b->nboxes);
        HIP_TRY(hipMemcpyAsync(st.data(), b->status, sizeof(int32_t) * b->nboxes,
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (int i = 0; i < b->nboxes; ++i)
            if (st[i] & 2) return fail(LLHMM_E_HIP, "box %d: a slab exchange wait gave up", i);
            else if (st[i] & 1) return fail(LLHMM_E_UNSTABLE, "box %d produced non-finite values", i);
            else if (st[i] & 4) return fail(LLHMM_E_UNSTABLE, "box %d: final state not resolved (neighbouring "
                                            "points differ by more than %g)", i, kRoughMax);
            else if (st[i] & 8) return fail(LLHMM_E_UNSTABLE, "box %d: final state left the unit sphere", i);
    }
    return LLHMM_OK;
}

llhmm_status llhmm_batch_run_graph(llhmm_ctx *ctx, llhmm_batch *b, const double *m_init_dev,
                                   const llhmm_macro *macro, const double *M_macro_dev,
                                   const double *coef_dev, double *m_final_dev, double *H_avg_dev,
                                   int32_t ld, int32_t *status_dev, hipStream_t stream) {
    if (!ctx || !b) return fail(LLHMM_E_INVALID, "ctx/batch is NULL");
    if (H_avg_dev && ld < 3 * b->dim_max) {
        for (const BoxPlan &P : b->plans_h)
            if (P.nq > ld) return fail(LLHMM_E_INVALID, "ld %d smaller than the outputs per box", ld);
    }
    GraphArgs ga;
    memset(&ga, 0, sizeof ga);
    ga.m_init = m_init_dev;
    ga.M_macro = M_macro_dev;
    ga.coef = coef_dev;
    ga.m_final = m_final_dev;
    ga.H = H_avg_dev;
    ga.status = status_dev;
    ga.ld = ld;
    ga.has_macro = macro != nullptr;
    if (macro) ga.macro = *macro;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!b->exec || !(ga == b->gargs)) {
        if (b->exec) {
            HIP_TRY(hipGraphExecDestroy(b->exec));
            b->exec = nullptr;
        }
        // everything that can fail on the host is checked before the capture opens
        PrologueArgs pa;
        llhmm_status st = prologue_args(b, m_init_dev, macro, M_macro_dev, coef_dev, pa);
        if (st != LLHMM_OK) return st;
        st = ensure_side_streams(b);
        if (st != LLHMM_OK) return st;
        if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        b->capturing = true;
        st = run_batch(ctx, b, m_init_dev, macro, M_macro_dev, coef_dev, m_final_dev, 0, b->cap_stream);
        if (st == LLHMM_OK) {
            const hipError_t e = launch_upscale(b->partials, b->wave_status, b->box_const, b->plans, b->nboxes,
                                                H_avg_dev, ld, b->status, status_dev, b->cap_stream);
            if (e != hipSuccess) st = fail(LLHMM_E_HIP, "upscale launch in capture: %s", hipGetErrorString(e));
        }
        b->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(b->cap_stream, &g);
        if (st != LLHMM_OK || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != LLHMM_OK ? st : fail(LLHMM_E_HIP, "graph capture: %s", hipGetErrorString(ee));
        }
        const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->exec = nullptr;
            return fail(LLHMM_E_HIP, "graph instantiation: %s", hipGetErrorString(ei));
        }
        b->gargs = ga;
    }
    const bool timed = b->timing;
    hipEvent_t *ev = b->ev[b->timed % LLHMM_TIMING_SLOTS];
    if (timed) {
        HIP_TRY(hipEventRecord(ev[0], stream));
        HIP_TRY(hipEventRecord(ev[1], stream));
    }
    HIP_TRY(hipGraphLaunch(b->exec, stream));
    if (timed) {
        HIP_TRY(hipEventRecord(ev[2], stream));
        ++b->timed;
    }
    return LLHMM_OK;
}

llhmm_status llhmm_batch_tune(llhmm_ctx *ctx, llhmm_batch *b, const double *m_init_dev,
                              const llhmm_macro *macro, const double *M_macro_dev, const double *coef_dev,
                              int32_t reps, hipStream_t stream) {
    if (!ctx || !b) return fail(LLHMM_E_INVALID, "ctx/batch is NULL");
    if (reps < 1) return fail(LLHMM_E_INVALID, "reps must be >= 1");
    if (b->slabs.empty()) return LLHMM_OK;
    PrologueArgs pa;
    llhmm_status st = prologue_args(b, m_init_dev, macro, M_macro_dev, coef_dev, pa);
    if (st != LLHMM_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_prologue(b->prec, pa, stream));  // tables the slab kernels read
    std::map<TuneKey, std::vector<int>> keys;
    for (int i = 0; i < b->nboxes; ++i)
        if (b->slab_tile[i]) {
            const BoxPlan &P = b->plans_h[i];
            keys[TuneKey{b->prec, P.n, P.bc, P.quantity, P.stages}].push_back(i);
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (auto &kv : keys) {
        const int i0 = kv.second[0];
        const BoxPlan &P0 = b->plans_h[i0];
        const auto &variants = slab_registry().at(SlabKey{b->prec, P0.n, P0.order, P0.bc, P0.quantity});
        int best_v = 0, best_spe = b->slab_spe[i0];
        for (size_t v = 0; v < variants.size(); ++v)
            if (variants[v] == b->slab_tile[i0]) best_v = (int)v;
        float best_ms = -1.f;
        for (int vs = 0; vs < (int)variants.size() * kNumSpe && st == LLHMM_OK; ++vs) {
            const int v = vs / kNumSpe, spe = kSlabSpe[vs % kNumSpe];
            const SlabTileInfo *t = variants[v];
            if (slab_geom(*t, P0.n, P0.stages, spe).ns == 0) continue;
            hipError_t e = hipStreamSynchronize(stream);  // no launch may still read the plans or jobs
            if (e != hipSuccess) { st = fail(LLHMM_E_HIP, "tune: %s", hipGetErrorString(e)); break; }
            for (int i : kv.second) {
                b->slab_tile[i] = t;
                b->slab_spe[i] = spe;
            }
            st = rebuild_slabs(b);
            if (st != LLHMM_OK) break;
            const SlabClass *sc = nullptr;
            for (const SlabClass &c : b->slabs)
                if (c.tile == t && c.geom.spe == spe && c.stages == P0.stages) sc = &c;
            if (!sc) continue;
            float ms = 0.f;
            for (int r = 0; r <= reps && st == LLHMM_OK; ++r) {  // round 0 warms up
                e = clear_slab_sync(b, stream);
                if (e == hipSuccess && r == 1) e = hipEventRecord(e0, stream);
                if (e == hipSuccess) st = launch_slab_class(b, *sc, 0, nullptr, stream);
                if (e != hipSuccess) st = fail(LLHMM_E_HIP, "tune: %s", hipGetErrorString(e));
            }
            if (st == LLHMM_OK) {
                hipError_t e2 = hipEventRecord(e1, stream);
                if (e2 == hipSuccess) e2 = hipEventSynchronize(e1);
                if (e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, e0, e1);
                if (e2 != hipSuccess) st = fail(LLHMM_E_HIP, "tune: %s", hipGetErrorString(e2));
            }
            if (st == LLHMM_OK && (best_ms < 0.f || ms < best_ms)) {
                best_ms = ms;
                best_v = v;
                best_spe = spe;
            }
        }
        if (st != LLHMM_OK) break;
        for (int i : kv.second) {
            b->slab_tile[i] = variants[best_v];
            b->slab_spe[i] = best_spe;
        }
        ctx->tuned[kv.first] = TuneVal{best_v, best_spe};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LLHMM_OK) return st;
    HIP_TRY(hipStreamSynchronize(stream));
    return rebuild_slabs(b);
}

llhmm_status llhmm_batch_slabs(const llhmm_batch *b, int32_t *slabs_out, int32_t *steps_per_exchange_out) {
    if (!b || !slabs_out) return fail(LLHMM_E_INVALID, "batch/slabs_out is NULL");
    for (int i = 0; i < b->nboxes; ++i) {
        slabs_out[i] = b->slab_tile[i] ? b->plans_h[i].strips : 0;
        if (steps_per_exchange_out) steps_per_exchange_out[i] = b->slab_tile[i] ? b->slab_spe[i] : 0;
    }
    return LLHMM_OK;
}

llhmm_status llhmm_tune_save(const llhmm_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(LLHMM_E_INVALID, "ctx/path is NULL");
    FILE *f = fopen(path, "w");
    if (!f) return fail(LLHMM_E_INVALID, "cannot write %s", path);
    fprintf(f, "# llhmm slab tuning: precision n bc quantity stages variant steps_per_exchange\n");
    for (const auto &kv : ctx->tuned)
        fprintf(f, "%d %d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                std::get<3>(kv.first), std::get<4>(kv.first), kv.second.first, kv.second.second);
    fclose(f);
    return LLHMM_OK;
}

llhmm_status llhmm_tune_load(llhmm_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(LLHMM_E_INVALID, "ctx/path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(LLHMM_E_INVALID, "cannot read %s", path);
    char line[256];
    std::map<TuneKey, TuneVal> got;
    llhmm_status st = LLHMM_OK;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        int v[7];
        if (sscanf(line, "%d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6]) != 7 ||
            v[5] < 0 || v[5] > 15 || std::find(std::begin(kSlabSpe), std::end(kSlabSpe), v[6]) == std::end(kSlabSpe)) {
            st = fail(LLHMM_E_INVALID, "%s: bad line: %s", path, line);
            break;
        }
        got[TuneKey{v[0], v[1], v[2], v[3], v[4]}] = TuneVal{v[5], v[6]};
    }
    fclose(f);
    if (st != LLHMM_OK) return st;
    for (const auto &kv : got) ctx->tuned[kv.first] = kv.second;
    return LLHMM_OK;
}

llhmm_status llhmm_macro_step(llhmm_ctx *ctx, int32_t npts, int32_t scheme, int32_t step_index,
                              int32_t stage, double dt, double alpha, double *M_dev,
                              const double *H_avg_dev, double *Y_dev, double *work_dev,
                              int32_t *next_stage_out, hipStream_t stream) {
    if (!ctx) return fail(LLHMM_E_INVALID, "ctx is NULL");
    if (npts <= 0 || !M_dev || !H_avg_dev || !Y_dev || !work_dev)
        return fail(LLHMM_E_INVALID, "macro step: empty grid or NULL buffer");
    if (!(dt > 0.0) || !(alpha >= 0.0)) return fail(LLHMM_E_INVALID, "macro step: dt > 0, alpha >= 0");
    int nst;
    if (scheme == LLHMM_MACRO_MPEA) {
        if (step_index < 2) return fail(LLHMM_E_INVALID, "MPEA needs two start-up steps (step_index >= 2)");
        nst = 1;
    } else if (scheme == LLHMM_MACRO_HEUNP) {
        nst = 2;
    } else if (scheme == LLHMM_MACRO_RK4P) {
        nst = 4;
    } else {
        return fail(LLHMM_E_INVALID, "unknown macro scheme %d", scheme);
    }
    if (stage < 0 || stage >= nst) return fail(LLHMM_E_INVALID, "stage %d out of range", stage);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_macro(npts, 0, scheme, step_index, stage, dt, alpha, M_dev, H_avg_dev, Y_dev, work_dev,
                         stream));
    if (next_stage_out) *next_stage_out = (stage + 1 < nst) ? stage + 1 : 0;
    return LLHMM_OK;
}

llhmm_status llhmm_macro_step_torque(llhmm_ctx *ctx, int32_t npts, int32_t scheme, int32_t stage, double dt,
                                     double alpha, double *M_dev, const double *T_avg_dev, double *Y_dev,
                                     double *work_dev, int32_t *next_stage_out, hipStream_t stream) {
    if (!ctx) return fail(LLHMM_E_INVALID, "ctx is NULL");
    if (npts <= 0 || !M_dev || !T_avg_dev || !Y_dev || !work_dev)
        return fail(LLHMM_E_INVALID, "macro step: empty grid or NULL buffer");
    if (!(dt > 0.0) || !(alpha >= 0.0)) return fail(LLHMM_E_INVALID, "macro step: dt > 0, alpha >= 0");
    int nst;
    if (scheme == LLHMM_MACRO_HEUNP) nst = 2;
    else if (scheme == LLHMM_MACRO_RK4P) nst = 4;
    else return fail(LLHMM_E_INVALID, "torque model: scheme must be HeunP or RK4P");
    if (stage < 0 || stage >= nst) return fail(LLHMM_E_INVALID, "stage %d out of range", stage);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_macro(npts, 1, scheme, 0, stage, dt, alpha, M_dev, T_avg_dev, Y_dev, work_dev, stream));
    if (next_stage_out) *next_stage_out = (stage + 1 < nst) ? stage + 1 : 0;
    return LLHMM_OK;
}

llhmm_status llhmm_flux_divergence(llhmm_ctx *ctx, const llhmm_macro *macro, int32_t order, const double *F_dev,
                                   int32_t ld, double *H_dev, hipStream_t stream) {
    if (!ctx || !macro) return fail(LLHMM_E_INVALID, "ctx/macro is NULL");
    if (macro->dim < 1 || macro->dim > 3 || macro->n < 5)
        return fail(LLHMM_E_INVALID, "flux divergence: dim 1, 2 or 3 and n >= 5 macro nodes");
    if (!(macro->dX > 0.0)) return fail(LLHMM_E_INVALID, "flux divergence: dX > 0");
    if (order != 2 && order != 4) return fail(LLHMM_E_INVALID, "flux divergence: order 2 or 4");
    if (!F_dev || !H_dev) return fail(LLHMM_E_INVALID, "flux divergence: NULL buffer");
    if (ld < 3 * macro->dim) return fail(LLHMM_E_INVALID, "flux divergence: ld %d < 3 dim", ld);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_flux_div(macro->dim, macro->n, macro->dX, order, F_dev, ld, H_dev, stream));
    return LLHMM_OK;
}

}  // extern "C"

// ===================================================================== serving
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ServeReq {
    llhmm_box box;
    int64_t id;
    double t_submit;                 // host steady clock, seconds
    const double *m_init, *M_macro;  // caller's device inputs for this request
    llhmm_macro macro;
    int32_t has_macro;
    int64_t bytes;                   // device memory its share of a micro-batch needs (upper bound)
};

// Results per request in the serving API: stride 6 (3 * dim for flux in 2-D;
// d = 3 flux requests are not served).
constexpr int kServeQ = 6;

struct ServeDone {
    int64_t id;
    double H[kServeQ];
    int32_t status;
    double latency_us;
};

struct ServeFlight {
    llhmm_batch *batch = nullptr;
    std::vector<ServeReq> reqs;
    double *H_dev = nullptr;
    int32_t *st_dev = nullptr;
    int64_t *ids_dev = nullptr;      // request ids, when results also go to the caller's device array
    hipEvent_t done = nullptr;
    int64_t bytes = 0, seq = 0;
    bool busy = false;
};

constexpr int64_t kBatchSlack = 32 * 256;  // alignment slack of one micro-batch's allocations

bool same_source(const ServeReq &a, const ServeReq &b) {
    return a.m_init == b.m_init && a.M_macro == b.M_macro && a.has_macro == b.has_macro &&
           (!a.has_macro || memcmp(&a.macro, &b.macro, sizeof a.macro) == 0);
}

}  // namespace

struct llhmm_server {
    llhmm_ctx *ctx = nullptr;
    llhmm_server_cfg cfg{};
    std::vector<llhmm_coef> coefs;
    Arena arena;
    std::deque<ServeReq> queue;
    std::vector<ServeFlight> slots;
    std::vector<hipStream_t> streams;
    double *H_host = nullptr;    // pinned [slots][max_batch_boxes][kServeQ]
    int32_t *st_host = nullptr;  // pinned [slots][max_batch_boxes]
    int64_t *ids_host = nullptr; // pinned [slots][max_batch_boxes], staging of the request ids
    double *out_H = nullptr;     // caller's device array of results (llhmm_server_set_output)
    int32_t out_ld = 0;
    int64_t out_rows = 0;
    std::deque<ServeDone> done;
    int64_t reserved = 0, seq = 0;
};

// Device memory one request adds to a micro-batch (tables, weights, set-up
// scratch, partial-sum slots, slab exchange rows, time weights, descriptors,
// its result, status and id), an upper bound of what the micro-batch allocates
// for it.
static llhmm_status request_bytes(const llhmm_server *sv, const llhmm_box &bx, int i, int64_t &bytes) {
    llhmm_status st = validate_box(bx, i, (int)sv->coefs.size());
    if (st != LLHMM_OK) return st;
    if (sv->coefs[bx.coef_index].dim != bx.dim)
        return fail(LLHMM_E_INVALID, "request %d: coefficient dimension differs from box", i);
    if (sv->coefs[bx.coef_index].sampled)
        return fail(LLHMM_E_NOTSUP, "request %d: sampled coefficients are not served", i);
    Planned pl{};
    st = plan_one(bx, i, pl);
    if (st != LLHMM_OK) return st;
    const int prec = sv->cfg.precision;
    st = check_fp32_domain(bx, i, prec);
    if (st != LLHMM_OK) return st;
    const int64_t tsize = (prec == LLHMM_FP32) ? 4 : 8;
    const int stages = (pl.integ == LLHMM_RK4P) ? 4 : 2;
    if (bx.dim == 3) {
        if (prec != LLHMM_FP64 || bx.order != 2 || bx.quantity == LLHMM_Q_FLUX)
            return fail(LLHMM_E_NOTSUP, "request %d: d = 3 needs FP64, order 2, field or torque", i);
        bytes = work3d_size(bx.n, bx.order) * 8 + 2 * bx.n * 8 + (kMaxQ * 8 + 4) + 2 * (int64_t)(pl.M + 1) * 8 +
                (int64_t)sizeof(BoxPlan) + 4 + kMaxQ * 8 + 4 + kMaxQ * 8 + 4 + (int64_t)sizeof(CoefDev) + 8 + 3 * 256;
        return LLHMM_OK;
    }
    auto it = registry().find(TileKey{prec, bx.dim, bx.n, bx.order, bx.bc, bx.quantity});
    bool slab = false;
    SlabReserve sres;
    if (it == registry().end() && bx.dim == 2) {
        auto bit = slab_registry().find(SlabKey{prec, bx.n, bx.order, bx.bc, bx.quantity});
        if (bit != slab_registry().end()) {
            slab = true;
            sres = slab_reserve(bit->second, bx.n, stages);
        }
    }
    if (it == registry().end() && !slab)
        return fail(LLHMM_E_NOTSUP, "request %d: no kernel for dim %d, n %d, order %d, bc %d, quantity %d", i,
                    bx.dim, bx.n, bx.order, bx.bc, bx.quantity);
    const int form = (prec == LLHMM_FP32 || slab || (!slab && (it->second->opt & kOptForm1))) ? 1 : 0;
    int64_t slots = (bx.dim == 2) ? 16 : 1;
    int64_t slab_bytes = 0;
    if (slab) {
        // exchange words, a work counter and an abort word, jobs
        slots = sres.slots;
        slab_bytes = sres.xwords * 8 + 2 * 4 + sres.items * (int64_t)sizeof(SlabJob) + 3 * 256;
    }
    bytes = tab_layout(bx.dim, bx.n, form).size * tsize + 2 * bx.n * 8 +
            (form == 1 ? scratch64_size(bx.dim, bx.n) * 8 : 0) + slots * (kMaxQ * 8 + 4) + slab_bytes +
            2 * (int64_t)(pl.M + 1) * 8 + (int64_t)sizeof(BoxPlan) + 4 + kMaxQ * 8 + 4 + kMaxQ * 8 + 4 +
            (int64_t)sizeof(CoefDev) + 8 + 2 * 256;
    return LLHMM_OK;
}

static void serve_release(llhmm_server *sv, ServeFlight &f) {
    if (f.batch) batch_free(f.batch);
    if (f.H_dev) sv->arena.release(f.H_dev);
    if (f.st_dev) sv->arena.release(f.st_dev);
    if (f.ids_dev) sv->arena.release(f.ids_dev);
    f.batch = nullptr;
    f.H_dev = nullptr;
    f.st_dev = nullptr;
    f.ids_dev = nullptr;
    sv->reserved -= f.bytes;
    f.bytes = 0;
    f.reqs.clear();
    f.busy = false;
}

// Completes finished micro-batches (non-blocking).
static llhmm_status serve_complete(llhmm_server *sv) {
    const int mb = sv->cfg.max_batch_boxes;
    for (size_t k = 0; k < sv->slots.size(); ++k) {
        ServeFlight &f = sv->slots[k];
        if (!f.busy) continue;
        const hipError_t e = hipEventQuery(f.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return fail(LLHMM_E_HIP, "serving: %s", hipGetErrorString(e));
        const double t = now_s();
        for (size_t r = 0; r < f.reqs.size(); ++r) {
            ServeDone d;
            d.id = f.reqs[r].id;
            memcpy(d.H, sv->H_host + ((size_t)k * mb + r) * kServeQ, sizeof d.H);
            d.status = sv->st_host[(size_t)k * mb + r];
            d.latency_us = (t - f.reqs[r].t_submit) * 1e6;
            sv->done.push_back(d);
        }
        serve_release(sv, f);
    }
    return LLHMM_OK;
}

static void serve_fail_front(llhmm_server *sv, size_t count, llhmm_status code) {
    const double t = now_s();
    for (size_t r = 0; r < count && !sv->queue.empty(); ++r) {
        ServeDone d{};
        d.id = sv->queue.front().id;
        d.status = code;
        d.latency_us = (t - sv->queue.front().t_submit) * 1e6;
        sv->done.push_back(d);
        sv->queue.pop_front();
    }
}

// Admits queued requests in arrival order while a stream slot is free and the
// server's memory can hold them; each admitted group is one micro-batch on
// its own stream: set-up, time stepping, upscale, copy of the results to
// pinned host memory, completion event.
static llhmm_status serve_admit(llhmm_server *sv) {
    const int mb = sv->cfg.max_batch_boxes;
    while (!sv->queue.empty()) {
        int slot = -1;
        bool any_busy = false;
        for (size_t k = 0; k < sv->slots.size(); ++k) {
            if (!sv->slots[k].busy && slot < 0) slot = (int)k;
            any_busy |= sv->slots[k].busy;
        }
        if (slot < 0) break;
        const ServeReq &head = sv->queue.front();
        const int64_t avail = (int64_t)sv->arena.size - sv->reserved - kBatchSlack;
        int64_t bytes = 0;
        size_t n = 0;
        for (const ServeReq &r : sv->queue) {
            if ((int)n == mb || !same_source(r, head) || bytes + r.bytes > avail) break;
            bytes += r.bytes;
            ++n;
        }
        if (n == 0) {
            if (any_busy) break;  // wait for memory to come back
            serve_fail_front(sv, 1, LLHMM_E_BUDGET);  // larger than the whole budget
            continue;
        }
        std::vector<llhmm_box> boxes(n);
        for (size_t r = 0; r < n; ++r) boxes[r] = sv->queue[r].box;
        ServeFlight &f = sv->slots[slot];
        llhmm_status st = batch_create_impl(sv->ctx, boxes.data(), (int32_t)n, &sv->cfg.K, sv->coefs.data(),
                                            (int32_t)sv->coefs.size(), sv->cfg.precision, &sv->arena, 1, &f.batch);
        if (st == LLHMM_E_NOMEM) {
            f.batch = nullptr;
            if (any_busy) break;
            serve_fail_front(sv, n, LLHMM_E_BUDGET);
            continue;
        }
        if (st != LLHMM_OK) {
            f.batch = nullptr;
            serve_fail_front(sv, n, st);
            continue;
        }
        f.H_dev = (double *)sv->arena.alloc(n * kServeQ * sizeof(double));
        f.st_dev = (int32_t *)sv->arena.alloc(n * sizeof(int32_t));
        if (sv->out_H) f.ids_dev = (int64_t *)sv->arena.alloc(n * sizeof(int64_t));
        f.bytes = bytes + kBatchSlack;
        sv->reserved += f.bytes;
        f.busy = true;
        if (!f.H_dev || !f.st_dev || (sv->out_H && !f.ids_dev)) {
            serve_release(sv, f);
            if (any_busy) break;
            serve_fail_front(sv, n, LLHMM_E_BUDGET);
            continue;
        }
        hipStream_t s = sv->streams[slot];
        st = run_batch(sv->ctx, f.batch, head.m_init, head.has_macro ? &head.macro : nullptr, head.M_macro,
                       nullptr, nullptr, 0, s);
        if (st != LLHMM_OK) {
            serve_release(sv, f);
            serve_fail_front(sv, n, st);
            continue;
        }
        HIP_TRY(launch_upscale(f.batch->partials, f.batch->wave_status, f.batch->box_const, f.batch->plans,
                               (int)n, f.H_dev, kServeQ, f.batch->status, f.st_dev, s));
        if (sv->out_H) {
            // results also to the caller's device array, before the completion event
            int64_t *ih = sv->ids_host + (size_t)slot * mb;
            for (size_t r = 0; r < n; ++r) ih[r] = sv->queue[r].id;
            HIP_TRY(hipMemcpyAsync(f.ids_dev, ih, n * sizeof(int64_t), hipMemcpyHostToDevice, s));
            HIP_TRY(launch_scatter_rows(f.H_dev, kServeQ, f.ids_dev, (int)n, std::min<int>(kServeQ, sv->out_ld),
                                        sv->out_H, sv->out_ld, sv->out_rows, s));
        }
        HIP_TRY(hipMemcpyAsync(sv->H_host + (size_t)slot * mb * kServeQ, f.H_dev, n * kServeQ * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(sv->st_host + (size_t)slot * mb, f.st_dev, n * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(f.done, s));
        f.seq = sv->seq++;
        f.reqs.assign(sv->queue.begin(), sv->queue.begin() + n);
        sv->queue.erase(sv->queue.begin(), sv->queue.begin() + n);
    }
    return LLHMM_OK;
}

static void server_free(llhmm_server *sv) {
    if (!sv) return;
    for (ServeFlight &f : sv->slots) {
        if (f.busy && f.done) (void)hipEventSynchronize(f.done);
        if (f.busy) serve_release(sv, f);
        if (f.done) (void)hipEventDestroy(f.done);
    }
    for (hipStream_t s : sv->streams)
        if (s) (void)hipStreamDestroy(s);
    if (sv->H_host) (void)hipHostFree(sv->H_host);
    if (sv->st_host) (void)hipHostFree(sv->st_host);
    if (sv->ids_host) (void)hipHostFree(sv->ids_host);
    if (sv->arena.base) (void)hipFree(sv->arena.base);
    delete sv;
}

extern "C" {

llhmm_status llhmm_server_create(llhmm_ctx *ctx, const llhmm_server_cfg *cfg, const llhmm_coef *coefs,
                                 int32_t ncoefs, llhmm_server **out) {
    if (!ctx || !cfg || !out) return fail(LLHMM_E_INVALID, "ctx/cfg/out is NULL");
    *out = nullptr;
    if (cfg->precision != LLHMM_FP32 && cfg->precision != LLHMM_FP64) return fail(LLHMM_E_INVALID, "bad precision");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 16) return fail(LLHMM_E_INVALID, "max_inflight in [1, 16]");
    if (cfg->max_batch_boxes < 1) return fail(LLHMM_E_INVALID, "max_batch_boxes >= 1");
    if (cfg->device_bytes < (1 << 20)) return fail(LLHMM_E_INVALID, "device_bytes >= 1 MiB");
    if (!coefs || ncoefs <= 0) return fail(LLHMM_E_INVALID, "coefficients missing");
    if (cfg->K.p_x > 7 || cfg->K.p_t > 7) return fail(LLHMM_E_INVALID, "kernel order p must be <= 7");
    HIP_TRY(hipSetDevice(ctx->device));
    llhmm_server *sv = new llhmm_server();
    sv->ctx = ctx;
    sv->cfg = *cfg;
    sv->coefs.assign(coefs, coefs + ncoefs);
    hipError_t e = sv->arena.init((size_t)cfg->device_bytes);
    const size_t mb = (size_t)cfg->max_batch_boxes;
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->H_host, sizeof(double) * cfg->max_inflight * mb * kServeQ);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->st_host, sizeof(int32_t) * cfg->max_inflight * mb);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->ids_host, sizeof(int64_t) * cfg->max_inflight * mb);
    sv->slots.resize(cfg->max_inflight);
    sv->streams.assign(cfg->max_inflight, nullptr);
    for (int k = 0; k < cfg->max_inflight && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&sv->streams[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->slots[k].done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        server_free(sv);
        return fail(e == hipErrorOutOfMemory ? LLHMM_E_NOMEM : LLHMM_E_HIP, "server: %s", hipGetErrorString(e));
    }
    *out = sv;
    return LLHMM_OK;
}

llhmm_status llhmm_server_destroy(llhmm_server *sv) {
    server_free(sv);
    return LLHMM_OK;
}

llhmm_status llhmm_server_submit(llhmm_server *sv, const llhmm_box *boxes, int32_t n, const int64_t *ids,
                                 const double *m_init_dev, const llhmm_macro *macro, const double *M_macro_dev) {
    if (!sv || (n > 0 && (!boxes || !ids))) return fail(LLHMM_E_INVALID, "server/boxes/ids is NULL");
    std::vector<ServeReq> reqs(n);
    const double t = now_s();
    for (int i = 0; i < n; ++i) {
        ServeReq &r = reqs[i];
        r.box = boxes[i];
        r.id = ids[i];
        r.t_submit = t;
        r.m_init = m_init_dev;
        r.M_macro = M_macro_dev;
        memset(&r.macro, 0, sizeof r.macro);
        r.has_macro = macro != nullptr;
        if (macro) r.macro = *macro;
        if (boxes[i].init_mode == LLHMM_INIT_EXPLICIT && !m_init_dev)
            return fail(LLHMM_E_INVALID, "request %d: explicit init needs m_init_dev", i);
        if (boxes[i].init_mode == LLHMM_INIT_MACRO_Q && (!macro || !M_macro_dev))
            return fail(LLHMM_E_INVALID, "request %d: macro init needs macro and M_macro_dev", i);
        llhmm_status st = request_bytes(sv, r.box, i, r.bytes);
        if (st != LLHMM_OK) return st;
    }
    for (ServeReq &r : reqs) sv->queue.push_back(r);
    return serve_admit(sv);
}

llhmm_status llhmm_server_poll(llhmm_server *sv, int32_t wait, int32_t max, int64_t *ids_out, double *H_out,
                               int32_t *status_out, double *latency_us_out, int32_t *ndone) {
    if (!sv || !ndone) return fail(LLHMM_E_INVALID, "server/ndone is NULL");
    *ndone = 0;
    HIP_TRY(hipSetDevice(sv->ctx->device));
    llhmm_status st = serve_complete(sv);
    if (st == LLHMM_OK) st = serve_admit(sv);
    while (st == LLHMM_OK && wait && sv->done.empty()) {
        ServeFlight *oldest = nullptr;
        for (ServeFlight &f : sv->slots)
            if (f.busy && (!oldest || f.seq < oldest->seq)) oldest = &f;
        if (!oldest) break;  // nothing in flight and nothing admissible
        HIP_TRY(hipEventSynchronize(oldest->done));
        st = serve_complete(sv);
        if (st == LLHMM_OK) st = serve_admit(sv);
    }
    if (st != LLHMM_OK) return st;
    int k = 0;
    while (k < max && !sv->done.empty()) {
        const ServeDone &d = sv->done.front();
        if (ids_out) ids_out[k] = d.id;
        if (H_out) memcpy(H_out + (size_t)k * kServeQ, d.H, sizeof d.H);
        if (status_out) status_out[k] = d.status;
        if (latency_us_out) latency_us_out[k] = d.latency_us;
        sv->done.pop_front();
        ++k;
    }
    *ndone = k;
    return LLHMM_OK;
}

llhmm_status llhmm_server_set_output(llhmm_server *sv, double *H_dev, int32_t ld, int64_t nrows) {
    if (!sv) return fail(LLHMM_E_INVALID, "server is NULL");
    if (H_dev && (ld < 1 || nrows < 1)) return fail(LLHMM_E_INVALID, "ld and nrows must be >= 1");
    sv->out_H = H_dev;
    sv->out_ld = H_dev ? ld : 0;
    sv->out_rows = H_dev ? nrows : 0;
    return LLHMM_OK;
}

llhmm_status llhmm_server_stats(const llhmm_server *sv, int64_t *queued, int64_t *inflight,
                                int64_t *bytes_in_use, int64_t *bytes_total) {
    if (!sv) return fail(LLHMM_E_INVALID, "server is NULL");
    int64_t fl = 0;
    for (const ServeFlight &f : sv->slots)
        if (f.busy) fl += (int64_t)f.reqs.size();
    if (queued) *queued = (int64_t)sv->queue.size();
    if (inflight) *inflight = fl;
    if (bytes_in_use) *bytes_in_use = (int64_t)sv->arena.used;
    if (bytes_total) *bytes_total = (int64_t)sv->arena.size;
    return LLHMM_OK;
}

}  // extern "C"

// ------------------------------------------------------------ allocation-free solve
// The scratch memory of llhmm_solve_noalloc: one array per device, holding a
// whole batch's descriptors, tables, slab exchange rows and partial sums.  In host code
// `scratch` names a host-side stand-in, never the device memory: its device
// address is taken once per device with hipGetSymbolAddress (with that device
// current) and only that address is used.
static __device__ __align__(256) char scratch[LLHMM_NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_of_device;

static llhmm_status scratch_address(int device, char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_of_device.find(device);
    if (it != g_scratch_of_device.end()) {
        *out = it->second;
        return LLHMM_OK;
    }
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    HIP_TRY(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
        return fail(LLHMM_E_HIP, "scratch array of device %d: hipGetSymbolAddress: %s", device,
                    hipGetErrorString(e));
    if ((uintptr_t)p % Arena::kAlign)
        return fail(LLHMM_E_HIP, "scratch array of device %d is not %zu-byte aligned", device, Arena::kAlign);
    g_scratch_of_device[device] = (char *)p;
    *out = (char *)p;
    return LLHMM_OK;
}

extern "C" {

int64_t llhmm_noalloc_bytes(void) { return (int64_t)LLHMM_NOALLOC_BYTES; }

llhmm_status llhmm_solve_noalloc(llhmm_ctx *ctx, const llhmm_box *boxes, int32_t nboxes,
                                 const llhmm_kernel *K, const llhmm_coef *coefs, int32_t ncoefs,
                                 int32_t precision, const double *m_init_dev, const llhmm_macro *macro,
                                 const double *M_macro_dev, const double *coef_dev, double *H_avg_dev,
                                 int32_t ld, int32_t *status_dev, hipStream_t stream) {
    if (!ctx) return fail(LLHMM_E_INVALID, "ctx is NULL");
    if (!ctx->scratch) return fail(LLHMM_E_HIP, "context has no scratch array");
    // The batch lives in the scratch array: a fresh first-fit arena over it per
    // call, one stream (no side streams, events or graphs), tables uploaded in
    // stream order so that a previous call still reading the array is not
    // overtaken.
    Arena arena;
    arena.init_external(ctx->scratch, (size_t)LLHMM_NOALLOC_BYTES);
    llhmm_batch *b = nullptr;
    llhmm_status st = batch_create_impl(ctx, boxes, nboxes, K, coefs, ncoefs, precision, &arena, 1, &b,
                                        stream, true);
    if (st == LLHMM_E_NOMEM)
        return fail(LLHMM_E_BUDGET, "batch does not fit the %lld-byte scratch array of the allocation-free "
                    "solve (%d boxes); use llhmm_batch_create or split the batch",
                    (long long)LLHMM_NOALLOC_BYTES, nboxes);
    if (st != LLHMM_OK) return st;
    if (H_avg_dev) {
        for (const BoxPlan &P : b->plans_h)
            if (P.nq > ld) {
                batch_free(b);
                return fail(LLHMM_E_INVALID, "ld %d smaller than the outputs per box", ld);
            }
    }
    st = run_batch(ctx, b, m_init_dev, macro, M_macro_dev, coef_dev, nullptr, 0, stream);
    if (st == LLHMM_OK) {
        const hipError_t e = launch_upscale(b->partials, b->wave_status, b->box_const, b->plans, b->nboxes,
                                            H_avg_dev, ld, b->status, status_dev, stream);
        if (e != hipSuccess) st = fail(LLHMM_E_HIP, "upscale launch: %s", hipGetErrorString(e));
    }
    batch_free(b);  // host bookkeeping only: the arena hands the array back, nothing is freed on the device
    return st;
}

}  // extern "C"
