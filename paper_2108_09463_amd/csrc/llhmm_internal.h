// Internal types shared by the host side (llhmm_host.cpp) and the gfx950
// kernels.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>
#include "../../include/llhmm.h"

namespace llhmm {

constexpr int kGhost = LLHMM_GHOST;
constexpr int kMaxWaves = 16;  // waves per block of the resident kernels
// Largest distance between neighbouring points of a final state that counts as
// resolved (status bit 4 above it)
constexpr double kRoughMax = 0.5;
constexpr int kMaxQ = 9;       // outputs per box (flux in 3-D: 3 axes x 3 components)
// Layout options of the resident kernels (bits of MicroLane's OPT):
constexpr int kOptForm1 = 1;  // reference + perturbation form in FP64 too (no boundary offsets)
constexpr int kOptRefG = 2;   // form-1 reference tables read from global memory instead of LDS
constexpr int kOptHReg = 4;   // H(r) of the own points in registers; LDS keeps r and |r|^2 - 1
constexpr int kMaxXcc = 8;     // accelerator complexes (XCDs) per device, each with its own L2
constexpr int kFaceHalo = 3;   // faces -2 .. n stored per line: n + 3 entries
// FP32 reference + perturbation form: every kRerefSteps time steps the state
// is re-expressed around a new reference r' = fl(r + u) (MicroLane::rereference).
constexpr int kRerefSteps = 8;
// Slab kernels: steps between the workgroup-wide checks for a wait that gave up
constexpr int kAbortCheckSteps = 8;

// Per-box plan as the kernels read it.
struct BoxPlan {
    int32_t dim, n, order, stages;       // stages: 2 (HeunP) or 4 (RK4P)
    int32_t bc, quantity, init_mode, M;  // M: number of time steps
    int32_t coef_index, mi0, mi1, nq;    // macro node; nq = outputs per box
    int32_t coef_sampled, nwaves, prec, form;   // form: 0 direct, 1 reference + perturbation
    int32_t slab, strips, mi2, pad1_;    // slab: box advanced in row slabs (large boxes), strips: their count; mi2: 3-D node
    double dt, alpha, dx, mu;
    double mu_box, a_scale, out_scale, cx;
    double cy, wsum;                     // wsum = sum_n w^n (time weights)
    double cz, pad2_;                    // 3-D: centre along x3
    int64_t init_offset, coef_offset, wt_offset, mfinal_offset;
    int64_t tab_offset;                  // element offset (in T) of the box's tables
    int64_t w_offset;                    // element offset (double) of the space weights
    int64_t s64_offset;                  // element offset (double) of the set-up scratch (form 1)
    int64_t part_offset;                 // first partial-sum slot of the box (nwaves slots)
    int64_t state_offset;                // unused
    int64_t ref_offset;                  // unused
};

// Per-box table layout (elements of T, starting at tab_offset), n = points per
// axis, C = n^dim points, lines = n^(dim-1).
//   form 0 (direct: the state is m itself; FP64 path)
//     m0   [3][C]                  initial micro state
//     ax   [lines][n + 3]          x1 faces f = -2..n (index f + 2), scaled a
//     ay   [n][n + 3]   (2-D)      x2 faces per column, index f + 2
//     tau1 [lines][2][3][8]        boundary flux offsets, x1 (west, east): per face
//                                  hi[3], 0, lo[3], 0 with tau = hi + lo (double word)
//     tau2 [n][2][3][8] (2-D)      boundary flux offsets, x2 (south, north)
//   form 1 (reference + perturbation: m = r + u; FP32 path)
//     u0   [3][C]                  m_init - r, the rounding residual of the reference
//     r    [3][C]                  reference r = fl(m_init) at the points
//     dm   [C]                     |r|^2 - 1 (computed in FP64)
//     H0   [3][C]                  H(r) with the boundary data, computed in FP64
//     ax, ay as in form 0 (no tau tables: u is periodic or zero on the ghosts)
// Space weights (double, at w_offset): wc [n] (points), wf [n] (east faces).
// Form-1 set-up scratch per box (doubles): FP64 scaled face coefficients
// ax [lines][n+3], ay [n][n+3] (2-D), then ghost references gx [lines][2][3][3]
// (x1: points -3..-1 and n..n+2 of each line), gy [n][2][3][3] (2-D).
__host__ __device__ inline int64_t scratch64_size(int d, int n) {
    const int64_t lines = (d == 1) ? 1 : n;
    return (lines + (d == 2 ? n : 0)) * (n + 3) + (lines + (d == 2 ? n : 0)) * 18;
}

struct TabLayout {
    int64_t m0, ref, dm, H0, ax, ay, tau1, tau2, size;
};
__host__ __device__ inline TabLayout tab_layout(int d, int n, int form) {
    TabLayout t;
    const int64_t C = (d == 1) ? (int64_t)n : (int64_t)n * n;
    const int64_t lines = (d == 1) ? 1 : n;
    t.m0 = 0;
    if (form == 1) {
        t.ref = 3 * C;
        t.dm = 6 * C;
        t.H0 = 7 * C;
        t.ax = 10 * C;
    } else {
        t.ref = t.dm = t.H0 = 0;
        t.ax = 3 * C;
    }
    t.ay = t.ax + lines * (n + kFaceHalo);
    t.tau1 = t.ay + (d == 1 ? 0 : (int64_t)n * (n + kFaceHalo));
    t.tau2 = t.tau1 + (form == 1 ? 0 : lines * 48);
    t.size = t.tau2 + (form == 1 || d == 1 ? 0 : (int64_t)n * 48);
    t.size = (t.size + 63) & ~(int64_t)63;
    return t;
}

// Kernel-side view of a material coefficient (same layout as llhmm_coef).
struct CoefDev {
    int32_t dim, n_terms, sampled, pad_;
    double c0;
    double amp[LLHMM_MAX_TERMS];
    double freq[LLHMM_MAX_TERMS][3];
    double phase[LLHMM_MAX_TERMS][3];
};
static_assert(sizeof(CoefDev) == sizeof(llhmm_coef), "coef layout");

// Grid indices (with ghosts) of the largest box whose micro data the set-up
// kernel interpolates from the macro field: 1-D boxes up to n = 256, 2-D up to 128.
constexpr int kLagMax = 256 + 2 * kGhost;
constexpr int kLagMax2 = 128 + 2 * kGhost;
constexpr int kMaxN3 = 64;  // largest d = 3 box (points per axis)

struct MacroDev {
    int32_t dim, n;
    double dX, x0[3];
};

struct PrologueArgs {
    const BoxPlan *plans;
    int32_t nboxes, mode_pad;
    const CoefDev *coefs;
    const double *m_init;
    const double *M_macro;
    MacroDev macro;
    const double *coef_samples;
    void *tabs;            // T tables
    double *wts;           // space weights
    double *box_const;     // [nboxes][kMaxQ]: average of the reference part (form 1)
    double *scratch64;     // form 1 set-up scratch: FP64 faces and ghost references per box
    double kc[8];          // space kernel coefficients c_0..c_p
    int32_t kp, kq;
};

// Everything a micro-kernel launch needs.  Passed by value.
struct MicroArgs {
    const BoxPlan *plans;      // [nboxes]
    const int32_t *box_ids;    // boxes of this tile class, in launch order
    int32_t nbox_class;        // entries in box_ids
    int32_t mode;              // 0 solve, 1 evaluate H(m0) only
    const void *tabs;          // per-box tables (T)
    const double *wts;         // space weights
    const double *wt;          // time-weight table
    double *partials;          // [slots][kMaxQ], box slots from part_offset
    int32_t *wave_status;      // [slots]
    double *out_field;         // m_final or H (nullable)
};

// Slab mode (large 2-D boxes): a box is cut into slabs of consecutive
// full-width rows, one workgroup per slab for the whole solve.  The workgroup
// holds a window of R * NG rows: its own rows and h halo rows on each side,
// which it advances redundantly; after every `spe` time steps it publishes
// the edge rows of its own rows and replaces its halo rows by its
// neighbours' published rows (global memory, tagged words).  One persistent
// launch per class; its workgroups take (box, slab) items from the queue of
// the XCD they run on.
struct SlabJob {
    int32_t box, slab, nslabs, o0;  // slab owns box rows [o0, o0 + rows)
    int32_t rows, pad_;
    int64_t xoff;                   // word offset of the box's exchange area
};

struct SlabArgs {
    const BoxPlan *plans;
    const SlabJob *jobs;        // items, in the order they are taken
    int32_t nqueues, mode;      // work queues (one per XCD); mode 0 solve, 1 evaluate H(m0) only
    int32_t qoff[kMaxXcc + 1];  // queue q holds items [qoff[q], qoff[q + 1]) of jobs
    int32_t *counter;           // next item of each queue [nqueues] (zero before the launch)
    int32_t *abort_word;        // set when a wait gives up (zero before the launch)
    long long spin_max;         // polls before a wait gives up
    int32_t h, spe;             // halo rows per side; time steps per exchange
    int32_t xdepth, pad_;       // rows per published edge
    const void *tabs;           // per-box tables (T)
    const double *wts;          // space weights
    const double *wt;           // time-weight table
    double *partials;           // [slots][kMaxQ]
    int32_t *wave_status;       // [slots]
    uint64_t *xbuf;             // per box [slabs][2 edges][2 parities][xdepth rows][3][n][words per value]
    double *out_field;          // m_final or H (nullable)
};

using SlabLaunchFn = hipError_t (*)(const SlabArgs &, int nblocks, hipStream_t);
using SlabOccFn = hipError_t (*)(int *blocks_per_cu);

struct SlabTileInfo {
    int n, order, bc, prec, qty;  // class it serves (2-D)
    int L, K, R, NG, NBUF;       // a window of R * NG rows of n = K * L points
    int threads;
    SlabLaunchFn launch;
    SlabOccFn occupancy;
    const char *name;
};

const SlabTileInfo *tiles_slab(int *count);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// dst[ids[r] * ld + q] = src[r * src_ld + q] for q < nq and 0 <= ids[r] < nrows
hipError_t launch_scatter_rows(const double *src, int src_ld, const int64_t *ids, int n, int nq, double *dst,
                               int ld, int64_t nrows, hipStream_t s);

using LaunchFn = hipError_t (*)(const MicroArgs &, int nblocks, hipStream_t);

struct TileInfo {
    int dim, n, order, bc, prec, qty; // class it serves
    int L, K, R, NG, NBUF;            // layout
    int threads, boxes_per_block;
    LaunchFn launch;
    const char *name;
    int opt;                          // layout options (kOpt* bits of the kernel)
};

const TileInfo *tiles_f32_2d(int *count);
const TileInfo *tiles_f64_2d(int *count);
const TileInfo *tiles_f32_1d(int *count);
const TileInfo *tiles_f64_1d(int *count);

hipError_t launch_prologue(int prec, const PrologueArgs &a, hipStream_t s);
hipError_t launch_upscale(const double *partials, const int32_t *wave_status,
                          const double *box_const, const BoxPlan *plans, int nboxes, double *H, int ld,
                          int32_t *status, int32_t *status_out, hipStream_t s);
hipError_t launch_macro(int npts, int model, int scheme, int step_index, int stage, double dt,
                        double alpha, double *M, const double *H, double *Y,
                        double *work, hipStream_t s);
hipError_t launch_flux_div(int dim, int n, double dX, int order, const double *F, int ld, double *H,
                           hipStream_t s);

}  // namespace llhmm
