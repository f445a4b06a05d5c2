// Time-stepping kernel for gfx950 (CDNA4): one workgroup per 2-D micro box
// (or several 1-D boxes per workgroup), the whole box resident on chip for all
// of its time steps.
//
// Method (Leitenmaier & Runborg): eq. (micro) of Section 2.2 time-stepped with
// HeunP / RK4P (Section 3.1), H = div(a grad m) by the second-order central
// difference of Section 2.3 (or a fourth-order conservative stencil), boundary
// data of Section 4.2, and the kernel average eq. (upscaling).
//
// Layout.  A "row group" of L lanes (L = 16: one DPP row; L = 64: a whole
// wavefront) spans a full box row of N = K*L points; lane j owns the K
// consecutive columns [jK, jK+K) of the R rows [gR, gR+R) of its group g.
// State m, stage input y and the Runge-Kutta accumulator live in VGPRs.
//   * x1 neighbours come from the adjacent lane through DPP row/wave rotations
//     (periodic m - m_init) or shifts with zero fill (Dirichlet), which the
//     compiler fuses into the consuming VALU instruction;
//   * x2 neighbours across row groups go through a small LDS halo buffer
//     (YH rows per group side; double buffered: one barrier per stage);
//   * boundary data enter as a constant offset tau_f = a_f G_f(delta) on the
//     fluxes of the faces whose stencil reaches a ghost point (delta = ghost
//     value minus wrapped value, or the ghost value for Dirichlet): the stencil
//     is linear, so wrapped or zero-filled neighbours plus tau_f reproduce the
//     ghost-point stencil exactly;
//   * the kernel-weighted average is accumulated per lane in FP64 (per step:
//     sum_j w_j Q_j(m^n) times the time weight w^n), reduced across the
//     wavefront by shuffles and written as one FP64 partial per wave.
#pragma once
#include "llhmm_internal.h"

namespace llhmm {

// ----------------------------------------------------------------- DPP
template <int L> struct DppCtl;
// FR: lane i <- lane i+1 ("from the right"); FL: lane i <- lane i-1.
template <> struct DppCtl<16> {
    static constexpr int ROT_FR = 0x12F;  // row_ror:15
    static constexpr int ROT_FL = 0x121;  // row_ror:1
    static constexpr int SH_FR = 0x101;   // row_shl:1 (lane 15 of the row reads 0)
    static constexpr int SH_FL = 0x111;   // row_shr:1 (lane 0 of the row reads 0)
};
template <> struct DppCtl<64> {
    static constexpr int ROT_FR = 0x134;  // wave_rol:1
    static constexpr int ROT_FL = 0x13C;  // wave_ror:1
    static constexpr int SH_FR = 0x130;   // wave_shl:1
    static constexpr int SH_FL = 0x138;   // wave_shr:1
};

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64 1/sqrt(x): the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2, each squaring the relative error, so the result is
// within about an ulp (the projection's argument is |m|^2 ~ 1, a normal number)
__device__ __forceinline__ double rsqrt_t(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double r = __builtin_fma(-x * y, y, 1.0);
        y = __builtin_fma(0.5 * y, r, y);
    }
    return y;
}
// 1/x: the hardware reciprocal in FP32 (the projection divides a perturbation-size
// quantity by 1 + sqrt(1 + e) ~ 2, where its 1-ulp error is far below the state's
// rounding); exact division in FP64.
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }


// ----------------------------------------------------------------- table copies
// Copies ROWS rows of N elements from global memory into LDS (row r to
// dst + r * N) with 16-byte accesses.  All of a thread's loads are issued
// before its first LDS store, so they are in flight together instead of each
// paying the full memory latency.  src_row(r) is the global start of row r
// (16-byte aligned).
template <typename T, int N, int ROWS, int NT, typename SrcRow>
__device__ __forceinline__ void copy_rows_to_lds(T *dst, SrcRow src_row, int tid) {
    constexpr int V = 16 / (int)sizeof(T);
    static_assert(N % V == 0, "rows must split into 16-byte vectors");
    typedef T VT __attribute__((ext_vector_type(V)));
    constexpr int RV = N / V, TOT = ROWS * RV, ITER = (TOT + NT - 1) / NT;
    VT buf[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int i = it * NT + tid;
        if (TOT % NT == 0 || i < TOT) {
            const int r = i / RV, cv = i - r * RV;
            buf[it] = *(const VT *)(src_row(r) + cv * V);
        }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int i = it * NT + tid;
        if (TOT % NT == 0 || i < TOT) {
            const int r = i / RV, cv = i - r * RV;
            *(VT *)(dst + r * N + cv * V) = buf[it];
        }
    }
}

enum { AVG_NONE = 0, AVG_FIELD = 1, AVG_TORQUE = 2, AVG_FLUX = 3, AVG_EVAL = 4, AVG_DREF = 5 };



// Cross-workgroup exchange words (slab mode).  A value travels with the
// index of the exchange that produced it in one 64-bit word (FP32: the value's
// bits and the index; FP64: two words, one per half), written and read as
// agent-scope atomics: each access is coherent across the XCDs' L2 caches
// without whole-cache write-back or invalidation, and a reader that sees the
// index it waits for has the value with it, so no separate flag is needed.
template <typename T>
__device__ __forceinline__ void xstore(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xload(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> struct XWords { static constexpr int n = sizeof(T) / 4; };  // words per value
// Exchange words go between workgroups on one XCD: a plain store leaves them in
// that XCD's L2, where the agent-scope loads of its other CUs find them,
// without the write-through to memory an agent-scope store makes.
__device__ __forceinline__ void xstore_xcd(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void xput(uint64_t *p, float v, uint32_t tag) {
    xstore_xcd(p, (uint64_t)__builtin_bit_cast(uint32_t, v) | ((uint64_t)tag << 32));
}
__device__ __forceinline__ void xput(uint64_t *p, double v, uint32_t tag) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    xstore_xcd(p, (uint64_t)((b & 0xffffffffu) | ((uint64_t)tag << 32)));
    xstore_xcd(p + 1, (uint64_t)((b >> 32) | ((uint64_t)tag << 32)));
}
// The accelerator complex (XCD) this wave runs on.
__device__ __forceinline__ int xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);  // HW_REG_XCC_ID, bits 3:0
}
// Reads a value whose words carry at least `tag`; false while any word is older.
__device__ __forceinline__ bool xget(const uint64_t *p, uint32_t tag, float &v) {
    const uint64_t w = xload(p);
    v = __builtin_bit_cast(float, (uint32_t)w);
    return (uint32_t)(w >> 32) >= tag;
}
__device__ __forceinline__ bool xget(const uint64_t *p, uint32_t tag, double &v) {
    const uint64_t a = xload(p), b = xload(p + 1);
    v = __builtin_bit_cast(double, (a & 0xffffffffull) | (b << 32));
    return (uint32_t)(a >> 32) >= tag && (uint32_t)(b >> 32) >= tag;
}

template <typename T, int D, int ORD, int BC, int QTY, int L, int K, int R, int NG, int NBUF,
          bool SLAB = false, int OPT = 0>
struct MicroLane {
    static constexpr int N = K * L;
    static constexpr int YH = (ORD == 2) ? 1 : 3;  // neighbour reach in points
    static constexpr int FW = (ORD == 2) ? 1 : 2;  // faces west/south of the first own point
    static constexpr int FE = (ORD == 2) ? 0 : 1;  // faces east/north of the last own point
    static constexpr int NF = K + FW + FE;         // x1 faces per lane row
    static constexpr int NFR = R + FW + FE;        // x2 faces per lane column
    static constexpr int GF = (ORD == 2) ? 1 : 3;  // faces per side touched by ghosts
    static constexpr int KD = (D == 2) ? K : 1;
    static constexpr int NFRD = (D == 2) ? NFR : 1;
    static constexpr int NQ = (QTY == LLHMM_Q_FLUX) ? 3 * D : 3;
    static constexpr int AVG = (QTY == LLHMM_Q_FIELD) ? 1 : ((QTY == LLHMM_Q_TORQUE) ? 2 : 3);
    // LDS halo per row group: its first and last YH rows, or all R rows once
    // when those overlap (R <= 2 YH); the last YH rows of a group's block are
    // its top rows either way
    static constexpr int HROWS = (2 * YH >= R) ? R : 2 * YH;
    static constexpr int HALO = (D == 2) ? NG * HROWS * 3 * N : 1;
    // 2-D boundary offsets in LDS: [2N lines/columns][2 sides][GF faces][hi 4, lo 4],
    // then a zero block read by lanes without boundary faces
    static constexpr int TAU_LDS = (D == 2) ? 4 * N * GF * 8 + 24 : 1;
    static constexpr int ZOFF = 4 * N * GF * 8;
    // FP64: face coefficients are read from LDS (x1 faces [lines][LF], 2-D x2
    // faces [N][LF] after them) instead of being held in registers
    static constexpr bool AXL = !SLAB && sizeof(T) == 8;
    static constexpr int LF = N + kFaceHalo;
    static constexpr int AX_LDS = AXL ? ((D == 2) ? 2 * N * LF : NG * LF) : 1;
    static constexpr int WLDS = (D == 2) ? 2 * N : NG * 2 * N;  // space weights in LDS
    // form 1 (FP32): m = r + u with the FP32 reference r = fl(m_init) and H(r)
    // precomputed in FP64; the state u starts at the rounding residual m_init - r
    // and stays periodic (or zero) on the ghosts, so no boundary offsets are needed.
    // Slab mode (a window of R * NG rows of a larger 2-D box) always uses form 1.
    static constexpr int FORM = (SLAB || sizeof(T) == 4 || (OPT & kOptForm1)) ? 1 : 0;
    static constexpr int CELLS = (D == 1) ? N : N * N;
    static constexpr int WR = R * NG;                       // rows held by the block
    static constexpr int CELLS_W = SLAB ? WR * N : CELLS;    // points held by the block
    // FP64 slab: the reference tables are read from global memory (box indexing)
    static constexpr bool REFG = (SLAB && sizeof(T) == 8) || (OPT & kOptRefG);
    // FP32 fourth-order slabs keep H(r) in registers too (the window's seven
    // planes and the wider halo would not fit the LDS)
    static constexpr bool HREG = ((OPT & kOptHReg) || (SLAB && ORD == 4)) && FORM && !REFG;
    static constexpr int RSTRIDE = REFG ? CELLS : CELLS_W;  // stride between reference planes
    static constexpr int REF_PLANES = HREG ? 4 : 7;          // planes held in LDS
    static constexpr int REF_LDS = (FORM && !REFG) ? ((D == 2) ? REF_PLANES * CELLS_W : NG * 7 * N) : 1;
    // x1 neighbours more than K points away come from lanes further off (several
    // DPP moves); the boundary offsets of form 0 assume one lane holds them all
    static_assert(K >= YH || FORM == 1, "lane tile narrower than the stencil reach");
    // periodic second-order 2-D form 0: x1 fluxes formed once per face (as in form 1)
    // with the seam offsets added by FMA; seam faces on both axes take the
    // offset's high word only
    static constexpr bool SEAM0 = (ORD == 2) && (FORM == 0) && (BC == LLHMM_BC_PERIODIC_PERT) && (D == 2);
    // second-order 2-D stages update the group's interior rows before waiting
    // for the other groups' halo rows
    static constexpr bool SPLIT = (ORD == 2) && (D == 2) && (R >= 3);
    // SEAM0 with one column per lane: a lane has at most one seam face, and its
    // x1 part is a_e g_e + (T - a_w g_w) by two FMAs, T the lane's seam offset
    // (held negated for the west seam in the unused low-word slots)
    static constexpr bool SEAMK1 = SEAM0 && (K == 1);
    static_assert(!HREG || D == 2, "H(r) in registers: 2-D");
    static_assert(D == 1 || R >= YH, "row group thinner than the stencil reach");
    static_assert(D == 1 || SLAB || R * NG == N, "row groups must tile the box");
    static_assert(!SLAB || D == 2, "slab mode: 2-D");
    static_assert(D == 2 || R == 1, "1-D boxes are one row");
    static_assert(L == 16 || L == 64, "row group is a DPP row or a wavefront");

    T m[R][K][3], y[R][K][3], acc[R][K][3];
    T hr[HREG ? R : 1][HREG ? K : 1][3];  // H(r) of the own points (kOptHReg)
    T ax[AXL ? 1 : R][AXL ? 1 : NF];
    T ay[AXL ? 1 : KD][AXL ? 1 : NFRD];
    const T *s_axl;  // AXL: this group's face coefficients in LDS
    T tauF[(D == 1) ? GF : 1][6], tauL[(D == 1) ? GF : 1][6];  // hi[3], lo[3]
    int tFb, tFs, tLb, tLs, tSb, tSs, tNb, tNs;  // LDS offsets: base + index * stride
    int tTb, tTs;  // SEAMT: the lane's seam offset (-tau west at lane 0, +tau east at lane L-1)
    double acc64[NQ];
    int g, c0, r0, gs, gn;
    bool zero_s, zero_n;
    T alpha, dt;
    T *s_halo, *s_zero, *s_tau;
    T *s_ref;          // form 1: this box's r [3][C], |r|^2-1 [C], H(r) [3][C] (LDS or global)
    const double *wl;  // this box's point weights [N] then east-face weights [N] (LDS)
    // slab mode: box row of each own row, whether the block owns it, and the
    // x2 point / face weights of the window rows (zero on rows it does not own)
    int brow[SLAB ? R : 1];
    bool own[SLAB ? R : 1];
    const double *s_wyl;
    const T *s_edge;   // slab: z of the box rows just outside the window (re-referencing)
    // slab, exchange at every stage (the window is the slab's own rows): the
    // neighbouring slabs' edge rows of each stage input come through tagged
    // words into LDS rows; the edge groups publish their first / last YH rows
    // of every stage result
    bool xs_on;                     // per-stage exchange
    bool xs_get[2], xs_put[2];      // [south, north]: read the neighbour's rows / publish own edge rows
    bool xs_pub;                    // publish this stage's result
    int xs_fail;                    // a wait gave up
    const uint64_t *xs_src[2];      // neighbours' edge words (parity 0; parity 1 at + xs_par)
    uint64_t *xs_dst[2];            // own edge words
    long xs_par;
    T *s_xrow;                      // LDS [2 sides][YH rows][3][N]
    int32_t *xs_abort;
    long long xs_spin;

    template <int CTRL_ROT, int CTRL_SH>
    __device__ __forceinline__ static T nb(T v) {
        return dpp_mov<(BC == LLHMM_BC_PERIODIC_PERT) ? CTRL_ROT : CTRL_SH>(v);
    }
    __device__ __forceinline__ double wv(int i) const { return wl[i]; }
    __device__ __forceinline__ double wy(int r) const {
        return SLAB ? s_wyl[r0 + r] : ((D == 2) ? wv(r0 + r) : 1.0);
    }
    __device__ __forceinline__ double wyf(int r) const { return SLAB ? s_wyl[WR + r0 + r] : wv(N + r0 + r); }
    __device__ __forceinline__ bool owned(int r) const { return SLAB ? own[SLAB ? r : 0] : true; }
    __device__ __forceinline__ int out_row(int r) const { return SLAB ? brow[SLAB ? r : 0] : r0 + r; }
    // index of own point (r, k) in the reference tables
    __device__ __forceinline__ int cell_of(int r, int k) const {
        return SLAB ? ((REFG ? brow[SLAB ? r : 0] : r0 + r) * N + c0 + k) : ((D == 1 ? 0 : (r0 + r) * N) + c0 + k);
    }
    __device__ __forceinline__ T tau_lds(int off) const {
        return FORM ? (T)0 : s_tau[off];
    }
    __device__ __forceinline__ T ref(int q, int cell) const { return s_ref[q * RSTRIDE + cell]; }
    // component c of H(r) at own point (r, k)
    __device__ __forceinline__ T href(int r, int k, int c, int cell) const {
        return HREG ? hr[HREG ? r : 0][HREG ? k : 0][c] : ref(4 + c, cell);
    }
    // face coefficient of x1 face lf of own row r / x2 face lr of own column k
    __device__ __forceinline__ T axv(int r, int lf) const {
        return AXL ? s_axl[(r0 + r) * LF + c0 - FW + lf + 2] : ax[AXL ? 0 : r][AXL ? 0 : lf];
    }
    __device__ __forceinline__ T ayv(int k, int lr) const {
        // x2 faces in LDS face-row major ([LF][N]): the lanes of a row group read
        // consecutive words, free of bank conflicts
        return AXL ? s_axl[N * LF + (r0 - FW + lr + 2) * N + c0 + k] : ay[AXL ? 0 : k][AXL ? 0 : lr];
    }

    // Per-stage exchange: reads the neighbours' edge rows that carry `tag` into
    // the LDS rows (a wait gives up after xs_spin polls or when another
    // workgroup has given up; the stage then goes on with whatever it read).
    __device__ __forceinline__ void xs_receive(uint32_t tag) {
        constexpr int XW = XWords<T>::n;
        const long par = (long)(tag & 1) * xs_par;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (!xs_get[side]) continue;
            const uint64_t *sb = xs_src[side] + par;
            T *dst = s_xrow + side * YH * 3 * N;
            long long polls = 0;
            {
                // first wait on the word this lane's publisher writes last
                T v;
                const uint64_t *sw = sb + ((long)((YH - 1) * 3 + 2) * N + c0 + K - 1) * XW;
                while (!xget(sw, tag, v)) {
                    if (xload(xs_abort) != 0 || ++polls > xs_spin) break;
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            for (;;) {
                bool all = true;
#pragma unroll
                for (int q = 0; q < YH; ++q)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            T v;
                            all &= xget(sb + ((long)(q * 3 + c) * N + c0 + k) * XW, tag, v);
                            dst[(q * 3 + c) * N + c0 + k] = v;
                        }
                if (all) break;
                if (xload(xs_abort) != 0 || ++polls > xs_spin) {
                    xs_fail = 1;
                    xstore(xs_abort, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    // Publishes the edge rows of the current y (the next stage's input) with `tag`.
    __device__ __forceinline__ void xs_publish(uint32_t tag) {
        constexpr int XW = XWords<T>::n;
        const long par = (long)(tag & 1) * xs_par;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (!xs_put[side]) continue;
            uint64_t *db = xs_dst[side] + par;
#pragma unroll
            for (int q = 0; q < YH; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        xput(db + ((long)(q * 3 + c) * N + c0 + k) * XW, y[side == 0 ? q : R - YH + q][k][c], tag);
        }
    }

    // One Runge-Kutta stage on stage input y: H(y), f(y), accumulator and
    // next stage input (or the projected new state when LAST).  With AVG != 0
    // this is stage 1 of a step: y == m^n and Q(m^n) is added to the average.
    template <int AVG, bool FIRST, bool LAST>
    __device__ __forceinline__ void stage(T bs, T cdt, double wn, int tstage, double *eval_out,
                                          long eval_cells) {
        asm volatile("" ::: "memory");  // keep per-cell LDS tables out of registers across stages
        // ---- x2 halo exchange through LDS
        const T *srcS = s_zero, *srcN = s_zero;
        if (D == 2) {
            T *hb = s_halo + (NBUF == 2 ? (tstage & 1) * HALO : 0);
            if (NBUF == 1) __syncthreads();
#pragma unroll
            for (int q = 0; q < YH; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        if (HROWS == 2 * YH) {
                            hb[((g * HROWS + q) * 3 + c) * N + c0 + k] = y[q][k][c];
                            hb[((g * HROWS + YH + q) * 3 + c) * N + c0 + k] = y[R - YH + q][k][c];
                        }
                    }
            if (HROWS == R && HROWS != 2 * YH) {
#pragma unroll
                for (int q = 0; q < R; ++q)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int k = 0; k < K; ++k) hb[((g * HROWS + q) * 3 + c) * N + c0 + k] = y[q][k][c];
            }
        }
        // the other groups' halo rows, readable after the barrier
        auto halo_ready = [&]() {
            if (D != 2) return;
            const T *hb = s_halo + (NBUF == 2 ? (tstage & 1) * HALO : 0);
            __syncthreads();
            // The edge groups wait for the neighbour slabs' rows after the
            // barrier, so the other groups go on meanwhile.  Each lane reads back
            // only the LDS words it wrote itself: no second barrier.  Stage 0
            // reads the neighbours' rows of the initial state, loaded from the
            // tables with the window.
            if (SLAB && xs_on && tstage > 0) xs_receive((uint32_t)tstage);
            srcS = zero_s ? s_zero : hb + (gs * HROWS + HROWS - YH) * 3 * N;
            srcN = zero_n ? s_zero : hb + (gn * HROWS + 0) * 3 * N;
            if (SLAB && xs_on) {
                if (xs_get[0]) srcS = s_xrow;
                if (xs_get[1]) srcN = s_xrow + YH * 3 * N;
            } else if (SLAB && AVG == AVG_DREF) {  // the reference change is known beyond the window
                if (g == 0) srcS = s_edge;
                if (g == NG - 1) srcN = s_edge + YH * 3 * N;
            }
        };
        if (!SPLIT) halo_ready();
        auto yat = [&](int q, int k, int c) -> T {  // local row q in [-YH, R+YH); halo rows from LDS
            if (q < 0) return *(const T *)(srcS + ((q + YH) * 3 + c) * N + c0 + k);
            if (q >= R) return *(const T *)(srcN + ((q - R) * 3 + c) * N + c0 + k);
            return y[(q < 0 || q >= R) ? 0 : q][k][c];
        };
        auto face2 = [&](int lr, int k, int c) -> T {  // flux on x2 face row lr
            const int q = lr - FW;                      // face between rows q and q+1
            T gr;
            if (ORD == 2) gr = yat(q + 1, k, c) - yat(q, k, c);
            else gr = (T)27 * (yat(q + 1, k, c) - yat(q, k, c)) - (yat(q + 2, k, c) - yat(q - 1, k, c));
            if (FORM == 1 || (lr >= GF && lr < NFR - GF)) return ayv(k, lr) * gr;
            const int off = (lr < GF) ? tSb + k * tSs + lr * 8 : tNb + k * tNs + (lr - (NFR - GF)) * 8;
            if constexpr (SEAM0) return fma_t(ayv(k, lr), gr, tau_lds(off + c));
            // boundary face: flux + tau as a double word (hi by FMA, then lo)
            return fma_t(ayv(k, lr), gr, tau_lds(off + c)) + tau_lds(off + 4 + c);
        };
        // sliding window of x2 face fluxes: faces lr = r .. r+FW+FE-1 before row r.
        // SPLIT: rows 1 .. R-2 first (their faces are the group's own), then the
        // barrier, then rows 0 and R-1 with the halo faces; face 1 (row 0's north
        // face) and face R-1 (row R-1's south face) are kept from the first pass.
        T F2[(D == 2) ? FW + FE : 1][KD][3];
        T Fk1[SPLIT ? KD : 1][3], FkL[SPLIT ? KD : 1][3];
        if (D == 2) {
#pragma unroll
            for (int w = 0; w < FW + FE; ++w)
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        F2[w][k][c] = face2(SPLIT ? w + 1 : w, k, c);
                        if (SPLIT) Fk1[SPLIT ? k : 0][c] = F2[w][k][c];
                    }
        }
        double sq[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) sq[q] = 0.0;

#pragma unroll
        for (int it = 0; it < R; ++it) {
            const int r = SPLIT ? ((it < R - 2) ? it + 1 : ((it == R - 2) ? 0 : R - 1)) : it;
            if (SPLIT && it == R - 2) {
                halo_ready();
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        FkL[SPLIT ? k : 0][c] = F2[0][k][c];
                        F2[0][k][c] = face2(0, k, c);
                    }
            }
            if (SPLIT && it == R - 1) {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) F2[0][k][c] = FkL[SPLIT ? k : 0][c];
            }
            // Periodic second order, form 1: every x1 face flux is formed once.  The
            // east gradients of the own columns (the last one reaches the right
            // neighbour), and the west flux of column 0 as the left neighbour's last
            // east gradient times this lane's own west-face coefficient, so the two
            // sides of the box's periodic seam keep their own coefficients.
            // Periodic second order, form 0: the same, with the box seam's flux offset
            // (lanes at the row's ends; zero elsewhere) taken into the seam faces'
            // FMA.  Its rounding residual is left out: the seam gradient itself is
            // rounded at that level.
            constexpr bool X1FAST = (ORD == 2) && (FORM == 1 || SEAM0) && (BC == LLHMM_BC_PERIODIC_PERT);
            constexpr bool SEAMT = SEAMK1 && AVG != AVG_FLUX;
            T ge[X1FAST ? K : 1][3], Fwest[3];
            auto tau_w = [&](int c) -> T { return SEAM0 ? tau_lds(tFb + r * tFs + c) : (T)0; };
            auto tau_e = [&](int c) -> T { return SEAM0 ? tau_lds(tLb + r * tLs + c) : (T)0; };
            if constexpr (X1FAST) {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        ge[k][c] = (k + 1 < K) ? y[r][(k + 1 < K) ? k + 1 : 0][c] - y[r][k][c]
                                               : dpp_mov<DppCtl<L>::ROT_FR>(y[r][0][c]) - y[r][K - 1][c];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T gw = dpp_mov<DppCtl<L>::ROT_FL>(ge[K - 1][c]);
                    if (SEAMT) Fwest[c] = fma_t(-axv(r, 0), gw, tau_lds(tTb + r * tTs + c));  // T - F_w
                    else Fwest[c] = SEAM0 ? fma_t(axv(r, 0), gw, tau_w(c)) : axv(r, 0) * gw;
                }
            }
            // x1 halo values from the neighbouring lanes (taken before any update of this row)
            T yw[YH][3], ye[YH][3];
            if constexpr (!X1FAST) {
#pragma unroll
                for (int i = 0; i < YH; ++i)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        // column c0 - YH + i: `hw` lanes to the west; c0 + K + i: `he` lanes east
                        constexpr int KK = K;
                        const int hw = (YH - i + KK - 1) / KK, he = i / KK + 1;
                        T vw = y[r][(K - YH + i + hw * K) % K][c], ve = y[r][i % K][c];
#pragma unroll
                        for (int hop = 0; hop < (YH + KK - 1) / KK; ++hop) {
                            if (hop < hw) vw = nb<DppCtl<L>::ROT_FL, DppCtl<L>::SH_FL>(vw);
                            if (hop < he) ve = nb<DppCtl<L>::ROT_FR, DppCtl<L>::SH_FR>(ve);
                        }
                        yw[i][c] = vw;
                        ye[i][c] = ve;
                    }
            }
            // row values at local column p in [-YH, K+YH)
            auto yrow = [&](int p, int c) -> T {
                return (p < 0) ? yw[p + YH][c] : ((p >= K) ? ye[p - K][c] : y[r][p][c]);
            };
            auto face1 = [&](int lf, int c) -> T {  // flux on x1 face lf (between p and p+1)
                const int p = lf - FW;
                T gr;
                if (ORD == 2) gr = yrow(p + 1, c) - yrow(p, c);
                else gr = (T)27 * (yrow(p + 1, c) - yrow(p, c)) - (yrow(p + 2, c) - yrow(p - 1, c));
                if (FORM == 1 || (lf >= GF && lf < NF - GF)) return axv(r, lf) * gr;
                // boundary face: flux + tau as a double word (hi by FMA, then lo)
                T hi, lo;
                if (lf < GF) {
                    hi = (D == 1) ? tauF[(D == 1) ? lf : 0][c] : tau_lds(tFb + r * tFs + lf * 8 + c);
                    lo = (D == 1) ? tauF[(D == 1) ? lf : 0][3 + c] : tau_lds(tFb + r * tFs + lf * 8 + 4 + c);
                } else {
                    const int q = lf - (NF - GF);
                    hi = (D == 1) ? tauL[(D == 1) ? q : 0][c] : tau_lds(tLb + r * tLs + q * 8 + c);
                    lo = (D == 1) ? tauL[(D == 1) ? q : 0][3 + c] : tau_lds(tLb + r * tLs + q * 8 + 4 + c);
                }
                return fma_t(axv(r, lf), gr, hi) + lo;
            };
            // rolling window of x1 fluxes: faces lf = k .. k+FW+FE-1 before cell k
            T Fw[FW + FE][3];
            if constexpr (!X1FAST) {
#pragma unroll
                for (int w = 0; w < FW + FE; ++w)
#pragma unroll
                    for (int c = 0; c < 3; ++c) Fw[w][c] = face1(w, c);
            }

#pragma unroll
            for (int k = 0; k < K; ++k) {
                T H[3], Fx_east[3];
                if constexpr (X1FAST) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (k + 1 < K || AVG == AVG_FLUX || (AVG == AVG_DREF && QTY == LLHMM_Q_FLUX)) {
                            const T fe = (SEAM0 && k + 1 == K) ? fma_t(axv(r, K), ge[k][c], tau_e(c))
                                                               : axv(r, k + 1) * ge[k][c];
                            H[c] = fe - Fwest[c];
                            Fx_east[c] = fe;
                            Fwest[c] = fe;
                        } else if (SEAMT) {
                            H[c] = fma_t(axv(r, K), ge[K - 1][c], Fwest[c]);
                            Fx_east[c] = (T)0;
                        } else if (SEAM0) {
                            H[c] = fma_t(axv(r, K), ge[K - 1][c], tau_e(c)) - Fwest[c];
                            Fx_east[c] = (T)0;
                        } else {
                            H[c] = fma_t(axv(r, K), ge[K - 1][c], -Fwest[c]);
                            Fx_east[c] = (T)0;
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < (X1FAST ? 0 : 3); ++c) {
                    const T fnew = face1(k + FW + FE, c);
                    if (ORD == 2) H[c] = fnew - Fw[0][c];
                    else H[c] = (T)27 * (Fw[(ORD == 2) ? 0 : 2][c] - Fw[(ORD == 2) ? 0 : 1][c]) - (fnew - Fw[0][c]);
                    Fx_east[c] = (FW == FW + FE) ? fnew : Fw[(FW < FW + FE) ? FW : 0][c];
#pragma unroll
                    for (int w = 0; w + 1 < FW + FE; ++w) Fw[w][c] = Fw[w + 1][c];
                    Fw[FW + FE - 1][c] = fnew;
                }
                T Fy_north[3];
                if (D == 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const T fnew = (SPLIT && r == 0) ? Fk1[SPLIT ? k : 0][c] : face2(r + FW + FE, k, c);
                        T h2;
                        if (ORD == 2) h2 = fnew - F2[0][k][c];
                        else h2 = (T)27 * (F2[(ORD == 2) ? 0 : 2][k][c] - F2[(ORD == 2) ? 0 : 1][k][c]) - (fnew - F2[0][k][c]);
                        H[c] = H[c] + h2;
                        Fy_north[c] = (FW == FW + FE) ? fnew : F2[(FW < FW + FE) ? FW : 0][k][c];
#pragma unroll
                        for (int w = 0; w + 1 < FW + FE; ++w) F2[w][k][c] = F2[w + 1][k][c];
                        F2[FW + FE - 1][k][c] = fnew;
                    }
                }
                if (AVG == AVG_DREF) {
                    // field of the reference change: kept in acc, and its average times
                    // the remaining time weight joins the constant part of the average
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[r][k][c] = H[c];
                    if (owned(r)) {
                        if (QTY == LLHMM_Q_FIELD) {
                            const double w = wv(c0 + k) * wy(r);
#pragma unroll
                            for (int c = 0; c < 3; ++c) sq[c] = fma(w, (double)H[c], sq[c]);
                        } else if (QTY == LLHMM_Q_FLUX) {
                            const double w1 = wv(N + c0 + k) * wy(r);
#pragma unroll
                            for (int c = 0; c < 3; ++c) sq[c] = fma(w1, (double)Fx_east[c], sq[c]);
                            if (D == 2) {
                                const double w2 = wv(c0 + k) * wyf(r);
#pragma unroll
                                for (int c = 0; c < 3; ++c)
                                    sq[(D == 2 ? 3 : 0) + c] = fma(w2, (double)Fy_north[c], sq[(D == 2 ? 3 : 0) + c]);
                            }
                        }
                    }
                    continue;
                }
                if (AVG == AVG_EVAL) {
                    const int cell = cell_of(r, k);
                    if (owned(r)) {
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            eval_out[c * eval_cells + (long)out_row(r) * N + c0 + k] =
                                (double)H[c] + (FORM ? (double)href(r, k, c, cell) : 0.0);
                    }
                    continue;
                }
                // ---- right-hand side f = -y x H - alpha y x (y x H), average, update
                const int cell = cell_of(r, k);
                // full state and field at this point: form 0 y, H; form 1 r + v, H(r) + D(v)
                T m0 = y[r][k][0], m1 = y[r][k][1], m2 = y[r][k][2];
                T h0 = H[0], h1 = H[1], h2 = H[2];
                if (FORM == 1) {
                    m0 += ref(0, cell);
                    m1 += ref(1, cell);
                    m2 += ref(2, cell);
                    h0 += href(r, k, 0, cell);
                    h1 += href(r, k, 1, cell);
                    h2 += href(r, k, 2, cell);
                }
                const T cx = m1 * h2 - m2 * h1;
                const T cy = m2 * h0 - m0 * h2;
                const T cz = m0 * h1 - m1 * h0;
                const T ex = m1 * cz - m2 * cy;
                const T ey = m2 * cx - m0 * cz;
                const T ez = m0 * cy - m1 * cx;
                const T f[3] = {-fma_t(alpha, ex, cx), -fma_t(alpha, ey, cy), -fma_t(alpha, ez, cz)};
                if ((AVG == AVG_FIELD || AVG == AVG_TORQUE) && owned(r)) {
                    // form 1 field: only D(u); the constant sum_j w_j H(r)_j is added at upscale
                    const double w = wv(c0 + k) * wy(r);
                    sq[0] = fma(w, (double)(AVG == AVG_FIELD ? H[0] : cx), sq[0]);
                    sq[1] = fma(w, (double)(AVG == AVG_FIELD ? H[1] : cy), sq[1]);
                    sq[2] = fma(w, (double)(AVG == AVG_FIELD ? H[2] : cz), sq[2]);
                } else if (AVG == AVG_FLUX && owned(r)) {
                    const double w1 = wv(N + c0 + k) * wy(r);
#pragma unroll
                    for (int c = 0; c < 3; ++c) sq[c] = fma(w1, (double)Fx_east[c], sq[c]);
                    if (D == 2) {
                        const double w2 = wv(c0 + k) * wyf(r);
#pragma unroll
                        for (int c = 0; c < 3; ++c) sq[(D == 2 ? 3 : 0) + c] = fma(w2, (double)Fy_north[c], sq[(D == 2 ? 3 : 0) + c]);
                    }
                }
                if constexpr (sizeof(T) == 8 && AVG >= AVG_FIELD && AVG <= AVG_FLUX) {
                    // FP64: the averages are finished point by point.  Left free, the
                    // scheduler moves the serial FMA chain of each sum to the end of
                    // the stage and keeps every point's field live until then, which
                    // spills to scratch in the 64-point-wide boxes.
#pragma unroll
                    for (int q = 0; q < NQ; ++q) asm volatile("" : "+v"(sq[q]));
                }
                if (!LAST) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        acc[r][k][c] = FIRST ? bs * f[c] : fma_t(bs, f[c], acc[r][k][c]);
                        y[r][k][c] = fma_t(cdt, f[c], m[r][k][c]);
                    }
                } else if (FORM == 0) {
                    T mt[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) mt[c] = fma_t(dt, fma_t(bs, f[c], acc[r][k][c]), m[r][k][c]);
                    const T inv = rsqrt_t(fma_t(mt[0], mt[0], fma_t(mt[1], mt[1], mt[2] * mt[2])));
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        m[r][k][c] = mt[c] * inv;
                        y[r][k][c] = m[r][k][c];
                    }
                } else {
                    // projection of r + ut onto the unit sphere, kept in perturbation form:
                    // e = |r + ut|^2 - 1 = 2 r.ut + |ut|^2 + (|r|^2 - 1), n = sqrt(1 + e),
                    // u = (r + ut)/n - r = (ut - r e / (1 + n)) / n
                    T ut[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) ut[c] = fma_t(dt, fma_t(bs, f[c], acc[r][k][c]), m[r][k][c]);
                    const T r0v = ref(0, cell), r1v = ref(1, cell), r2v = ref(2, cell);
                    const T e = fma_t((T)2, fma_t(r0v, ut[0], fma_t(r1v, ut[1], r2v * ut[2])),
                                      fma_t(ut[0], ut[0], fma_t(ut[1], ut[1], fma_t(ut[2], ut[2], ref(3, cell)))));
                    const T inv = rsqrt_t((T)1 + e);
                    const T nn = ((T)1 + e) * inv;
                    const T q = e * rcp_t((T)1 + nn);
                    m[r][k][0] = (ut[0] - r0v * q) * inv;
                    m[r][k][1] = (ut[1] - r1v * q) * inv;
                    m[r][k][2] = (ut[2] - r2v * q) * inv;
#pragma unroll
                    for (int c = 0; c < 3; ++c) y[r][k][c] = m[r][k][c];
                }
            }
        }
        if ((AVG >= AVG_FIELD && AVG <= AVG_FLUX) || (AVG == AVG_DREF && QTY != LLHMM_Q_TORQUE)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc64[q] = fma(wn, sq[q], acc64[q]);
        }
        if (SLAB && xs_on && xs_pub && AVG != AVG_DREF && AVG != AVG_EVAL) xs_publish((uint32_t)tstage + 1);
    }

    // Status bits of the final state of this lane's own points (every lane of
    // the group calls it; `live`: the lane holds box points):
    //   4  two neighbouring points differ by more than kRoughMax (an
    //      unresolved, grid-scale state: what an unstable run leaves, since
    //      the projection keeps it on the unit sphere);
    //   8  ||m|^2 - 1| exceeds the precision's drift tolerance.
    // Neighbours along x1 (the next lane's first column through DPP; the pair
    // across the box edge is skipped) and along x2 within the lane's rows.
    __device__ __forceinline__ int health(bool live) const {
        T mf[R][K][3];
        int bits = 0;
        // an opaque zero: keeps the table addresses below from being computed
        // ahead of the time loop, where they would only add register pressure
        int opaque;
        asm volatile("v_mov_b32 %0, 0" : "=v"(opaque));
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cell = cell_of(r, k) + opaque;
                T e;
                if (FORM == 1) {
                    const T r0v = ref(0, cell), r1v = ref(1, cell), r2v = ref(2, cell);
                    const T u0 = m[r][k][0], u1 = m[r][k][1], u2 = m[r][k][2];
                    e = fma_t((T)2, fma_t(r0v, u0, fma_t(r1v, u1, r2v * u2)),
                              fma_t(u0, u0, fma_t(u1, u1, fma_t(u2, u2, ref(3, cell)))));
                    mf[r][k][0] = r0v + u0;
                    mf[r][k][1] = r1v + u1;
                    mf[r][k][2] = r2v + u2;
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) mf[r][k][c] = m[r][k][c];
                    e = fma_t(mf[r][k][0], mf[r][k][0], fma_t(mf[r][k][1], mf[r][k][1],
                                                             fma_t(mf[r][k][2], mf[r][k][2], (T)-1)));
                }
                const T tol = (sizeof(T) == 4) ? (T)1e-4 : (T)1e-10;
                if (live && owned(r) && !(__builtin_fabs(e) <= tol)) bits |= 8;
            }
        const bool edge_lane = (L == 16) ? ((threadIdx.x & 15) == 15) : ((threadIdx.x & 63) == 63);
        auto far = [](T a0, T a1, T a2, T b0, T b1, T b2) {
            const T d0 = a0 - b0, d1 = a1 - b1, d2 = a2 - b2;
            return !(fma_t(d0, d0, fma_t(d1, d1, d2 * d2)) <= (T)(kRoughMax * kRoughMax));
        };
#pragma unroll
        for (int r = 0; r < R; ++r) {
            T east[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) east[c] = dpp_mov<DppCtl<L>::ROT_FR>(mf[r][0][c]);
            if (!(live && owned(r))) continue;
#pragma unroll
            for (int k = 0; k + 1 < K; ++k)
                if (far(mf[r][k][0], mf[r][k][1], mf[r][k][2], mf[r][k + 1][0], mf[r][k + 1][1], mf[r][k + 1][2]))
                    bits |= 4;
            if (!edge_lane && far(mf[r][K - 1][0], mf[r][K - 1][1], mf[r][K - 1][2], east[0], east[1], east[2]))
                bits |= 4;
            if (D == 2 && r + 1 < R && owned(r + 1 < R ? r + 1 : r) &&
                far(mf[r][0][0], mf[r][0][1], mf[r][0][2], mf[(r + 1 < R) ? r + 1 : r][0][0],
                    mf[(r + 1 < R) ? r + 1 : r][0][1], mf[(r + 1 < R) ? r + 1 : r][0][2]))
                bits |= 4;
        }
        return bits;
    }

    // FP32 form 1 only.  Over many small steps the FP32 perturbation u keeps
    // only the top bits of each step's increment once |u| has grown, and the
    // stencil's 1/dx^2 turns the lost bits into field error.  Re-referencing
    // moves the representable part of u into the reference: r' = fl(r + u),
    // z = r' - r and u' = u - z are exact (Fast2Sum, |r| >= |u|), so r' + u' =
    // r + u and |u'| <= ulp(r)/2.  The tables follow: |r'|^2 - 1 from exact
    // FP64 squares, H(r') = H(r) + D(z) (D linear; D(z) through the stage's
    // stencil with z in the stage-input registers and the result in the
    // accumulator, both free at a step boundary), and the average's constant
    // part gains w_tail * sum_j w_j D(z)_j, w_tail = sum_{n' >= n} w^n'.
    // Every lane writes only its own points' table entries.
    __device__ __forceinline__ void rereference(double w_tail, int tstage) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cell = cell_of(r, k);
                double n2 = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T rv = s_ref[c * RSTRIDE + cell];
                    const T sv = rv + m[r][k][c];
                    const T z = sv - rv;
                    m[r][k][c] = m[r][k][c] - z;
                    y[r][k][c] = z;
                    s_ref[c * RSTRIDE + cell] = sv;
                    n2 = fma((double)sv, (double)sv, n2);
                }
                s_ref[3 * RSTRIDE + cell] = (T)(n2 - 1.0);
            }
        // per-stage slab exchange: the neighbours take this z for their edge rows
        if (SLAB && xs_on) xs_publish((uint32_t)tstage);
        stage<AVG_DREF, true, false>((T)0, (T)0, w_tail, tstage, nullptr, 0);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int cell = cell_of(r, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (HREG) hr[HREG ? r : 0][HREG ? k : 0][c] = hr[HREG ? r : 0][HREG ? k : 0][c] + acc[r][k][c];
                    else s_ref[(4 + c) * RSTRIDE + cell] = s_ref[(4 + c) * RSTRIDE + cell] + acc[r][k][c];
                    y[r][k][c] = m[r][k][c];
                }
            }
        if (SLAB && xs_on) xs_publish((uint32_t)tstage + 1);
    }
};

template <typename T, int D, int ORD, int BC, int QTY, int L, int K, int R, int NG, int NBUF, int MINW,
          int OPT = 0>
__global__ void __launch_bounds__(L * NG, MINW) k_micro(MicroArgs A) {
    using Lane = MicroLane<T, D, ORD, BC, QTY, L, K, R, NG, NBUF, false, OPT>;
    constexpr int N = Lane::N, NF = Lane::NF, FW = Lane::FW, GF = Lane::GF;
    constexpr int YH = Lane::YH, NQ = Lane::NQ;
    __shared__ T s_halo[NBUF * Lane::HALO];
    __shared__ T s_zero[(D == 2) ? YH * 3 * N : 1];
    __shared__ T s_tau[Lane::FORM ? 1 : Lane::TAU_LDS];
    __shared__ T s_refl[Lane::REF_LDS];
    __shared__ double s_w[Lane::WLDS];
    __shared__ T s_ax[Lane::AX_LDS];
    constexpr int FORM = Lane::FORM;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // the wavefront index is uniform across the wave: in a scalar register, the
    // row group of a 64-lane group and everything derived from it are too
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = (L == 16) ? (lane & 15) : lane;
    Lane S;
    S.g = (L == 16) ? (wave * 4 + (lane >> 4)) : wave;
    S.c0 = j * K;
    S.r0 = (D == 2) ? S.g * R : 0;
    const int g = S.g, c0 = S.c0, r0 = S.r0;

    // 2-D: one box per block.  1-D: NG boxes per block (one per row group); the
    // host groups 1-D boxes so that a block's boxes share M, the integrator and
    // the time weights, and pads the last block with -1 (inactive groups).
    const int slot = (D == 2) ? (int)blockIdx.x : (int)blockIdx.x * NG + g;
    const int lead = A.box_ids[(D == 2) ? (int)blockIdx.x : (int)blockIdx.x * NG];
    int box = (slot < A.nbox_class) ? A.box_ids[slot] : -1;
    const bool active = box >= 0;
    if (!active) box = lead;
    const BoxPlan &P = A.plans[box];
    const BoxPlan &PU = A.plans[lead];  // block-uniform controls
    const T *tab = (const T *)A.tabs + P.tab_offset;
    constexpr long CELLS = (D == 1) ? (long)N : (long)N * N;
    const TabLayout TL = tab_layout(D, N, FORM);
    constexpr int LF = N + kFaceHalo;  // faces stored per line

    // ---------------- load the box tables
    if (Lane::AXL) {
        // x1 faces then (2-D) x2 faces; ay follows ax in the table
        if (D == 2) {
            // x1 faces as stored ([lines][LF]); x2 faces transposed to [LF][N]
            for (int i = tid; i < N * LF; i += L * NG) s_ax[i] = tab[TL.ax + i];
            for (int i = tid; i < N * LF; i += L * NG) {
                const int f = i / N, col = i - f * N;
                s_ax[N * LF + i] = tab[TL.ay + (long)col * LF + f];
            }
            S.s_axl = s_ax;
        } else {
            for (int i = j; i < LF; i += L) s_ax[g * LF + i] = tab[TL.ax + i];
            S.s_axl = s_ax + g * LF;
        }
    } else {
        S.s_axl = nullptr;
#pragma unroll
        for (int r = 0; r < (Lane::AXL ? 0 : R); ++r)
#pragma unroll
            for (int lf = 0; lf < NF; ++lf)
                S.ax[Lane::AXL ? 0 : r][Lane::AXL ? 0 : lf] = tab[TL.ax + (long)(r0 + r) * LF + (c0 - FW + lf) + 2];
        if (D == 2) {
#pragma unroll
            for (int k = 0; k < (Lane::AXL ? 0 : Lane::KD); ++k)
#pragma unroll
                for (int lr = 0; lr < Lane::NFRD; ++lr)
                    S.ay[Lane::AXL ? 0 : k][Lane::AXL ? 0 : lr] = tab[TL.ay + (long)(c0 + k) * LF + (r0 - FW + lr) + 2];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                S.m[r][k][c] = tab[TL.m0 + c * CELLS + (long)(r0 + r) * N + c0 + k];
                S.y[r][k][c] = S.m[r][k][c];
                S.acc[r][k][c] = (T)0;
            }
    // space weights of this box into LDS
    const double *wsrc = A.wts + P.w_offset;
    if (D == 2) {
        for (int i = tid; i < 2 * N; i += L * NG) s_w[i] = wsrc[i];
        S.wl = s_w;
    } else {
        for (int i = j; i < 2 * N; i += L) s_w[g * 2 * N + i] = wsrc[i];
        S.wl = s_w + g * 2 * N;
    }
    S.s_ref = nullptr;
    if (FORM == 1) {
        // reference, |r|^2 - 1 and H(r) of this box into LDS (7 values per point);
        // kOptHReg: H(r) of the own points into registers; kOptRefG: read in place
        if (D == 2 && Lane::REFG) {
            S.s_ref = const_cast<T *>(tab) + TL.ref;
        } else if (D == 2) {
            const T *src = tab + TL.ref;
            copy_rows_to_lds<T, N, (D == 2) ? Lane::REF_PLANES * N : 1, L * NG>(
                s_refl, [&](int r) { return src + (long)r * N; }, tid);
            S.s_ref = s_refl;
            if (Lane::HREG) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            S.hr[Lane::HREG ? r : 0][Lane::HREG ? k : 0][c] =
                                src[(4 + c) * CELLS + (long)(r0 + r) * N + c0 + k];
            }
        } else {
            for (int i = j; i < 7 * N; i += L) s_refl[g * 7 * N + i] = tab[TL.ref + i];
            S.s_ref = s_refl + g * 7 * N;
        }
        for (int i = tid; i < ((D == 2) ? YH * 3 * N : 0); i += L * NG) s_zero[i] = (T)0;
#pragma unroll
        for (int q = 0; q < ((D == 1) ? GF : 1); ++q)
#pragma unroll
            for (int c = 0; c < 6; ++c) S.tauF[q][c] = S.tauL[q][c] = (T)0;
        S.tFb = S.tFs = S.tLb = S.tLs = S.tSb = S.tSs = S.tNb = S.tNs = S.tTb = S.tTs = 0;
    } else {
        // boundary offsets: 1-D in registers (lanes 0 and L-1), 2-D in LDS
        if (D == 1) {
#pragma unroll
            for (int q = 0; q < ((D == 1) ? GF : 1); ++q)
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const int e = (c < 3) ? c : c + 1;  // hi[0..2] at 0..2, lo[0..2] at 4..6
                    T tf = tab[TL.tau1 + (0 * 3 + q) * 8 + e];
                    T tl = tab[TL.tau1 + (1 * 3 + q) * 8 + e];
                    S.tauF[q][c] = (j == 0) ? tf : (T)0;
                    S.tauL[q][c] = (j == L - 1) ? tl : (T)0;
                }
        } else {
            // tables hold [2N][2 sides][3][8]; LDS keeps the GF faces that are used
            constexpr int TS = GF * 8;
            for (int i = tid; i < 4 * N * TS; i += L * NG) {
                const int pr = i / TS, e = i % TS;  // (line, side) pair, entry
                // SEAMK1: the west x1 offsets' low-word slots hold -hi
                const bool neg = Lane::SEAMK1 && pr < 2 * N && (pr & 1) == 0 && e >= 4 && e < 7;
                s_tau[i] = neg ? -tab[TL.tau1 + pr * 24 + e - 4] : tab[TL.tau1 + pr * 24 + e];
            }
            for (int i = tid; i < 24; i += L * NG) s_tau[Lane::ZOFF + i] = (T)0;
            for (int i = tid; i < YH * 3 * N; i += L * NG) s_zero[i] = (T)0;
            S.tFb = (j == 0) ? (r0 * 2 + 0) * TS : Lane::ZOFF;
            S.tFs = (j == 0) ? 2 * TS : 0;
            S.tLb = (j == L - 1) ? (r0 * 2 + 1) * TS : Lane::ZOFF;
            S.tLs = (j == L - 1) ? 2 * TS : 0;
            S.tSb = (g == 0) ? 2 * N * TS + (c0 * 2 + 0) * TS : Lane::ZOFF;
            S.tSs = (g == 0) ? 2 * TS : 0;
            S.tNb = (g == NG - 1) ? 2 * N * TS + (c0 * 2 + 1) * TS : Lane::ZOFF;
            S.tNs = (g == NG - 1) ? 2 * TS : 0;
            S.tTb = (j == 0) ? (r0 * 2 + 0) * TS + 4 : ((j == L - 1) ? (r0 * 2 + 1) * TS : Lane::ZOFF);
            S.tTs = (j == 0 || j == L - 1) ? 2 * TS : 0;
        }
    }
    __syncthreads();
    S.gs = (g + NG - 1) % NG;
    S.gn = (g + 1) % NG;
    S.zero_s = (BC == LLHMM_BC_DIRICHLET) && (g == 0);
    S.zero_n = (BC == LLHMM_BC_DIRICHLET) && (g == NG - 1);
    S.s_halo = s_halo;
    S.s_zero = s_zero;
    S.s_tau = s_tau;
    S.alpha = (T)P.alpha;
    S.dt = (T)P.dt;
#pragma unroll
    for (int q = 0; q < NQ; ++q) S.acc64[q] = 0.0;

    if (A.mode == 1) {  // evaluate H(m0) only
        if (active)
            S.template stage<AVG_EVAL, true, false>((T)0, (T)0, 0.0, 0, A.out_field + P.mfinal_offset, CELLS);
        return;
    }

    const int M = PU.M;
    const bool rk4 = (PU.stages == 4);
    constexpr bool REREF = (FORM == 1) && (sizeof(T) == 4);
    // stage-1 data: b_1 and c_2 dt; RK4P b = (1,2,2,1)/6, c = (1/2, 1/2, 1); HeunP b = (1/2, 1/2), c = (1)
    const T b1 = rk4 ? (T)(1.0 / 6.0) : (T)0.5;
    const T c2dt = rk4 ? (T)(0.5 * P.dt) : (T)P.dt;  // per box (1-D lanes may differ)
    const T third = (T)(1.0 / 3.0);
    const T half_dt = (T)(0.5 * P.dt);
    const double *wtab = A.wt + PU.wt_offset;  // w^0..w^M, then the tails sum_{n' >= n} w^n'
    int ts = 0;
    for (int n = 0; n < M; ++n) {
        const double wn = wtab[n];
        if (REREF && n > 0 && n % kRerefSteps == 0) S.rereference(wtab[M + 1 + n], ts++);
        asm volatile("" ::: "memory");
        S.template stage<Lane::AVG, true, false>(b1, c2dt, wn, ts, nullptr, 0);
        ++ts;
        // RK4P: two middle stages (b = 1/3; c = 1/2, 1), then the last (b = 1/6).
        // HeunP: only the last stage (b = 1/2).
        const int nmid = rk4 ? 2 : 0;
        for (int sm = 0; sm < nmid; ++sm) {
            S.template stage<AVG_NONE, false, false>(third, sm == 0 ? half_dt : S.dt, 0.0, ts++, nullptr, 0);
        }
        S.template stage<AVG_NONE, false, true>(rk4 ? (T)(1.0 / 6.0) : (T)0.5, (T)0, 0.0, ts++, nullptr, 0);
    }

    // ---------------- outputs
    if (A.out_field && active) {
        double *dst = A.out_field + P.mfinal_offset;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    dst[c * CELLS + (long)(r0 + r) * N + c0 + k] =
                        (double)S.m[r][k][c] +
                        (FORM ? (double)S.s_ref[c * CELLS + (D == 1 ? 0 : (r0 + r) * N) + c0 + k] : 0.0);
    }
    // reduce over the row group (1-D: one box) or the wavefront (2-D)
    constexpr int RED = (D == 1) ? L : 64;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = S.acc64[q];
#pragma unroll
        for (int off = 1; off < RED; off <<= 1) v += __shfl_xor(v, off, 64);
        S.acc64[q] = v;
    }
    // final-state checks over the row group (1-D: one box) or the wavefront (2-D)
    const int hb = S.health(active);
    const uint64_t gmask = (D == 1 && L == 16) ? (0xFFFFull << ((lane >> 4) * 16)) : ~0ull;
    const int hbits = ((__ballot((hb & 4) != 0) & gmask) ? 4 : 0) | ((__ballot((hb & 8) != 0) & gmask) ? 8 : 0);
    const bool writer = (D == 1) ? (j == 0) : (lane == 0);
    if (writer && active) {
        const int wslot = (D == 1) ? 0 : wave;
        double *dst = A.partials + (P.part_offset + wslot) * kMaxQ;
        int bad = hbits;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            dst[q] = S.acc64[q];
            if (!__builtin_isfinite(S.acc64[q])) bad |= 1;
        }
        A.wave_status[P.part_offset + wslot] = bad;
    }
}


// A block-uniform copy of *p in scalar registers.  Loads inside a loop that
// also stores to global memory are not provably unclobbered, so the compiler
// would keep them (and every address derived from them) in vector registers.
template <typename S>
__device__ __forceinline__ S uniform_load(const S *p) {
    static_assert(sizeof(S) % 4 == 0, "whole words");
    S out;
    int *o = reinterpret_cast<int *>(&out);
    const int *in = reinterpret_cast<const int *>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / 4); ++k) o[k] = __builtin_amdgcn_readfirstlane(in[k]);
    return out;
}

// Slab mode: one persistent grid advances the large 2-D boxes of one tile
// class.  A box is cut into slabs of consecutive full-width rows, one
// workgroup per slab for all of the box's time steps.  The workgroup holds a
// window of R * NG rows: the slab's own rows and at least h halo rows on each
// side (periodic images of box rows, or Dirichlet ghost rows held at u = 0).
// The window's outermost rows see zeros beyond it; the error that causes
// moves inwards one row per stage, so the own rows stay exact for h stages
// (h >= spe * stages).  After every spe time steps the workgroup publishes
// its edge rows and replaces its halo rows with its neighbours' published
// rows: box state never leaves the chip, and only those rows cross between
// workgroups.  Re-referencing (FP32) happens only at exchange steps, when
// every window row is exact, so a halo row's reference stays the one its
// owner computes (only the outermost row's H(r) update misses the point
// beyond the window, which stays inside the same error cone).
// Each XCD has its own queue of (box, slab) items, taken through an atomic
// counter by the workgroups running on it, so all slabs of a box share one L2
// and exchange through it.  In a queue the items of a box are consecutive and
// the boxes longest first.  A workgroup waiting for a neighbour's rows only
// waits for an item of its own box, which is taken before any later item, so
// a queue makes progress with any number of resident workgroups on its XCD
// >= slabs per box.  Every wait polls at most A.spin_max times; a wait that runs out sets
// the grid-wide abort word, every later wait ends at once on it, every
// workgroup stops at its next check (every kAbortCheckSteps steps and after
// the last step), and the boxes it touched report status 2.
// EVAL (a separate instantiation, so that the solve's register allocation
// does not carry the evaluation's): evaluate H(m0) on the own rows instead of
// solving; A.mode must agree.
template <typename T, int ORD, int QTY, int BC, int L, int K, int R, int NG, int NBUF, int MINW, bool EVAL, int OPT = 0>
__global__ void __launch_bounds__(L * NG, MINW) k_slab(SlabArgs A) {
    constexpr int D = 2;
    using Lane = MicroLane<T, D, ORD, BC, QTY, L, K, R, NG, NBUF, true, OPT>;
    constexpr int N = Lane::N, NF = Lane::NF, NFR = Lane::NFR, FW = Lane::FW, NQ = Lane::NQ;
    constexpr int YH = Lane::YH, WR = Lane::WR;
    constexpr long C = (long)N * N;
    constexpr int LF = N + kFaceHalo;
    constexpr int WAVES = L * NG / 64;
    constexpr int XW = XWords<T>::n;
    __shared__ T s_halo[NBUF * Lane::HALO];
    __shared__ T s_zero[2 * YH * 3 * N];   // zero rows: beyond Dirichlet edges, and both window edges
    __shared__ T s_refl[Lane::REF_LDS];
    __shared__ double s_w[2 * N];
    __shared__ double s_wyl[2 * WR];
    // per-stage exchange (second order): the neighbours' edge rows
    __shared__ T s_xrow[(ORD == 2) ? 2 * YH * 3 * N : 1];
    __shared__ int s_item, s_abort;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar register
    const int j = (L == 16) ? (lane & 15) : lane;
    for (int i = tid; i < 2 * YH * 3 * N; i += L * NG) s_zero[i] = (T)0;
    const int h = A.h, spe = A.spe, xd = A.xdepth;
    // spe == 0: exchange at every stage; the window holds only the slab's own
    // rows (h == 0) and the edge groups read their neighbours' rows from LDS
    const bool xs = (ORD == 2) && (spe == 0);
    const int queue = __builtin_amdgcn_readfirstlane(xcc_id() % A.nqueues);
    auto wrap = [](int br) { return ((br % N) + N) % N; };

    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(A.counter + queue, 1);
            s_abort = xload(A.abort_word);
        }
        __syncthreads();
        // block-uniform: in scalar registers, and so is everything derived from the item
        const int item = A.qoff[queue] + __builtin_amdgcn_readfirstlane(s_item);
        if (item >= A.qoff[queue + 1]) break;
        const SlabJob job = uniform_load(A.jobs + item);
        const BoxPlan P = uniform_load(A.plans + job.box);
        if (__builtin_amdgcn_readfirstlane(s_abort) != 0) {
            // a wait has given up: the remaining items only report it
            if (!EVAL && lane == 0) A.wave_status[P.part_offset + (long)job.slab * WAVES + wave] = 2;
            __syncthreads();
            continue;
        }
        const T *tab = (const T *)A.tabs + P.tab_offset;
        const TabLayout TL = tab_layout(D, N, 1);
        const int w0 = job.o0 - h;  // box row of window row 0, before wrapping
        const int own_end = h + job.rows;
        // Dead row groups, held at u = 0 and never exchanged: Dirichlet ghost rows
        // outside the box, and the window rows beyond the north halo (a slab with
        // fewer own rows than the window allows keeps an h-row halo on each side)
        auto dead = [&](int gg) {
            const int br = w0 + gg * R;
            return (BC == LLHMM_BC_DIRICHLET && (br < 0 || br >= N)) || gg * R >= own_end + h;
        };

        Lane S;
        S.g = (L == 16) ? (wave * 4 + (lane >> 4)) : wave;
        S.c0 = j * K;
        S.r0 = S.g * R;
        const int g = S.g, c0 = S.c0, r0 = S.r0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int wr = r0 + r;
            S.brow[r] = wrap(w0 + wr);
            S.own[r] = (wr >= h) && (wr < own_end);
        }
        const bool gdead = dead(g);
        // the group's role in the exchange (h, rows and xdepth are multiples of R)
        const bool halo_s = (r0 < h) && !gdead, halo_n = (r0 >= own_end) && !gdead;
        const bool pub_s = (r0 >= h) && (r0 < h + xd), pub_n = (r0 >= own_end - xd) && (r0 < own_end);
        const int ns = job.nslabs, sl = job.slab;
        const int s_south = (sl + ns - 1) % ns, s_north = (sl + 1) % ns;
        const bool has_s = (BC != LLHMM_BC_DIRICHLET) || (sl > 0);
        const bool has_n = (BC != LLHMM_BC_DIRICHLET) || (sl < ns - 1);
        constexpr long XROW = 3L * N * XW;   // words of one exchanged row
        uint64_t *xbox = A.xbuf + job.xoff;
        auto edge = [&](int slab, int side, int par) { return xbox + ((long)(slab * 2 + side) * 2 + par) * xd * XROW; };

        // space weights; window-row weights (zero on rows this block does not own)
        const double *wsrc = A.wts + P.w_offset;
        for (int i = tid; i < 2 * N; i += L * NG) s_w[i] = wsrc[i];
        for (int i = tid; i < WR; i += L * NG) {
            const bool own = (i >= h) && (i < own_end);
            const int br = wrap(w0 + i);
            s_wyl[i] = own ? wsrc[br] : 0.0;
            s_wyl[WR + i] = own ? wsrc[N + br] : 0.0;
        }
        S.wl = s_w;
        S.s_wyl = s_wyl;
        // reference r, |r|^2 - 1 and H(r): window copy in LDS (FP32) or the box tables (FP64)
        if (Lane::REFG) {
            S.s_ref = const_cast<T *>(tab) + TL.ref;
        } else {
            const T *src = tab + TL.ref;
            copy_rows_to_lds<T, N, Lane::REFG ? 1 : Lane::REF_PLANES * WR, L * NG>(
                s_refl,
                [&](int r) {
                    const int q = r / WR, wr = r - q * WR;
                    return src + q * C + (long)wrap(w0 + wr) * N;
                },
                tid);
            S.s_ref = s_refl;
            if (Lane::HREG) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            S.hr[Lane::HREG ? r : 0][Lane::HREG ? k : 0][c] =
                                src[(4 + c) * C + (long)S.brow[r] * N + c0 + k];
            }
        }
        // face coefficients of the own rows (x1) and of the own column segment (x2)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int lf = 0; lf < NF; ++lf) S.ax[r][lf] = tab[TL.ax + (long)S.brow[r] * LF + (c0 - FW + lf) + 2];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int lr = 0; lr < NFR; ++lr)
                S.ay[k][lr] = tab[TL.ay + (long)(c0 + k) * LF + (S.brow[0] - FW + lr) + 2];
        // state: u0 from the set-up tables on every window row
        const T *src = tab + TL.m0;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    S.m[r][k][c] = gdead ? (T)0 : src[c * C + (long)S.brow[r] * N + c0 + k];
                    S.y[r][k][c] = S.m[r][k][c];
                    S.acc[r][k][c] = (T)0;
                }
#pragma unroll
        for (int c = 0; c < 6; ++c) S.tauF[0][c] = S.tauL[0][c] = (T)0;
        S.tFb = S.tFs = S.tLb = S.tLs = S.tSb = S.tSs = S.tNb = S.tNs = S.tTb = S.tTs = 0;
        S.gs = (g > 0) ? g - 1 : 0;
        S.gn = (g < NG - 1) ? g + 1 : 0;
        S.zero_s = (g == 0) || dead(g - 1);
        S.zero_n = (g == NG - 1) || dead(g + 1);
        S.s_halo = s_halo;
        S.s_zero = s_zero;
        S.s_edge = s_zero;   // re-referencing sees zeros beyond the window too
        {
            const int g_last = (own_end + R - 1) / R - 1;  // last own group (h == 0 with xs)
            S.xs_on = xs;
            S.xs_get[0] = S.xs_put[0] = xs && (g == 0) && has_s;
            S.xs_get[1] = S.xs_put[1] = xs && (g == g_last) && has_n;
            S.xs_pub = true;
            S.xs_fail = 0;
            S.xs_src[0] = edge(s_south, 1, 0);
            S.xs_src[1] = edge(s_north, 0, 0);
            S.xs_dst[0] = edge(sl, 0, 0);
            S.xs_dst[1] = edge(sl, 1, 0);
            S.xs_par = (long)xd * XROW;
            S.s_xrow = s_xrow;
            S.xs_abort = A.abort_word;
            S.xs_spin = A.spin_max;
            // stage 0 reads the neighbours' initial rows straight from the tables
            for (int i = tid; i < (xs ? 2 * YH * 3 * N : 0); i += L * NG) {
                const int side = i / (YH * 3 * N), rem = i - side * (YH * 3 * N);
                const int q = rem / (3 * N), c = (rem / N) % 3, col = rem % N;
                const int br = (side == 0) ? job.o0 - YH + q : job.o0 + job.rows + q;
                s_xrow[i] = (br >= 0 && br < N) || BC != LLHMM_BC_DIRICHLET ? src[c * C + (long)wrap(br) * N + col]
                                                                             : (T)0;
            }
        }
        S.s_tau = nullptr;
        S.alpha = (T)P.alpha;
        S.dt = (T)P.dt;
#pragma unroll
        for (int q = 0; q < NQ; ++q) S.acc64[q] = 0.0;
        __syncthreads();

        bool aborted = false;
        if constexpr (EVAL) {
            S.template stage<AVG_EVAL, true, false>((T)0, (T)0, 0.0, 0, A.out_field + P.mfinal_offset, C);
        } else {
            const int M = P.M;
            const bool rk4 = (P.stages == 4);
            const T b1 = rk4 ? (T)(1.0 / 6.0) : (T)0.5;
            const T c2dt = rk4 ? (T)(0.5 * P.dt) : (T)P.dt;
            const T third = (T)(1.0 / 3.0);
            const T half_dt = (T)(0.5 * P.dt);
            const double *wtab = A.wt + P.wt_offset;  // w^0..w^M, then the tails
            constexpr bool REREF = !Lane::REFG && (sizeof(T) == 4);
            int ts = 0;
            for (int n = 0; n < M; ++n) {
                if (!xs && n > 0 && n % spe == 0) {
                    // replace the halo rows with the neighbours' rows of exchange e
                    const uint32_t e = (uint32_t)(n / spe);
                    const int par = (int)(e & 1);
                    int fail = 0;
                    if ((halo_s && has_s) || (halo_n && has_n)) {
                        const uint64_t *sb = halo_s ? edge(s_south, 1, par) : edge(s_north, 0, par);
                        // south halo rows come from the neighbour's last xd own rows, north
                        // halo rows from its first ones
                        const int q0 = halo_s ? xd - h + r0 : r0 - own_end;
                        long long polls = 0;
                        // first wait on one word per lane (the last its publisher writes),
                        // then read the rest
                        {
                            T v;
                            const uint64_t *sw = sb + (q0 + R - 1) * XROW + ((long)2 * N + c0 + K - 1) * XW;
                            while (!xget(sw, e, v)) {
                                if (xload(A.abort_word) != 0 || ++polls > A.spin_max) break;
                                __builtin_amdgcn_s_sleep(1);
                            }
                        }
                        for (;;) {
                            // read straight into the halo rows' state: a word that is
                            // still old is read again on the next poll
                            bool all = true;
#pragma unroll
                            for (int r = 0; r < R; ++r)
#pragma unroll
                                for (int c = 0; c < 3; ++c)
#pragma unroll
                                    for (int k = 0; k < K; ++k)
                                        all &= xget(sb + (q0 + r) * XROW + ((long)c * N + c0 + k) * XW, e, S.m[r][k][c]);
                            if (all) break;
                            if (xload(A.abort_word) != 0 || ++polls > A.spin_max) {
                                fail = 1;
                                xstore(A.abort_word, 1);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int k = 0; k < K; ++k)
#pragma unroll
                                for (int c = 0; c < 3; ++c) S.y[r][k][c] = S.m[r][k][c];
                    }
                    S.xs_fail |= fail;
                }
                const double wn = wtab[n];
                if (REREF && n > 0 && n % kRerefSteps == 0) S.rereference(wtab[M + 1 + n], ts++);
                asm volatile("" ::: "memory");
                S.template stage<Lane::AVG, true, false>(b1, c2dt, wn, ts, nullptr, 0);
                ++ts;
                const int nmid = rk4 ? 2 : 0;
                for (int sm = 0; sm < nmid; ++sm)
                    S.template stage<AVG_NONE, false, false>(third, sm == 0 ? half_dt : S.dt, 0.0, ts++, nullptr, 0);
                // per-stage exchange: the last stage's result goes out unless the next
                // step starts by re-referencing (which publishes its own rows)
                S.xs_pub = !(REREF && (n + 1) % kRerefSteps == 0);
                S.template stage<AVG_NONE, false, true>(rk4 ? (T)(1.0 / 6.0) : (T)0.5, (T)0, 0.0, ts++, nullptr, 0);
                S.xs_pub = true;
                // a wait that gave up is seen by the whole workgroup every few
                // steps and after the last one (the other waits end at once on
                // the abort word meanwhile)
                if ((n + 1) % kAbortCheckSteps == 0 || n + 1 == M) {
                    aborted = __syncthreads_or(S.xs_fail) != 0;
                    if (aborted) break;
                }
                if (xs) continue;
                if ((n + 1) % spe == 0 && n + 1 < M) {
                    // publish the edge rows of exchange e = (n + 1) / spe: the first xd own
                    // rows (south edge) and the last xd (north edge; a group may be in both)
                    const uint32_t e = (uint32_t)((n + 1) / spe);
#pragma unroll
                    for (int side = 0; side < 2; ++side) {
                        if (side == 0 ? !(pub_s && has_s) : !(pub_n && has_n)) continue;
                        uint64_t *db = edge(sl, side, (int)(e & 1));
                        const int q0 = (side == 0) ? r0 - h : r0 - (own_end - xd);
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int c = 0; c < 3; ++c)
#pragma unroll
                                for (int k = 0; k < K; ++k)
                                    xput(db + (q0 + r) * XROW + ((long)c * N + c0 + k) * XW, S.m[r][k][c], e);
                    }
                }
            }
            if (A.out_field && !aborted) {
                double *dst = A.out_field + P.mfinal_offset;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (S.own[r] && !gdead)
#pragma unroll
                        for (int k = 0; k < K; ++k)
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const long cell = (long)S.brow[r] * N + c0 + k;
                                dst[c * C + cell] = (double)S.m[r][k][c] + (double)S.ref(c, S.cell_of(r, k));
                            }
            }
            // per-wave partial sums (the window-row weights select the own rows)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double v = S.acc64[q];
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
                S.acc64[q] = v;
            }
            const int hb = aborted ? 0 : S.health(!gdead);
            const int hbits = (__ballot((hb & 4) != 0) ? 4 : 0) | (__ballot((hb & 8) != 0) ? 8 : 0);
            if (lane == 0) {
                const long slot = P.part_offset + (long)job.slab * WAVES + wave;
                double *dst = A.partials + slot * kMaxQ;
                bool finite = true;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    dst[q] = S.acc64[q];
                    finite = finite && __builtin_isfinite(S.acc64[q]);
                }
                A.wave_status[slot] = aborted ? 2 : (hbits | (finite ? 0 : 1));
            }
        }
        __syncthreads();  // LDS of this item is dead before the next item loads its own
    }
}

}  // namespace llhmm
