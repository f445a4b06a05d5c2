// Small pointwise kernels around the micro solve.
//
//   k_upscale: forms the upscaled quantity of each box (eq. (upscaling)) from
//              the FP64 per-wave partial sums in a fixed order, times the
//              physical scale of the averaged quantity; writes a status word.
//   k_macro:   one stage of the macro field model eq. (macro_disc) per macro
//              point: MPEA (eqs. (h_mpea), (mpe_update)) or HeunP / RK4P
//              start-up stages (Section 3.1); or one HeunP / RK4P stage of the
//              torque model eq. (macro_torque).  FP64.
//   k_flux_div: the divergence of the averaged flux of the flux model
//              eq. (macro_flux) at the macro nodes from the fluxes at the
//              staggered points x_i + dX/2 e_j.  FP64.
//   k_fill_i32: sets an int32 array (the slab kernels' counters and exchange words) to a value;
//              a kernel rather than a memset, so that graph replays reset it.
//   k_scatter_rows: copies each served request's upscaled values into the
//              caller's device array at the row the request's id names.
#include <algorithm>

#include "llhmm_internal.h"

namespace llhmm {

__global__ void __launch_bounds__(256) k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_scatter_rows(const double *src, int src_ld, const int64_t *ids, int n,
                                                      int nq, double *dst, int ld, int64_t nrows) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nq) return;
    const int r = i / nq, q = i - r * nq;
    const int64_t id = ids[r];
    if (id >= 0 && id < nrows) dst[id * ld + q] = src[(int64_t)r * src_ld + q];
}

hipError_t launch_scatter_rows(const double *src, int src_ld, const int64_t *ids, int n, int nq, double *dst,
                               int ld, int64_t nrows, hipStream_t s) {
    if (n <= 0 || nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((n * nq + 255) / 256)), dim3(256), 0, s, src, src_ld, ids,
                       n, nq, dst, ld, nrows);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_upscale(const double *partials, const int32_t *wave_status,
                                                 const double *box_const, const BoxPlan *plans,
                                                 int nboxes, double *H, int ld,
                                                 int32_t *status, int32_t *status_out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nboxes) return;
    const BoxPlan &P = plans[b];
    int bad = 0;
    for (int q = 0; q < P.nq; ++q) {
        double s = 0.0;
        for (int w = 0; w < P.nwaves; ++w) s += partials[(P.part_offset + w) * kMaxQ + q];
        // form 1: add the time-independent average of the reference part, times sum_n w^n
        s = (s + P.wsum * box_const[(long)b * kMaxQ + q]) * P.out_scale;
        if (!__builtin_isfinite(s)) bad = 1;
        if (H) H[(long)b * ld + q] = s;
    }
    for (int w = 0; w < P.nwaves; ++w) bad |= wave_status[P.part_offset + w];
    status[b] = bad;
    if (status_out) status_out[b] = bad;
}

hipError_t launch_upscale(const double *partials, const int32_t *wave_status, const double *box_const,
                          const BoxPlan *plans, int nboxes, double *H, int ld, int32_t *status,
                          int32_t *status_out, hipStream_t s) {
    if (nboxes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_upscale, dim3((nboxes + 255) / 256), dim3(256), 0, s, partials,
                       wave_status, box_const, plans, nboxes, H, ld, status, status_out);
    return hipGetLastError();
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// f(M, H) = -M x H - alpha M x (M x H)
__device__ __forceinline__ void ll_rhs(const double m[3], const double h[3], double alpha, double f[3]) {
    double c[3], e[3];
    cross3(m, h, c);
    cross3(m, c, e);
    for (int i = 0; i < 3; ++i) f[i] = -c[i] - alpha * e[i];
}

// model 0: field (and flux) model, H = H_avg; model 1: torque model, H = T_avg.
__global__ void __launch_bounds__(256) k_macro(int npts, int model, int scheme, int step, int stage,
                                               double dt, double alpha, double *M, const double *H,
                                               double *Y, double *work) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const long np = npts;
    auto W = [&](int slot, int c) -> double & { return work[((long)slot * 3 + c) * np + i]; };
    double m[3], h[3], y[3];
    for (int c = 0; c < 3; ++c) {
        m[c] = M[c * np + i];
        h[c] = H[(long)i * 3 + c];
        y[c] = Y[c * np + i];
    }
    if (stage == 0 && model == 0) {  // h^j = H_avg + alpha M^j x H_avg, eq. (h_term), kept for MPEA
        double mh[3];
        cross3(m, h, mh);
        for (int c = 0; c < 3; ++c) W(step % 3, c) = h[c] + alpha * mh[c];
    }
    if (scheme == LLHMM_MACRO_MPEA) {
        double hb[3];
        for (int c = 0; c < 3; ++c)
            hb[c] = (23.0 * W(step % 3, c) - 16.0 * W((step + 2) % 3, c) + 5.0 * W((step + 1) % 3, c)) / 12.0;
        // (I - s[hb]x) M' = (I + s[hb]x) M, s = dt/2: rotation about hb (Cayley transform)
        const double s = 0.5 * dt;
        const double hh = hb[0] * hb[0] + hb[1] * hb[1] + hb[2] * hb[2];
        const double hm = hb[0] * m[0] + hb[1] * m[1] + hb[2] * m[2];
        double hxm[3];
        cross3(hb, m, hxm);
        const double den = 1.0 + s * s * hh;
        for (int c = 0; c < 3; ++c) {
            const double v = ((1.0 - s * s * hh) * m[c] + 2.0 * s * hxm[c] + 2.0 * s * s * hm * hb[c]) / den;
            M[c * np + i] = v;
            Y[c * np + i] = v;
        }
        return;
    }
    double k[3];
    if (model == 0) {
        ll_rhs(stage == 0 ? m : y, h, alpha, k);
    } else {  // -T - alpha Y x T
        double yt[3];
        cross3(stage == 0 ? m : y, h, yt);
        for (int c = 0; c < 3; ++c) k[c] = -h[c] - alpha * yt[c];
    }
    const int nst = (scheme == LLHMM_MACRO_HEUNP) ? 2 : 4;
    if (stage < nst - 1) {
        for (int c = 0; c < 3; ++c) W(3 + stage, c) = k[c];
        double cfac = (scheme == LLHMM_MACRO_HEUNP) ? 1.0 : (stage == 2 ? 1.0 : 0.5);
        for (int c = 0; c < 3; ++c) Y[c * np + i] = m[c] + cfac * dt * k[c];
        return;
    }
    double mt[3];
    if (scheme == LLHMM_MACRO_HEUNP) {
        for (int c = 0; c < 3; ++c) mt[c] = m[c] + 0.5 * dt * (W(3, c) + k[c]);
    } else {
        for (int c = 0; c < 3; ++c)
            mt[c] = m[c] + dt / 6.0 * (W(3, c) + 2.0 * W(4, c) + 2.0 * W(5, c) + k[c]);
    }
    const double nr = sqrt(mt[0] * mt[0] + mt[1] * mt[1] + mt[2] * mt[2]);
    for (int c = 0; c < 3; ++c) {
        M[c * np + i] = mt[c] / nr;
        Y[c * np + i] = mt[c] / nr;
    }
}

hipError_t launch_macro(int npts, int model, int scheme, int step, int stage, double dt, double alpha,
                        double *M, const double *H, double *Y, double *work, hipStream_t s) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_macro, dim3((npts + 255) / 256), dim3(256), 0, s, npts, model, scheme, step,
                       stage, dt, alpha, M, H, Y, work);
    return hipGetLastError();
}

// One thread per macro node i: H_i = sum_j D_j F_j with F_j at x_i + dX/2 e_j in
// row j * npts + (staggered index) of F.  Node index: the last coordinate
// runs fastest, p = (i0 * n + i1) * n + i2 in 3-D.
__global__ void __launch_bounds__(256) k_flux_div(int dim, int n, double dX, int order, const double *F,
                                                  int ld, double *H) {
    long npts = n;
    for (int d = 1; d < dim; ++d) npts *= n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    int idx[3] = {0, 0, 0};
    {
        long r = p;
        for (int d = dim - 1; d >= 0; --d) {
            idx[d] = (int)(r % n);
            r /= n;
        }
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < dim; ++j) {
        // F_j at staggered index i + k along axis j (periodic)
        auto at = [&](int k, int c) -> double {
            int a[3] = {idx[0], idx[1], idx[2]};
            a[j] = ((a[j] + k) % n + n) % n;
            long q = 0;
            for (int d = 0; d < dim; ++d) q = q * n + a[d];
            return F[((long)j * npts + q) * ld + j * 3 + c];
        };
        for (int c = 0; c < 3; ++c) {
            double v;
            if (order == 4) v = (27.0 * (at(0, c) - at(-1, c)) - (at(1, c) - at(-2, c))) / (24.0 * dX);
            else v = (at(0, c) - at(-1, c)) / dX;
            acc[c] += v;
        }
    }
    for (int c = 0; c < 3; ++c) H[p * 3 + c] = acc[c];
}

hipError_t launch_flux_div(int dim, int n, double dX, int order, const double *F, int ld, double *H,
                           hipStream_t s) {
    long npts = n;
    for (int d = 1; d < dim; ++d) npts *= n;
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flux_div, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, dim, n, dX, order,
                       F, ld, H);
    return hipGetLastError();
}

}  // namespace llhmm
