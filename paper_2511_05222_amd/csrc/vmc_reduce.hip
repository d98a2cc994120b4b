// vmc_reduce.hip -- deterministic FP64 reductions over walkers and the
// conjugate-gradient kernels of the Z-vector solve (gfx950).
#include <algorithm>

#include "vmc_kernels.hpp"

namespace vmcx {

template <int BS>
__device__ inline double block_sum(double v, double *red) {
    // deterministic: fixed shuffle tree inside each wave, then waves in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += red[i];
    return s;
}

// ---------------------------------------------------------------------------
// Reductions over walkers (deterministic two-level sums).
// Element space of the estimator sums (per measured walker k, e_k = E_L - s):
//   [0] e, [1] e^2, [2..) H (3A), P = dlnpsi + dlnjac/2 (3A), e P (3A),
//   O (M n), e O (M n), G (M n).
// Element space of the vector-Jacobian product:
//   [0..Mn) dC = gE G + gPsi O, [Mn..Mn+3A) dR = gE dEdR + gPsi dPdR + gJ dJdR.
// ---------------------------------------------------------------------------
__device__ inline double est_term(const EstArgs &a, int64_t o, int64_t k) {
    const double e = a.EL[k] - a.shift[0];
    const int64_t A3 = a.A3, Mn = a.Mn;
    if (o == 0) return e;
    if (o == 1) return e * e;
    o -= 2;
    if (o < A3) return a.dEdR[k * A3 + o];
    o -= A3;
    if (o < A3) return a.dPdR[k * A3 + o] + 0.5 * a.dJdR[k * A3 + o];
    o -= A3;
    if (o < A3) return e * (a.dPdR[k * A3 + o] + 0.5 * a.dJdR[k * A3 + o]);
    o -= A3;
    if (o < Mn) return a.O[k * Mn + o];
    o -= Mn;
    if (o < Mn) return e * a.O[k * Mn + o];
    o -= Mn;
    return a.G[k * Mn + o];
}

__device__ inline double vjp_term(const EstArgs &a, int64_t o, int64_t k) {
    const int64_t A3 = a.A3, Mn = a.Mn;
    if (o < Mn) return a.gE[k] * a.G[k * Mn + o] + a.gP[k] * a.O[k * Mn + o];
    o -= Mn;
    return a.gE[k] * a.dEdR[k * A3 + o] + a.gP[k] * a.dPdR[k * A3 + o] + a.gJ[k] * a.dJdR[k * A3 + o];
}

// partial[seg][o] = sum over walkers of segment seg (Neumaier, fixed order)
__global__ void k_partial_sums(EstArgs a, int mode, int64_t n_out, int64_t W, int64_t seg_len,
                               double *partial) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t seg = blockIdx.y;
    if (o >= n_out) return;
    const int64_t k0 = seg * seg_len, k1 = min(W, k0 + seg_len);
    double s = 0.0, c = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        const double x = mode == 0 ? est_term(a, o, k) : vjp_term(a, o, k);
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    partial[seg * n_out + o] = s + c;
}

// acc[o] (+ comp[o]) += sum_seg partial[seg][o]  (Neumaier, fixed order);
// if blk != nullptr, element 0's chunk sum is also added to *blk.
__global__ void k_accumulate(const double *partial, int64_t n_out, int64_t n_seg, double *acc,
                             double *comp, double *blk) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_out) return;
    double s = 0.0, c = 0.0;
    for (int64_t g = 0; g < n_seg; ++g) {
        const double x = partial[g * n_out + o];
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    const double x = s + c;
    const double a0 = acc[o];
    const double t = a0 + x;
    comp[o] += (fabs(a0) >= fabs(x)) ? ((a0 - t) + x) : ((x - t) + a0);
    acc[o] = t;
    if (o == 0 && blk != nullptr) blk[0] += x;
}

// shift s = mean E_L of the first measured chunk (set once)
__global__ void k_set_shift(const double *EL, int64_t W, double *shift, int *shift_set) {
    __shared__ double red[4];
    if (shift_set[0]) return;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < W; k += 256) s += EL[k];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) {
        shift[0] = s / (double)W;
        shift_set[0] = 1;
    }
}

// reweighting weights of the fixed-sample estimator and E_hat
__global__ void k_eval_weights(const double *EL, const double *lnpsi, const double *lnjac,
                               const double *lnpsi0, int64_t W, double *wnorm, double *Ehat) {
    __shared__ double red[4];
    // max log-weight first for a safe exponent
    double mx = -1e308;
    for (int64_t k = threadIdx.x; k < W; k += 256)
        mx = fmax(mx, 2.0 * (lnpsi[k] - lnpsi0[k]) + lnjac[k]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    double sw = 0.0;
    for (int64_t k = threadIdx.x; k < W; k += 256) sw += exp(2.0 * (lnpsi[k] - lnpsi0[k]) + lnjac[k] - mx);
    sw = block_sum<256>(sw, red);
    double se = 0.0;
    for (int64_t k = threadIdx.x; k < W; k += 256) {
        const double wk = exp(2.0 * (lnpsi[k] - lnpsi0[k]) + lnjac[k] - mx) / sw;
        wnorm[k] = wk;
        se += wk * EL[k];
    }
    se = block_sum<256>(se, red);
    if (threadIdx.x == 0) Ehat[0] = se;
}

__global__ void k_energy_cotangents(int64_t W, double gE, const double *EL, const double *wnorm,
                                    const double *Ehat, double *gEL, double *gPsi, double *gJac) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= W) return;
    const double w = wnorm[k];
    const double d = EL[k] - Ehat[0];
    gEL[k] = gE * w;
    gPsi[k] = 2.0 * gE * w * d;
    gJac[k] = gE * w * d;
}

__global__ void k_combine(const double *acc, const double *comp, int64_t n, double *out) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) out[o] = acc[o] + comp[o];
}

// ---------------------------------------------------------------------------
// Conjugate gradients (FP64, HBM-bound matrix-vector products).
// ---------------------------------------------------------------------------
// y = H x, one 256-thread block per row group: each wave owns one row.
__global__ __launch_bounds__(256) void k_matvec(const double *__restrict__ H, const double *__restrict__ x,
                                                double *__restrict__ y, int64_t d) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= d) return;
    const double *h = H + row * d;
    double s = 0.0;
    for (int64_t c = lane; c < d; c += 64) s += h[c] * x[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) y[row] = s;
}

// partial dot products (fixed order) of n_seg segments
__global__ void k_dot_partial(const double *a, const double *b, int64_t d, double *part) {
    __shared__ double red[4];
    const int64_t seg = blockIdx.x;
    const int64_t len = (d + gridDim.x - 1) / gridDim.x;
    const int64_t k0 = seg * len, k1 = min(d, k0 + len);
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += a[k] * b[k];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) part[seg] = s;
}

__global__ void k_dot_final(const double *part, int n, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s;
    }
}

// CG vector updates with alpha = rr / pHp:  x += alpha p, r -= alpha Hp
__global__ void k_cg_update_xr(double *x, double *r, const double *p, const double *Hp, int64_t d,
                               const double *rr, const double *pHp) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d) return;
    const double alpha = rr[0] / pHp[0];
    x[k] += alpha * p[k];
    r[k] -= alpha * Hp[k];
}

// p = r + beta p, beta = rr_new / rr
__global__ void k_cg_update_p(double *p, const double *r, int64_t d, const double *rr_new, const double *rr) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d) return;
    p[k] = r[k] + (rr_new[0] / rr[0]) * p[k];
}

__global__ void k_cg_init(double *x, double *r, double *p, const double *b, int64_t d) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d) return;
    x[k] = 0.0;
    r[k] = -b[k];
    p[k] = -b[k];
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_reduce(const EstArgs &a, int mode, int64_t n_out, int64_t W, double *partial,
                         int64_t max_seg, double *acc, double *comp, double *blk, hipStream_t st) {
    int64_t n_seg = std::min<int64_t>(max_seg, std::max<int64_t>(1, (W + 63) / 64));
    const int64_t seg_len = (W + n_seg - 1) / n_seg;
    n_seg = (W + seg_len - 1) / seg_len;
    dim3 g1((unsigned)((n_out + 255) / 256), (unsigned)n_seg);
    hipLaunchKernelGGL(k_partial_sums, g1, dim3(256), 0, st, a, mode, n_out, W, seg_len, partial);
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, partial, n_out,
                       n_seg, acc, comp, blk);
    return hipGetLastError();
}

hipError_t launch_set_shift(const double *EL, int64_t W, double *shift, int *shift_set, hipStream_t st) {
    hipLaunchKernelGGL(k_set_shift, dim3(1), dim3(256), 0, st, EL, W, shift, shift_set);
    return hipGetLastError();
}

hipError_t launch_eval_weights(const double *EL, const double *lnpsi, const double *lnjac,
                               const double *lnpsi0, int64_t W, double *wnorm, double *Ehat, hipStream_t st) {
    hipLaunchKernelGGL(k_eval_weights, dim3(1), dim3(256), 0, st, EL, lnpsi, lnjac, lnpsi0, W, wnorm, Ehat);
    return hipGetLastError();
}

hipError_t launch_energy_cotangents(int64_t W, double gE, const double *EL, const double *wnorm,
                                    const double *Ehat, double *gEL, double *gPsi, double *gJac,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_energy_cotangents, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, st, W, gE, EL,
                       wnorm, Ehat, gEL, gPsi, gJac);
    return hipGetLastError();
}

hipError_t launch_combine(const double *acc, const double *comp, int64_t n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc, comp, n, out);
    return hipGetLastError();
}

hipError_t launch_matvec(const double *H, const double *x, double *y, int64_t d, hipStream_t st) {
    hipLaunchKernelGGL(k_matvec, dim3((unsigned)((d + 3) / 4)), dim3(256), 0, st, H, x, y, d);
    return hipGetLastError();
}

hipError_t launch_dot(const double *a, const double *b, int64_t d, double *part, int n_part, double *out,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial, dim3(n_part), dim3(256), 0, st, a, b, d, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, st, part, n_part, out);
    return hipGetLastError();
}

hipError_t launch_cg_init(double *x, double *r, double *p, const double *b, int64_t d, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, x, r, p, b, d);
    return hipGetLastError();
}

hipError_t launch_cg_update_xr(double *x, double *r, const double *p, const double *Hp, int64_t d,
                               const double *rr, const double *pHp, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_update_xr, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, x, r, p, Hp, d, rr,
                       pHp);
    return hipGetLastError();
}

hipError_t launch_cg_update_p(double *p, const double *r, int64_t d, const double *rr_new, const double *rr,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_cg_update_p, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, p, r, d, rr_new, rr);
    return hipGetLastError();
}

}  // namespace vmcx
