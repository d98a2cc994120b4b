// vmc_reduce.hip -- deterministic FP64 reductions over walkers and the
// conjugate-gradient kernels of the Z-vector solve (gfx950).
#include <algorithm>

#include "vmc_kernels.hpp"
#include "vmc_mfma.hpp"

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
// Element space of the estimator sums (per measured walker k, e_k = E_L - s,
// every term multiplied by the walker's weight w_k, 1 unless given):
//   [0] e, [1] e^2, [2..) H (3A), P = dlnpsi + dlnjac/2 (3A), e P (3A),
//   O (M n), e O (M n), G (M n), and last the weight w itself.
// Element space of the vector-Jacobian product:
//   [0..Mn) dC = gE G + gPsi O, [Mn..Mn+3A) dR = gE dEdR + gPsi dPdR + gJ dJdR.
// ---------------------------------------------------------------------------
__device__ inline double est_O(const EstArgs &a, int64_t i) { return a.Of ? (double)a.Of[i] : a.O[i]; }
__device__ inline double est_G(const EstArgs &a, int64_t i) { return a.Gf ? (double)a.Gf[i] : a.G[i]; }

__device__ inline double est_term_1(const EstArgs &a, int64_t o, int64_t k) {
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
    if (o < Mn) return est_O(a, k * Mn + o);
    o -= Mn;
    if (o < Mn) return e * est_O(a, k * Mn + o);
    o -= Mn;
    if (o < Mn) return est_G(a, k * Mn + o);
    return 1.0;   // the weight element
}

__device__ inline double est_term(const EstArgs &a, int64_t o, int64_t k) {
    const double t = est_term_1(a, o, k);
    return a.wt ? a.wt[k] * t : t;
}

__device__ inline double vjp_term(const EstArgs &a, int64_t o, int64_t k) {
    const int64_t A3 = a.A3, Mn = a.Mn;
    if (o < Mn) return a.gE[k] * a.G[k * Mn + o] + a.gP[k] * a.O[k * Mn + o];
    o -= Mn;
    return a.gE[k] * a.dEdR[k * A3 + o] + a.gP[k] * a.dPdR[k * A3 + o] + a.gJ[k] * a.dJdR[k * A3 + o];
}

// Neumaier step: s + c accumulates x
__device__ inline void neumaier(double &s, double &c, double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

// partial[seg][o] = sum over walkers of segment seg (Neumaier, fixed order).
// Partial sums over one walker segment (blockIdx.y) of elements [0, n_elem)
// of a partial row of n_out elements; in mode 0 only the leading elements
// (everything before O), the O / e O / G elements going to k_partial_sums_og.
constexpr int PS_U = 8;

__global__ void k_partial_sums(EstArgs a, int mode, int64_t n_elem, int64_t n_out, int64_t W, int64_t seg_len,
                               double *partial) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t seg = blockIdx.y;
    if (o >= n_elem) return;
    const int64_t k0 = seg * seg_len, k1 = min(W, k0 + seg_len);
    // estimator element of this thread: the leading ones, then the weight
    const int64_t oe = (mode == 0 && o == n_elem - 1) ? n_out - 1 : o;
    double s = 0.0, c = 0.0;
    int64_t k = k0;
    for (; k + PS_U <= k1; k += PS_U) {
        double x[PS_U];
#pragma unroll
        for (int u = 0; u < PS_U; ++u) x[u] = mode == 0 ? est_term(a, oe, k + u) : vjp_term(a, o, k + u);
#pragma unroll
        for (int u = 0; u < PS_U; ++u) neumaier(s, c, x[u]);
    }
    for (; k < k1; ++k) neumaier(s, c, mode == 0 ? est_term(a, oe, k) : vjp_term(a, o, k));
    partial[seg * n_out + oe] = s + c;
}

// Mode 0, the O, e O and G elements (most of the element space): thread
// t < Mn takes O element t and forms e O from the same load, Mn <= t < 2 Mn
// takes G element t - Mn.  PS_OG walkers are loaded ahead; their energies are
// the same in every lane (scalar loads).  Few registers, so that enough
// wavefronts are resident to keep HBM busy.
constexpr int PS_OG = 16;

template <typename S>
__global__ __launch_bounds__(256) void k_partial_sums_og(const S *__restrict__ O, const S *__restrict__ G,
                                                         EstArgs a, int64_t n_out, int64_t W, int64_t seg_len,
                                                         double *partial) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Mn = a.Mn, oO = 2 + 3 * a.A3;
    if (t >= 2 * Mn) return;
    const bool isO = t < Mn;
    const int64_t i = isO ? t : t - Mn;
    const S *src = isO ? O : G;
    const int64_t seg = blockIdx.y, k0 = seg * seg_len, k1 = min(W, k0 + seg_len);
    const double sh = ldc(a.shift);
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    int64_t k = k0;
    const double *wt = a.wt;
    for (; k + PS_OG <= k1; k += PS_OG) {
        S x[PS_OG];
#pragma unroll
        for (int u = 0; u < PS_OG; ++u) x[u] = src[(k + u) * Mn + i];
#pragma unroll
        for (int u = 0; u < PS_OG; ++u) {
            const double xv = wt ? ldc(wt + k + u) * (double)x[u] : (double)x[u];
            neumaier(s1, c1, xv);
            if (isO) neumaier(s2, c2, (ldc(a.EL + k + u) - sh) * xv);
        }
    }
    for (; k < k1; ++k) {
        const double xv = wt ? ldc(wt + k) * (double)src[k * Mn + i] : (double)src[k * Mn + i];
        neumaier(s1, c1, xv);
        if (isO) neumaier(s2, c2, (ldc(a.EL + k) - sh) * xv);
    }
    partial[seg * n_out + oO + (isO ? i : 2 * Mn + i)] = s1 + c1;
    if (isO) partial[seg * n_out + oO + Mn + i] = s2 + c2;
}

// acc[o] (+ comp[o]) += sum_seg partial[seg][o]  (Neumaier, fixed order);
// if blk / blkw != nullptr, element 0's / the last element's chunk sum is
// also added to *blk / *blkw.
__global__ void k_accumulate(const double *partial, int64_t n_out, int64_t n_seg, double *acc,
                             double *comp, double *blk, double *blkw, double *blk_all) {
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
    if (o == n_out - 1 && blkw != nullptr) blkw[0] += x;
    if (blk_all != nullptr) blk_all[o] += x;
}

// Leave-one-block-out (jackknife) replicas of the estimators over nb complete
// blocks with per-block sums bs[b][*] (weight sums cnt[b] = bs[b][n_est - 1]):
//   S^(-b) = sum_{b' != b} S_b' (formed as the fixed-order total minus S_b),
//   dE/dC^(-b) = 2 (S_EO/K - (S_E/K)(S_O/K)),  F^(-b) = -S_H/K - 2 (S_EP/K - (S_E/K)(S_P/K)),
//   E^(-b) = s + S_E/K,  K = K^(-b).
__global__ void k_jackknife(const double *__restrict__ bs, int nb, int64_t n_est, int64_t A3, int64_t Mn,
                            const double *__restrict__ shift, double *E_jk, double *F_jk, double *dC_jk) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // output element of one replica
    const int b = blockIdx.y;
    const int64_t n_out = 1 + A3 + Mn;
    if (o >= n_out) return;
    double Kt = 0.0;
    for (int q = 0; q < nb; ++q) Kt += bs[(size_t)q * n_est + n_est - 1];
    const double K = Kt - bs[(size_t)b * n_est + n_est - 1];
    auto loo = [&](int64_t i) {
        double t = 0.0;
        for (int q = 0; q < nb; ++q) t += bs[(size_t)q * n_est + i];
        return (t - bs[(size_t)b * n_est + i]) / K;
    };
    const double vE = loo(0);
    if (o == 0) {
        if (E_jk) E_jk[b] = shift[0] + vE;
    } else if (o <= A3) {
        const int64_t i = o - 1;
        if (F_jk) F_jk[(size_t)b * A3 + i] = -loo(2 + i) - 2.0 * (loo(2 + 2 * A3 + i) - vE * loo(2 + A3 + i));
    } else {
        const int64_t i = o - 1 - A3;
        if (dC_jk) dC_jk[(size_t)b * Mn + i] = 2.0 * (loo(2 + 3 * A3 + Mn + i) - vE * loo(2 + 3 * A3 + i));
    }
}

// Jackknife mean and standard error of nb replicas of len values:
//   mean = sum_b x_b / nb,  sigma = sqrt((nb - 1)/nb * sum_b (x_b - mean)^2)
__global__ void k_jackknife_stats(const double *__restrict__ x, int64_t nb, int64_t len, double *mean,
                                  double *sigma) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double m = 0.0;
    for (int64_t b = 0; b < nb; ++b) m += x[b * len + i];
    m /= (double)nb;
    double v = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        const double d = x[b * len + i] - m;
        v += d * d;
    }
    if (mean) mean[i] = m;
    if (sigma) sigma[i] = sqrt((double)(nb - 1) / (double)nb * v);
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
// Conjugate gradients for H z = -b (FP64; Hestenes-Stiefel with an optional
// Jacobi preconditioner M = diag H), stopping at ||r|| <= rtol ||b||.  The
// iteration state lives on the device so that the host queues batches of
// iterations and reads the state once per batch; every kernel returns at once
// when the state says the solve has ended, so iterations queued after the end
// change nothing.
// ---------------------------------------------------------------------------
constexpr int CG_BS = 1024;   // threads of the single-block vector kernels
constexpr int CG_RW = 2;      // matrix rows per matvec wavefront
constexpr int CG_U = 8;       // column groups of 64 per row in flight
constexpr int CG_ROWS = 4 * CG_RW;   // matrix rows per matvec block

template <int BS>
__device__ inline void block_sum2(double &a, double &b, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[2 * wid] = a;
        red[2 * wid + 1] = b;
    }
    __syncthreads();
    a = b = 0.0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) {
        a += red[2 * i];
        b += red[2 * i + 1];
    }
}

// x = 0, r = -b, dinv = 1 / H_kk (or 1), p = dinv r; rz = r.(dinv r),
// tol2 = rtol^2 ||b||^2.
__global__ __launch_bounds__(CG_BS) void k_cg_setup(const double *__restrict__ H, const double *__restrict__ b,
                                                    int64_t d, int jacobi, double rtol, int maxit, double *x,
                                                    double *r, double *p, double *dinv, CgState *cs) {
    // right-hand side blockIdx.x of a batch (vectors stored one after another)
    {
        const int64_t o = (int64_t)blockIdx.x * d;
        b += o, x += o, r += o, p += o, dinv += o;
        cs += blockIdx.x;
    }
    __shared__ double red[2 * CG_BS / 64];
    double rr = 0.0, rz = 0.0;
    for (int64_t k = threadIdx.x; k < d; k += CG_BS) {
        const double rk = -b[k];
        const double di = jacobi ? 1.0 / H[k * d + k] : 1.0;
        x[k] = 0.0;
        r[k] = rk;
        dinv[k] = di;
        p[k] = di * rk;
        rr += rk * rk;
        rz += rk * (di * rk);
    }
    block_sum2<CG_BS>(rr, rz, red);
    if (threadIdx.x == 0) {
        cs->rz = rz;
        cs->tol2 = rtol * rtol * rr;
        cs->maxit = maxit;
        cs->it = 0;
        cs->done = !(std::isfinite(rr) && std::isfinite(rz)) ? CG_NONFINITE : (rr == 0.0 ? CG_CONVERGED : 0);
    }
}

// Hp = H p, CG_RW rows per wavefront (each p element is loaded once for
// them), CG_U column groups of 64 in flight per row, plus the block's partial
// of p.Hp over its rows in row order.
__global__ __launch_bounds__(256) void k_cg_matvec(const double *__restrict__ H, const double *__restrict__ p,
                                                   double *__restrict__ Hp, double *__restrict__ part, int64_t d,
                                                   const CgState *cs) {
    if (cs->done) return;
    __shared__ double rp[CG_ROWS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * CG_ROWS + wv * CG_RW;
    const double *h[CG_RW];
#pragma unroll
    for (int i = 0; i < CG_RW; ++i) h[i] = H + min(r0 + i, d - 1) * d;   // rows past the end repeat the last
    double s[CG_RW];
#pragma unroll
    for (int i = 0; i < CG_RW; ++i) s[i] = 0.0;
    const int64_t dm = d - d % (64 * CG_U);
    for (int64_t c = lane; c < dm; c += 64 * CG_U) {
        double xv[CG_U], hv[CG_RW][CG_U];
#pragma unroll
        for (int u = 0; u < CG_U; ++u) xv[u] = p[c + 64 * u];
#pragma unroll
        for (int i = 0; i < CG_RW; ++i)
#pragma unroll
            for (int u = 0; u < CG_U; ++u) hv[i][u] = __builtin_nontemporal_load(h[i] + c + 64 * u);
#pragma unroll
        for (int i = 0; i < CG_RW; ++i)
#pragma unroll
            for (int u = 0; u < CG_U; ++u) s[i] = fma(hv[i][u], xv[u], s[i]);
    }
    for (int64_t c = dm + lane; c < d; c += 64) {
        const double xv = p[c];
#pragma unroll
        for (int i = 0; i < CG_RW; ++i) s[i] = fma(h[i][c], xv, s[i]);
    }
#pragma unroll
    for (int i = 0; i < CG_RW; ++i)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s[i] += __shfl_down(s[i], off, 64);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < CG_RW; ++i) {
            const int64_t row = r0 + i;
            const bool ok = row < d;
            if (ok) Hp[row] = s[i];
            rp[wv * CG_RW + i] = ok ? s[i] * p[min(row, d - 1)] : 0.0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < CG_ROWS; ++i) t += rp[i];
        part[blockIdx.x] = t;
    }
}

// alpha = rz / p.Hp; x += alpha p; r -= alpha Hp; stop test on ||r||^2; then
// beta = rz_new / rz and p = dinv r + beta p.
__global__ __launch_bounds__(CG_BS) void k_cg_update(double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ p, const double *__restrict__ Hp,
                                                     const double *__restrict__ dinv,
                                                     const double *__restrict__ part, int n_part, int64_t d,
                                                     CgState *cs) {
    if (cs->done) return;
    __shared__ double red[2 * CG_BS / 64];
    double pHp = 0.0, unused = 0.0;
    for (int j = threadIdx.x; j < n_part; j += CG_BS) pHp += part[j];
    block_sum2<CG_BS>(pHp, unused, red);
    const double rz = cs->rz;
    const double alpha = rz / pHp;
    double rr = 0.0, rzn = 0.0;
    for (int64_t k = threadIdx.x; k < d; k += CG_BS) {
        x[k] += alpha * p[k];
        const double rk = r[k] - alpha * Hp[k];
        r[k] = rk;
        rr += rk * rk;
        rzn += rk * (dinv[k] * rk);
    }
    block_sum2<CG_BS>(rr, rzn, red);
    const int it = cs->it + 1;
    int done = 0;
    if (!(std::isfinite(rr) && std::isfinite(rzn))) done = CG_NONFINITE;
    else if (rr <= cs->tol2) done = CG_CONVERGED;
    else if (it >= cs->maxit) done = CG_MAXIT;
    if (!done) {
        const double beta = rzn / rz;
        for (int64_t k = threadIdx.x; k < d; k += CG_BS) p[k] = dinv[k] * r[k] + beta * p[k];
    }
    __syncthreads();   // every thread has read the state
    if (threadIdx.x == 0) {
        cs->rz = rzn;
        cs->it = it;
        cs->done = done;
    }
}

// ---------------------------------------------------------------------------
// Several right-hand sides at once (e.g. jackknife replicas): every read of H
// serves up to 64 of them.  HP = H P^T is a tall-skinny FP64 product on the
// matrix cores: a block stages 64 rows x 32 columns of H and the 16*NRT
// right-hand sides' 32 columns in LDS, each wavefront accumulates 16 rows x
// 16*NRT right-hand sides, and the columns are split over ksplit blocks whose
// partial products the update kernel adds in a fixed order.  The per-RHS
// vector work runs one block per right-hand side.
// ---------------------------------------------------------------------------
constexpr int CGB_ROWS = 64;          // rows of H per block (16 per wavefront)
constexpr int CGB_KC = 32;            // columns per LDS stage
constexpr int CGB_LD = CGB_KC + 1;    // padded LDS row stride (doubles)

template <int NRT>
__global__ __launch_bounds__(256) void k_cgb_matvec(const double *__restrict__ H, const double *__restrict__ P,
                                                    double *__restrict__ HPp, int64_t d, int nrhs, int ksplit,
                                                    const CgState *cs) {
    typedef Mfma<double> MF;
    __shared__ double Hs[CGB_ROWS * CGB_LD];
    __shared__ double Ps[16 * NRT * CGB_LD];
    int running = 0;
    for (int k = 0; k < nrhs; ++k) running |= cs[k].done == 0;
    if (!running) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ml = lane & 15, kg = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * CGB_ROWS;
    const int split = blockIdx.y;
    // this block's share of the columns, in whole stages
    const int64_t nst = (d + CGB_KC - 1) / CGB_KC;
    const int64_t s0 = nst * split / ksplit, s1 = nst * (split + 1) / ksplit;
    MF::acc_t acc[NRT];
#pragma unroll
    for (int t = 0; t < NRT; ++t) acc[t] = MF::zero();
    // stage st+1 is loaded into registers while stage st is multiplied
    constexpr int HQ = CGB_ROWS * CGB_KC / 256, PQ = 16 * NRT * CGB_KC / 256;
    double hr[HQ], pr[PQ];
    auto load = [&](int64_t st) {
        const int64_t c0 = st * CGB_KC;
        // clamped, unconditional loads (selected afterwards)
#pragma unroll
        for (int q = 0; q < HQ; ++q) {
            const int i = tid + 256 * q, rr = i / CGB_KC, cc = i % CGB_KC;
            const int64_t row = r0 + rr, col = c0 + cc;
            const double v = H[min(row, d - 1) * d + min(col, d - 1)];
            hr[q] = (row < d && col < d) ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int i = tid + 256 * q, kk = i / CGB_KC, cc = i % CGB_KC;
            const int64_t col = c0 + cc;
            const double v = P[(int64_t)min(kk, nrhs - 1) * d + min(col, d - 1)];
            pr[q] = (kk < nrhs && col < d) ? v : 0.0;
        }
    };
    if (s0 < s1) load(s0);
    for (int64_t st = s0; st < s1; ++st) {
#pragma unroll
        for (int q = 0; q < HQ; ++q) {
            const int i = tid + 256 * q;
            Hs[(i / CGB_KC) * CGB_LD + i % CGB_KC] = hr[q];
        }
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int i = tid + 256 * q;
            Ps[(i / CGB_KC) * CGB_LD + i % CGB_KC] = pr[q];
        }
        __syncthreads();
        if (st + 1 < s1) load(st + 1);
        const double *ha = Hs + (16 * wv + ml) * CGB_LD + kg;
#pragma unroll
        for (int ks = 0; ks < CGB_KC / 4; ++ks) {
            const double a = ha[4 * ks];
#pragma unroll
            for (int t = 0; t < NRT; ++t) acc[t] = MF::fma(a, Ps[(16 * t + ml) * CGB_LD + 4 * ks + kg], acc[t]);
        }
        __syncthreads();
    }
    // D[i][j] = sum_c H[row i][c] P[rhs j][c]: register v of lane l holds row
    // l/16 + 4v, right-hand side l%16 of tile t
#pragma unroll
    for (int t = 0; t < NRT; ++t) {
        const int j = 16 * t + ml;
        if (j >= nrhs) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + 16 * wv + kg + 4 * v;
            if (row < d) HPp[((int64_t)split * nrhs + j) * d + row] = acc[t][v];
        }
    }
}

// HP[k][i] = the ksplit partial products added in a fixed order, written over
// the first partial (all right-hand sides and rows in parallel)
__global__ void k_cgb_sum(double *__restrict__ HPp, int64_t d, int nrhs, int ksplit, const CgState *cs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nrhs * d || cs[t / d].done) return;
    double v = 0.0;
    for (int s = 0; s < ksplit; ++s) v += HPp[(int64_t)s * nrhs * d + t];
    HPp[t] = v;
}

// per right-hand side k (one block each): alpha = rz / p.Hp; x += alpha p;
// r -= alpha Hp; stop test; p = dinv r + beta p
__global__ __launch_bounds__(CG_BS) void k_cgb_update(double *__restrict__ X, double *__restrict__ R,
                                                      double *__restrict__ P, const double *__restrict__ HP,
                                                      const double *__restrict__ Dinv, int64_t d, CgState *css) {
    const int k = blockIdx.x;
    CgState *cs = css + k;
    if (cs->done) return;
    __shared__ double red[2 * CG_BS / 64];
    double *x = X + (int64_t)k * d, *r = R + (int64_t)k * d, *p = P + (int64_t)k * d;
    const double *dinv = Dinv + (int64_t)k * d;
    const double *hpk = HP + (int64_t)k * d;
    auto hp = [&](int64_t i) { return hpk[i]; };
    double pHp = 0.0, unused = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += CG_BS) pHp += p[i] * hp(i);
    block_sum2<CG_BS>(pHp, unused, red);
    const double rz = cs->rz;
    const double alpha = rz / pHp;
    double rr = 0.0, rzn = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += CG_BS) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * hp(i);
        r[i] = ri;
        rr += ri * ri;
        rzn += ri * (dinv[i] * ri);
    }
    block_sum2<CG_BS>(rr, rzn, red);
    const int it = cs->it + 1;
    int done = 0;
    if (!(std::isfinite(rr) && std::isfinite(rzn))) done = CG_NONFINITE;
    else if (rr <= cs->tol2) done = CG_CONVERGED;
    else if (it >= cs->maxit) done = CG_MAXIT;
    if (!done) {
        const double beta = rzn / rz;
        for (int64_t i = threadIdx.x; i < d; i += CG_BS) p[i] = dinv[i] * r[i] + beta * p[i];
    }
    __syncthreads();   // every thread has read the state
    if (threadIdx.x == 0) {
        cs->rz = rzn;
        cs->it = it;
        cs->done = done;
    }
}

// b[a][i] = sum_mu Cv[mu][a] G[mu][i] (the virtual-occupied block of C^T G)
__global__ void k_zv_rhs(const double *__restrict__ Cv, const double *__restrict__ G, int64_t M, int64_t nv,
                         int64_t n, double *__restrict__ b) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    G += (size_t)blockIdx.y * M * n;   // batch item
    b += (size_t)blockIdx.y * nv * n;
    if (o >= nv * n) return;
    const int64_t a = o / n, i = o % n;
    double s = 0.0;
    for (int64_t mu = 0; mu < M; ++mu) s = fma(Cv[mu * nv + a], G[mu * n + i], s);
    b[o] = s;
}

// Z[mu][i] = sum_a Cv[mu][a] z[a][i]
__global__ void k_zv_backmap(const double *__restrict__ Cv, const double *__restrict__ z, int64_t M, int64_t nv,
                             int64_t n, double *__restrict__ Z) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    z += (size_t)blockIdx.y * nv * n;   // batch item
    Z += (size_t)blockIdx.y * M * n;
    if (o >= M * n) return;
    const int64_t mu = o / n, i = o % n;
    double s = 0.0;
    for (int64_t a = 0; a < nv; ++a) s = fma(Cv[mu * nv + a], z[a * n + i], s);
    Z[o] = s;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_reduce(const EstArgs &a, int mode, int64_t n_out, int64_t W, double *partial,
                         int64_t max_seg, double *acc, double *comp, double *blk, double *blkw, double *blk_all,
                         hipStream_t st) {
    int64_t n_seg = std::min<int64_t>(max_seg, std::max<int64_t>(1, (W + 63) / 64));
    const int64_t seg_len = (W + n_seg - 1) / n_seg;
    n_seg = (W + seg_len - 1) / seg_len;
    // mode 0: the leading elements and the weight (last) here, O / e O / G
    // in k_partial_sums_og
    const int64_t n_elem = mode == 0 ? 3 + 3 * a.A3 : n_out;
    dim3 g1((unsigned)((n_elem + 255) / 256), (unsigned)n_seg);
    hipLaunchKernelGGL(k_partial_sums, g1, dim3(256), 0, st, a, mode, n_elem, n_out, W, seg_len, partial);
    if (mode == 0) {
        dim3 g2((unsigned)((2 * a.Mn + 255) / 256), (unsigned)n_seg);
        if (a.Of != nullptr)
            hipLaunchKernelGGL(k_partial_sums_og<float>, g2, dim3(256), 0, st, a.Of, a.Gf, a, n_out, W, seg_len,
                               partial);
        else
            hipLaunchKernelGGL(k_partial_sums_og<double>, g2, dim3(256), 0, st, a.O, a.G, a, n_out, W, seg_len,
                               partial);
    }
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, partial, n_out,
                       n_seg, acc, comp, blk, blkw, blk_all);
    return hipGetLastError();
}

hipError_t launch_jackknife(const double *bs, int nb, int64_t n_est, int64_t A3, int64_t Mn, const double *shift,
                            double *E_jk, double *F_jk, double *dC_jk, hipStream_t st) {
    const int64_t n_out = 1 + A3 + Mn;
    hipLaunchKernelGGL(k_jackknife, dim3((unsigned)((n_out + 255) / 256), (unsigned)nb), dim3(256), 0, st, bs, nb,
                       n_est, A3, Mn, shift, E_jk, F_jk, dC_jk);
    return hipGetLastError();
}

hipError_t launch_jackknife_stats(const double *x, int64_t nb, int64_t len, double *mean, double *sigma,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_jackknife_stats, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, x, nb, len, mean,
                       sigma);
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

int cg_matvec_blocks(int64_t d) { return (int)((d + CG_ROWS - 1) / CG_ROWS); }

hipError_t launch_cg_setup(const double *H, const double *b, int64_t d, int nrhs, int jacobi, double rtol,
                           int maxit, double *x, double *r, double *p, double *dinv, CgState *cs, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_setup, dim3((unsigned)nrhs), dim3(CG_BS), 0, st, H, b, d, jacobi, rtol, maxit, x, r, p,
                       dinv, cs);
    return hipGetLastError();
}

int cgb_ksplit(int64_t d) {
    const int64_t rb = (d + CGB_ROWS - 1) / CGB_ROWS, nst = (d + CGB_KC - 1) / CGB_KC;
    int64_t ks = (2048 + rb - 1) / rb;   // about 2048 blocks in all
    return (int)std::max<int64_t>(1, std::min<int64_t>({ks, 32, nst}));
}

hipError_t launch_cgb_iteration(const double *H, int64_t d, int nrhs, double *X, double *R, double *P, double *HPp,
                                const double *dinv, CgState *cs, hipStream_t st) {
    const int ks = cgb_ksplit(d);
    const dim3 g((unsigned)((d + CGB_ROWS - 1) / CGB_ROWS), (unsigned)ks);
    switch ((nrhs + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_cgb_matvec<1>, g, dim3(256), 0, st, H, P, HPp, d, nrhs, ks, cs); break;
        case 2: hipLaunchKernelGGL(k_cgb_matvec<2>, g, dim3(256), 0, st, H, P, HPp, d, nrhs, ks, cs); break;
        case 3: hipLaunchKernelGGL(k_cgb_matvec<3>, g, dim3(256), 0, st, H, P, HPp, d, nrhs, ks, cs); break;
        default: hipLaunchKernelGGL(k_cgb_matvec<4>, g, dim3(256), 0, st, H, P, HPp, d, nrhs, ks, cs); break;
    }
    hipLaunchKernelGGL(k_cgb_sum, dim3((unsigned)(((int64_t)nrhs * d + 255) / 256)), dim3(256), 0, st, HPp, d, nrhs,
                       ks, cs);
    hipLaunchKernelGGL(k_cgb_update, dim3((unsigned)nrhs), dim3(CG_BS), 0, st, X, R, P, HPp, dinv, d, cs);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const double *H, int64_t d, double *x, double *r, double *p, double *Hp,
                               const double *dinv, double *part, CgState *cs, hipStream_t st) {
    const int nb = cg_matvec_blocks(d);
    hipLaunchKernelGGL(k_cg_matvec, dim3((unsigned)nb), dim3(256), 0, st, H, p, Hp, part, d, cs);
    hipLaunchKernelGGL(k_cg_update, dim3(1), dim3(CG_BS), 0, st, x, r, p, Hp, dinv, part, nb, d, cs);
    return hipGetLastError();
}

hipError_t launch_zv_rhs(const double *Cv, const double *G, int64_t M, int64_t nv, int64_t n, int64_t nbat,
                         double *b, hipStream_t st) {
    hipLaunchKernelGGL(k_zv_rhs, dim3((unsigned)((nv * n + 255) / 256), (unsigned)nbat), dim3(256), 0, st, Cv, G, M,
                       nv, n, b);
    return hipGetLastError();
}

hipError_t launch_zv_backmap(const double *Cv, const double *z, int64_t M, int64_t nv, int64_t n, int64_t nbat,
                             double *Z, hipStream_t st) {
    hipLaunchKernelGGL(k_zv_backmap, dim3((unsigned)((M * n + 255) / 256), (unsigned)nbat), dim3(256), 0, st, Cv, z,
                       M, nv, n, Z);
    return hipGetLastError();
}

}  // namespace vmcx
