// vmc_kernels.hip -- gfx950 kernels of the VMC force hot path (FP64 path).
//
// One workgroup owns one walker: the walker's Slater inverses and its
// per-electron intermediates live in LDS; the walkers of a launch are
// independent Markov chains (Appendix A, MCMC over independent chains).
#include <algorithm>

#include "vmc_kernels.hpp"

namespace vmcx {

// ---------------------------------------------------------------------------
// block helpers
// ---------------------------------------------------------------------------
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

// In-place Gauss-Jordan inversion with partial pivoting of a[n][n] (LDS,
// row-major).  After it a holds a^-1; logabs/sign of det(a) are returned in
// every thread.  col (>= n doubles) and perm (>= n ints) are LDS scratch.
template <int BS>
__device__ void gj_invert(double *a, int n, double *col, int *perm, double &logabs, double &sign,
                          bool &singular) {
    const int tid = threadIdx.x;
    double la = 0.0, sg = 1.0;
    bool sing = false;
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < n; i += 64) {
                const double v = fabs(a[i * n + k]);
                if (v > best) {
                    best = v;
                    bi = i;
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_down(best, off, 64);
                const int oi = __shfl_down(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (tid == 0) perm[k] = bi;
        }
        __syncthreads();
        const int p = perm[k];
        if (p != k) {
            for (int j = tid; j < n; j += BS) {
                const double t = a[k * n + j];
                a[k * n + j] = a[p * n + j];
                a[p * n + j] = t;
            }
            __syncthreads();
        }
        for (int i = tid; i < n; i += BS) col[i] = a[i * n + k];
        __syncthreads();
        const double piv = col[k];
        if (!(fabs(piv) > 1e-300)) sing = true;
        la += log(fabs(piv));
        sg *= (piv < 0.0) ? -1.0 : 1.0;
        if (p != k) sg = -sg;
        const double inv = 1.0 / piv;
        for (int j = tid; j < n; j += BS) a[k * n + j] = (j == k) ? inv : a[k * n + j] * inv;
        __syncthreads();
        for (int idx = tid; idx < n * n; idx += BS) {
            const int i = idx / n, j = idx - (idx / n) * n;
            if (i == k) continue;
            const double f = col[i];
            a[idx] = (j == k) ? -f * inv : a[idx] - f * a[k * n + j];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k) {
            for (int i = tid; i < n; i += BS) {
                const double t = a[i * n + k];
                a[i * n + k] = a[i * n + p];
                a[i * n + p] = t;
            }
            __syncthreads();
        }
    }
    logabs = la;
    sign = sg;
    singular = sing;
}

// Slater matrix of one spin block into a[n][n] (a[e][i] = phi_i(r_{off+e})),
// by tiles of 16 electrons x 64 AOs staged in LDS (aot: 1024 doubles).
template <int BS>
__device__ void build_slater(const SysDev &S, const double *__restrict__ C, const double *__restrict__ R,
                             const double *pos, int off, int n, double *a, double *aot) {
    const int tid = threadIdx.x;
    constexpr int ET = 16, MT = 64;
    constexpr int NO = (ET * 64 + BS - 1) / BS;
    for (int e0 = 0; e0 < n; e0 += ET) {
        double acc[NO];
#pragma unroll
        for (int q = 0; q < NO; ++q) acc[q] = 0.0;
        for (int m0 = 0; m0 < S.M; m0 += MT) {
            for (int idx = tid; idx < ET * MT; idx += BS) {
                const int el = idx / MT, ml = idx - el * MT;
                const int e = e0 + el, mu = m0 + ml;
                double v = 0.0;
                if (e < n && mu < S.M) {
                    const double *r = pos + 3 * (off + e);
                    ao_eval<1>(S.basis, R, mu, r[0], r[1], r[2], &v);
                }
                aot[idx] = v;
            }
            __syncthreads();
            const int mlim = min(MT, S.M - m0);
#pragma unroll
            for (int q = 0; q < NO; ++q) {
                const int o = tid + q * BS;
                const int el = o >> 6, i = o & 63;
                if (el < ET && i < n && e0 + el < n) {
                    double s = acc[q];
                    for (int ml = 0; ml < mlim; ++ml) s += aot[el * MT + ml] * C[(m0 + ml) * S.n_occ + i];
                    acc[q] = s;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < NO; ++q) {
            const int o = tid + q * BS;
            const int el = o >> 6, i = o & 63;
            if (el < ET && i < n && e0 + el < n) a[(e0 + el) * n + i] = acc[q];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Sweep kernel: N single-electron Metropolis moves of one walker per block.
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(BS) void k_sweep(SysDev S, const double *__restrict__ C,
                                              const double *__restrict__ R, double *walkers, int W,
                                              uint32_t sweep, uint64_t seed, double sigma,
                                              int refresh_period, uint8_t *accept, int *status,
                                              SweepLayout L) {
    extern __shared__ double smem[];
    const int w = blockIdx.x;
    if (w >= W) return;
    const int tid = threadIdx.x;
    const int N = S.N, nu = S.n_up, nd = S.n_dn;
    double *pos = smem + L.pos;
    double *K0 = smem + L.K0;
    double *K1 = smem + L.K1;
    double *aor = smem + L.aor;
    double *phin = smem + L.phin;
    double *vrow = smem + L.vrow;
    double *colj = smem + L.colj;
    double *part = smem + L.part;
    double *red = smem + L.red;
    double *misc = smem + L.misc;
    int *perm = (int *)(smem + L.perm);

    double *wp = walkers + (size_t)w * N * 3;
    for (int i = tid; i < 3 * N; i += BS) pos[i] = wp[i];
    __syncthreads();

    bool bad = false;
    auto refresh = [&]() {
        double la, sg;
        bool sing;
        build_slater<BS>(S, C, R, pos, 0, nu, K0, aor);
        gj_invert<BS>(K0, nu, colj, perm, la, sg, sing);
        bad |= sing;
        if (nd > 0) {
            build_slater<BS>(S, C, R, pos, nu, nd, K1, aor);
            gj_invert<BS>(K1, nd, colj, perm, la, sg, sing);
            bad |= sing;
        }
    };
    refresh();

    constexpr int NP = BS / 64;
    for (int e = 0; e < N; ++e) {
        const int b = e < nu ? 0 : 1;
        const int j = e - (b ? nu : 0);
        const int nb = b ? nd : nu;
        double *K = b ? K1 : K0;
        if (tid == 0) {
            double z[3], u;
            move_draws(seed, (uint32_t)w, sweep, (uint32_t)e, z, u);
            misc[0] = pos[3 * e + 0] + sigma * z[0];
            misc[1] = pos[3 * e + 1] + sigma * z[1];
            misc[2] = pos[3 * e + 2] + sigma * z[2];
            misc[3] = u;
        }
        __syncthreads();
        const double rx = misc[0], ry = misc[1], rz = misc[2];
        for (int mu = tid; mu < S.M; mu += BS) {
            double v;
            ao_eval<1>(S.basis, R, mu, rx, ry, rz, &v);
            aor[mu] = v;
        }
        double dj = 0.0;
        for (int k = tid; k < N; k += BS) {
            if (k == e) continue;
            const double ax = rx - pos[3 * k], ay = ry - pos[3 * k + 1], az = rz - pos[3 * k + 2];
            const double bx = pos[3 * e] - pos[3 * k], by = pos[3 * e + 1] - pos[3 * k + 1],
                         bz = pos[3 * e + 2] - pos[3 * k + 2];
            dj += pade_u(sqrt(ax * ax + ay * ay + az * az), S.ee_a, S.ee_F) -
                  pade_u(sqrt(bx * bx + by * by + bz * bz), S.ee_a, S.ee_F);
        }
        dj = block_sum<BS>(dj, red);   // contains barriers: aor is visible after
        {
            const int i = tid & 63, pp = tid >> 6;
            double acc = 0.0;
            if (i < nb)
                for (int mu = pp; mu < S.M; mu += NP) acc += aor[mu] * C[mu * S.n_occ + i];
            part[pp * 64 + i] = acc;
        }
        __syncthreads();
        if (tid < nb) {
            double s = 0.0;
            for (int pp = 0; pp < NP; ++pp) s += part[pp * 64 + tid];
            phin[tid] = s;
        }
        __syncthreads();
        {
            const int c = tid & 63, pp = tid >> 6;
            double acc = 0.0;
            if (c < nb)
                for (int i = pp; i < nb; i += NP) acc += phin[i] * K[i * nb + c];
            part[pp * 64 + c] = acc;
        }
        __syncthreads();
        if (tid < nb) {
            double s = 0.0;
            for (int pp = 0; pp < NP; ++pp) s += part[pp * 64 + tid];
            vrow[tid] = s;
        }
        __syncthreads();
        const double ratio = vrow[j];
        const double qv = ratio * exp(dj);
        const bool acc = misc[3] < qv * qv;
        if (acc) {
            if (tid < nb) colj[tid] = K[tid * nb + j];
            __syncthreads();
            if (tid < 3) pos[3 * e + tid] = misc[tid];
            const double inv = 1.0 / ratio;
            for (int idx = tid; idx < nb * nb; idx += BS) {
                const int i = idx / nb, c = idx - (idx / nb) * nb;
                K[idx] -= colj[i] * (vrow[c] - (c == j ? 1.0 : 0.0)) * inv;
            }
            __syncthreads();
            if (fabs(ratio) < FORCED_REFRESH_RATIO) refresh();
        }
        if (accept != nullptr && tid == 0) accept[(size_t)e * W + w] = acc ? 1 : 0;
        const uint64_t m = (uint64_t)sweep * (uint64_t)N + (uint64_t)e;
        if (((m + 1) % (uint64_t)refresh_period) == 0 && e < N - 1) refresh();
        __syncthreads();
    }
    for (int i = tid; i < 3 * N; i += BS) wp[i] = pos[i];
    if (bad && tid == 0) atomicOr(status, STATUS_SINGULAR);
}

// ---------------------------------------------------------------------------
// Space warp weights omega_a(r) = kappa_a / sum kappa, kappa = d^-4, with
// gradient.  Written as 1 / sum_b (d_a^2/d_b^2)^2 so that it stays finite at
// a nucleus; within 1e-12 bohr of a nucleus omega is 1 there, gradient 0.
// ---------------------------------------------------------------------------
__device__ inline int near_nucleus(const double *R0, int A, double x, double y, double z) {
    for (int b = 0; b < A; ++b) {
        const double dx = x - R0[3 * b], dy = y - R0[3 * b + 1], dz = z - R0[3 * b + 2];
        if (dx * dx + dy * dy + dz * dz < 1e-24) return b;
    }
    return -1;
}

__device__ inline double swct_omega(const double *R0, int A, int a, double x, double y, double z) {
    const double ax = x - R0[3 * a], ay = y - R0[3 * a + 1], az = z - R0[3 * a + 2];
    const double da = ax * ax + ay * ay + az * az;
    double s = 0.0;
    for (int b = 0; b < A; ++b) {
        const double bx = x - R0[3 * b], by = y - R0[3 * b + 1], bz = z - R0[3 * b + 2];
        const double q = da / (bx * bx + by * by + bz * bz);
        s += q * q;
    }
    return 1.0 / s;
}

// grad omega_a = omega_a (g_a - sum_b omega_b g_b), g_b = grad ln kappa_b = -4 (r - R_b)/d_b^2.
// sgx,sgy,sgz = sum_b omega_b g_b (precomputed per electron).
__device__ inline void swct_grad(const double *R0, int a, double om, double x, double y, double z,
                                 double sgx, double sgy, double sgz, double g[3]) {
    const double ax = x - R0[3 * a], ay = y - R0[3 * a + 1], az = z - R0[3 * a + 2];
    const double f = -4.0 / (ax * ax + ay * ay + az * az);
    g[0] = om * (f * ax - sgx);
    g[1] = om * (f * ay - sgy);
    g[2] = om * (f * az - sgz);
}

// ---------------------------------------------------------------------------
// Measurement kernel: one walker per block.
//   forward : MO values/gradients/Laplacians, Slater inverses, E_L, ln|Psi|
//   adjoint : dE_L/dC, dln|Psi|/dC, dE_L/dR, dln|Psi|/dR, dln Jac/dR
// (hand-written reverse mode; AO derivatives recomputed, never stored).
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(BS) void k_measure(SysDev S, const double *__restrict__ C,
                                                const double *__restrict__ R,
                                                const double *__restrict__ R0, int warp,
                                                const double *__restrict__ walkers, int W, int full,
                                                WalkerOut out, double *__restrict__ slab,
                                                int *status, MeasLayout L) {
    extern __shared__ double smem[];
    const int wl = blockIdx.x;   // walker within this launch
    if (wl >= W) return;
    const int tid = threadIdx.x;
    const int N = S.N, nu = S.n_up, nd = S.n_dn, no = S.n_occ, M = S.M, A = S.A;
    double *p0 = smem + L.p0;
    double *p = smem + L.p;
    double *Kb[2] = {smem + L.K0, smem + L.K1};
    double *X = smem + L.X;
    double *U = smem + L.U;
    double *g = smem + L.g;
    double *h = smem + L.h;
    double *bD = smem + L.bD;
    double *lapD = smem + L.lapD;
    double *dEdr = smem + L.dEdr;
    double *tAOE = smem + L.tAOE;
    double *tAOP = smem + L.tAOP;
    double *Minv = smem + L.Minv;
    double *sg = smem + L.sg;
    double *red = smem + L.red;
    double *misc = smem + L.misc;
    int *perm = (int *)(smem + L.perm);
    double *ph = slab + (size_t)wl * N * 5 * no;   // Phi5[e][c][i]

    // ---- positions, warp, Jacobian ---------------------------------------
    const double *wp = walkers + (size_t)wl * N * 3;
    for (int i = tid; i < 3 * N; i += BS) p0[i] = wp[i];
    __syncthreads();
    double lnj_part = 0.0;
    for (int i = tid; i < N; i += BS) {
        const double x = p0[3 * i], y = p0[3 * i + 1], z = p0[3 * i + 2];
        double M3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        double px = x, py = y, pz = z;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        const int nn = near_nucleus(R0, A, x, y, z);
        if (nn < 0) {
            for (int b = 0; b < A; ++b) {
                const double om = swct_omega(R0, A, b, x, y, z);
                const double bx = x - R0[3 * b], by = y - R0[3 * b + 1], bz = z - R0[3 * b + 2];
                const double f = -4.0 / (bx * bx + by * by + bz * bz);
                sx += om * f * bx;
                sy += om * f * by;
                sz += om * f * bz;
            }
        }
        sg[3 * i] = sx;
        sg[3 * i + 1] = sy;
        sg[3 * i + 2] = sz;
        if (warp) {
            for (int a = 0; a < A; ++a) {
                const double dx = R[3 * a] - R0[3 * a], dy = R[3 * a + 1] - R0[3 * a + 1],
                             dz = R[3 * a + 2] - R0[3 * a + 2];
                double om, gw[3] = {0.0, 0.0, 0.0};
                if (nn >= 0) {
                    om = (a == nn) ? 1.0 : 0.0;
                } else {
                    om = swct_omega(R0, A, a, x, y, z);
                    swct_grad(R0, a, om, x, y, z, sx, sy, sz, gw);
                }
                px += om * dx;
                py += om * dy;
                pz += om * dz;
                // M[k][l] = d r'_k / d r_l = delta + dR_k grad_l omega
                const double d3[3] = {dx, dy, dz};
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) M3[3 * k + l] += d3[k] * gw[l];
            }
        }
        p[3 * i] = px;
        p[3 * i + 1] = py;
        p[3 * i + 2] = pz;
        const double det = M3[0] * (M3[4] * M3[8] - M3[5] * M3[7]) -
                           M3[1] * (M3[3] * M3[8] - M3[5] * M3[6]) +
                           M3[2] * (M3[3] * M3[7] - M3[4] * M3[6]);
        lnj_part += log(det);
        const double id = 1.0 / det;
        double *Mi = Minv + 9 * i;
        Mi[0] = (M3[4] * M3[8] - M3[5] * M3[7]) * id;
        Mi[1] = (M3[2] * M3[7] - M3[1] * M3[8]) * id;
        Mi[2] = (M3[1] * M3[5] - M3[2] * M3[4]) * id;
        Mi[3] = (M3[5] * M3[6] - M3[3] * M3[8]) * id;
        Mi[4] = (M3[0] * M3[8] - M3[2] * M3[6]) * id;
        Mi[5] = (M3[2] * M3[3] - M3[0] * M3[5]) * id;
        Mi[6] = (M3[3] * M3[7] - M3[4] * M3[6]) * id;
        Mi[7] = (M3[1] * M3[6] - M3[0] * M3[7]) * id;
        Mi[8] = (M3[0] * M3[4] - M3[1] * M3[3]) * id;
    }
    const double lnjac = block_sum<BS>(lnj_part, red);

    // ---- phase A: MO value/gradient/Laplacian rows into the slab ----------
    {
        constexpr int ET = 4, MT = BS / 4;
        const int nout = ET * 5 * no;
        constexpr int NQ = (4 * 5 * VMC_MAX_OCC_K + BS - 1) / BS;
        double *aot = U;   // [ET*MT][5]
        for (int e0 = 0; e0 < N; e0 += ET) {
            double acc[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
            for (int m0 = 0; m0 < M; m0 += MT) {
                {
                    const int el = tid / MT, ml = tid - (tid / MT) * MT;
                    const int e = e0 + el, mu = m0 + ml;
                    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                    if (e < N && mu < M) ao_eval<5>(S.basis, R, mu, p[3 * e], p[3 * e + 1], p[3 * e + 2], v);
#pragma unroll
                    for (int c = 0; c < 5; ++c) aot[tid * 5 + c] = v[c];
                }
                __syncthreads();
                const int mlim = min(MT, M - m0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int o = tid + q * BS;
                    if (o < nout) {
                        const int el = o / (5 * no);
                        const int rem = o - el * 5 * no;
                        const int c = rem / no, i = rem - (rem / no) * no;
                        if (e0 + el < N) {
                            double s = acc[q];
                            const double *at = aot + (el * MT) * 5 + c;
                            for (int ml = 0; ml < mlim; ++ml) s += at[ml * 5] * C[(m0 + ml) * no + i];
                            acc[q] = s;
                        }
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int o = tid + q * BS;
                if (o < nout) {
                    const int el = o / (5 * no);
                    if (e0 + el < N) ph[(size_t)e0 * 5 * no + o] = acc[q];
                }
            }
        }
        __syncthreads();
    }

    // ---- phase B: Slater inverses ------------------------------------------
    double logdet = 0.0;
    bool bad = false;
    for (int b = 0; b < 2; ++b) {
        const int nb = b ? nd : nu, off = b ? nu : 0;
        if (nb == 0) continue;
        double *K = Kb[b];
        for (int idx = tid; idx < nb * nb; idx += BS) {
            const int e = idx / nb, i = idx - (idx / nb) * nb;
            K[idx] = ph[(size_t)(off + e) * 5 * no + i];
        }
        __syncthreads();
        double la, sgn;
        bool sing;
        gj_invert<BS>(K, nb, U, perm, la, sgn, sing);
        logdet += la;
        bad |= sing;
    }

    // ---- phase C: per-electron terms and E_L --------------------------------
    double el_part = 0.0, j_part = 0.0;
    for (int e = tid; e < N; e += BS) {
        const int b = e < nu ? 0 : 1;
        const int nb = b ? nd : nu, j = e - (b ? nu : 0);
        const double *K = Kb[b];
        const double *row = ph + (size_t)e * 5 * no;
        double bx = 0.0, by = 0.0, bz = 0.0, lp = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double kk = K[i * nb + j];
            bx += kk * row[no + i];
            by += kk * row[2 * no + i];
            bz += kk * row[3 * no + i];
            lp += kk * row[4 * no + i];
        }
        const double x = p[3 * e], y = p[3 * e + 1], z = p[3 * e + 2];
        double gx = 0.0, gy = 0.0, gz = 0.0, hh = 0.0, vee = 0.0, jj = 0.0;
        for (int k = 0; k < N; ++k) {
            if (k == e) continue;
            const double dx = x - p[3 * k], dy = y - p[3 * k + 1], dz = z - p[3 * k + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const PadeD pd = pade_all(r, S.ee_a, S.ee_F);
            const double f = pd.u1 / r;
            gx += f * dx;
            gy += f * dy;
            gz += f * dz;
            hh += pd.u2 + 2.0 * f;
            vee += 1.0 / r;
            jj += pd.u;
        }
        double ven = 0.0;
        for (int a = 0; a < A; ++a) {
            const double dx = x - R[3 * a], dy = y - R[3 * a + 1], dz = z - R[3 * a + 2];
            ven -= S.Z[a] / sqrt(dx * dx + dy * dy + dz * dz);
        }
        g[3 * e] = gx;
        g[3 * e + 1] = gy;
        g[3 * e + 2] = gz;
        h[e] = hh;
        bD[3 * e] = bx;
        bD[3 * e + 1] = by;
        bD[3 * e + 2] = bz;
        lapD[e] = lp;
        const double kin = lp + 2.0 * (bx * gx + by * gy + bz * gz) + hh + gx * gx + gy * gy + gz * gz;
        el_part += -0.5 * kin + ven + 0.5 * vee;
        j_part += 0.5 * jj;
    }
    double vnn = 0.0;
    if (tid == 0) {
        for (int a = 0; a < A; ++a)
            for (int c = a + 1; c < A; ++c) {
                const double dx = R[3 * a] - R[3 * c], dy = R[3 * a + 1] - R[3 * c + 1],
                             dz = R[3 * a + 2] - R[3 * c + 2];
                vnn += S.Z[a] * S.Z[c] / sqrt(dx * dx + dy * dy + dz * dz);
            }
    }
    const double EL = block_sum<BS>(el_part + vnn, red);
    const double J = block_sum<BS>(j_part, red);
    const double lnpsi = logdet + J;
    const size_t wg = (size_t)wl;
    if (tid == 0) {
        if (out.EL) out.EL[wg] = EL;
        if (out.lnpsi) out.lnpsi[wg] = lnpsi;
        if (out.lnjac) out.lnjac[wg] = lnjac;
        if (bad) atomicOr(status, STATUS_SINGULAR);
        if (!isfinite(EL) || !isfinite(lnpsi)) atomicOr(status, STATUS_NONFINITE);
    }
    if (!full) return;

    // ---- phase D: X = lap phi + 2 gradJ . grad phi;  Abar = 1/2 (K X K)^T ----
    for (int idx = tid; idx < N * no; idx += BS) {
        const int e = idx / no, i = idx - (idx / no) * no;
        const double *row = ph + (size_t)e * 5 * no;
        X[idx] = row[4 * no + i] + 2.0 * (g[3 * e] * row[no + i] + g[3 * e + 1] * row[2 * no + i] +
                                          g[3 * e + 2] * row[3 * no + i]);
    }
    __syncthreads();
    for (int b = 0; b < 2; ++b) {
        const int nb = b ? nd : nu, off = b ? nu : 0;
        if (nb == 0) continue;
        const double *K = Kb[b];
        double *T = U;   // T[e'][e] = sum_i X[e'][i] K[i][e]
        for (int idx = tid; idx < nb * nb; idx += BS) {
            const int ep = idx / nb, e = idx - (idx / nb) * nb;
            double s = 0.0;
            for (int i = 0; i < nb; ++i) s += X[(off + ep) * no + i] * K[i * nb + e];
            T[idx] = s;
        }
        __syncthreads();
        for (int idx = tid; idx < nb * nb; idx += BS) {
            const int e = idx / nb, i = idx - (idx / nb) * nb;
            double s = 0.0;
            for (int ep = 0; ep < nb; ++ep) s += K[i * nb + ep] * T[ep * nb + e];
            X[(off + e) * no + i] = 0.5 * s;   // Abar[e][i]
        }
        __syncthreads();
    }
    const double *Abar = X;

    // ---- phase E: AO-space adjoint contractions and outer products --------
    for (int i = tid; i < 3 * N; i += BS) dEdr[i] = 0.0;
    for (int i = tid; i < 3 * M; i += BS) {
        tAOE[i] = 0.0;
        tAOP[i] = 0.0;
    }
    __syncthreads();
    {
        constexpr int ET = 4, MT = BS / 4;
        double *tl = U;                  // [ET*MT][6]
        double *psi_t = U + 6 * BS;      // [ET*MT]
        double *q_t = U + 7 * BS;        // [ET*MT]
        constexpr int NG = BS / 64;      // groups of AOs for the outer products
        constexpr int MPT = (MT + NG - 1) / NG;
        const int il = tid & 63, mg = tid >> 6;
        for (int m0 = 0; m0 < M; m0 += MT) {
            double aO[MPT], aG[MPT];
#pragma unroll
            for (int k = 0; k < MPT; ++k) {
                aO[k] = 0.0;
                aG[k] = 0.0;
            }
            for (int e0 = 0; e0 < N; e0 += ET) {
                {
                    const int el = tid / MT, ml = tid - (tid / MT) * MT;
                    const int e = e0 + el, mu = m0 + ml;
                    double t6[6] = {0, 0, 0, 0, 0, 0}, psi = 0.0, q = 0.0;
                    if (e < N && mu < M) {
                        double v[14];
                        ao_eval<14>(S.basis, R, mu, p[3 * e], p[3 * e + 1], p[3 * e + 2], v);
                        const int b = e < nu ? 0 : 1;
                        const int nb = b ? nd : nu, j = e - (b ? nu : 0);
                        const double *K = Kb[b];
                        const double *Crow = C + (size_t)mu * no;
                        double kap = 0.0, aa = 0.0;
                        for (int i = 0; i < nb; ++i) {
                            const double c = Crow[i];
                            kap += c * K[i * nb + j];
                            aa += c * Abar[e * no + i];
                        }
                        const double gx = g[3 * e], gy = g[3 * e + 1], gz = g[3 * e + 2];
                        // hessian order xx,xy,xz,yy,yz,zz at v[5..10]
                        const double hgx = gx * v[5] + gy * v[6] + gz * v[7];
                        const double hgy = gx * v[6] + gy * v[8] + gz * v[9];
                        const double hgz = gx * v[7] + gy * v[9] + gz * v[10];
                        t6[0] = aa * v[1] - kap * (hgx + 0.5 * v[11]);
                        t6[1] = aa * v[2] - kap * (hgy + 0.5 * v[12]);
                        t6[2] = aa * v[3] - kap * (hgz + 0.5 * v[13]);
                        t6[3] = kap * v[1];
                        t6[4] = kap * v[2];
                        t6[5] = kap * v[3];
                        psi = v[0];
                        q = -(gx * v[1] + gy * v[2] + gz * v[3]) - 0.5 * v[4];
                    }
#pragma unroll
                    for (int c = 0; c < 6; ++c) tl[tid * 6 + c] = t6[c];
                    psi_t[tid] = psi;
                    q_t[tid] = q;
                }
                __syncthreads();
                // per-electron sums over the AO tile (fixed order)
                for (int idx = tid; idx < ET * 3 + MT * 6; idx += BS) {
                    if (idx < ET * 3) {
                        const int el = idx / 3, k = idx - (idx / 3) * 3;
                        if (e0 + el < N) {
                            double s = 0.0;
                            for (int ml = 0; ml < MT; ++ml) s += tl[(el * MT + ml) * 6 + k];
                            dEdr[3 * (e0 + el) + k] += s;
                        }
                    } else {
                        const int t2 = idx - ET * 3;
                        const int ml = t2 / 6, c = t2 - (t2 / 6) * 6;
                        if (m0 + ml < M) {
                            double s = 0.0;
                            for (int el = 0; el < ET; ++el) s += tl[(el * MT + ml) * 6 + c];
                            if (c < 3)
                                tAOE[3 * (m0 + ml) + c] += s;
                            else
                                tAOP[3 * (m0 + ml) + c - 3] += s;
                        }
                    }
                }
                // outer products: thread (il, mg) owns AOs m0 + mg + NG*k, orbital il
                for (int el = 0; el < ET; ++el) {
                    const int e = e0 + el;
                    if (e >= N) break;
                    const int b = e < nu ? 0 : 1;
                    const int nb = b ? nd : nu, j = e - (b ? nu : 0);
                    if (il < nb) {
                        const double kk = Kb[b][il * nb + j];
                        const double ab = Abar[e * no + il];
#pragma unroll
                        for (int k = 0; k < MPT; ++k) {
                            const int ml = mg + NG * k;
                            if (ml < MT) {
                                const double ps = psi_t[el * MT + ml];
                                aO[k] += ps * kk;
                                aG[k] += ps * ab + q_t[el * MT + ml] * kk;
                            }
                        }
                    }
                }
                __syncthreads();
            }
            if (il < no) {
#pragma unroll
                for (int k = 0; k < MPT; ++k) {
                    const int mu = m0 + mg + NG * k;
                    if (mg + NG * k < MT && mu < M) {
                        const size_t o = (wg * M + mu) * no + il;
                        if (out.O) out.O[o] = aO[k];
                        if (out.G) out.G[o] = aG[k];
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- phase F: electron-position derivatives (Jastrow, potential) -------
    for (int e = tid; e < N; e += BS) {
        const double x = p[3 * e], y = p[3 * e + 1], z = p[3 * e + 2];
        const double gbe[3] = {-(bD[3 * e] + g[3 * e]), -(bD[3 * e + 1] + g[3 * e + 1]),
                               -(bD[3 * e + 2] + g[3 * e + 2])};
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        for (int k = 0; k < N; ++k) {
            if (k == e) continue;
            const double dx = x - p[3 * k], dy = y - p[3 * k + 1], dz = z - p[3 * k + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double ir = 1.0 / r;
            const double ux = dx * ir, uy = dy * ir, uz = dz * ir;
            const PadeD pd = pade_all(r, S.ee_a, S.ee_F);
            // H(d) v = u'' dhat (dhat.v) + u'/r (v - dhat (dhat.v)),  v = gbar_e - gbar_k
            const double vx = gbe[0] + (bD[3 * k] + g[3 * k]);
            const double vy = gbe[1] + (bD[3 * k + 1] + g[3 * k + 1]);
            const double vz = gbe[2] + (bD[3 * k + 2] + g[3 * k + 2]);
            const double dv = ux * vx + uy * vy + uz * vz;
            const double f1 = pd.u1 * ir;
            d0 += pd.u2 * ux * dv + f1 * (vx - ux * dv);
            d1 += pd.u2 * uy * dv + f1 * (vy - uy * dv);
            d2 += pd.u2 * uz * dv + f1 * (vz - uz * dv);
            // d/dr_e of -1/2 sum lapJ: -w'(r) dhat, w = u'' + 2u'/r
            const double wp1 = pd.u3 + 2.0 * pd.u2 * ir - 2.0 * pd.u1 * ir * ir;
            d0 -= wp1 * ux;
            d1 -= wp1 * uy;
            d2 -= wp1 * uz;
            // electron-electron Coulomb
            const double ir3 = ir * ir * ir;
            d0 -= dx * ir3;
            d1 -= dy * ir3;
            d2 -= dz * ir3;
        }
        for (int a = 0; a < A; ++a) {
            const double dx = x - R[3 * a], dy = y - R[3 * a + 1], dz = z - R[3 * a + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double f = S.Z[a] / (r2 * sqrt(r2));
            d0 += f * dx;
            d1 += f * dy;
            d2 += f * dz;
        }
        dEdr[3 * e] += d0;
        dEdr[3 * e + 1] += d1;
        dEdr[3 * e + 2] += d2;
    }
    __syncthreads();

    // ---- phase G: nuclear derivatives with the space warp --------------------
    for (int idx = tid; idx < 3 * A; idx += BS) {
        const int a = idx / 3, k = idx - (idx / 3) * 3;
        double sE = 0.0, sP = 0.0, sJ = 0.0;
        for (int mu = 0; mu < M; ++mu)
            if (S.basis.shell_atom[S.basis.ao_shell[mu]] == a) {
                sE -= tAOE[3 * mu + k];
                sP -= tAOP[3 * mu + k];
            }
        for (int e = 0; e < N; ++e) {
            const double dx = p[3 * e] - R[3 * a], dy = p[3 * e + 1] - R[3 * a + 1],
                         dz = p[3 * e + 2] - R[3 * a + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double dk = k == 0 ? dx : (k == 1 ? dy : dz);
            sE -= S.Z[a] * dk / (r2 * sqrt(r2));
        }
        for (int c = 0; c < A; ++c) {
            if (c == a) continue;
            const double dx = R[3 * a] - R[3 * c], dy = R[3 * a + 1] - R[3 * c + 1],
                         dz = R[3 * a + 2] - R[3 * c + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double dk = k == 0 ? dx : (k == 1 ? dy : dz);
            sE -= S.Z[a] * S.Z[c] * dk / (r2 * sqrt(r2));
        }
        for (int e = 0; e < N; ++e) {
            const double x = p0[3 * e], y = p0[3 * e + 1], z = p0[3 * e + 2];
            const int nn = near_nucleus(R0, A, x, y, z);
            double om, gw[3] = {0.0, 0.0, 0.0};
            if (nn >= 0) {
                om = (nn == a) ? 1.0 : 0.0;
            } else {
                om = swct_omega(R0, A, a, x, y, z);
                swct_grad(R0, a, om, x, y, z, sg[3 * e], sg[3 * e + 1], sg[3 * e + 2], gw);
            }
            sE += om * dEdr[3 * e + k];
            sP += om * (bD[3 * e + k] + g[3 * e + k]);
            const double *Mi = Minv + 9 * e;
            sJ += Mi[k] * gw[0] + Mi[3 + k] * gw[1] + Mi[6 + k] * gw[2];
        }
        const size_t o = wg * 3 * A + idx;
        if (out.dEL_dR) out.dEL_dR[o] = sE;
        if (out.dlnpsi_dR) out.dlnpsi_dR[o] = sP;
        if (out.dlnjac_dR) out.dlnjac_dR[o] = sJ;
    }
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
hipError_t configure_kernels(size_t sweep_lds, size_t meas_lds) {
    hipError_t e = hipFuncSetAttribute((const void *)k_sweep<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sweep_lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_measure<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)meas_lds);
}

hipError_t launch_sweep(const SysDev &S, const double *C, const double *R, double *walkers, int W,
                        uint32_t sweep, uint64_t seed, double sigma, int refresh_period,
                        uint8_t *accept, int *status, const SweepLayout &L, hipStream_t st) {
    hipLaunchKernelGGL(k_sweep<256>, dim3(W), dim3(256), L.bytes, st, S, C, R, walkers, W, sweep, seed,
                       sigma, refresh_period, accept, status, L);
    return hipGetLastError();
}

hipError_t launch_measure(const SysDev &S, const double *C, const double *R, const double *R0, int warp,
                          const double *walkers, int W, int full, const WalkerOut &out, double *slab,
                          int *status, const MeasLayout &L, hipStream_t st) {
    hipLaunchKernelGGL(k_measure<256>, dim3(W), dim3(256), L.bytes, st, S, C, R, R0, warp, walkers, W,
                       full, out, slab, status, L);
    return hipGetLastError();
}

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
