// vmc_pipeline.hip -- batched gfx950 kernels of the VMC force hot path.
//
//   k_mo_rows      MO values (and gradients/Laplacians) of every (walker,
//                  electron) row: a GEMM over AOs whose left operand is
//                  produced in LDS by a shell-major GTO evaluation
//   k_warp         space-warped electron positions and ln Jac per walker
//   k_walker_dense per walker: Slater inverses, E_L, ln|Psi|, Abar = (K X K)^T/2
//   k_adjoint_ao   AO-space adjoint per (AO tile, walker): back-projection,
//                  GTO third derivatives, electron-position sums, outer
//                  products dln|Psi|/dC and dE_L/dC
//   k_finalize     per walker: Jastrow/potential terms of dE_L/dr, SWCT force
//                  terms dE_L/dR, dln|Psi|/dR, dln Jac/dR
//
// T is the arithmetic type of the AO/MO/Sherman-Morrison/back-projection
// work; inverses, local-energy assembly and all sums over walkers are FP64.
#include <algorithm>
#include <type_traits>

#include "vmc_pipeline.hpp"

namespace vmcx {

template <int BS>
__device__ inline double block_sum_p(double v, double *red) {
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
// Gauss-Jordan inversion with partial pivoting of a[n][n] (LDS, FP64) by a
// block of BS threads; the pivot of column k is the largest |a[i][k]|, i >= k.
// col: n doubles of scratch.  log|det| and the singular flag are uniform.
// ---------------------------------------------------------------------------
template <int BS>
__device__ void gj_invert_block(double *a, int n, double *col, int *perm, double &logabs, bool &singular) {
    constexpr int NW = BS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool on = lane < n;
    double la = 0.0;
    bool sing = false;
    for (int k = 0; k < n; ++k) {
        if (wave == 0) {
            double best = (on && lane >= k) ? fabs(a[lane * n + k]) : -1.0;
            int bi = lane;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (bi >= n) bi = k;   // no comparable pivot (non-finite column): keep the row order
            if (lane == 0) perm[k] = bi;
            if (bi != k && on) {
                const double t = a[k * n + lane];
                a[k * n + lane] = a[bi * n + lane];
                a[bi * n + lane] = t;
            }
        }
        __syncthreads();
        if (tid < n) col[tid] = a[tid * n + k];
        __syncthreads();
        const double piv = col[k];
        if (!(fabs(piv) > 1e-300)) sing = true;
        la += log(fabs(piv));
        const double inv = 1.0 / piv;
        const double rk = on ? ((lane == k) ? inv : a[k * n + lane] * inv) : 0.0;
        __syncthreads();
        if (on) {
            if (wave == k % NW) a[k * n + lane] = rk;
            for (int i = wave; i < n; i += NW) {
                if (i == k) continue;
                const double f = col[i];
                a[i * n + lane] = (lane == k) ? -f * inv : a[i * n + lane] - f * rk;
            }
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges (each thread owns a row)
    for (int i = tid; i < n; i += BS)
        for (int k = n - 1; k >= 0; --k) {
            const int p = perm[k];
            if (p != k) {
                const double t = a[i * n + k];
                a[i * n + k] = a[i * n + p];
                a[i * n + p] = t;
            }
        }
    __syncthreads();
    logabs = la;
    singular = sing;
}

// ---------------------------------------------------------------------------
// k_mo_rows: out[row][c][i] = sum_mu AO_c(r_row)[mu] C[mu][i], c < NC.
// 32 rows per block; AO tiles of whole shells (<= 32 AOs) staged in LDS.
// Thread (ty, tx): rows 2ty, 2ty+1; orbitals tx + 16 q.
// ---------------------------------------------------------------------------
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_mo_rows(SysDev S, const T *__restrict__ C, const double *__restrict__ R,
                                                 const double *__restrict__ pos, int64_t n_rows, AoTiles tiles,
                                                 T *__restrict__ out) {
    constexpr int RT = 32, MT = 32;
    __shared__ double sp[RT * 3];
    __shared__ T aot[RT][MT][NC];
    __shared__ T ct[MT][64];
    const int tid = threadIdx.x;
    const int n = S.n_occ;
    const int64_t row0 = (int64_t)blockIdx.x * RT;
    for (int k = tid; k < RT * 3; k += 256) {
        const int64_t r = row0 + k / 3;
        sp[k] = r < n_rows ? pos[row0 * 3 + k] : 0.0;
    }
    const int ty = tid >> 4, tx = tid & 15;
    T acc[2][NC][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[r][c][q] = T(0);
    for (int t = 0; t < tiles.n_tiles; ++t) {
        const int s0 = tiles.s0[t], s1 = tiles.s1[t], mu0 = tiles.mu0[t], mu1 = tiles.mu1[t];
        const int nsh = s1 - s0, nmu = mu1 - mu0;
        __syncthreads();
        for (int p = tid; p < RT * nsh; p += 256) {
            const int r = p / nsh, s = s0 + (p - (p / nsh) * nsh);
            T v[6 * NC];
            const int nc = shell_eval<NC, T>(S.basis, R, s, sp[3 * r], sp[3 * r + 1], sp[3 * r + 2], v);
            const int m0 = S.basis.shell_mu0[s] - mu0;
            for (int q = 0; q < nc; ++q)
#pragma unroll
                for (int c = 0; c < NC; ++c) aot[r][m0 + q][c] = v[q * NC + c];
        }
        for (int p = tid; p < nmu * 64; p += 256) {
            const int m = p >> 6, i = p & 63;
            ct[m][i] = i < n ? C[(size_t)(mu0 + m) * n + i] : T(0);
        }
        __syncthreads();
        for (int m = 0; m < nmu; ++m) {
            T a[2][NC], cc[4];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c) a[r][c] = aot[2 * ty + r][m][c];
#pragma unroll
            for (int q = 0; q < 4; ++q) cc[q] = ct[m][tx + 16 * q];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[r][c][q] += a[r][c] * cc[q];
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int64_t row = row0 + 2 * ty + r;
        if (row >= n_rows) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = tx + 16 * q;
                if (i < n) out[(row * NC + c) * n + i] = acc[r][c][q];
            }
    }
}

// ---------------------------------------------------------------------------
// Space-warp helpers: omega_a(r) = kappa_a / sum_b kappa_b, kappa = d^-4;
// grad omega_a = omega_a (g_a - sum_b omega_b g_b), g_b = -4 (r - R_b)/d_b^2.
// Within 1e-12 bohr of nucleus c: omega = delta_ac, gradient 0.
// ---------------------------------------------------------------------------
struct WarpE {
    double invS;      // 1 / sum_b d_b^-4
    double sg[3];     // sum_b omega_b g_b
    int near;         // nucleus within 1e-12 bohr, else -1
};

__device__ inline WarpE warp_electron(const double *R0, int A, double x, double y, double z) {
    WarpE o;
    o.near = -1;
    double S = 0.0;
    for (int b = 0; b < A; ++b) {
        const double dx = x - R0[3 * b], dy = y - R0[3 * b + 1], dz = z - R0[3 * b + 2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < 1e-24) o.near = b;
        S += 1.0 / (d2 * d2);
    }
    o.invS = 1.0 / S;
    o.sg[0] = o.sg[1] = o.sg[2] = 0.0;
    if (o.near < 0)
        for (int b = 0; b < A; ++b) {
            const double dx = x - R0[3 * b], dy = y - R0[3 * b + 1], dz = z - R0[3 * b + 2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            const double om = o.invS / (d2 * d2);
            const double f = -4.0 / d2;
            o.sg[0] += om * f * dx;
            o.sg[1] += om * f * dy;
            o.sg[2] += om * f * dz;
        }
    return o;
}

__device__ inline double warp_omega(const WarpE &we, const double *R0, int a, double x, double y, double z,
                                    double g[3]) {
    if (we.near >= 0) {
        g[0] = g[1] = g[2] = 0.0;
        return we.near == a ? 1.0 : 0.0;
    }
    const double dx = x - R0[3 * a], dy = y - R0[3 * a + 1], dz = z - R0[3 * a + 2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double om = we.invS / (d2 * d2);
    const double f = -4.0 / d2;
    g[0] = om * (f * dx - we.sg[0]);
    g[1] = om * (f * dy - we.sg[1]);
    g[2] = om * (f * dz - we.sg[2]);
    return om;
}

// r' = r + sum_a omega_a(r; R0) (R_a - R0_a); ln Jac = sum_i ln det(dr'_i/dr_i).
__global__ __launch_bounds__(128) void k_warp(SysDev S, const double *__restrict__ R, const double *__restrict__ R0,
                                              const double *__restrict__ pos0, double *__restrict__ posw,
                                              double *__restrict__ lnjac, int W) {
    __shared__ double red[4];
    const int w = blockIdx.x;
    if (w >= W) return;
    const int N = S.N, A = S.A;
    double part = 0.0;
    for (int e = threadIdx.x; e < N; e += 128) {
        const double *p = pos0 + ((size_t)w * N + e) * 3;
        const double x = p[0], y = p[1], z = p[2];
        const WarpE we = warp_electron(R0, A, x, y, z);
        double px = x, py = y, pz = z;
        double M3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int a = 0; a < A; ++a) {
            double g[3];
            const double om = warp_omega(we, R0, a, x, y, z, g);
            const double d3[3] = {R[3 * a] - R0[3 * a], R[3 * a + 1] - R0[3 * a + 1], R[3 * a + 2] - R0[3 * a + 2]};
            px += om * d3[0];
            py += om * d3[1];
            pz += om * d3[2];
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) M3[3 * k + l] += d3[k] * g[l];
        }
        double *q = posw + ((size_t)w * N + e) * 3;
        q[0] = px;
        q[1] = py;
        q[2] = pz;
        const double det = M3[0] * (M3[4] * M3[8] - M3[5] * M3[7]) - M3[1] * (M3[3] * M3[8] - M3[5] * M3[6]) +
                           M3[2] * (M3[3] * M3[7] - M3[4] * M3[6]);
        part += log(det);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) lnjac[w] = red[0] + red[1];
}

// ---------------------------------------------------------------------------
// Block-wide FP64 GEMM in LDS with 4x4 register tiles and general strides:
//   C[i*ldc + j] = scale * sum_k A(i,k) B(k,j),  A(i,k) = A[i*sai + k*sak],
//   B(k,j) = B[k*sbk + j*sbj],  i < m, j < nn, k < kk.
// ---------------------------------------------------------------------------
template <int BS>
__device__ void lds_gemm44(const double *A, int sai, int sak, const double *B, int sbk, int sbj, double *C, int ldc,
                           int m, int nn, int kk, double scale) {
    const int tm = (m + 3) >> 2, tn = (nn + 3) >> 2;
    for (int t = threadIdx.x; t < tm * tn; t += BS) {
        const int i0 = (t / tn) * 4, j0 = (t - (t / tn) * tn) * 4;
        double acc[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
        int ia[4], jb[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            ia[r] = min(i0 + r, m - 1);
            jb[r] = min(j0 + r, nn - 1);
        }
        for (int k = 0; k < kk; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r] = A[ia[r] * sai + k * sak];
                b[r] = B[k * sbk + jb[r] * sbj];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (i0 + r < m && j0 + c < nn) C[(i0 + r) * ldc + j0 + c] = scale * acc[r][c];
    }
}

// ---------------------------------------------------------------------------
// k_walker_dense: one block per walker (FP64 inside).
//   Slater inverses K (Gauss-Jordan), Jastrow gradient g and Laplacian,
//   det gradient b_e = sum_i K[i][e] grad phi_i(r_e), lapD_e likewise,
//   E_L and ln|Psi|; with the adjoint: X = lap phi + 2 g.grad phi and
//   Abar = 1/2 (K X K)^T, written with K~[e][i] = K[i][e] for k_adjoint_ao.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_walker_dense(SysDev S, const double *__restrict__ R,
                                                      MeasBufs<T> mb, WalkerOut out, int *status, DenseLayout L) {
    extern __shared__ double smem[];
    const int w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N = S.N, nu = S.n_up, nd = S.n_dn, n = S.n_occ, A = S.A;
    double *p = smem + L.p;
    double *Kb[2] = {smem + L.K0, smem + L.K1};
    double *X = smem + L.X;
    double *U = smem + L.U;
    double *g = smem + L.g;
    double *red = smem + L.red;
    int *perm = (int *)(smem + L.perm);
    const T *ph = mb.phi + (size_t)w * N * 5 * n;
    for (int i = tid; i < 3 * N; i += 256) p[i] = mb.pos[(size_t)w * N * 3 + i];
    __syncthreads();
    // Jastrow and potential terms per electron
    double el_part = 0.0, j_part = 0.0;
    for (int e = tid; e < N; e += 256) {
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
        el_part += -0.5 * (hh + gx * gx + gy * gy + gz * gz) + ven + 0.5 * vee;
        j_part += 0.5 * jj;
    }
    // Slater inverses
    double logdet = 0.0;
    bool bad = false;
    for (int b = 0; b < 2; ++b) {
        const int nb = b ? nd : nu, off = b ? nu : 0;
        if (nb == 0) continue;
        double *K = Kb[b];
        if (lane < nb)
            for (int e = wave; e < nb; e += 4) K[e * nb + lane] = (double)ph[(size_t)(off + e) * 5 * n + lane];
        __syncthreads();
        double la;
        bool sing;
        gj_invert_block<256>(K, nb, U, perm, la, sing);
        logdet += la;
        bad |= sing;
    }
    __syncthreads();
    // one wavefront per electron row: lanes over orbitals
    double *gb = mb.gb + (size_t)w * N * 6;
    for (int e = wave; e < N; e += 4) {
        const int b = e < nu ? 0 : 1;
        const int nb = b ? nd : nu, j = e - (b ? nu : 0);
        const T *row = ph + (size_t)e * 5 * n;
        const double gx = g[3 * e], gy = g[3 * e + 1], gz = g[3 * e + 2];
        double bx = 0.0, by = 0.0, bz = 0.0, lp = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double Gx = (double)row[n + i], Gy = (double)row[2 * n + i], Gz = (double)row[3 * n + i];
            const double Lp = (double)row[4 * n + i];
            X[e * n + i] = Lp + 2.0 * (gx * Gx + gy * Gy + gz * Gz);
            if (i < nb) {
                const double kk = Kb[b][i * nb + j];
                bx += kk * Gx;
                by += kk * Gy;
                bz += kk * Gz;
                lp += kk * Lp;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            bx += __shfl_xor(bx, o, 64);
            by += __shfl_xor(by, o, 64);
            bz += __shfl_xor(bz, o, 64);
            lp += __shfl_xor(lp, o, 64);
        }
        if (lane == 0) {
            gb[6 * e + 0] = gx;
            gb[6 * e + 1] = gy;
            gb[6 * e + 2] = gz;
            gb[6 * e + 3] = bx;
            gb[6 * e + 4] = by;
            gb[6 * e + 5] = bz;
            el_part += -0.5 * (lp + 2.0 * (bx * gx + by * gy + bz * gz));
        }
    }
    double vnn = 0.0;
    if (tid == 0)
        for (int a = 0; a < A; ++a)
            for (int c = a + 1; c < A; ++c) {
                const double dx = R[3 * a] - R[3 * c], dy = R[3 * a + 1] - R[3 * c + 1],
                             dz = R[3 * a + 2] - R[3 * c + 2];
                vnn += S.Z[a] * S.Z[c] / sqrt(dx * dx + dy * dy + dz * dz);
            }
    const double EL = block_sum_p<256>(el_part + vnn, red);
    const double J = block_sum_p<256>(j_part, red);
    if (tid == 0) {
        if (out.EL) out.EL[w] = EL;
        if (out.lnpsi) out.lnpsi[w] = logdet + J;
        if (bad) atomicOr(status, STATUS_SINGULAR);
        if (!isfinite(EL) || !isfinite(logdet + J)) atomicOr(status, STATUS_NONFINITE);
    }
    if (mb.ktil == nullptr) return;
    // Abar = 1/2 (K X K)^T per spin:  T = X K,  Abar[e][i] = 1/2 sum_e' T[e'][e] K[i][e']
    T *kt = mb.ktil + (size_t)w * N * n;
    T *ab = mb.abar + (size_t)w * N * n;
    for (int b = 0; b < 2; ++b) {
        const int nb = b ? nd : nu, off = b ? nu : 0;
        if (nb == 0) continue;
        const double *K = Kb[b];
        lds_gemm44<256>(X + off * n, n, 1, K, nb, 1, U, nb, nb, nb, nb, 1.0);
        __syncthreads();
        lds_gemm44<256>(U, 1, nb, K, 1, nb, X + off * n, n, nb, nb, nb, 0.5);
        __syncthreads();
        for (int idx = tid; idx < nb * n; idx += 256) {
            const int e = idx / n, i = idx - (idx / n) * n;
            ab[(size_t)(off + e) * n + i] = i < nb ? (T)X[(off + e) * n + i] : T(0);
            kt[(size_t)(off + e) * n + i] = i < nb ? (T)K[i * nb + e] : T(0);
        }
    }
}

// ---------------------------------------------------------------------------
// k_adjoint_ao: block (AO tile t, walker w).  Thread (ml = AO in tile,
// es = electron slot 0..7).  Per electron chunk of 16:
//   kappa[e][mu] = sum_i C[mu][i] K~[e][i],  a[e][mu] = sum_i C[mu][i] Abar[e][i]
//   t_k = a d_k psi - kappa (sum_d g_d d_k d_d psi + 1/2 d_k lap psi)   (-> dE_L/dr_e, dE_L/dR)
//   s_k = kappa d_k psi                                                 (-> dln|Psi|/dR)
//   O[mu][i] += psi K~[e][i];  G[mu][i] += psi Abar[e][i] + q K~[e][i],
//   q = -g . grad psi - 1/2 lap psi
// ---------------------------------------------------------------------------
template <typename T, int NMAX>
__global__ __launch_bounds__(256) void k_adjoint_ao(SysDev S, const T *__restrict__ C, const double *__restrict__ R,
                                                    MeasBufs<T> mb, AoTiles tiles, WalkerOut out) {
    constexpr int EC = 16;
    __shared__ double sp[EC * 3];
    __shared__ double sg[EC * 3];
    __shared__ T kt[EC][NMAX];
    __shared__ T ab[EC][NMAX];
    __shared__ T rad[EC][32][4];
    __shared__ T psi_t[EC][32];
    __shared__ T q_t[EC][32];
    __shared__ double red6[8][32][6];
    const int t = blockIdx.x;
    const int w = blockIdx.y;
    const int tid = threadIdx.x;
    const int ml = tid & 31, es = tid >> 5;
    const int N = S.N, n = S.n_occ, M = S.M;
    const int s0 = tiles.s0[t], s1 = tiles.s1[t], mu0 = tiles.mu0[t], mu1 = tiles.mu1[t];
    const int nsh = s1 - s0, nmu = mu1 - mu0;
    const int mu = mu0 + ml;
    const bool mok = ml < nmu;
    // this thread's AO: C row, shell, monomial, eta
    T crow[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) crow[i] = (mok && i < n) ? C[(size_t)mu * n + i] : T(0);
    int shl = 0, pw = 0;
    T eta = T(0);
    int atom = 0;
    if (mok) {
        const int s = S.basis.ao_shell[mu];
        shl = s - s0;
        pw = S.basis.ao_pow[mu];
        eta = (T)S.basis.ao_eta[mu];
        atom = S.basis.shell_atom[s];
    }
    const double Rx = R[3 * atom], Ry = R[3 * atom + 1], Rz = R[3 * atom + 2];
    double tsum[6] = {0, 0, 0, 0, 0, 0};
    constexpr int NI = (NMAX + 7) / 8;   // orbitals per thread in the outer products
    T aO[NI], aG[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) aO[k] = aG[k] = T(0);
    const double *posw = mb.pos + (size_t)w * N * 3;
    const double *gbw = mb.gb + (size_t)w * N * 6;
    const T *ktw = mb.ktil + (size_t)w * N * n;
    const T *abw = mb.abar + (size_t)w * N * n;
    double *dpart = mb.dedr_part + ((size_t)w * tiles.n_tiles + t) * N * 3;
    for (int e0 = 0; e0 < N; e0 += EC) {
        const int ne = min(EC, N - e0);
        __syncthreads();
        for (int k = tid; k < ne * 3; k += 256) {
            sp[k] = posw[(size_t)e0 * 3 + k];
            sg[k] = gbw[(size_t)(e0 + k / 3) * 6 + (k % 3)];
        }
        for (int k = tid; k < ne * NMAX; k += 256) {
            const int e = k / NMAX, i = k - (k / NMAX) * NMAX;
            kt[e][i] = i < n ? ktw[(size_t)(e0 + e) * n + i] : T(0);
            ab[e][i] = i < n ? abw[(size_t)(e0 + e) * n + i] : T(0);
        }
        __syncthreads();
        for (int k = tid; k < ne * nsh; k += 256) {
            const int e = k / nsh, s = s0 + (k - (k / nsh) * nsh);
            const int at = S.basis.shell_atom[s];
            const T x = (T)(sp[3 * e] - R[3 * at]), y = (T)(sp[3 * e + 1] - R[3 * at + 1]),
                    z = (T)(sp[3 * e + 2] - R[3 * at + 2]);
            T R0, R1, R2, R3;
            shell_radial<14, T>(S.basis, s, x * x + y * y + z * z, R0, R1, R2, R3);
            rad[e][s - s0][0] = R0;
            rad[e][s - s0][1] = R1;
            rad[e][s - s0][2] = R2;
            rad[e][s - s0][3] = R3;
        }
        __syncthreads();
        for (int el = es; el < EC; el += 8) {
            T psi = T(0), q = T(0);
            double t6[6] = {0, 0, 0, 0, 0, 0};
            if (el < ne && mok) {
                T kap = T(0), aa = T(0);
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    kap += crow[i] * kt[el][i];
                    aa += crow[i] * ab[el][i];
                }
                const T x = (T)(sp[3 * el] - Rx), y = (T)(sp[3 * el + 1] - Ry), z = (T)(sp[3 * el + 2] - Rz);
                T v[14];
                ao_components<14, T>(x, y, z, x * x + y * y + z * z, rad[el][shl][0], rad[el][shl][1],
                                     rad[el][shl][2], rad[el][shl][3], pw, eta, v);
                const T gx = (T)sg[3 * el], gy = (T)sg[3 * el + 1], gz = (T)sg[3 * el + 2];
                const T hgx = gx * v[5] + gy * v[6] + gz * v[7];
                const T hgy = gx * v[6] + gy * v[8] + gz * v[9];
                const T hgz = gx * v[7] + gy * v[9] + gz * v[10];
                const T half = T(0.5);
                t6[0] = (double)(aa * v[1] - kap * (hgx + half * v[11]));
                t6[1] = (double)(aa * v[2] - kap * (hgy + half * v[12]));
                t6[2] = (double)(aa * v[3] - kap * (hgz + half * v[13]));
                t6[3] = (double)(kap * v[1]);
                t6[4] = (double)(kap * v[2]);
                t6[5] = (double)(kap * v[3]);
                psi = v[0];
                q = -(gx * v[1] + gy * v[2] + gz * v[3]) - half * v[4];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) tsum[c] += t6[c];
            // sum over the AOs of the tile (32 lanes of this half-wave) -> dE_L/dr_e partial
            double d0 = t6[0], d1 = t6[1], d2 = t6[2];
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) {
                d0 += __shfl_xor(d0, off, 64);
                d1 += __shfl_xor(d1, off, 64);
                d2 += __shfl_xor(d2, off, 64);
            }
            if (ml == 0 && el < ne) {
                dpart[(size_t)(e0 + el) * 3 + 0] = d0;
                dpart[(size_t)(e0 + el) * 3 + 1] = d1;
                dpart[(size_t)(e0 + el) * 3 + 2] = d2;
            }
            psi_t[el][ml] = psi;
            q_t[el][ml] = q;
        }
        __syncthreads();
        if (mok)
            for (int el = 0; el < ne; ++el) {
                const T ps = psi_t[el][ml], qq = q_t[el][ml];
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    const int i = es + 8 * k;
                    if (i < NMAX) {
                        const T kk = kt[el][i];
                        aO[k] += ps * kk;
                        aG[k] += ps * ab[el][i] + qq * kk;
                    }
                }
            }
    }
    // outer products of this walker for the tile
    if (mok) {
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int i = es + 8 * k;
            if (i < n) {
                const size_t o = ((size_t)w * M + mu) * n + i;
                if (out.O) out.O[o] = (double)aO[k];
                if (out.G) out.G[o] = (double)aG[k];
            }
        }
    }
    // per-AO sums over electrons (fixed order over es)
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; ++c) red6[es][ml][c] = tsum[c];
    __syncthreads();
    if (tid < 32 * 6) {
        const int m = tid / 6, c = tid - (tid / 6) * 6;
        if (m < nmu) {
            double s = 0.0;
            for (int k = 0; k < 8; ++k) s += red6[k][m][c];
            mb.tao[((size_t)w * M + mu0 + m) * 6 + c] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// k_finalize: one block per walker.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_finalize(SysDev S, const double *__restrict__ R,
                                                  const double *__restrict__ R0, MeasBufsD mb, int n_tiles,
                                                  WalkerOut out, int warp) {
    extern __shared__ double smem[];
    const int w = blockIdx.x;
    const int tid = threadIdx.x;
    const int N = S.N, A = S.A, M = S.M;
    double *p = smem;              // [N][3] evaluation positions
    double *p0 = p + 3 * N;        // [N][3] sampling positions
    double *gb = p0 + 3 * N;       // [N][6]
    double *dEdr = gb + 6 * N;     // [N][3]
    double *Minv = dEdr + 3 * N;   // [N][9]
    double *wS = Minv + 9 * N;     // [N][4]: invS, sg
    int *wnear = (int *)(wS + 4 * N);
    for (int i = tid; i < 3 * N; i += 128) {
        p[i] = mb.pos[(size_t)w * N * 3 + i];
        p0[i] = mb.pos0[(size_t)w * N * 3 + i];
    }
    for (int i = tid; i < 6 * N; i += 128) gb[i] = mb.gb[(size_t)w * N * 6 + i];
    __syncthreads();
    for (int e = tid; e < N; e += 128) {
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        for (int t = 0; t < n_tiles; ++t) {
            const double *dp = mb.dedr_part + (((size_t)w * n_tiles + t) * N + e) * 3;
            d0 += dp[0];
            d1 += dp[1];
            d2 += dp[2];
        }
        const double x = p[3 * e], y = p[3 * e + 1], z = p[3 * e + 2];
        const double ge[3] = {-(gb[6 * e + 3] + gb[6 * e]), -(gb[6 * e + 4] + gb[6 * e + 1]),
                              -(gb[6 * e + 5] + gb[6 * e + 2])};
        for (int k = 0; k < N; ++k) {
            if (k == e) continue;
            const double dx = x - p[3 * k], dy = y - p[3 * k + 1], dz = z - p[3 * k + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double ir = 1.0 / r;
            const double ux = dx * ir, uy = dy * ir, uz = dz * ir;
            const PadeD pd = pade_all(r, S.ee_a, S.ee_F);
            const double vx = ge[0] + (gb[6 * k + 3] + gb[6 * k]);
            const double vy = ge[1] + (gb[6 * k + 4] + gb[6 * k + 1]);
            const double vz = ge[2] + (gb[6 * k + 5] + gb[6 * k + 2]);
            const double dv = ux * vx + uy * vy + uz * vz;
            const double f1 = pd.u1 * ir;
            d0 += pd.u2 * ux * dv + f1 * (vx - ux * dv);
            d1 += pd.u2 * uy * dv + f1 * (vy - uy * dv);
            d2 += pd.u2 * uz * dv + f1 * (vz - uz * dv);
            const double wp1 = pd.u3 + 2.0 * pd.u2 * ir - 2.0 * pd.u1 * ir * ir;
            d0 -= wp1 * ux;
            d1 -= wp1 * uy;
            d2 -= wp1 * uz;
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
        dEdr[3 * e] = d0;
        dEdr[3 * e + 1] = d1;
        dEdr[3 * e + 2] = d2;
        // warp weights at the sampling positions
        const double x0 = p0[3 * e], y0 = p0[3 * e + 1], z0 = p0[3 * e + 2];
        const WarpE we = warp_electron(R0, A, x0, y0, z0);
        wS[4 * e] = we.invS;
        wS[4 * e + 1] = we.sg[0];
        wS[4 * e + 2] = we.sg[1];
        wS[4 * e + 3] = we.sg[2];
        wnear[e] = we.near;
        double M3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (warp)
            for (int a = 0; a < A; ++a) {
                double g[3];
                warp_omega(we, R0, a, x0, y0, z0, g);
                const double d3[3] = {R[3 * a] - R0[3 * a], R[3 * a + 1] - R0[3 * a + 1],
                                      R[3 * a + 2] - R0[3 * a + 2]};
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) M3[3 * k + l] += d3[k] * g[l];
            }
        const double det = M3[0] * (M3[4] * M3[8] - M3[5] * M3[7]) - M3[1] * (M3[3] * M3[8] - M3[5] * M3[6]) +
                           M3[2] * (M3[3] * M3[7] - M3[4] * M3[6]);
        const double id = 1.0 / det;
        double *Mi = Minv + 9 * e;
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
    __syncthreads();
    for (int idx = tid; idx < 3 * A; idx += 128) {
        const int a = idx / 3, k = idx - (idx / 3) * 3;
        double sE = 0.0, sP = 0.0, sJ = 0.0;
        for (int m = 0; m < M; ++m)
            if (S.basis.shell_atom[S.basis.ao_shell[m]] == a) {
                sE -= mb.tao[((size_t)w * M + m) * 6 + k];
                sP -= mb.tao[((size_t)w * M + m) * 6 + 3 + k];
            }
        for (int e = 0; e < N; ++e) {
            const double dx = p[3 * e] - R[3 * a], dy = p[3 * e + 1] - R[3 * a + 1], dz = p[3 * e + 2] - R[3 * a + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double dk = k == 0 ? dx : (k == 1 ? dy : dz);
            sE -= S.Z[a] * dk / (r2 * sqrt(r2));
        }
        for (int c = 0; c < A; ++c) {
            if (c == a) continue;
            const double dx = R[3 * a] - R[3 * c], dy = R[3 * a + 1] - R[3 * c + 1], dz = R[3 * a + 2] - R[3 * c + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double dk = k == 0 ? dx : (k == 1 ? dy : dz);
            sE -= S.Z[a] * S.Z[c] * dk / (r2 * sqrt(r2));
        }
        for (int e = 0; e < N; ++e) {
            WarpE we;
            we.invS = wS[4 * e];
            we.sg[0] = wS[4 * e + 1];
            we.sg[1] = wS[4 * e + 2];
            we.sg[2] = wS[4 * e + 3];
            we.near = wnear[e];
            double g[3];
            const double om = warp_omega(we, R0, a, p0[3 * e], p0[3 * e + 1], p0[3 * e + 2], g);
            sE += om * dEdr[3 * e + k];
            sP += om * (gb[6 * e + 3 + k] + gb[6 * e + k]);
            const double *Mi = Minv + 9 * e;
            sJ += Mi[k] * g[0] + Mi[3 + k] * g[1] + Mi[6 + k] * g[2];
        }
        const size_t o = (size_t)w * 3 * A + idx;
        if (out.dEL_dR) out.dEL_dR[o] = sE;
        if (out.dlnpsi_dR) out.dlnpsi_dR[o] = sP;
        if (out.dlnjac_dR) out.dlnjac_dR[o] = sJ;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_mo_rows(const SysDev &S, const T *C, const double *R, const double *pos, int64_t n_rows,
                          const AoTiles &tiles, T *out, int nc, hipStream_t st) {
    const dim3 g((unsigned)((n_rows + 31) / 32));
    if (nc == 1)
        hipLaunchKernelGGL((k_mo_rows<T, 1>), g, dim3(256), 0, st, S, C, R, pos, n_rows, tiles, out);
    else
        hipLaunchKernelGGL((k_mo_rows<T, 5>), g, dim3(256), 0, st, S, C, R, pos, n_rows, tiles, out);
    return hipGetLastError();
}

hipError_t launch_warp(const SysDev &S, const double *R, const double *R0, const double *pos0, double *posw,
                       double *lnjac, int W, hipStream_t st) {
    hipLaunchKernelGGL(k_warp, dim3(W), dim3(128), 0, st, S, R, R0, pos0, posw, lnjac, W);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_walker_dense(const SysDev &S, const double *R, const MeasBufs<T> &mb, const WalkerOut &out,
                               int *status, const DenseLayout &L, int W, hipStream_t st) {
    hipLaunchKernelGGL(k_walker_dense<T>, dim3(W), dim3(256), L.bytes, st, S, R, mb, out, status, L);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_ao(const SysDev &S, const T *C, const double *R, const MeasBufs<T> &mb,
                             const AoTiles &tiles, const WalkerOut &out, int W, hipStream_t st) {
    const dim3 g((unsigned)tiles.n_tiles, (unsigned)W);
    const int n = S.n_occ;
    if (n <= 16)
        hipLaunchKernelGGL((k_adjoint_ao<T, 16>), g, dim3(256), 0, st, S, C, R, mb, tiles, out);
    else if (n <= 32)
        hipLaunchKernelGGL((k_adjoint_ao<T, 32>), g, dim3(256), 0, st, S, C, R, mb, tiles, out);
    else if (n <= 48)
        hipLaunchKernelGGL((k_adjoint_ao<T, 48>), g, dim3(256), 0, st, S, C, R, mb, tiles, out);
    else
        hipLaunchKernelGGL((k_adjoint_ao<T, 64>), g, dim3(256), 0, st, S, C, R, mb, tiles, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const SysDev &S, const double *R, const double *R0, const MeasBufsD &mb, int n_tiles,
                           const WalkerOut &out, int warp, int W, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)S.N * (3 + 3 + 6 + 3 + 9 + 4) + sizeof(int) * (size_t)S.N;
    hipLaunchKernelGGL(k_finalize, dim3(W), dim3(128), lds, st, S, R, R0, mb, n_tiles, out, warp);
    return hipGetLastError();
}

hipError_t configure_pipeline(size_t dense_lds) {
    return hipFuncSetAttribute((const void *)k_walker_dense<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)dense_lds);
}

template hipError_t launch_mo_rows<double>(const SysDev &, const double *, const double *, const double *, int64_t,
                                           const AoTiles &, double *, int, hipStream_t);
template hipError_t launch_walker_dense<double>(const SysDev &, const double *, const MeasBufs<double> &,
                                                const WalkerOut &, int *, const DenseLayout &, int, hipStream_t);
template hipError_t launch_adjoint_ao<double>(const SysDev &, const double *, const double *,
                                              const MeasBufs<double> &, const AoTiles &, const WalkerOut &, int,
                                              hipStream_t);

}  // namespace vmcx
