// vmc_pipeline.hip -- batched gfx950 kernels of the VMC force hot path.
//
//   k_warp         space-warped electron positions and ln Jac per walker
//   k_walker_dense per walker: Slater inverses, E_L, ln|Psi|, Abar = (K X K)^T/2
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
//   Abar = 1/2 (K X K)^T, written with K~[e][i] = K[i][e] for the adjoint.
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
// k_finalize: one block per walker.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_finalize(SysDev S, const double *__restrict__ R,
                                                  const double *__restrict__ R0, MeasBufsD mb,
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
        const double *dp = mb.dedr_part + ((size_t)w * N + e) * 3;
        double d0 = dp[0], d1 = dp[1], d2 = dp[2];
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

hipError_t launch_finalize(const SysDev &S, const double *R, const double *R0, const MeasBufsD &mb,
                           const WalkerOut &out, int warp, int W, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)S.N * (3 + 3 + 6 + 3 + 9 + 4) + sizeof(int) * (size_t)S.N;
    hipLaunchKernelGGL(k_finalize, dim3(W), dim3(128), lds, st, S, R, R0, mb, out, warp);
    return hipGetLastError();
}

hipError_t configure_pipeline(size_t dense_lds) {
    return hipFuncSetAttribute((const void *)k_walker_dense<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)dense_lds);
}

template hipError_t launch_walker_dense<double>(const SysDev &, const double *, const MeasBufs<double> &,
                                                const WalkerOut &, int *, const DenseLayout &, int, hipStream_t);

}  // namespace vmcx
