// vmc_pipeline.hip -- batched gfx950 kernels of the VMC force hot path.
//
//   k_warp         space-warped electron positions and ln Jac per walker
//   k_finalize     per walker: Jastrow/potential terms of dE_L/dr, SWCT force
//                  terms dE_L/dR, dln|Psi|/dR, dln Jac/dR
//
// Both work in FP64.
#include <algorithm>
#include <type_traits>

#include "vmc_pipeline.hpp"
#include "vmc_regs.hpp"

namespace vmcx {

// ---------------------------------------------------------------------------
// Space-warp helpers: omega_a(r) = kappa_a / sum_b kappa_b, kappa = d^-4;
// grad omega_a = omega_a (g_a - sum_b omega_b g_b), g_b = -4 (r - R_b)/d_b^2.
// Within 1e-12 bohr of nucleus c: omega = delta_ac, gradient 0.  The
// reciprocals 1/d^2 come from rcp_nr (a few ulp from the rounded quotient).
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
        double id2 = 0.0;
        if (d2 < 1e-24)
            o.near = b;
        else
            id2 = rcp_nr(d2);
        S += id2 * id2;
    }
    o.invS = 1.0 / S;
    o.sg[0] = o.sg[1] = o.sg[2] = 0.0;
    if (o.near < 0)
        for (int b = 0; b < A; ++b) {
            const double dx = x - R0[3 * b], dy = y - R0[3 * b + 1], dz = z - R0[3 * b + 2];
            const double id2 = rcp_nr(dx * dx + dy * dy + dz * dz);
            const double om = o.invS * id2 * id2;
            const double f = -4.0 * id2;
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
    const double id2 = rcp_nr(dx * dx + dy * dy + dz * dz);
    const double om = we.invS * id2 * id2;
    const double f = -4.0 * id2;
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
// k_finalize: one block per walker.
// ---------------------------------------------------------------------------
// doubles of the region that holds Minv [N][9] and wS [N][4], then the
// [128][9] partial sums of the per-nucleus phase
__host__ __device__ inline int finalize_region(int N) { return 13 * N > 128 * 9 ? 13 * N : 128 * 9; }

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
    // (Minv and wS, at least 128 x 9 doubles, later hold the partial sums)
    double *bw = Minv + finalize_region(N);   // [2][N][3] pair terms gathered by each wavefront
    int *wnear = (int *)(bw + 6 * N);
    const int wave = tid >> 6;
    for (int i = tid; i < 3 * N; i += 128) {
        p[i] = mb.pos[(size_t)w * N * 3 + i];
        p0[i] = mb.pos0[(size_t)w * N * 3 + i];
    }
    for (int i = tid; i < 6 * N; i += 128) gb[i] = mb.gb[(size_t)w * N * 6 + i];
    for (int i = tid; i < 6 * N; i += 128) bw[i] = 0.0;
    __syncthreads();
    // Electron-electron terms of dE_L/dr, each pair once: the term of pair
    // (e, k) is odd under the exchange of e and k (bit for bit: every
    // difference and product in it changes sign exactly), so round s pairs
    // thread e with k = (e + s) mod N, adds the term to e and subtracts it
    // from k's slot in its wavefront's table (a permutation of the slots in
    // every round, read and written in program order).  Rounds s = 1 .. N/2
    // cover every pair once; in round N/2 of an even N only e < N/2 takes part.
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (tid < N) {
        const int e = tid;
        const double x = p[3 * e], y = p[3 * e + 1], z = p[3 * e + 2];
        const double ge[3] = {-(gb[6 * e + 3] + gb[6 * e]), -(gb[6 * e + 4] + gb[6 * e + 1]),
                              -(gb[6 * e + 5] + gb[6 * e + 2])};
        double *bme = bw + (size_t)wave * 3 * N;
        for (int s = 1; 2 * s <= N; ++s) {
            if (2 * s == N && e >= s) break;
            int k = e + s;
            if (k >= N) k -= N;
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            const double dx = x - p[3 * k], dy = y - p[3 * k + 1], dz = z - p[3 * k + 2];
            const double ir = rsqrt_nr(dx * dx + dy * dy + dz * dz);
            const double r = (dx * dx + dy * dy + dz * dz) * ir;
            const double ux = dx * ir, uy = dy * ir, uz = dz * ir;
            const JasD pd = jas_all(r, S.ee_a, S.ee_F, S.ee_form);
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
            a0 += d0;
            a1 += d1;
            a2 += d2;
            bme[3 * k] -= d0;
            bme[3 * k + 1] -= d1;
            bme[3 * k + 2] -= d2;
            // the next round's partner slot of lane e - 1 is this round's of
            // lane e: keep the rounds' LDS accesses in order
            wave_sync_s();
        }
    }
    __syncthreads();
    if (tid < N) {
        const int e = tid;
        const double *dp = mb.dedr_part + ((size_t)w * N + e) * 3;
        double d0 = dp[0] + (a0 + (bw[3 * e] + bw[3 * N + 3 * e]));
        double d1 = dp[1] + (a1 + (bw[3 * e + 1] + bw[3 * N + 3 * e + 1]));
        double d2 = dp[2] + (a2 + (bw[3 * e + 2] + bw[3 * N + 3 * e + 2]));
        const double x = p[3 * e], y = p[3 * e + 1], z = p[3 * e + 2];
        for (int a = 0; a < A; ++a) {
            const double dx = x - R[3 * a], dy = y - R[3 * a + 1], dz = z - R[3 * a + 2];
            const double ir = rsqrt_nr(dx * dx + dy * dy + dz * dz);
            const double f = S.Z[a] * ir * ir * ir;
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
    // per-nucleus sums: thread (a, j) takes electrons and AOs congruent to j
    // modulo tpa; the tpa partials of a nucleus are added in a fixed order
    double *part = Minv;   // [128][9] once Minv and wS are read
    const int tpa = 128 / A;
    double sE[3] = {0, 0, 0}, sP[3] = {0, 0, 0}, sJ[3] = {0, 0, 0};
    if (tid < tpa * A) {
        const int a = tid / tpa, j = tid - (tid / tpa) * tpa;
        // this nucleus's AOs (congruent to j modulo tpa in its list)
        const int q0 = S.basis.atom_ao_ptr[a], q1 = S.basis.atom_ao_ptr[a + 1];
        for (int q = q0 + j; q < q1; q += tpa) {
            const double *t = mb.tao + ((size_t)w * M + S.basis.atom_ao[q]) * 6;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sE[k] -= t[k];
                sP[k] -= t[3 + k];
            }
        }
        if (mb.jtao) {
            // the one-/three-body Jastrow functions on this nucleus
            const int MJ = mb.jb.n_ao, j0 = mb.jb.atom_ao_ptr[a], j1 = mb.jb.atom_ao_ptr[a + 1];
            for (int q = j0 + j; q < j1; q += tpa) {
                const double *t = mb.jtao + ((size_t)w * MJ + mb.jb.atom_ao[q]) * 6;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    sE[k] -= t[k];
                    sP[k] -= t[3 + k];
                }
            }
        }
        const double Rx = R[3 * a], Ry = R[3 * a + 1], Rz = R[3 * a + 2], Za = S.Z[a];
        for (int e = j; e < N; e += tpa) {
            const double dx = p[3 * e] - Rx, dy = p[3 * e + 1] - Ry, dz = p[3 * e + 2] - Rz;
            const double ir = rsqrt_nr(dx * dx + dy * dy + dz * dz);
            const double f = Za * ir * ir * ir;
            sE[0] -= f * dx;
            sE[1] -= f * dy;
            sE[2] -= f * dz;
            WarpE we;
            we.invS = wS[4 * e];
            we.sg[0] = wS[4 * e + 1];
            we.sg[1] = wS[4 * e + 2];
            we.sg[2] = wS[4 * e + 3];
            we.near = wnear[e];
            double g[3];
            const double om = warp_omega(we, R0, a, p0[3 * e], p0[3 * e + 1], p0[3 * e + 2], g);
            const double *Mi = Minv + 9 * e;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sE[k] += om * dEdr[3 * e + k];
                sP[k] += om * (gb[6 * e + 3 + k] + gb[6 * e + k]);
                sJ[k] += Mi[k] * g[0] + Mi[3 + k] * g[1] + Mi[6 + k] * g[2];
            }
        }
        if (j == 0 && mb.ecp_dR) {
            // the pseudopotential's explicit derivative in this nucleus
            const double *q = mb.ecp_dR + ((size_t)w * A + a) * 3;
            sE[0] += q[0];
            sE[1] += q[1];
            sE[2] += q[2];
        }
        if (j == 0)
            for (int c = 0; c < A; ++c) {
                if (c == a) continue;
                const double dx = Rx - R[3 * c], dy = Ry - R[3 * c + 1], dz = Rz - R[3 * c + 2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double f = Za * S.Z[c] / (r2 * sqrt(r2));
                sE[0] -= f * dx;
                sE[1] -= f * dy;
                sE[2] -= f * dz;
            }
    }
    __syncthreads();   // Minv and wS are read: the partials replace them
    if (tid < tpa * A) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            part[9 * tid + k] = sE[k];
            part[9 * tid + 3 + k] = sP[k];
            part[9 * tid + 6 + k] = sJ[k];
        }
    }
    __syncthreads();
    for (int idx = tid; idx < 3 * A; idx += 128) {
        const int a = idx / 3, k = idx - (idx / 3) * 3;
        double sE = 0.0, sP = 0.0, sJ = 0.0;
        for (int j = 0; j < tpa; ++j) {
            const double *q = part + 9 * (a * tpa + j);
            sE += q[k];
            sP += q[3 + k];
            sJ += q[6 + k];
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

hipError_t launch_finalize(const SysDev &S, const double *R, const double *R0, const MeasBufsD &mb,
                           const WalkerOut &out, int warp, int W, hipStream_t st) {
    // one electron per thread of the 128 (the spin blocks hold at most 64 each)
    if (S.N > 128) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * ((size_t)S.N * (3 + 3 + 6 + 3 + 6) + (size_t)finalize_region(S.N)) +
                       sizeof(int) * (size_t)S.N;
    hipLaunchKernelGGL(k_finalize, dim3(W), dim3(128), lds, st, S, R, R0, mb, out, warp);
    return hipGetLastError();
}

__global__ void k_round_f32(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

hipError_t launch_round_f32(const double *x, float *y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_round_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

// The k walkers with the largest keys, by a most-significant-digit radix
// select on the bit patterns of the keys (non-negative doubles order like
// their bits; NaN counts as +inf), 8 bits per pass, then a pass over index
// segments that lists the keys above the k-th largest and as many equal to
// it as needed, lowest indices first, in index order.  One block.
__device__ inline unsigned long long promote_bits(double x) {
    return (unsigned long long)__double_as_longlong(x > 0.0 ? x : (x <= 0.0 ? 0.0 : __builtin_inf()));
}

template <int BS>
__device__ inline int block_excl_scan(int v, int *buf, int &total) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int o = 1; o < BS; o <<= 1) {
        const int a = t >= o ? buf[t - o] : 0;
        __syncthreads();
        buf[t] += a;
        __syncthreads();
    }
    const int incl = buf[t];
    total = buf[BS - 1];
    __syncthreads();
    return incl - v;
}

constexpr int SEL_BS = 1024;

__global__ __launch_bounds__(SEL_BS) void k_promote_select(const double *__restrict__ key, int W, int k,
                                                           int *__restrict__ list) {
    __shared__ unsigned hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_rem;
    __shared__ int buf[SEL_BS];
    const int tid = threadIdx.x;
    unsigned long long prefix = 0, mask = 0;
    int rem = k;
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
        for (int w = tid; w < W; w += SEL_BS) {
            const unsigned long long u = promote_bits(key[w]);
            if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int cum = 0, b = 255;
            for (; b > 0; --b) {
                if (cum + (int)hist[b] >= rem) break;
                cum += (int)hist[b];
            }
            s_rem = rem - cum;
            s_prefix = prefix | ((unsigned long long)b << shift);
        }
        __syncthreads();
        rem = s_rem;
        prefix = s_prefix;
        mask |= 255ull << shift;
        __syncthreads();
    }
    // prefix: the k-th largest key; rem: how many keys equal to it to take
    const int seg = (W + SEL_BS - 1) / SEL_BS;
    const int w0 = min(W, tid * seg), w1 = min(W, w0 + seg);
    int gt = 0, eq = 0;
    for (int w = w0; w < w1; ++w) {
        const unsigned long long u = promote_bits(key[w]);
        gt += u > prefix;
        eq += u == prefix;
    }
    int tot;
    const int eq_before = block_excl_scan<SEL_BS>(eq, buf, tot);
    const int take = max(0, min(eq, rem - eq_before));
    int off = block_excl_scan<SEL_BS>(gt + take, buf, tot);
    int taken = 0;
    for (int w = w0; w < w1; ++w) {
        const unsigned long long u = promote_bits(key[w]);
        if (u > prefix || (u == prefix && taken++ < take)) list[off++] = w;
    }
}

hipError_t launch_promote_select(const double *key, int W, int k, int *list, hipStream_t st) {
    if (k <= 0 || W <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_promote_select, dim3(1), dim3(SEL_BS), 0, st, key, W, min(k, W), list);
    return hipGetLastError();
}

// dst[k][j] = src[list[k]][j] and its inverse, rows of len doubles.
__global__ void k_gather_rows(const double *__restrict__ src, const int *__restrict__ list, int64_t kc, int64_t len,
                              double *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kc * len) return;
    const int64_t k = t / len, j = t - (t / len) * len;
    dst[t] = src[(int64_t)list[k] * len + j];
}

__global__ void k_scatter_rows(const double *__restrict__ src, const int *__restrict__ list, int64_t kc, int64_t len,
                               double *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kc * len) return;
    const int64_t k = t / len, j = t - (t / len) * len;
    dst[(int64_t)list[k] * len + j] = src[t];
}

__global__ void k_scatter_rows_f32(const double *__restrict__ src, const int *__restrict__ list, int64_t kc,
                                   int64_t len, float *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kc * len) return;
    const int64_t k = t / len, j = t - (t / len) * len;
    dst[(int64_t)list[k] * len + j] = (float)src[t];
}

hipError_t launch_scatter_rows_f32(const double *src, const int *list, int64_t kc, int64_t len, float *dst,
                                   hipStream_t st) {
    const int64_t n = kc * len;
    hipLaunchKernelGGL(k_scatter_rows_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, list, kc, len,
                       dst);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const double *src, const int *list, int64_t kc, int64_t len, double *dst,
                              hipStream_t st) {
    const int64_t n = kc * len;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, list, kc, len, dst);
    return hipGetLastError();
}

hipError_t launch_scatter_rows(const double *src, const int *list, int64_t kc, int64_t len, double *dst,
                               hipStream_t st) {
    const int64_t n = kc * len;
    hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, list, kc, len, dst);
    return hipGetLastError();
}

}  // namespace vmcx
