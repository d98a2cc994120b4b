// vmc_adjoint.hip -- AO-space adjoint of one measurement on the matrix cores.
//
// One block per walker; the block's wavefronts take 16-AO sub-tiles in turn.
// For a sub-tile (AOs mu) and 16-electron row tile (electrons e):
//   kappa[e][mu] = sum_i K~[e][i] C[mu][i],  a[e][mu] = sum_i Abar[e][i] C[mu][i]
// on 16x16x4 MFMA (A = K~ or Abar from LDS, B = C held in registers).  The
// accumulator of that product holds, in every lane, the (e, mu) pairs that
// the lane then evaluates (AO value, gradient, Hessian, grad-Laplacian):
//   t_k = a d_k psi - kappa (sum_d g_d d_k d_d psi + 1/2 d_k lap psi)
//   s_k = kappa d_k psi,   q = -g . grad psi - 1/2 lap psi
// and those per-lane values are exactly the A operand (rows mu, k = e) of the
// outer products
//   O[mu][i] = sum_e psi[e][mu] K~[e][i]
//   G[mu][i] = sum_e psi[e][mu] Abar[e][i] + q[e][mu] K~[e][i]
// whose B operand (K~, Abar rows e) comes from LDS.  Per AO the electron sums
// of t_k and s_k go to tao; per electron the AO sums of t_k (dE_L/dr_e, the
// determinant part) go to dedr_part, in a fixed order.
#include "vmc_pipeline.hpp"
#include "vmc_mfma.hpp"

namespace vmcx {

template <typename T, int NT>
__global__ __launch_bounds__(512) void k_adjoint_mfma(SysDev S, const T *__restrict__ C,
                                                      const double *__restrict__ R, MeasBufs<T> mb, WalkerOut out,
                                                      AdjLayout L) {
    typedef Mfma<T> MF;
    constexpr int KS = 4 * NT;        // k-steps over orbitals (4 per step)
    constexpr int NPR = sizeof(T) == 4 ? 3 : 0;   // primitives held in registers (FP32)
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int N = S.N, n = S.n_occ, M = S.M;
    const int ldk = L.ldk, RT = L.rt;
    T *Ks = (T *)(smem + L.off_k);    // [RT*16][ldk]  K~[e][i]
    T *As = (T *)(smem + L.off_a);    // [RT*16][ldk]  Abar[e][i]
    double *sp = (double *)(smem + L.off_p);    // [N][3]
    T *sg = (T *)(smem + L.off_g);              // [N][3] Jastrow gradient (arithmetic type)
    double *dpw = (double *)(smem + L.off_d);   // [nw][N][3] per-wave dE_L/dr_e partials
    const T *ktw = mb.ktil + (size_t)w * N * n;
    const T *abw = mb.abar + (size_t)w * N * n;
    // K~ and Abar into LDS, eight elements per thread in flight (clamped,
    // unconditional loads; the padding is selected afterwards)
    for (int k0 = tid; k0 < RT * 16 * ldk; k0 += 8 * (int)blockDim.x) {
        T kv[8], av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u * (int)blockDim.x;
            const int e = min(k / ldk, N - 1), i = min(k - (k / ldk) * ldk, n - 1);
            kv[u] = ktw[(size_t)e * n + i];
            av[u] = abw[(size_t)e * n + i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u * (int)blockDim.x;
            if (k < RT * 16 * ldk) {
                const int e = k / ldk, i = k - (k / ldk) * ldk;
                const bool on = e < N && i < n;
                Ks[k] = on ? kv[u] : T(0);
                As[k] = on ? av[u] : T(0);
            }
        }
    }
    for (int k = tid; k < 3 * N; k += blockDim.x) {
        sp[k] = mb.pos[(size_t)w * N * 3 + k];
        sg[k] = (T)mb.gb[(size_t)w * N * 6 + 6 * (k / 3) + (k - (k / 3) * 3)];
    }
    for (int k = tid; k < nw * 3 * N; k += blockDim.x) dpw[k] = 0.0;
    __syncthreads();
    double *dw = dpw + (size_t)wave * 3 * N;
    const int ml = lane & 15, kg = lane >> 4;
    const int n_sub = (M + 15) >> 4;
    for (int st = wave; st < n_sub; st += nw) {
        const int mu = 16 * st + ml;
        const bool vm = mu < M;
        // this lane's AO: monomial and primitives in registers for the sub-tile
        AoLane<T, NPR> al;
        ao_lane_load<T, NPR>(S.basis, vm ? mu : M - 1, al);
        if (!vm) al.c0[0] = al.c1[0] = al.c2[0] = al.c22[0] = T(0);   // no AO: every component 0
        const int atom = S.basis.shell_atom[S.basis.ao_shell[vm ? mu : M - 1]];
        const double Rx = R[3 * atom], Ry = R[3 * atom + 1], Rz = R[3 * atom + 2];
        T cB[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int i = 4 * ks + kg;
            cB[ks] = (vm && i < n) ? C[(size_t)mu * n + i] : T(0);
        }
        typename MF::acc_t accO[NT], accG[NT];
#pragma unroll
        for (int it = 0; it < NT; ++it) accO[it] = accG[it] = MF::zero();
        // per-AO sums over this lane's 4 RT electrons in T, then over the
        // four row groups in FP64
        T tl[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        for (int rt = 0; rt < RT; ++rt) {
            typename MF::acc_t kap = MF::zero(), aa = MF::zero();
            const T *kr = Ks + (16 * rt + ml) * ldk + kg;
            const T *ar = As + (16 * rt + ml) * ldk + kg;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                kap = MF::fma(kr[4 * ks], cB[ks], kap);
                aa = MF::fma(ar[4 * ks], cB[ks], aa);
            }
            // one (e, mu) evaluation at a time: unrolled, four would be live.
            // Every lane evaluates: past the last AO all components are 0,
            // past the last electron (position of electron N - 1) kappa, a
            // and the K~ / Abar rows are 0, so nothing of it reaches a sum.
#pragma unroll 1
            for (int v = 0; v < 4; ++v) {
                const int e = 16 * rt + MF::row(lane, v), ec = min(e, N - 1);
                const double dx = sp[3 * ec] - Rx, dy = sp[3 * ec + 1] - Ry, dz = sp[3 * ec + 2] - Rz;
                const double rho_d = dx * dx + dy * dy + dz * dz;
                const T x = (T)dx, y = (T)dy, z = (T)dz, rho = (T)rho_d;
                T R0, u1, u2, u3;
                ao_lane_radial<T, NPR>(al, S.basis, rho_d, R0, u1, u2, u3);
                T d[14];
                ao_lane_components<T, NPR>(al, x, y, z, rho, R0, u1, u2, u3, d);
                const T gx = sg[3 * ec], gy = sg[3 * ec + 1], gz = sg[3 * ec + 2];
                const T hgx = gx * d[5] + gy * d[6] + gz * d[7];
                const T hgy = gx * d[6] + gy * d[8] + gz * d[9];
                const T hgz = gx * d[7] + gy * d[9] + gz * d[10];
                const T half = T(0.5);
                const T kv = kap[v], av = aa[v];
                const T t6[6] = {av * d[1] - kv * (hgx + half * d[11]), av * d[2] - kv * (hgy + half * d[12]),
                                 av * d[3] - kv * (hgz + half * d[13]), kv * d[1], kv * d[2], kv * d[3]};
                const T psi = d[0];
                const T q = -(gx * d[1] + gy * d[2] + gz * d[3]) - half * d[4];
#pragma unroll
                for (int c = 0; c < 6; ++c) tl[c] += t6[c];
                // AO sum of t_k for electron e over the 16 lanes of this row
                // group (a DPP row), left in its last lane
                const double d0 = (double)row16_sum_last<T>(t6[0]), d1 = (double)row16_sum_last<T>(t6[1]),
                             d2 = (double)row16_sum_last<T>(t6[2]);
                if (ml == 15 && e < N) {
                    dw[3 * e] += d0;
                    dw[3 * e + 1] += d1;
                    dw[3 * e + 2] += d2;
                }
                const T *kb = Ks + e * ldk + ml;
                const T *ab = As + e * ldk + ml;
#pragma unroll
                for (int it = 0; it < NT; ++it) {
                    const T bk = kb[16 * it], ba = ab[16 * it];
                    accO[it] = MF::fma(psi, bk, accO[it]);
                    accG[it] = MF::fma(psi, ba, accG[it]);
                    accG[it] = MF::fma(q, bk, accG[it]);
                }
            }
        }
        // outer products of the walker for this sub-tile
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int mr = 16 * st + MF::row(lane, v);
            if (mr >= M) continue;
#pragma unroll
            for (int it = 0; it < NT; ++it) {
                const int i = 16 * it + ml;
                if (i < n) {
                    const size_t o = ((size_t)w * M + mr) * n + i;
                    if (out.O) out.O[o] = (double)accO[it][v];
                    if (out.G) out.G[o] = (double)accG[it][v];
                    if (out.Of) out.Of[o] = (float)accO[it][v];
                    if (out.Gf) out.Gf[o] = (float)accG[it][v];
                }
            }
        }
        // electron sums per AO: add the four row groups
        double td[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            td[c] = (double)tl[c];
            td[c] += __shfl_xor(td[c], 16, 64);
            td[c] += __shfl_xor(td[c], 32, 64);
        }
        if (kg == 0 && vm)
#pragma unroll
            for (int c = 0; c < 6; ++c) mb.tao[((size_t)w * M + mu) * 6 + c] = td[c];
    }
    __syncthreads();
    // dE_L/dr_e (determinant part): the wavefronts' partials in a fixed order
    double *dpart = mb.dedr_part + (size_t)w * N * 3;
    for (int k = tid; k < 3 * N; k += blockDim.x) {
        double acc = 0.0;
        for (int q = 0; q < nw; ++q) acc += dpw[(size_t)q * 3 * N + k];
        dpart[k] = acc;
    }
}

template <typename T>
hipError_t launch_adjoint(const SysDev &S, const T *C, const double *R, const MeasBufs<T> &mb,
                          const WalkerOut &out, const AdjLayout &L, int W, hipStream_t st) {
    const dim3 g((unsigned)W), b((unsigned)(64 * L.waves));
    switch ((S.n_occ + 15) / 16) {
        case 1: hipLaunchKernelGGL((k_adjoint_mfma<T, 1>), g, b, L.bytes, st, S, C, R, mb, out, L); break;
        case 2: hipLaunchKernelGGL((k_adjoint_mfma<T, 2>), g, b, L.bytes, st, S, C, R, mb, out, L); break;
        case 3: hipLaunchKernelGGL((k_adjoint_mfma<T, 3>), g, b, L.bytes, st, S, C, R, mb, out, L); break;
        default: hipLaunchKernelGGL((k_adjoint_mfma<T, 4>), g, b, L.bytes, st, S, C, R, mb, out, L); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t configure_adjoint(size_t lds) {
    const void *f[4] = {(const void *)k_adjoint_mfma<T, 1>, (const void *)k_adjoint_mfma<T, 2>,
                        (const void *)k_adjoint_mfma<T, 3>, (const void *)k_adjoint_mfma<T, 4>};
    for (const void *g : f) {
        const hipError_t e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_adjoint<double>(const SysDev &, const double *, const double *, const MeasBufs<double> &,
                                           const WalkerOut &, const AdjLayout &, int, hipStream_t);
template hipError_t configure_adjoint<double>(size_t);

template hipError_t launch_adjoint<float>(const SysDev &, const float *, const double *, const MeasBufs<float> &,
                                          const WalkerOut &, const AdjLayout &, int, hipStream_t);
template hipError_t configure_adjoint<float>(size_t);

}  // namespace vmcx
