// vmc_dense.hip -- per-walker dense part of one measurement (gfx950).
//
// One block of four wavefronts per walker.
//   phase A  waves 0 and 1: the inverse K of the up and down Slater blocks by
//            in-register Gauss-Jordan (FP64, partial pivoting), log|det|; or,
//            after a sweep, the sweep's inverse of the block followed by one
//            FP64 Newton step K + K (I - A K) on MFMA (then without log|det|);
//            every wave: Jastrow gradient g_e, Laplacian and value, e-e and
//            e-n potentials, each electron pair evaluated once (in rounds,
//            the partner's gradient share gathered per wavefront) and
//            combined in a fixed order.
//   phase B  per spin block, one wavefront per electron row: the determinant
//            gradient b_e = sum_i K[i][e] grad phi_i(r_e), lap D/D likewise,
//            and (with the adjoint) X[e][i] = lap phi_i + 2 g_e . grad phi_i;
//            then on 16x16x4 FP64 MFMA T = X K and
//            Abar = 1/2 (K X K)^T = 1/2 T^T K^T, written with K~[e][i] = K[i][e].
//            Abar is the sensitivity of E_L to the orbital values, so its
//            largest magnitude is the key by which the mixed path picks the
//            walkers it measures again in FP64 (formed, not stored, when
//            only that key is wanted).
//   phase C  block sums: E_L, ln|Psi| = log|det up| + log|det dn| + J.
// K, X and T stay FP64; K~ and Abar are stored in the arithmetic type T.
#include <cfloat>

#include "vmc_mfma.hpp"
#include "vmc_pipeline.hpp"
#include "vmc_regs.hpp"

namespace vmcx {

__device__ inline double block_max4(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__device__ inline double block_sum4(double v, double *red) {
    v = wave_sum_dpp(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T, int KN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_dense(SysDev S, const double *__restrict__ R, MeasBufs<T> mb, WalkerOut out,
                                               int *status, DenseLayout L) {
    typedef Mfma<double> MF;
    constexpr int RTS = KN / 16;                    // 16-row tiles of a spin block
    constexpr int TPW = (RTS * RTS + 3) / 4;        // output tiles per wavefront
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N = S.N, nu = S.n_up, nd = S.n_dn, n = S.n_occ, A = S.A;
    const int ldk = L.ldk;
    double *p = (double *)(smem + L.off_p);      // [N][3]
    double *g = (double *)(smem + L.off_g);      // [N][3] Jastrow gradient
    double *Ks = (double *)(smem + L.off_k);     // [2][KN][ldk]  K[i][e]
    double *Xs = (double *)(smem + L.off_x);     // [KN][ldk]     X, then T
    int *perm = (int *)(smem + L.off_perm);      // [2][64]
    double *red = (double *)(smem + L.off_red);  // [8]
    const T *ph = mb.phi + (size_t)w * N * 5 * n;
    for (int i = tid; i < 3 * N; i += 256) p[i] = mb.pos[(size_t)w * N * 3 + i];
    __syncthreads();
    double el_part = 0.0, j_part = 0.0;
    bool bad = false;
    if (wave < 2) {
        const int b = wave, off = b ? nu : 0, nb = b ? nd : nu;
        // B = A^T of the block: lane c holds orbital c at the block's electrons
        int lz = lane;
        asm volatile("" : "+v"(lz));
        int sig;
        double la = 0.0;
        double Br[KN];
        const bool from_state = mb.kst != nullptr && mb.kstale[2 * w + b] == 0;
        if (from_state) {
            // the sweep's inverse, in its register layout
            const T *kk = mb.kst + ((size_t)w * 2 + b) * KN * KN + min(lane, KN - 1);
#pragma unroll
            for (int r = 0; r < KN; ++r) {
                const double v = (double)kk[r * KN];
                Br[r] = lane < KN ? v : 0.0;
            }
            const int sg = (int)mb.ksig[((size_t)w * 2 + b) * KN + min(lane, KN - 1)];
            sig = lane < KN ? sg : lane;
        } else {
            // (clamped, unconditional loads: a guarded load per register would
            // be issued and waited for one at a time)
            const T *pa = ph + (size_t)off * 5 * n + min(lz, nb - 1);
            T av[KN];
#pragma unroll
            for (int r = 0; r < KN; ++r) av[r] = pa[(size_t)min(r, nb - 1) * 5 * n];
            double mx = 0.0;
#pragma unroll
            for (int r = 0; r < KN; ++r) {
                const bool in = lz < nb && r < nb;
                Br[r] = in ? (double)av[r] : ((lz == r) ? 1.0 : 0.0);   // identity padding
                mx = fmax(mx, in ? fabs(Br[r]) : 0.0);
            }
            gj_regs<KN, true>(Br, sig, bad, la, gj_tol(mx));
        }
        if (lane == 0) {
            red[4 + b] = la;
            red[8 + b] = from_state ? 1.0 : 0.0;
        }
        // natural layout: lane p_k holds column k with register j = orbital p_j
        if (lane < KN) perm[64 * b + sig] = lane;
        wave_sync_s();
        double *K = Ks + (size_t)b * KN * ldk;
        if (lane < KN)
#pragma unroll
            for (int j = 0; j < KN; ++j) K[perm[64 * b + j] * ldk + sig] = Br[j];
    }
    // Jastrow and potential, each electron pair once.  Round s pairs electron
    // e with k = (e + s) mod N; rounds 1 .. N/2 cover every pair once (in
    // round N/2 of an even N only e < N/2 takes part).  Threads 0-127 (waves 0
    // and 1, after the inverses) take rounds 1 .. N/4, threads 128-255 the
    // rest, electron e = tid % 128.  The pair's gradient term f (r_e - r_k) is
    // odd under exchange, bit for bit: e keeps it, and k's share is gathered
    // in the wavefront's own table (all lanes of a wavefront are in the same
    // round, so their slots differ; reads and writes in program order).  The
    // even terms (Laplacian, potential, J) enter the block sums once per pair
    // with weight 2 relative to the per-electron form.
    double *jp = (double *)(smem + L.off_jas);   // [2][N][3] own gradient partials
    double *bw = jp + 6 * N;                     // [4][N][3] partners' gradient partials
    {
        double *bme = bw + (size_t)wave * 3 * N;
        for (int i = lane; i < 3 * N; i += 64) bme[i] = 0.0;
        wave_sync_s();
        const int h = tid >> 7, e = tid & 127;
        const int s0 = N / 4, sb = h ? s0 + 1 : 1, se = h ? N / 2 : s0;
        if (e < N) {
            const double x = p[3 * e], y = p[3 * e + 1], z = p[3 * e + 2];
            double gx = 0.0, gy = 0.0, gz = 0.0;
            for (int s = sb; s <= se; ++s) {
                if (2 * s == N && e >= s) break;
                int k = e + s;
                if (k >= N) k -= N;
                const double dx = x - p[3 * k], dy = y - p[3 * k + 1], dz = z - p[3 * k + 2];
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double ir = rsqrt_nr(d2), r = d2 * ir;
                double u, u1, u2;
                if (S.ee_form == 1) {
                    const double ex = exp(-S.ee_F * r);
                    u1 = S.ee_a * ex;
                    u2 = -S.ee_F * u1;
                    u = S.ee_a * (1.0 - ex) / S.ee_F;
                } else {
                    const double q = rcp_nr(1.0 + S.ee_F * r);
                    u1 = S.ee_a * q * q;
                    u2 = -2.0 * S.ee_F * u1 * q;
                    u = S.ee_a * r * q;
                }
                const double f = u1 * ir;
                const double tx = f * dx, ty = f * dy, tz = f * dz;
                gx += tx;
                gy += ty;
                gz += tz;
                bme[3 * k] -= tx;
                bme[3 * k + 1] -= ty;
                bme[3 * k + 2] -= tz;
                el_part += ir - (u2 + 2.0 * f);
                j_part += u;
                // the next round's partner slot of lane e - 1 is this round's
                // of lane e: keep the rounds' LDS accesses in order
                wave_sync_s();
            }
            if (h)
                for (int a = 0; a < A; ++a) {
                    const double ax = x - R[3 * a], ay = y - R[3 * a + 1], az = z - R[3 * a + 2];
                    el_part -= S.Z[a] * rsqrt_nr(ax * ax + ay * ay + az * az);
                }
            double *o = jp + 3 * ((size_t)h * N + e);
            o[0] = gx;
            o[1] = gy;
            o[2] = gz;
        }
    }
    __syncthreads();
    for (int e = tid; e < N; e += 256) {
        double gq[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            gq[c] = (jp[3 * e + c] + jp[3 * N + 3 * e + c]) +
                    ((bw[3 * e + c] + bw[3 * N + 3 * e + c]) + (bw[6 * N + 3 * e + c] + bw[9 * N + 3 * e + c]));
        if (mb.jg) {
            // one-/three-body terms: gradient into the total, Laplacian
            const double *jg = mb.jg + ((size_t)w * N + e) * 4;
#pragma unroll
            for (int c = 0; c < 3; ++c) gq[c] += jg[c];
            el_part += -0.5 * jg[3];
        }
        g[3 * e] = gq[0];
        g[3 * e + 1] = gq[1];
        g[3 * e + 2] = gq[2];
        el_part += -0.5 * (gq[0] * gq[0] + gq[1] * gq[1] + gq[2] * gq[2]);
    }
    __syncthreads();
    const int ml = lane & 15, kg = lane >> 4;
    // a block started from the sweep's inverse: one FP64 Newton step
    // K <- K + K (I - A K) on the matrix cores (quadratic in the drift)
    for (int b = 0; b < 2; ++b) {
        if (red[8 + b] == 0.0) continue;
        const int nb = b ? nd : nu, off = b ? nu : 0;
        double *K = Ks + (size_t)b * KN * ldk;
        // (all of this thread's loads first: one latency, not one per element)
        constexpr int PER = (KN * KN + 255) / 256;
        T av[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = min(tid + 256 * q, KN * KN - 1);
            const int e = idx / KN, i = idx - (idx / KN) * KN;
            av[q] = ph[(size_t)(off + min(e, nb - 1)) * 5 * n + min(i, nb - 1)];
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q;
            if (idx < KN * KN) {
                const int e = idx / KN, i = idx - (idx / KN) * KN;
                const bool in = e < nb && i < nb;
                Xs[e * ldk + i] = in ? (double)av[q] : (e == i ? 1.0 : 0.0);
            }
        }
        __syncthreads();
        MF::acc_t tacc[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            tacc[q] = MF::zero();
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
                const double *xa = Xs + (16 * rt + ml) * ldk + kg;
                const double *kb = K + kg * ldk + 16 * ct + ml;
#pragma unroll
                for (int ks = 0; ks < KN / 4; ++ks) tacc[q] = MF::fma(xa[4 * ks], kb[4 * ks * ldk], tacc[q]);
            }
        }
        __syncthreads();   // A is read: R = I - A K replaces it
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + MF::row(lane, v), c = 16 * ct + ml;
                    Xs[r * ldk + c] = (r == c ? 1.0 : 0.0) - tacc[q][v];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            tacc[q] = MF::zero();
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
                const double *ka = K + (16 * rt + ml) * ldk + kg;
                const double *rb = Xs + kg * ldk + 16 * ct + ml;
#pragma unroll
                for (int ks = 0; ks < KN / 4; ++ks) tacc[q] = MF::fma(ka[4 * ks], rb[4 * ks * ldk], tacc[q]);
            }
        }
        __syncthreads();   // K is read: add the correction
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
#pragma unroll
                for (int v = 0; v < 4; ++v) K[(16 * rt + MF::row(lane, v)) * ldk + 16 * ct + ml] += tacc[q][v];
            }
        }
        __syncthreads();
    }
    const bool have_ld = red[8] == 0.0 && red[9] == 0.0;   // ln|det| known
    const double logdet = red[4] + red[5];
    const bool full = mb.ktil != nullptr;
    // Abar is also formed, not stored, when it decides the FP64 re-measurement
    const bool need_abar = full || mb.promote_key != nullptr;
    double abar_max = 0.0;
    double *gb = mb.gb + (size_t)w * N * 6;
    for (int b = 0; b < 2; ++b) {
        const int nb = b ? nd : nu, off = b ? nu : 0;
        const double *K = Ks + (size_t)b * KN * ldk;
        // one wavefront per electron row j of the block (rows nb..KN-1:
        // zeros).  The wavefront's gradient and Laplacian rows are loaded
        // together first (clamped, unconditional loads), so that their
        // latency is paid once rather than once per row.
        constexpr int JPW = (KN + 3) / 4;
        T rG[JPW][4];
        const int lc = min(lane, n - 1);
#pragma unroll
        for (int q = 0; q < JPW; ++q) {
            const T *row = ph + (size_t)(off + min(wave + 4 * q, nb - 1)) * 5 * n + lc;
#pragma unroll
            for (int c = 0; c < 4; ++c) rG[q][c] = row[(c + 1) * n];
        }
#pragma unroll
        for (int q = 0; q < JPW; ++q) {
            const int j = wave + 4 * q;
            if (j >= nb) {
                if (lane < KN) Xs[j * ldk + lane] = 0.0;
                continue;
            }
            const int e = off + j;
            const double gx = g[3 * e], gy = g[3 * e + 1], gz = g[3 * e + 2];
            double bx = 0.0, by = 0.0, bz = 0.0, lp = 0.0, xv = 0.0;
            if (lane < n) {
                const double Gx = (double)rG[q][0], Gy = (double)rG[q][1], Gz = (double)rG[q][2],
                             Lp = (double)rG[q][3];
                xv = Lp + 2.0 * (gx * Gx + gy * Gy + gz * Gz);
                if (lane < nb) {
                    const double kk = K[lane * ldk + j];
                    bx = kk * Gx;
                    by = kk * Gy;
                    bz = kk * Gz;
                    lp = kk * Lp;
                }
            }
            if (lane < KN) Xs[j * ldk + lane] = xv;
            bx = wave_sum_dpp(bx);
            by = wave_sum_dpp(by);
            bz = wave_sum_dpp(bz);
            lp = wave_sum_dpp(lp);
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
        if (!need_abar) continue;
        __syncthreads();
        // T = X K  (rows e', columns e)
        MF::acc_t tacc[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            tacc[q] = MF::zero();
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
                const double *xa = Xs + (16 * rt + ml) * ldk + kg;
                const double *kb = K + kg * ldk + 16 * ct + ml;
#pragma unroll
                for (int ks = 0; ks < KN / 4; ++ks) tacc[q] = MF::fma(xa[4 * ks], kb[4 * ks * ldk], tacc[q]);
            }
        }
        __syncthreads();   // every read of X is done: T replaces it
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[(16 * rt + MF::row(lane, v)) * ldk + 16 * ct + ml] = tacc[q][v];
            }
        }
        __syncthreads();
        // Abar[e][i] = 1/2 sum_e' T[e'][e] K[i][e']
        T *abw = full ? mb.abar + ((size_t)w * N + off) * n : nullptr;
        T *ktw = full ? mb.ktil + ((size_t)w * N + off) * n : nullptr;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = wave + 4 * q;
            if (t < RTS * RTS) {
                const int rt = t / RTS, ct = t - (t / RTS) * RTS;
                const double *ta = Xs + kg * ldk + 16 * rt + ml;
                const double *kb = K + (16 * ct + ml) * ldk + kg;
                MF::acc_t acc = MF::zero();
#pragma unroll
                for (int ks = 0; ks < KN / 4; ++ks) acc = MF::fma(ta[4 * ks * ldk], kb[4 * ks], acc);
                const int i = 16 * ct + ml;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int e = 16 * rt + MF::row(lane, v);
                    if (e < nb && i < n) {
                        abar_max = fmax(abar_max, fabs(0.5 * acc[v]));
                        if (full) {
                            abw[(size_t)e * n + i] = (T)(0.5 * acc[v]);
                            ktw[(size_t)e * n + i] = (T)K[i * ldk + e];
                        }
                    }
                }
            }
        }
        __syncthreads();   // the next block rewrites X
    }
    if (mb.promote_key) abar_max = block_max4(abar_max, red + 12);
    // nuclear repulsion: the A^2 ordered pairs spread over the block
    double vnn = 0.0;
    for (int q = tid; q < A * A; q += 256) {
        const int a = q / A, c = q - (q / A) * A;
        if (c <= a) continue;
        const double dx = R[3 * a] - R[3 * c], dy = R[3 * a + 1] - R[3 * c + 1], dz = R[3 * a + 2] - R[3 * c + 2];
        vnn += S.Z[a] * S.Z[c] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    const double EL = block_sum4(el_part + vnn, red);
    const double J = block_sum4(j_part, red) + (mb.ju ? mb.ju[w] : 0.0);
    const int anybad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) {
        if (mb.promote_key) mb.promote_key[w] = abar_max <= DBL_MAX ? abar_max : __builtin_inf();
        if (out.EL) out.EL[w] = EL;
        if (out.lnpsi) out.lnpsi[w] = have_ld ? logdet + J : __builtin_nan("");
        if (anybad) atomicOr(status, STATUS_SINGULAR);
        if (!isfinite(EL) || !isfinite(J) || (have_ld && !isfinite(logdet))) atomicOr(status, STATUS_NONFINITE);
    }
}

template <typename T>
hipError_t launch_dense(const SysDev &S, const double *R, const MeasBufs<T> &mb, const WalkerOut &out, int *status,
                        const DenseLayout &L, int W, hipStream_t st) {
    const dim3 g((unsigned)W), b(256);
    switch (sweep_kn(S.n_occ)) {
        case 16: hipLaunchKernelGGL((k_dense<T, 16>), g, b, L.bytes, st, S, R, mb, out, status, L); break;
        case 32: hipLaunchKernelGGL((k_dense<T, 32>), g, b, L.bytes, st, S, R, mb, out, status, L); break;
        case 48: hipLaunchKernelGGL((k_dense<T, 48>), g, b, L.bytes, st, S, R, mb, out, status, L); break;
        default: hipLaunchKernelGGL((k_dense<T, 64>), g, b, L.bytes, st, S, R, mb, out, status, L); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t configure_dense(size_t lds) {
    const void *f[4] = {(const void *)k_dense<T, 16>, (const void *)k_dense<T, 32>, (const void *)k_dense<T, 48>,
                        (const void *)k_dense<T, 64>};
    for (const void *g : f) {
        const hipError_t e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_dense<double>(const SysDev &, const double *, const MeasBufs<double> &, const WalkerOut &,
                                         int *, const DenseLayout &, int, hipStream_t);
template hipError_t configure_dense<double>(size_t);

template hipError_t launch_dense<float>(const SysDev &, const double *, const MeasBufs<float> &, const WalkerOut &,
                                        int *, const DenseLayout &, int, hipStream_t);
template hipError_t configure_dense<float>(size_t);

}  // namespace vmcx
