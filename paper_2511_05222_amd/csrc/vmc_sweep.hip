// vmc_sweep.hip -- single-electron Metropolis sweeps on gfx950.
//
// One wavefront per walker, L.wpb walkers per block.  Shared by the block in
// LDS: the MO coefficients C (transposed, odd row stride; every proposed move
// needs phi(r') = psi(r')^T C, i.e. all of C) and the basis tables (atom
// centres, primitives, packed shell descriptors).  Per wavefront in LDS: the
// AO values psi(r') and two broadcast vectors.  Everything else of the walker
// lives in registers:
//   * positions: lane l holds electrons l and l + 64;
//   * the draws of this sweep: lane l holds those of electrons l and l + 64;
//   * the inverse K of the spin block being swept: KN registers per lane,
//     lane p_k holding column k (electron k of the block), register r holding
//     orbital p_r, where p is the pivot order of the last rebuild (gj_regs).
// The MO matrix A[e][i] = phi_i(r_e) of every walker lives in HBM (type T);
// row e is rewritten on each accepted move of e.  Both blocks' inverses
// persist across sweeps: at the end of a block the registers go to HBM (Kst,
// with the layout permutation and a flag for a rebuild still due), and at the
// block's next start they come back.  A block's inverse is rebuilt from A in
// FP64 at the first sweep of a call (fresh), after every refresh_period-th
// proposed move of that block (its own move index sweep * nb + j), and after
// an accepted move with |ratio| < 1e-8; a rebuild that falls due after the
// block's last move is carried to its next start by the flag.
#include "vmc_pipeline.hpp"
#include "vmc_regs.hpp"

namespace vmcx {

// Rebuild the inverse of spin block [off, off + nb) from the walker's MO
// matrix Aw ([N][n], type T) into Kr, in the layout of gj_regs.
template <typename T, int KN>
__device__ inline void rebuild(const T *Aw, int n, int off, int nb, T (&Kr)[KN], int &sig, bool &bad) {
    const int lane = threadIdx.x & 63;
    // rows of A were written by this wavefront: make them visible to its loads
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    // an opaque copy of the lane id keeps the KN padding values from being
    // hoisted out of the sweep loop (they would stay live in registers)
    int lz = lane;
    asm volatile("" : "+v"(lz));
    // (clamped, unconditional loads: a guarded load per register would be
    // issued and waited for one at a time)
    const T *pa = Aw + (size_t)off * n + min(lz, nb - 1);
    T av[KN];
#pragma unroll
    for (int r = 0; r < KN; ++r) av[r] = pa[(size_t)min(r, nb - 1) * n];
    double Br[KN];
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < KN; ++r) {
        const bool in = lz < nb && r < nb;
        Br[r] = in ? (double)av[r] : ((lz == r) ? 1.0 : 0.0);   // padding
        mx = fmax(mx, in ? fabs(Br[r]) : 0.0);
    }
    double la;
    gj_regs<KN, false>(Br, sig, bad, la, gj_tol(mx));
#pragma unroll
    for (int r = 0; r < KN; ++r) Kr[r] = (T)Br[r];
}

// Values of the AOs of shell s at (rx, ry, rz) into psi, from the basis tables
// in LDS.  Component factors: 1/sqrt(3) for xx, yy, zz; 1 otherwise.
template <typename T>
__device__ inline void shell_values_lds(const SweepBasisLds &B, int s, double rx, double ry, double rz, T *psi) {
    const int sa = B.sha[s], sb = B.shb[s];
    const int atom = sa & 255, l = (sa >> 8) & 15, np = sa >> 12;
    const int mu0 = sb & 0xFFFF, p0 = sb >> 16;
    const T x = (T)(rx - B.R[3 * atom]), y = (T)(ry - B.R[3 * atom + 1]), z = (T)(rz - B.R[3 * atom + 2]);
    const T rho = x * x + y * y + z * z;
    const T *pe = (const T *)B.pexp + p0, *pc = (const T *)B.pcp + p0;
    T r0 = T(0);
    // (FP32, ratios only: the hardware exponential, relative error of order
    // |a rho| 2^-23, negligible on the terms that are not already tiny)
    for (int k = 0; k < np; ++k) {
        if constexpr (sizeof(T) == sizeof(float))
            r0 += pc[k] * __expf(-pe[k] * rho);
        else
            r0 += pc[k] * exp(-pe[k] * rho);
    }
    T *o = psi + mu0;
    if (l == 0) {
        o[0] = r0;
    } else if (l == 1) {
        o[0] = x * r0;
        o[1] = y * r0;
        o[2] = z * r0;
    } else {
        const T e3 = T(0.57735026918962576451);   // 1/sqrt(3)
        o[0] = e3 * (x * x) * r0;
        o[1] = (x * y) * r0;
        o[2] = (x * z) * r0;
        o[3] = e3 * (y * y) * r0;
        o[4] = (y * z) * r0;
        o[5] = e3 * (z * z) * r0;
    }
}

// 16-byte vectors of the MO-row product (four FP32 or two FP64 lanes of LDS
// per load; the element-wise products are plain scalar FMAs).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
    __device__ static float sum(type v) { return (v.x + v.y) + (v.z + v.w); }
};
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
    __device__ static double sum(type v) { return v.x + v.y; }
};

// Sum over the pairs (e, k) of u(|r' - r_k|) - u(|r_e - r_k|), the lane's k
// being lane and lane + 64, reduced over the wavefront.  FP64: exact sqrt and
// division.  FP32 (the mixed sweep, where it only enters the acceptance
// ratio): differences of FP64 positions rounded to FP32, hardware square root
// and reciprocal (about one ulp each), so the sum carries a relative error of
// order 1e-7, far below what moves a Metropolis decision.
template <typename T>
__device__ inline double jastrow_delta(const SysDev &S, int N, int e, int lane, double rx, double ry, double rz,
                                       double ex, double ey, double ez, const double *px, const double *py,
                                       const double *pz) {
    if constexpr (sizeof(T) == sizeof(float)) {
        const float a = (float)S.ee_a, F = (float)S.ee_F;
        const float aF = S.ee_form == 1 ? (float)(S.ee_a / S.ee_F) : 0.0f;
        float d = 0.0f;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int k = lane + 64 * hh;
            const float ax = (float)(rx - px[hh]), ay = (float)(ry - py[hh]), az = (float)(rz - pz[hh]);
            const float bx = (float)(ex - px[hh]), by = (float)(ey - py[hh]), bz = (float)(ez - pz[hh]);
            const float ra = __builtin_amdgcn_sqrtf(ax * ax + ay * ay + az * az);
            const float rb = __builtin_amdgcn_sqrtf(bx * bx + by * by + bz * bz);
            const float t = S.ee_form == 1
                                ? aF * (__expf(-F * rb) - __expf(-F * ra))
                                : a * ra * __builtin_amdgcn_rcpf(1.0f + F * ra) -
                                      a * rb * __builtin_amdgcn_rcpf(1.0f + F * rb);
            d += (k < N && k != e) ? t : 0.0f;
        }
        // wavefront sum in FP32: DPP sums of the four rows, then their totals
        d = row16_sum_last<float>(d);
        const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 15));
        const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 31));
        const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 47));
        const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 63));
        return (double)((r0 + r1) + (r2 + r3));
    } else {
        double dj = 0.0;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int k = lane + 64 * hh;
            if (k < N && k != e) {
                const double ax = rx - px[hh], ay = ry - py[hh], az = rz - pz[hh];
                const double bx = ex - px[hh], by = ey - py[hh], bz = ez - pz[hh];
                dj += jas_u(sqrt(ax * ax + ay * ay + az * az), S.ee_a, S.ee_F, S.ee_form) -
                      jas_u(sqrt(bx * bx + by * by + bz * bz), S.ee_a, S.ee_F, S.ee_form);
            }
        }
        return wave_sum_dpp(dj);
    }
}

// FP32 with KN <= 48 fits three wavefronts per SIMD (spilling a little in the
// FP64 rebuild); the rest runs two.
template <typename T, int KN>
constexpr int sweep_waves() {
    return (sizeof(T) == 4 && KN <= 48) ? 3 : 2;
}

template <typename T, int KN>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sweep_waves<T, KN>()))) void k_sweep_r(SysDev S, const T *__restrict__ Cg, const double *__restrict__ R,
                                                  double *walkers, int W, T *Amo, KState<T> ks, int fresh,
                                                  uint32_t sweep, uint64_t seed, double sigma, int refresh_period,
                                                  uint8_t *accept, int *status, SweepLayout L) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int N = S.N, nu = S.n_up, n = S.n_occ, M = S.M, NS = S.basis.n_shells;
    // block-shared: C transposed (Ct[i*ldc + mu] = C[mu][i]) and the basis
    T *Ct = (T *)smem;
    const int ldc = L.ldc;
    SweepBasisLds B{(double *)(smem + L.off_R), smem + L.off_pexp, smem + L.off_pcp, (int *)(smem + L.off_sha),
                    (int *)(smem + L.off_shb)};
    for (int k = threadIdx.x; k < M * n; k += blockDim.x) {
        const int mu = k / n, i = k - (k / n) * n;
        Ct[i * ldc + mu] = Cg[k];
    }
    // zero padding of the rows up to mpad (the vector loop reads it)
    for (int k = threadIdx.x; k < n * (L.mpad - M); k += blockDim.x) {
        const int i = k / (L.mpad - M), mu = M + k - (k / (L.mpad - M)) * (L.mpad - M);
        Ct[i * ldc + mu] = T(0);
    }
    for (int k = threadIdx.x; k < 3 * S.A; k += blockDim.x) B.R[k] = R[k];
    for (int k = threadIdx.x; k < NS; k += blockDim.x) {
        const int p0 = S.basis.shell_p0[k], np = S.basis.shell_np[k];
        B.sha[k] = S.basis.shell_atom[k] | (S.basis.shell_l[k] << 8) | (np << 12);
        B.shb[k] = S.basis.shell_mu0[k] | (p0 << 16);
        for (int q = 0; q < np; ++q) {
            ((T *)B.pexp)[p0 + q] = (T)S.basis.prim_exp[p0 + q];
            ((T *)B.pcp)[p0 + q] = (T)S.basis.prim_cp[p0 + q];
        }
    }
    __syncthreads();
    const int w = blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (w >= W) return;   // no block barrier follows
    unsigned char *wbase = smem + L.block_bytes + (size_t)wave * L.wave_bytes;
    T *psi = (T *)(wbase + L.off_psi);
    T *phin = (T *)(wbase + L.off_phin);   // phin[r] = phi_{p_r}
    T *colj = (T *)(wbase + L.off_colj);   // column of the moved electron
    for (int k = M + lane; k < L.mpad; k += 64) psi[k] = T(0);
    double *wp = walkers + (size_t)w * N * 3;
    T *Aw = Amo + (size_t)w * N * n;
    // positions and this sweep's draws: lane l holds electrons l and l + 64
    double px[2], py[2], pz[2], dz[2][3], du[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;
        const bool on = e < N;
        px[h] = on ? wp[3 * e] : 0.0;
        py[h] = on ? wp[3 * e + 1] : 0.0;
        pz[h] = on ? wp[3 * e + 2] : 0.0;
        move_draws(seed, (uint32_t)w, sweep, (uint32_t)(on ? e : 0), dz[h], du[h]);
    }
    bool bad = false;
    T Kr[KN];
    int sig = lane;

    const int npad = n <= 16 ? 16 : (n <= 32 ? 32 : 64);
    const int G = 64 / npad;
    const int li = lane & (npad - 1), lg = lane / npad;
    // lane group lg of the phi product covers AOs [lg*mchunk, (lg+1)*mchunk)
    // of the zero-padded range [0, mpad), in 16-byte vectors
    typedef typename Vec16<T>::type V;
    const int nvec = L.mchunk / Vec16<T>::W;
    const V *cvec = (const V *)(Ct + li * ldc + lg * L.mchunk);
    const V *svec = (const V *)(psi + lg * L.mchunk);
    bool need = true;
    for (int e = 0; e < N; ++e) {
        const int b = e < nu ? 0 : 1;
        const int off = b ? nu : 0;
        const int jj = e - off;
        const int nb = b ? S.n_dn : nu;
        T *kst = ks.K + ((size_t)w * 2 + b) * KN * KN;
        if (jj == 0) {
            // the block's inverse: rebuilt, or as left at its last move
            need = fresh || ks.stale[2 * w + b] != 0;
            if (!need) {
                const T *kk = kst + min(lane, KN - 1);
#pragma unroll
                for (int r = 0; r < KN; ++r) {
                    const T v = kk[r * KN];
                    Kr[r] = lane < KN ? v : T(0);
                }
                const int sg = (int)ks.sig[((size_t)w * 2 + b) * KN + min(lane, KN - 1)];
                sig = lane < KN ? sg : lane;
            }
        }
        if (need) {
            rebuild<T, KN>(Aw, n, off, nb, Kr, sig, bad);
            need = false;
        }
        const int src = e & 63, h = e >> 6;
        const double z0 = readlane_d(h ? dz[1][0] : dz[0][0], src);
        const double z1 = readlane_d(h ? dz[1][1] : dz[0][1], src);
        const double z2 = readlane_d(h ? dz[1][2] : dz[0][2], src);
        const double u = readlane_d(h ? du[1] : du[0], src);
        const double ex = readlane_d(h ? px[1] : px[0], src);
        const double ey = readlane_d(h ? py[1] : py[0], src);
        const double ez = readlane_d(h ? pz[1] : pz[0], src);
        const double rx = ex + sigma * z0, ry = ey + sigma * z1, rz = ez + sigma * z2;
        for (int s = lane; s < NS; s += 64) shell_values_lds<T>(B, s, rx, ry, rz, psi);
        // Jastrow difference over the pairs (e, k), k held by this lane (in
        // the arithmetic type: it only enters the acceptance ratio)
        double dj = jastrow_delta<T>(S, N, e, lane, rx, ry, rz, ex, ey, ez, px, py, pz);
        wave_sync_s();
        // phi_i(r') = sum_mu psi_mu C[mu][i]; lane group lg sums its AO range
        T ph = T(0);
        if (li < nb) {
            // up to KN = 48: four vectors per step (16 FP32 or 8 FP64
            // products per address increment); otherwise two (four would
            // spill in the rebuild)
            V a0 = V(T(0)), a1 = V(T(0));
            int k = 0;
            if constexpr (KN <= 48) {
                V a2 = V(T(0)), a3 = V(T(0));
                for (; k + 4 <= nvec; k += 4) {
                    a0 += svec[k] * cvec[k];
                    a1 += svec[k + 1] * cvec[k + 1];
                    a2 += svec[k + 2] * cvec[k + 2];
                    a3 += svec[k + 3] * cvec[k + 3];
                }
                a0 += a2;
                a1 += a3;
            } else {
                for (; k + 2 <= nvec; k += 2) {
                    a0 += svec[k] * cvec[k];
                    a1 += svec[k + 1] * cvec[k + 1];
                }
            }
            for (; k < nvec; ++k) a0 += svec[k] * cvec[k];
            a0 += a1;
            ph = Vec16<T>::sum(a0);
        }
        for (int o = npad; o < 64; o <<= 1) ph += __shfl_xor(ph, o, 64);
        // lane i < KN holds phi_i (zero from nb on): store it at the register
        // slot of orbital i
        if (lane < KN) phin[sig] = ph;
        wave_sync_s();
        // v = phi^T K for the column this lane holds
        T v0 = T(0), v1 = T(0);
#pragma unroll
        for (int r = 0; r < KN; r += 2) {
            v0 += phin[r] * Kr[r];
            v1 += phin[r + 1] * Kr[r + 1];
        }
        const T v = v0 + v1;
        // the lane holding electron jj of the block
        const int pj = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(sig == jj)));
        const double ratio = (double)readlane_t(v, pj);
        // (FP32 sweep: the FP32 exponential, as accurate as its ratio)
        const double qv = ratio * (sizeof(T) == sizeof(float) ? (double)expf((float)dj) : exp(dj));
        const bool acc = u < qv * qv;
        if (acc) {
            if (lane < nb && lg == 0) Aw[(size_t)e * n + lane] = ph;
            if (lane == src) {
                if (h) {
                    px[1] = rx;
                    py[1] = ry;
                    pz[1] = rz;
                } else {
                    px[0] = rx;
                    py[0] = ry;
                    pz[0] = rz;
                }
            }
            if (lane == pj) {
#pragma unroll
                for (int r = 0; r < KN; ++r) colj[r] = Kr[r];
            }
            wave_sync_s();
            const T rr = sizeof(T) == sizeof(float) ? (T)__builtin_amdgcn_rcpf((float)ratio) : (T)rcp_nr(ratio);
            const T t = (v - (lane == pj ? T(1) : T(0))) * rr;
#pragma unroll
            for (int r = 0; r < KN; ++r) Kr[r] -= colj[r] * t;
            if (fabs(ratio) < S.forced_ratio) need = true;
        }
        if (accept != nullptr && lane == 0) accept[(size_t)e * W + w] = acc ? 1 : 0;
        // refresh_period-th move of this block: rebuild before its next move
        const uint64_t m = (uint64_t)sweep * (uint64_t)nb + (uint64_t)jj;
        if (((m + 1) % (uint64_t)refresh_period) == 0) need = true;
        if (jj == nb - 1) {
            // end of the block: keep its inverse (and a rebuild still due)
#pragma unroll
            for (int r = 0; r < KN; ++r)
                if (lane < KN) kst[r * KN + lane] = Kr[r];
            if (lane < KN) ks.sig[((size_t)w * 2 + b) * KN + lane] = (uint8_t)sig;
            if (lane == 0) ks.stale[2 * w + b] = need ? 1 : 0;
            need = false;
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;
        if (e < N) {
            wp[3 * e] = px[h];
            wp[3 * e + 1] = py[h];
            wp[3 * e + 2] = pz[h];
        }
    }
    if (bad && lane == 0) atomicOr(status, STATUS_SINGULAR);
}

template <typename T, int KN>
static hipError_t launch_kn(const SysDev &S, const T *C, const double *R, double *walkers, int W, T *Amo,
                            const KState<T> &ks, int fresh, uint32_t sweep, uint64_t seed, double sigma,
                            int refresh_period, uint8_t *accept, int *status, const SweepLayout &L, hipStream_t st) {
    hipLaunchKernelGGL((k_sweep_r<T, KN>), dim3((unsigned)((W + L.wpb - 1) / L.wpb)), dim3(64 * L.wpb), L.bytes, st,
                       S, C, R, walkers, W, Amo, ks, fresh, sweep, seed, sigma, refresh_period, accept, status, L);
    return hipGetLastError();
}

int sweep_kn(int n_occ) { return n_occ <= 16 ? 16 : (n_occ <= 32 ? 32 : (n_occ <= 48 ? 48 : 64)); }

template <typename T>
hipError_t launch_sweep(const SysDev &S, const T *C, const double *R, double *walkers, int W, T *Amo,
                        const KState<T> &ks, int fresh, uint32_t sweep, uint64_t seed, double sigma,
                        int refresh_period, uint8_t *accept, int *status, const SweepLayout &L, hipStream_t st) {
    switch (sweep_kn(S.n_occ)) {
        case 16:
            return launch_kn<T, 16>(S, C, R, walkers, W, Amo, ks, fresh, sweep, seed, sigma, refresh_period, accept,
                                    status, L, st);
        case 32:
            return launch_kn<T, 32>(S, C, R, walkers, W, Amo, ks, fresh, sweep, seed, sigma, refresh_period, accept,
                                    status, L, st);
        case 48:
            return launch_kn<T, 48>(S, C, R, walkers, W, Amo, ks, fresh, sweep, seed, sigma, refresh_period, accept,
                                    status, L, st);
        default:
            return launch_kn<T, 64>(S, C, R, walkers, W, Amo, ks, fresh, sweep, seed, sigma, refresh_period, accept,
                                    status, L, st);
    }
}

template <typename T>
hipError_t configure_sweep(size_t lds) {
    const void *f[4] = {(const void *)k_sweep_r<T, 16>, (const void *)k_sweep_r<T, 32>,
                        (const void *)k_sweep_r<T, 48>, (const void *)k_sweep_r<T, 64>};
    for (const void *g : f) {
        const hipError_t e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_sweep<double>(const SysDev &, const double *, const double *, double *, int, double *,
                                         const KState<double> &, int, uint32_t, uint64_t, double, int, uint8_t *,
                                         int *, const SweepLayout &, hipStream_t);
template hipError_t launch_sweep<float>(const SysDev &, const float *, const double *, double *, int, float *,
                                        const KState<float> &, int, uint32_t, uint64_t, double, int, uint8_t *,
                                        int *, const SweepLayout &, hipStream_t);
template <typename T>
int sweep_blocks_per_cu(int n_occ, int wpb, size_t lds) {
    const void *f[4] = {(const void *)k_sweep_r<T, 16>, (const void *)k_sweep_r<T, 32>,
                        (const void *)k_sweep_r<T, 48>, (const void *)k_sweep_r<T, 64>};
    const int kn = sweep_kn(n_occ), k = kn == 16 ? 0 : (kn == 32 ? 1 : (kn == 48 ? 2 : 3));
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f[k], 64 * wpb, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

template int sweep_blocks_per_cu<double>(int, int, size_t);
template int sweep_blocks_per_cu<float>(int, int, size_t);
template hipError_t configure_sweep<double>(size_t);
template hipError_t configure_sweep<float>(size_t);

}  // namespace vmcx
