// vmc_sweep.hip -- single-electron Metropolis sweeps on gfx950.
//
// Every electron moves once per sweep, from its position at the start of the
// sweep, so all N proposals r'_e = r_e + sigma z_e of a sweep are known before
// its first move and none depends on an earlier move's outcome.  A sweep is
// therefore three launches:
//   k_propose      the proposals of every (walker, electron) (Philox normals);
//   k_mo_rows_mfma their MO rows phi(r'_e) = psi(r'_e)^T C, one product of
//                  [W N x M] by [M x n] on the matrix cores (vmc_mo.hip);
//   k_sweep_r      the moves in order, per walker: ratio, Jastrow difference,
//                  accept, Sherman-Morrison update, refreshes.
// k_sweep_r runs one wavefront per walker, L.wpb walkers per block.  Per
// wavefront in LDS: two broadcast vectors.  Everything else of the walker
// lives in registers:
//   * positions and proposals: lane l holds electrons l and l + 64;
//   * the uniforms of this sweep: lane l holds those of electrons l and l + 64;
//   * the inverse K of the spin block being swept: KN registers per lane,
//     lane p_k holding column k (electron k of the block), register r holding
//     orbital p_r, where p is the pivot order of the last rebuild (gj_regs).
// The MO matrix A[e][i] = phi_i(r_e) of every walker lives in HBM (type T);
// row e is rewritten (from the proposal's row) on each accepted move of e.
// Both blocks' inverses persist across sweeps: at the end of a block the
// registers go to HBM (Kst, with the layout permutation and a flag for a
// rebuild still due), and at the block's next start they come back.  A
// block's inverse is rebuilt from A in FP64 at the first sweep of a call
// (fresh), after every refresh_period-th proposed move of that block (its own
// move index sweep * nb + j), and after an accepted move with |ratio| below
// the forced-refresh threshold; a rebuild that falls due after the block's
// last move is carried to its next start by the flag.
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

// Proposals of one sweep: prop[w][e] = r_e + sigma z_e, z_e the Philox
// normals of (walker w, sweep, electron e).
__global__ __launch_bounds__(256) void k_propose(const double *__restrict__ walkers, int64_t n_rows, int N,
                                                 uint32_t sweep, uint64_t seed, double sigma,
                                                 double *__restrict__ prop) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rows) return;
    const uint32_t w = (uint32_t)(k / N), e = (uint32_t)(k - (int64_t)w * N);
    double z[3];
    move_normals(seed, w, sweep, e, z);
#pragma unroll
    for (int d = 0; d < 3; ++d) prop[3 * k + d] = fma(sigma, z[d], walkers[3 * k + d]);
}

// Sum over the pairs (e, k) of u(|r' - r_k|) - u(|r_e - r_k|), the lane's k
// being lane and lane + 64, reduced over the wavefront together with a term
// of each lane (extra: the lane's part of the one-/three-body difference).  FP64: exact sqrt and
// division.  FP32 (the mixed sweep, where it only enters the acceptance
// ratio): differences of FP64 positions rounded to FP32, hardware square root
// and reciprocal (about one ulp each), so the sum carries a relative error of
// order 1e-7, far below what moves a Metropolis decision.
template <typename T>
__device__ inline double jastrow_delta(const SysDev &S, int N, int e, int lane, double rx, double ry, double rz,
                                       double ex, double ey, double ez, const double *px, const double *py,
                                       const double *pz, T extra) {
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
        d += (float)extra;
        // wavefront sum in FP32: DPP sums of the four rows, then their totals
        d = row16_sum_last<float>(d);
        const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 15));
        const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 31));
        const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 47));
        const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), 63));
        return (double)((r0 + r1) + (r2 + r3));
    } else {
        double dj = (double)extra;
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

// The one-/three-body Jastrow slots of a lane: basis functions 4 lane + u,
// u < JQ (at most 256 functions).  Row e of chi(r') - chi(r) times
// [xi3 | xi1] is row-major with the xi1 column at MJ and a row stride of MJ + 1
// rounded up to a multiple of 4.  jrow4 reads a lane's four entries of a row
// as one vector when the row starts are 16-byte aligned (vec), else one by one;
// entries past n read 0.
constexpr int JQ = 4;

template <typename T>
__device__ inline void jrow4(const T *row, int mu0, int n, bool vec, T *d) {
    typedef T V4 __attribute__((ext_vector_type(4)));
    if (vec) {
        const V4 v = *(const V4 *)(row + mu0);
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = mu0 + u < n ? v[u] : T(0);
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = mu0 + u < n ? row[mu0 + u] : T(0);
    }
}

template <typename T, int KN, bool J13>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sweep_waves<T, KN>()))) void k_sweep_r(
    SysDev S, const T *__restrict__ Phip, const double *__restrict__ prop, double *walkers, int W, T *Amo,
    KState<T> ks, int fresh, uint32_t sweep, uint64_t seed, int refresh_period, uint8_t *accept, int *status,
    SweepLayout L, JasSweep<T> js) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int N = S.N, nu = S.n_up, n = S.n_occ;
    const int w = blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (w >= W) return;   // no block barrier in this kernel
    unsigned char *wbase = smem + (size_t)wave * L.wave_bytes;
    T *phin = (T *)(wbase + L.off_phin);   // phin[r] = phi_{p_r}
    T *colj = (T *)(wbase + L.off_colj);   // column of the moved electron
    double *wp = walkers + (size_t)w * N * 3;
    const double *pp = prop + (size_t)w * N * 3;
    const T *phw = Phip + (size_t)w * N * n;
    T *Aw = Amo + (size_t)w * N * n;
    // positions, proposals and this sweep's uniforms: lane l holds electrons
    // l and l + 64
    double px[2], py[2], pz[2], qx[2], qy[2], qz[2], du[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;
        const bool on = e < N;
        const int ec = on ? e : 0;
        px[h] = on ? wp[3 * e] : 0.0;
        py[h] = on ? wp[3 * e + 1] : 0.0;
        pz[h] = on ? wp[3 * e + 2] : 0.0;
        qx[h] = pp[3 * ec];
        qy[h] = pp[3 * ec + 1];
        qz[h] = pp[3 * ec + 2];
        du[h] = move_uniform(seed, (uint32_t)w, sweep, (uint32_t)ec);
    }
    bool bad = false;
    T Kr[KN];
    int sig = lane;
    // one-/three-body Jastrow: s = the sum of chi over the electrons' current
    // positions, over this lane's basis slots (kept current by the accepted
    // moves; rebuilt from the start positions every sweep)
    T sq[JQ];
    // (the lane's first slot; the rows' vector reads: X rows need MJ % 4 == 0,
    // the product rows are padded)
    const int jm0 = 4 * lane, jld = (js.MJ + 4) & ~3;
    const bool jvx = (js.MJ & 3) == 0 && jm0 < js.MJ, jvp = jm0 < js.MJ;
    if constexpr (J13) {
        // (two partial sums per slot: the electrons' loads in flight together)
        const T *x0 = js.X0 + (size_t)w * N * js.MJ;
        T a[2][JQ];
#pragma unroll
        for (int u = 0; u < JQ; ++u) a[0][u] = a[1][u] = T(0);
        int e = 0;
        for (; e + 2 <= N; e += 2) {
            T v0[JQ], v1[JQ];
            jrow4<T>(x0 + (size_t)e * js.MJ, jm0, js.MJ, jvx, v0);
            jrow4<T>(x0 + (size_t)(e + 1) * js.MJ, jm0, js.MJ, jvx, v1);
#pragma unroll
            for (int u = 0; u < JQ; ++u) {
                a[0][u] += v0[u];
                a[1][u] += v1[u];
            }
        }
        if (e < N) {
            T v0[JQ];
            jrow4<T>(x0 + (size_t)e * js.MJ, jm0, js.MJ, jvx, v0);
#pragma unroll
            for (int u = 0; u < JQ; ++u) a[0][u] += v0[u];
        }
#pragma unroll
        for (int u = 0; u < JQ; ++u) sq[u] = a[0][u] + a[1][u];
    }

    // the proposal's MO row of the first move (later rows are loaded one move
    // ahead, so that the load overlaps the move before)
    T ph_next = lane < nu ? phw[lane] : T(0);
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
        const double u = readlane_d(h ? du[1] : du[0], src);
        const double ex = readlane_d(h ? px[1] : px[0], src);
        const double ey = readlane_d(h ? py[1] : py[0], src);
        const double ez = readlane_d(h ? pz[1] : pz[0], src);
        const double rx = readlane_d(h ? qx[1] : qx[0], src);
        const double ry = readlane_d(h ? qy[1] : qy[0], src);
        const double rz = readlane_d(h ? qz[1] : qz[0], src);
        // phi_i(r') of lane i (zero from nb on); the next move's row in flight
        const T ph = ph_next;
        if (e + 1 < N) {
            const int nb1 = e + 1 < nu ? nu : S.n_dn;
            ph_next = lane < nb1 ? phw[(size_t)(e + 1) * n + lane] : T(0);
        }
        // Jastrow difference over the pairs (e, k), k held by this lane (in
        // the arithmetic type: it only enters the acceptance ratio)
        // one-/three-body difference, with d = chi' - chi_e and xi3 symmetric:
        // d^T xi3 (s - chi_e) = (xi3 d) . (s - chi_e) over the basis (this
        // lane's part, summed over the wavefront with the two-body terms),
        // plus xi1 . d from the last column of the products
        // (chi(r') itself is read only on an accepted move, for s += d)
        T x0[JQ], loc = T(0), p1 = T(0);
        if constexpr (J13) {
            const size_t row = (size_t)w * N + e;
            const T *pr = js.Pd + row * jld;
            T pd[JQ];
            jrow4<T>(pr, jm0, js.MJ, jvp, pd);
            jrow4<T>(js.X0 + row * js.MJ, jm0, js.MJ, jvx, x0);
            p1 = pr[js.MJ];   // the same in every lane
#pragma unroll
            for (int u = 0; u < JQ; ++u) loc += pd[u] * (sq[u] - x0[u]);
        }
        double dj = jastrow_delta<T>(S, N, e, lane, rx, ry, rz, ex, ey, ez, px, py, pz, loc) + (double)p1;
        // lane i < KN holds phi_i (zero from nb on): store it at the register
        // slot of orbital i
        if (lane < KN) phin[sig] = ph;
        wave_sync_s();
        // v = phi^T K for the column this lane holds (the broadcast vector
        // read 16 bytes at a time: the regions are 16-byte aligned)
        typedef T V16 __attribute__((ext_vector_type(16 / sizeof(T))));
        constexpr int VL = 16 / sizeof(T);
        T v0 = T(0), v1 = T(0);
#pragma unroll
        for (int r = 0; r < KN; r += VL) {
            const V16 a = *(const V16 *)(phin + r);
#pragma unroll
            for (int u = 0; u < VL; u += 2) {
                v0 += a[u] * Kr[r + u];
                v1 += a[u + 1] * Kr[r + u + 1];
            }
        }
        const T v = v0 + v1;
        // the lane holding electron jj of the block
        const int pj = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(__ballot(sig == jj)));
        const double ratio = (double)readlane_t(v, pj);
        // (FP32 sweep: the FP32 exponential, as accurate as its ratio)
        const double qv = ratio * (sizeof(T) == sizeof(float) ? (double)expf((float)dj) : exp(dj));
        const bool acc = u < qv * qv;
        if (acc) {
            T xp[JQ];
            if constexpr (J13) jrow4<T>(js.Xp + ((size_t)w * N + e) * js.MJ, jm0, js.MJ, jvx, xp);
            if (lane < nb) Aw[(size_t)e * n + lane] = ph;
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
                for (int r = 0; r < KN; r += VL) {
                    V16 c;
#pragma unroll
                    for (int u = 0; u < VL; ++u) c[u] = Kr[r + u];
                    *(V16 *)(colj + r) = c;
                }
            }
            wave_sync_s();
            if constexpr (J13) {
#pragma unroll
                for (int u = 0; u < JQ; ++u) sq[u] += xp[u] - x0[u];
            }
            const T rr = sizeof(T) == sizeof(float) ? (T)__builtin_amdgcn_rcpf((float)ratio) : (T)rcp_nr(ratio);
            const T t = (v - (lane == pj ? T(1) : T(0))) * rr;
#pragma unroll
            for (int r = 0; r < KN; r += VL) {
                const V16 c = *(const V16 *)(colj + r);
#pragma unroll
                for (int u = 0; u < VL; ++u) Kr[r + u] -= c[u] * t;
            }
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
static hipError_t launch_kn(const SysDev &S, const T *Phip, const double *prop, double *walkers, int W, T *Amo,
                            const KState<T> &ks, int fresh, uint32_t sweep, uint64_t seed, int refresh_period,
                            uint8_t *accept, int *status, const SweepLayout &L, const JasSweep<T> &js,
                            hipStream_t st) {
    const dim3 g((unsigned)((W + L.wpb - 1) / L.wpb)), b(64 * L.wpb);
    if (js.Xp)
        hipLaunchKernelGGL((k_sweep_r<T, KN, true>), g, b, L.bytes, st, S, Phip, prop, walkers, W, Amo, ks, fresh,
                           sweep, seed, refresh_period, accept, status, L, js);
    else
        hipLaunchKernelGGL((k_sweep_r<T, KN, false>), g, b, L.bytes, st, S, Phip, prop, walkers, W, Amo, ks, fresh,
                           sweep, seed, refresh_period, accept, status, L, js);
    return hipGetLastError();
}

int sweep_kn(int n_occ) { return n_occ <= 16 ? 16 : (n_occ <= 32 ? 32 : (n_occ <= 48 ? 48 : 64)); }

hipError_t launch_propose(const double *walkers, int64_t W, int N, uint32_t sweep, uint64_t seed, double sigma,
                          double *prop, hipStream_t st) {
    const int64_t rows = W * N;
    hipLaunchKernelGGL(k_propose, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, walkers, rows, N, sweep,
                       seed, sigma, prop);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SysDev &S, const T *Phip, const double *prop, double *walkers, int W, T *Amo,
                        const KState<T> &ks, int fresh, uint32_t sweep, uint64_t seed, int refresh_period,
                        uint8_t *accept, int *status, const SweepLayout &L, const JasSweep<T> &js, hipStream_t st) {
    switch (sweep_kn(S.n_occ)) {
        case 16:
            return launch_kn<T, 16>(S, Phip, prop, walkers, W, Amo, ks, fresh, sweep, seed, refresh_period, accept,
                                    status, L, js, st);
        case 32:
            return launch_kn<T, 32>(S, Phip, prop, walkers, W, Amo, ks, fresh, sweep, seed, refresh_period, accept,
                                    status, L, js, st);
        case 48:
            return launch_kn<T, 48>(S, Phip, prop, walkers, W, Amo, ks, fresh, sweep, seed, refresh_period, accept,
                                    status, L, js, st);
        default:
            return launch_kn<T, 64>(S, Phip, prop, walkers, W, Amo, ks, fresh, sweep, seed, refresh_period, accept,
                                    status, L, js, st);
    }
}

template <typename T>
hipError_t configure_sweep(size_t lds) {
    const void *f[4] = {(const void *)k_sweep_r<T, 16, false>, (const void *)k_sweep_r<T, 32, false>,
                        (const void *)k_sweep_r<T, 48, false>, (const void *)k_sweep_r<T, 64, false>};
    for (const void *g : f) {
        const hipError_t e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_sweep<double>(const SysDev &, const double *, const double *, double *, int, double *,
                                         const KState<double> &, int, uint32_t, uint64_t, int, uint8_t *, int *,
                                         const SweepLayout &, const JasSweep<double> &, hipStream_t);
template hipError_t launch_sweep<float>(const SysDev &, const float *, const double *, double *, int, float *,
                                        const KState<float> &, int, uint32_t, uint64_t, int, uint8_t *, int *,
                                        const SweepLayout &, const JasSweep<float> &, hipStream_t);
template <typename T>
int sweep_blocks_per_cu(int n_occ, int wpb, size_t lds) {
    const void *f[4] = {(const void *)k_sweep_r<T, 16, false>, (const void *)k_sweep_r<T, 32, false>,
                        (const void *)k_sweep_r<T, 48, false>, (const void *)k_sweep_r<T, 64, false>};
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
