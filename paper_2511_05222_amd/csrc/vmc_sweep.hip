// vmc_sweep.hip -- single-electron Metropolis sweeps on gfx950.
//
// One wavefront per walker, L.wpb walkers per block.  The MO coefficients C
// stay resident in LDS for the whole sweep and are shared by the block's
// walkers (every proposed move needs phi(r') = psi(r')^T C, i.e. all of C).
// The MO matrix A[e][i] = phi_i(r_e) of every walker lives in HBM (built by
// k_mo_rows before the sweep; row e rewritten on each accepted move of e).
// Only the inverse K of the spin block being swept is kept in LDS; it is
// rebuilt from A in FP64 when the sweep reaches the block's first electron
// (no electron of that block has moved yet in this sweep, so this equals an
// inverse built at the start of the sweep), after every refresh_period-th
// proposed move, and after an accepted move with |ratio| < 1e-8.
// The random numbers of all N moves are drawn lane-parallel at sweep start
// (lane l draws for electrons l and l + 64) and read with readlane per move.
#include <type_traits>

#include "vmc_pipeline.hpp"

namespace vmcx {

__device__ inline void wave_sync_s() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline double readlane_d(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Gauss-Jordan inversion with partial pivoting (FP64, n <= 64) by one
// wavefront, on a matrix stored transposed: at[j*ld + i] = a[i][j] (ld odd,
// so that lanes walking their own column are free of LDS bank conflicts).
// The pivot of column k is the largest |a[i][k]|, i >= k.  On return
// at[j*ld + i] = inverse[i][j].  col: n doubles.  log|det|, the singular
// flag and the permutation are uniform across the wavefront.
__device__ void gj_invert_wave_t(double *at, int n, int ld, double *col, int *perm, double &logabs, bool &singular) {
    const int lane = threadIdx.x & 63;
    const bool on = lane < n;
    double *mine = at + lane * ld;   // column `lane` of a
    double la = 0.0;
    bool sing = false;
    for (int k = 0; k < n; ++k) {
        const double *ck = at + k * ld;   // column k of a
        double best = (on && lane >= k) ? fabs(ck[lane]) : -1.0;
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
        const int p = bi < n ? bi : k;   // no comparable pivot (non-finite column): keep the row order
        if (lane == 0) perm[k] = p;
        if (p != k && on) {
            const double t = mine[k];
            mine[k] = mine[p];
            mine[p] = t;
        }
        wave_sync_s();
        double cv = 0.0;
        if (on) {
            cv = ck[lane];
            col[lane] = lane == k ? 0.0 : cv;
        }
        wave_sync_s();
        const double piv = readlane_d(cv, k);
        if (!(fabs(piv) > 1e-300)) sing = true;
        la += log(fabs(piv));
        const double inv = 1.0 / piv;
        if (on) {
            const double rk = (lane == k) ? inv : mine[k] * inv;
            if (lane == k)
                for (int i = 0; i < n; ++i) mine[i] = 0.0;
            mine[k] = rk;
            // a[i][lane] -= col[i] rk (col[k] = 0 keeps row k)
            int i = 0;
            for (; i + 4 <= n; i += 4) {
                mine[i] -= col[i] * rk;
                mine[i + 1] -= col[i + 1] * rk;
                mine[i + 2] -= col[i + 2] * rk;
                mine[i + 3] -= col[i + 3] * rk;
            }
            for (; i < n; ++i) mine[i] -= col[i] * rk;
        }
        wave_sync_s();
    }
    // undo the row interchanges as column interchanges: lane = row
    for (int k = n - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k && on) {
            const double t = at[k * ld + lane];
            at[k * ld + lane] = at[p * ld + lane];
            at[p * ld + lane] = t;
        }
        wave_sync_s();
    }
    logabs = la;
    singular = sing;
}

// Kt = inverse of the spin block [off, off + nb) of the walker's MO matrix,
// stored transposed: Kt[c*ld + i] = K[i][c] (K[i][c] pairs orbital i with
// electron c of the block).
template <typename T>
__device__ void refresh_spin(const T *Aw, int n, int off, int nb, T *Kt, int ld, double *gjs, double *col, int *perm,
                             bool &bad) {
    const int lane = threadIdx.x & 63;
    // rows of A were written by this wavefront: make them visible to its loads
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    constexpr bool in_place = std::is_same<T, double>::value;
    double *at = in_place ? (double *)Kt : gjs;
    // at[i*ld + e] = A[e][i]: column i of the Slater matrix (orbital i)
    if (lane < nb)
        for (int e = 0; e < nb; ++e) at[lane * ld + e] = (double)Aw[(size_t)(off + e) * n + lane];
    wave_sync_s();
    double la;
    bool sing;
    gj_invert_wave_t(at, nb, ld, col, perm, la, sing);
    bad |= sing;
    if (!in_place) {
        if (lane < nb)
            for (int i = 0; i < nb; ++i) Kt[lane * ld + i] = (T)at[lane * ld + i];
        wave_sync_s();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sweep_w(SysDev S, const T *__restrict__ Cg, const double *__restrict__ R,
                                                  double *walkers, int W, T *Amo, uint32_t sweep, uint64_t seed,
                                                  double sigma, int refresh_period, uint8_t *accept, int *status,
                                                  SweepWLayout L) {
    extern __shared__ double smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int N = S.N, nu = S.n_up, n = S.n_occ, M = S.M;
    // C resident in LDS for the block, transposed: Ct[i*L.ldc + mu] = C[mu][i]
    T *Ct = (T *)smem;
    const int ldc = L.ldc;
    for (int k = threadIdx.x; k < M * n; k += blockDim.x) {
        const int mu = k / n, i = k - (k / n) * n;
        Ct[i * ldc + mu] = Cg[k];
    }
    __syncthreads();
    const int w = blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (w >= W) return;   // no block barrier follows
    double *base = smem + L.cdoubles + (size_t)wave * L.per_wave;
    double *pos = base + L.pos;
    T *K = (T *)(base + L.K);
    T *psi = (T *)(base + L.psi);
    T *phin = (T *)(base + L.phin);
    T *colj = (T *)(base + L.colj);
    double *gjs = base + L.gjs;
    double *col = base + L.col;
    int *perm = (int *)(base + L.perm);
    double *wp = walkers + (size_t)w * N * 3;
    T *Aw = Amo + (size_t)w * N * n;
    for (int i = lane; i < 3 * N; i += 64) pos[i] = wp[i];
    // this sweep's draws: lane l holds those of electrons l and l + 64
    double dz[2][3], du[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h;
        move_draws(seed, (uint32_t)w, sweep, (uint32_t)(e < N ? e : 0), dz[h], du[h]);
    }
    wave_sync_s();
    bool bad = false;

    const int npad = n <= 16 ? 16 : (n <= 32 ? 32 : 64);
    const int G = 64 / npad;
    const int li = lane & (npad - 1), lg = lane / npad;
    const int ldk = L.ldk;
    // lane group lg of the phi product covers AOs [m_lo, m_hi)
    const int mchunk = (M + G - 1) / G;
    const int m_lo = min(M, lg * mchunk), m_hi = min(M, m_lo + mchunk);
    for (int e = 0; e < N; ++e) {
        const int b = e < nu ? 0 : 1;
        const int off = b ? nu : 0;
        const int j = e - off;
        const int nb = b ? S.n_dn : nu;
        if (j == 0) refresh_spin<T>(Aw, n, off, nb, K, ldk, gjs, col, perm, bad);
        const int src = e & 63, h = e >> 6;
        const double z0 = readlane_d(h ? dz[1][0] : dz[0][0], src);
        const double z1 = readlane_d(h ? dz[1][1] : dz[0][1], src);
        const double z2 = readlane_d(h ? dz[1][2] : dz[0][2], src);
        const double u = readlane_d(h ? du[1] : du[0], src);
        const double rx = pos[3 * e] + sigma * z0, ry = pos[3 * e + 1] + sigma * z1, rz = pos[3 * e + 2] + sigma * z2;
        for (int s = lane; s < S.basis.n_shells; s += 64) {
            T v[6];
            const int nc = shell_eval<1, T>(S.basis, R, s, rx, ry, rz, v);
            const int m0 = S.basis.shell_mu0[s];
            for (int q = 0; q < nc; ++q) psi[m0 + q] = v[q];
        }
        double dj = 0.0;
        {
            const double ex = pos[3 * e], ey = pos[3 * e + 1], ez = pos[3 * e + 2];
            for (int k = lane; k < N; k += 64) {
                if (k == e) continue;
                const double px = pos[3 * k], py = pos[3 * k + 1], pz = pos[3 * k + 2];
                const double ax = rx - px, ay = ry - py, az = rz - pz;
                const double bx = ex - px, by = ey - py, bz = ez - pz;
                dj += pade_u(sqrt(ax * ax + ay * ay + az * az), S.ee_a, S.ee_F) -
                      pade_u(sqrt(bx * bx + by * by + bz * bz), S.ee_a, S.ee_F);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dj += __shfl_xor(dj, o, 64);
        wave_sync_s();
        // phi_i(r') = sum_mu psi_mu C[mu][i]; lane group lg sums mu = lg (mod G)
        T ph = T(0);
        if (li < nb) {
            T p0 = T(0), p1 = T(0), p2 = T(0), p3 = T(0);
            const T *cp = Ct + li * ldc + m_lo;
            const T *sp = psi + m_lo;
            const int len = m_hi - m_lo;
            int k = 0;
            for (; k + 8 <= len; k += 8) {
                p0 += sp[k] * cp[k];
                p1 += sp[k + 1] * cp[k + 1];
                p2 += sp[k + 2] * cp[k + 2];
                p3 += sp[k + 3] * cp[k + 3];
                p0 += sp[k + 4] * cp[k + 4];
                p1 += sp[k + 5] * cp[k + 5];
                p2 += sp[k + 6] * cp[k + 6];
                p3 += sp[k + 7] * cp[k + 7];
            }
            for (; k < len; ++k) p0 += sp[k] * cp[k];
            ph = (p0 + p1) + (p2 + p3);
        }
        for (int o = npad; o < 64; o <<= 1) ph += __shfl_xor(ph, o, 64);
        if (lg == 0 && li < nb) phin[li] = ph;
        wave_sync_s();
        // v_c = sum_i phi_i K[i][c]; ratio = v_j
        T v = T(0);
        if (lane < nb) {
            // v_c = sum_i phi_i K[i][c], lane c walks column c of K (contiguous in Kt)
            T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
            const T *kp = K + lane * ldk;
            int i = 0;
            for (; i + 4 <= nb; i += 4) {
                v0 += phin[i] * kp[i];
                v1 += phin[i + 1] * kp[i + 1];
                v2 += phin[i + 2] * kp[i + 2];
                v3 += phin[i + 3] * kp[i + 3];
            }
            for (; i < nb; ++i) v0 += phin[i] * kp[i];
            v = (v0 + v1) + (v2 + v3);
        }
        const double ratio = (double)__shfl(v, j, 64);
        const double qv = ratio * exp(dj);
        const bool acc = u < qv * qv;
        if (acc) {
            // lane c < nb: column c of K; colj = old column j
            if (lane < nb) {
                colj[lane] = K[j * ldk + lane];   // K[lane][j]
                Aw[(size_t)e * n + lane] = ph;
            }
            if (lane < 3) pos[3 * e + lane] = lane == 0 ? rx : (lane == 1 ? ry : rz);
            wave_sync_s();
            if (lane < nb) {
                const T t = (v - (lane == j ? T(1) : T(0))) * (T)(1.0 / ratio);
                T *kp = K + lane * ldk;
                int i = 0;
                for (; i + 4 <= nb; i += 4) {
                    kp[i] -= colj[i] * t;
                    kp[i + 1] -= colj[i + 1] * t;
                    kp[i + 2] -= colj[i + 2] * t;
                    kp[i + 3] -= colj[i + 3] * t;
                }
                for (; i < nb; ++i) kp[i] -= colj[i] * t;
            }
            wave_sync_s();
            if (fabs(ratio) < FORCED_REFRESH_RATIO) refresh_spin<T>(Aw, n, off, nb, K, ldk, gjs, col, perm, bad);
        }
        if (accept != nullptr && lane == 0) accept[(size_t)e * W + w] = acc ? 1 : 0;
        const uint64_t m = (uint64_t)sweep * (uint64_t)N + (uint64_t)e;
        // the next move of this spin block needs a fresh inverse; a block that
        // has no further move in this sweep is rebuilt at the next sweep anyway
        if (((m + 1) % (uint64_t)refresh_period) == 0 && j < nb - 1)
            refresh_spin<T>(Aw, n, off, nb, K, ldk, gjs, col, perm, bad);
    }
    for (int i = lane; i < 3 * N; i += 64) wp[i] = pos[i];
    if (bad && lane == 0) atomicOr(status, STATUS_SINGULAR);
}

template <typename T>
hipError_t launch_sweep_w(const SysDev &S, const T *C, const double *R, double *walkers, int W, T *Amo,
                          uint32_t sweep, uint64_t seed, double sigma, int refresh_period, uint8_t *accept,
                          int *status, const SweepWLayout &L, hipStream_t st) {
    hipLaunchKernelGGL(k_sweep_w<T>, dim3((unsigned)((W + L.wpb - 1) / L.wpb)), dim3(64 * L.wpb), L.bytes, st, S, C,
                       R, walkers, W, Amo, sweep, seed, sigma, refresh_period, accept, status, L);
    return hipGetLastError();
}

hipError_t configure_sweep(size_t sweep_lds) {
    return hipFuncSetAttribute((const void *)k_sweep_w<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sweep_lds);
}

template hipError_t launch_sweep_w<double>(const SysDev &, const double *, const double *, double *, int, double *,
                                           uint32_t, uint64_t, double, int, uint8_t *, int *, const SweepWLayout &,
                                           hipStream_t);

}  // namespace vmcx
