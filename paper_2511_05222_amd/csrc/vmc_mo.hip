// vmc_mo.hip -- MO rows of every (walker, electron) on the matrix cores.
//
//   out[row][c][i] = sum_mu AO_c(r_row)[mu] C[mu][i],   c < NC
//   (NC = 1: values;  NC = 5: value, gradient, Laplacian)
//
// A block owns 64 rows (one 16-row tile per wavefront) and all n orbitals
// (NT tiles of 16 columns).  C is read from a copy padded to 64 columns and
// 16 extra zero rows (k_pad_c), one 16-byte vector per thread and tile.  The
// AO tile is zeroed once: its AOs past the tile's last one then hold finite
// values of earlier tiles, which meet zero rows of the C tile.  AO tiles of whole shells (<= 16 AOs) are
// produced in LDS by a GTO evaluation that gives each wavefront one shell at
// all 64 rows (uniform angular momentum) and consumed in k-steps of
// 4 AOs by 16x16x4 MFMA (FP64: v_mfma_f64_16x16x4_f64; FP32:
// v_mfma_f32_16x16x4_f32), accumulating in the arithmetic type T.
#include "vmc_mfma.hpp"
#include "vmc_pipeline.hpp"

namespace vmcx {

// Cp[mu][i] = C[mu][i] for mu < M, i < n; zero elsewhere ([M + 16][64]).
template <typename T>
__global__ void k_pad_c(const T *__restrict__ C, int M, int n, T *__restrict__ Cp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (M + 16) * 64) return;
    const int mu = k >> 6, i = k & 63;
    Cp[k] = (mu < M && i < n) ? C[(size_t)mu * n + i] : T(0);
}

// All cartesian components of shell s at one position, evaluated in FP64 and
// rounded once to FP32 (the angular momentum fixed at compile time per
// branch, so that the FP64 values stay in registers).  For the FP32
// measurement rows: components formed in FP32 from FP32 radial sums lose
// digits to cancellation (the Laplacian near its radial nodes), and that
// rounding, second order through the inverse, shifts the walker-averaged
// E_L by several 1e-6 Ha; formed in FP64 and rounded once they leave a few
// 1e-7 Ha.
template <int NC, int L>
__device__ inline void shell_round_l(const BasisDev &B, int mu0, double x, double y, double z, double rho, double R0,
                                     double R1, double R2, double R3, float *dst) {
    double t[(L + 1) * (L + 2) / 2 * NC];
    shell_components<NC, double, L>(B, mu0, x, y, z, rho, R0, R1, R2, R3, t);
#pragma unroll
    for (int i = 0; i < (L + 1) * (L + 2) / 2 * NC; ++i) dst[i] = (float)t[i];
}

template <int NC>
__device__ inline void shell_eval_rounded(const BasisDev &B, const double *R, int s, double rx, double ry, double rz,
                                          float *dst) {
    const int atom = ldc(B.shell_atom + s);
    const double x = rx - ldc(R + 3 * atom), y = ry - ldc(R + 3 * atom + 1), z = rz - ldc(R + 3 * atom + 2);
    const double rho = x * x + y * y + z * z;
    // radial sums in FP64 around the FP32 exponential of the split argument
    // (its relative error, ~1e-7, is the one the FP32 path has; the
    // derivative combinations below are where FP32 would lose digits)
    double R0 = 0.0, R1 = 0.0, R2 = 0.0, R3 = 0.0;
    const int p0 = ldc(B.shell_p0 + s), np = ldc(B.shell_np + s);
    for (int k = 0; k < np; ++k) {
        const double al = ldc(B.prim_exp + p0 + k);
        const double e = ldc(B.prim_cp + p0 + k) * (double)exp_neg(al, rho, 0.0f);
        R0 += e;
        R1 -= al * e;
        R2 += al * al * e;
    }
    const int l = ldc(B.shell_l + s), mu0 = ldc(B.shell_mu0 + s);
    if (l == 0)
        shell_round_l<NC, 0>(B, mu0, x, y, z, rho, R0, R1, R2, R3, dst);
    else if (l == 1)
        shell_round_l<NC, 1>(B, mu0, x, y, z, rho, R0, R1, R2, R3, dst);
    else
        shell_round_l<NC, 2>(B, mu0, x, y, z, rho, R0, R1, R2, R3, dst);
}

template <typename T, int NC, int NT>
__global__ __launch_bounds__(256) void k_mo_rows_mfma(SysDev S, const T *__restrict__ Cp, const double *__restrict__ R,
                                                      const double *__restrict__ pos, int64_t n_rows, AoTiles tiles,
                                                      T *__restrict__ out, const int *__restrict__ rows_dev) {
    constexpr int RB = 64, MT = 16;
    constexpr int RS = MT * NC + 1;    // odd row stride of the AO tile
    constexpr int CS = 80;             // row stride of the C tile (lane groups hit disjoint banks)
    __shared__ double sp[RB * 3];
    __shared__ T aot[RB * RS];
    __shared__ T ct[MT * CS];
    typedef Mfma<T> MF;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = S.n_occ;
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    // (a row count known only on the device: the blocks past it leave)
    if (rows_dev) n_rows = min(n_rows, (int64_t)*rows_dev);
    if (row0 >= n_rows) return;
    for (int k = tid; k < RB * 3; k += 256) sp[k] = (row0 + k / 3) < n_rows ? pos[row0 * 3 + k] : 0.0;
    for (int k = tid; k < RB * RS; k += 256) aot[k] = T(0);
    typename MF::acc_t acc[NC][NT];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[c][t] = MF::zero();
    const int ar = wave * 16 + (lane & 15);   // A-operand row of this lane
    const int ak = lane >> 4;                 // A-operand k (AO within the k-step)
    for (int tile = 0; tile < tiles.n_tiles; ++tile) {
        const int s0 = tiles.s0[tile], s1 = tiles.s1[tile], mu0 = tiles.mu0[tile], mu1 = tiles.mu1[tile];
        const int nsh = s1 - s0, nmu = mu1 - mu0;
        __syncthreads();
        // shell-major: a wavefront evaluates one shell at its 64 rows, so the
        // angular momentum (and the shell's tables) are uniform over it
        for (int p = tid; p < RB * nsh; p += 256) {
            // p / RB is the same in every lane of a wavefront: scalar tables
            const int s = __builtin_amdgcn_readfirstlane(s0 + p / RB), r = p % RB;
            T *dst = aot + r * RS + (ldc(S.basis.shell_mu0 + s) - mu0) * NC;
            if constexpr (sizeof(T) == 4 && NC == 5) {
                // FP32 measurement rows: the AO components in FP64, rounded once
                shell_eval_rounded<NC>(S.basis, R, s, sp[3 * r], sp[3 * r + 1], sp[3 * r + 2], dst);
            } else {
                shell_eval_to<NC, T>(S.basis, R, s, sp[3 * r], sp[3 * r + 1], sp[3 * r + 2], dst);
            }
        }
        // C tile: rows of the tile's AOs, zero rows past its last AO
        constexpr int VW = 16 / sizeof(T);
        typedef T V __attribute__((ext_vector_type(VW)));
        for (int p = tid; p < MT * 64 / VW; p += 256) {
            const int m = p / (64 / VW), i = (p - m * (64 / VW)) * VW;
            const V v = *(const V *)(Cp + (size_t)(mu0 + m) * 64 + i);
            *(V *)(ct + m * CS + i) = m < nmu ? v : V(T(0));
        }
        __syncthreads();
        const int ksteps = (nmu + 3) >> 2;
        for (int ks = 0; ks < ksteps; ++ks) {
            const int m = ks * 4 + ak;
            T a[NC], b[NT];
#pragma unroll
            for (int c = 0; c < NC; ++c) a[c] = aot[ar * RS + m * NC + c];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = ct[m * CS + t * 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[c][t] = MF::fma(a[c], b[t], acc[c][t]);
        }
    }
    const int col = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wave * 16 + MF::row(lane, v);
        if (row >= n_rows) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int i = t * 16 + col;
                if (i < n) out[(row * NC + c) * n + i] = acc[c][t][v];
            }
    }
}

template <typename T, int NC>
static hipError_t launch_nc(const SysDev &S, const T *C, const double *R, const double *pos, int64_t n_rows,
                            const AoTiles &tiles, T *out, const int *rows_dev, hipStream_t st) {
    // (C here is the padded copy)
    const dim3 g((unsigned)((n_rows + 63) / 64));
    const int nt = (S.n_occ + 15) / 16;
    if (nt == 1)
        hipLaunchKernelGGL((k_mo_rows_mfma<T, NC, 1>), g, dim3(256), 0, st, S, C, R, pos, n_rows, tiles, out,
                           rows_dev);
    else if (nt == 2)
        hipLaunchKernelGGL((k_mo_rows_mfma<T, NC, 2>), g, dim3(256), 0, st, S, C, R, pos, n_rows, tiles, out,
                           rows_dev);
    else if (nt == 3)
        hipLaunchKernelGGL((k_mo_rows_mfma<T, NC, 3>), g, dim3(256), 0, st, S, C, R, pos, n_rows, tiles, out,
                           rows_dev);
    else
        hipLaunchKernelGGL((k_mo_rows_mfma<T, NC, 4>), g, dim3(256), 0, st, S, C, R, pos, n_rows, tiles, out,
                           rows_dev);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mo_rows_mfma(const SysDev &S, const T *C, const double *R, const double *pos, int64_t n_rows,
                               const AoTiles &tiles16, T *out, int nc, T *cpad, hipStream_t st,
                               const int *rows_dev) {
    if (S.n_occ > 64) return hipErrorInvalidValue;
    const int np = (S.M + 16) * 64;
    hipLaunchKernelGGL(k_pad_c<T>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, C, S.M, S.n_occ, cpad);
    return nc == 1 ? launch_nc<T, 1>(S, cpad, R, pos, n_rows, tiles16, out, rows_dev, st)
                   : launch_nc<T, 5>(S, cpad, R, pos, n_rows, tiles16, out, rows_dev, st);
}

template hipError_t launch_mo_rows_mfma<double>(const SysDev &, const double *, const double *, const double *,
                                                int64_t, const AoTiles &, double *, int, double *, hipStream_t,
                                                const int *);

template hipError_t launch_mo_rows_mfma<float>(const SysDev &, const float *, const double *, const double *,
                                               int64_t, const AoTiles &, float *, int, float *, hipStream_t,
                                               const int *);

}  // namespace vmcx
