// vmc_regs.hpp -- wavefront register-level helpers (gfx950): lane reads and
// the in-register Gauss-Jordan inversion shared by the sweep and the
// measurement.
#pragma once

#include <hip/hip_runtime.h>

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

__device__ inline float readlane_t(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double readlane_t(double v, int src) { return readlane_d(v, src); }

// In-register Gauss-Jordan inversion (FP64) with partial pivoting by implicit
// row choice.  The matrix is B = A^T of the spin block, padded to KN x KN with
// an identity block: on entry lane c holds row c of B in Br[0..KN) (lanes >=
// KN hold zeros and never pivot).  Step k eliminates column k, which a
// rotation keeps in Br[0]: after the step every register moves down by one and
// the new column k enters at Br[KN-1], so after KN steps the registers are
// back in order.  The pivot of step k is the unused lane with the largest
// |B[.][k]| (ties: lowest lane).  With p_k the pivot lane of step k the result
// is R[p_k][j] = B^-1[k][p_j], i.e. lane p_k holds column k of K = A^-1 with
// register j holding orbital p_j.  On return sig = k on lane p_k (lanes >= KN:
// sig = lane).  A pivot with |pivot| <= 1e-300 or NaN sets bad.  With LOGDET,
// logabs = sum_k log|pivot_k| = log|det B| (the identity padding adds 0).
template <int KN, bool LOGDET>
__device__ inline void gj_regs(double (&Br)[KN], int &sig, bool &bad, double &logabs) {
    const int lane = threadIdx.x & 63;
    bool used = lane >= KN;
    sig = lane;
    logabs = 0.0;
    for (int k = 0; k < KN; ++k) {
        const double a0 = Br[0];
        const double fa = fabs(a0);
        double best = used ? -1.0 : (fa == fa ? fa : -0.5);
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
        const int p = __builtin_amdgcn_readfirstlane(bi);
        const double piv = readlane_d(a0, p);
        if (!(fabs(piv) > 1e-300)) bad = true;
        if (LOGDET) logabs += log(fabs(piv));
        const double inv = 1.0 / piv;
        const bool me = lane == p;
        if (me) {
            used = true;
            sig = k;
        }
        // pivot row: B[p][j] / piv;  other rows: B[i][j] - (B[i][k] / piv) B[p][j]
        const double g = me ? -inv : a0 * inv;
        const double h = me ? 0.0 : 1.0;
#pragma unroll
        for (int r = 0; r + 1 < KN; ++r) {
            const double pr = readlane_d(Br[r + 1], p);
            Br[r] = fma(-g, pr, h * Br[r + 1]);
        }
        Br[KN - 1] = me ? inv : -a0 * inv;
    }
}

}  // namespace vmcx
