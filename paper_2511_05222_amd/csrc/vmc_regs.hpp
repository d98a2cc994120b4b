// vmc_regs.hpp -- wavefront register-level helpers (gfx950): lane reads and
// the in-register Gauss-Jordan inversion shared by the sweep and the
// measurement.
#pragma once

#include <hip/hip_runtime.h>

#include "vmc_device.hpp"

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

// Maximum of an unsigned value over the wavefront (uniform result): DPP
// within each row of 16 lanes (quad swaps, half-row and row mirrors), then the
// four row results by lane reads.
__device__ inline unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));    // quad [1,0,3,2]
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));    // quad [2,3,0,1]
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));   // half-row mirror
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));   // row mirror
    const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16),
                   c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

// In-register Gauss-Jordan inversion (FP64) with partial pivoting by implicit
// row choice.  The matrix is B = A^T of the spin block, padded to KN x KN with
// an identity block: on entry lane c holds row c of B in Br[0..KN) (lanes >=
// KN hold zeros and never pivot).  Step k eliminates column k, which a
// rotation keeps in Br[0]: after the step every register moves down by one and
// the new column k enters at Br[KN-1], so after KN steps the registers are
// back in order.  The pivot of step k is an unused lane with the largest
// |B[.][k]| compared on a 32-bit key: |B| rounded to FP32 with its six low
// mantissa bits replaced by (63 - lane), so that values within 2^-17 of each
// other count as equal and the lowest such lane wins (any such pivot is a
// partial-pivoting choice; NaN and 0 rank lowest among the unused lanes).
// The pivot row is broadcast by lane reads.  With p_k the pivot lane of step k the result is
// R[p_k][j] = B^-1[k][p_j], i.e. lane p_k holds column k of K = A^-1 with
// register j holding orbital p_j.  On return sig = k on lane p_k (lanes >= KN:
// sig = lane).  The block counts as singular (bad set) when a pivot is no
// larger than tol (gj_tol below: 2^-40 of the block's largest entry), so a
// row that is a linear combination of the others to working precision, e.g.
// two coincident same-spin electrons, or an all-zero row is reported.  A NaN
// pivot is not: it leaves non-finite results, reported as such.  With LOGDET,
// logabs = sum_k log|pivot_k| = log|det B| (the identity padding adds 0).
template <int KN, bool LOGDET>
__device__ inline void gj_regs(double (&Br)[KN], int &sig, bool &bad, double &logabs, double tol) {
    const int lane = threadIdx.x & 63;
    bool used = lane >= KN;
    sig = lane;
    logabs = 0.0;
    for (int k = 0; k < KN; ++k) {
        const double a0 = Br[0];
        const double fa = fabs(a0);
        unsigned key = 0u;
        if (!used) {
            const unsigned fb = fa == fa ? __float_as_uint((float)fa) : 0u;
            key = max(fb & ~63u, 64u) | (unsigned)(63 - lane);
        }
        const int p = 63 - (int)(wave_max_u32(key) & 63u);
        const bool me = lane == p;
        const double piv = readlane_d(a0, p);
        if (fabs(piv) <= tol) bad = true;
        if (LOGDET) logabs += log(fabs(piv));
        const double inv = rcp_nr(piv);   // a few ulp; a zero pivot is flagged above
        if (me) {
            used = true;
            sig = k;
        }
        // other rows: B[i][j] - (B[i][k] / piv) B[p][j];  pivot row: B[p][j] / piv,
        // formed by the same fma as B[p][j] - (1 - 1/piv) B[p][j] (its own
        // row; relative error |piv - 1| 2^-53 from rounding 1 - 1/piv)
        const double g = me ? 1.0 - inv : a0 * inv;
#pragma unroll
        for (int r = 0; r + 1 < KN; ++r) Br[r] = fma(-g, readlane_d(Br[r + 1], p), Br[r + 1]);
        Br[KN - 1] = me ? inv : -a0 * inv;
    }
}

// Singularity threshold of gj_regs from each lane's largest |entry| of the
// block (padding excluded): 2^-40 of the block's largest entry, i.e. a pivot
// that lost 40 of the 53 significant bits.  The wavefront maximum is taken
// on the high words of the non-negative doubles (monotonic in the value),
// rounded up; NaN entries must be left out by the caller (fmax does).
__device__ inline double gj_tol(double lane_max) {
    const unsigned hi = wave_max_u32((unsigned)__double2hiint(lane_max));
    return __hiloint2double((int)hi, -1) * 0x1p-40;
}

}  // namespace vmcx
