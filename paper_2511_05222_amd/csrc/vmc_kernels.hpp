// vmc_kernels.hpp -- kernel argument structs and launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vmc_device.hpp"

#define VMC_MAX_OCC_K 64

namespace vmcx {

// default threshold of the forced inverse refresh after an accepted move
constexpr double FORCED_REFRESH_RATIO = 1e-8;
constexpr int STATUS_SINGULAR = 1;
constexpr int STATUS_NONFINITE = 2;
constexpr int STATUS_CAPACITY = 4;   // a walker had more pseudopotential pairs than the capacity

struct SysDev {
    int N, n_up, n_dn, n_occ, M, A;
    double ee_a, ee_F;
    int ee_form;   // 0: a r / (1 + F r); 1: a (1 - e^{-F r}) / F
    double forced_ratio;   // an accepted move with |ratio| below it rebuilds the block's inverse
    BasisDev basis;
    const double *Z;
};

struct WalkerOut {
    double *EL, *lnpsi, *lnjac, *dEL_dR, *dlnpsi_dR, *dlnjac_dR, *O, *G;
    // O and G kept in FP32 instead (internal staging of the mixed path)
    float *Of = nullptr, *Gf = nullptr;
};

struct EstArgs {
    const double *EL, *dEdR, *dPdR, *dJdR, *O, *G;
    const double *shift;
    const double *gE, *gP, *gJ;
    int64_t A3, Mn;
    // when set, O and G are read from these FP32 arrays
    const float *Of = nullptr, *Gf = nullptr;
    // per-walker weights |Psi/Psi_G|^2 of the estimator sums (null: all 1)
    const double *wt = nullptr;
};

// blk / blkw: the running block's energy and weight sums (elements 0 and
// n_out - 1); blk_all: its sums of every element (all nullable)
hipError_t launch_reduce(const EstArgs &a, int mode, int64_t n_out, int64_t W, double *partial,
                         int64_t max_seg, double *acc, double *comp, double *blk, double *blkw, double *blk_all,
                         hipStream_t st);
// leave-one-block-out replicas E_jk[nb], F_jk[nb][A3], dC_jk[nb][Mn] (nullable)
// from per-block sums bs[nb][n_est] (the last element of a block's sums is
// its weight sum)
hipError_t launch_jackknife(const double *bs, int nb, int64_t n_est, int64_t A3, int64_t Mn, const double *shift,
                            double *E_jk, double *F_jk, double *dC_jk, hipStream_t st);
hipError_t launch_jackknife_stats(const double *x, int64_t nb, int64_t len, double *mean, double *sigma,
                                  hipStream_t st);
hipError_t launch_set_shift(const double *EL, int64_t W, double *shift, int *shift_set, hipStream_t st);
hipError_t launch_eval_weights(const double *EL, const double *lnpsi, const double *lnjac,
                               const double *lnpsi0, int64_t W, double *wnorm, double *Ehat, hipStream_t st);
hipError_t launch_energy_cotangents(int64_t W, double gE, const double *EL, const double *wnorm,
                                    const double *Ehat, double *gEL, double *gPsi, double *gJac,
                                    hipStream_t st);
hipError_t launch_combine(const double *acc, const double *comp, int64_t n, double *out, hipStream_t st);
// device state of a conjugate-gradient solve
enum { CG_CONVERGED = 1, CG_NONFINITE = 2, CG_MAXIT = 3 };
struct CgState {
    double rz;     // r . (M^-1 r) of the current residual
    double tol2;   // (rtol ||b||)^2
    int maxit;
    int it;        // iterations done
    int done;      // 0 while running, else CG_*
};
int cg_matvec_blocks(int64_t d);   // partial sums the iteration writes
// nrhs right-hand sides, vectors stored one after another (states cs[nrhs])
hipError_t launch_cg_setup(const double *H, const double *b, int64_t d, int nrhs, int jacobi, double rtol,
                           int maxit, double *x, double *r, double *p, double *dinv, CgState *cs, hipStream_t st);
// several right-hand sides (2..64) sharing the reads of H; HPp holds
// cgb_ksplit(d) * nrhs * d doubles of partial products
int cgb_ksplit(int64_t d);
hipError_t launch_cgb_iteration(const double *H, int64_t d, int nrhs, double *X, double *R, double *P, double *HPp,
                                const double *dinv, CgState *cs, hipStream_t st);
hipError_t launch_cg_iteration(const double *H, int64_t d, double *x, double *r, double *p, double *Hp,
                               const double *dinv, double *part, CgState *cs, hipStream_t st);
hipError_t launch_zv_rhs(const double *Cv, const double *G, int64_t M, int64_t nv, int64_t n, int64_t nbat,
                         double *b, hipStream_t st);
hipError_t launch_zv_backmap(const double *Cv, const double *z, int64_t M, int64_t nv, int64_t n, int64_t nbat,
                             double *Z, hipStream_t st);

}  // namespace vmcx
