// vmc_kernels.hpp -- kernel argument structs and launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vmc_device.hpp"

#define VMC_MAX_OCC_K 64

namespace vmcx {

constexpr double FORCED_REFRESH_RATIO = 1e-8;
constexpr int STATUS_SINGULAR = 1;
constexpr int STATUS_NONFINITE = 2;

struct SysDev {
    int N, n_up, n_dn, n_occ, M, A;
    double ee_a, ee_F;
    BasisDev basis;
    const double *Z;
};

struct WalkerOut {
    double *EL, *lnpsi, *lnjac, *dEL_dR, *dlnpsi_dR, *dlnjac_dR, *O, *G;
};

struct EstArgs {
    const double *EL, *dEdR, *dPdR, *dJdR, *O, *G;
    const double *shift;
    const double *gE, *gP, *gJ;
    int64_t A3, Mn;
};

hipError_t launch_reduce(const EstArgs &a, int mode, int64_t n_out, int64_t W, double *partial,
                         int64_t max_seg, double *acc, double *comp, double *blk, hipStream_t st);
hipError_t launch_set_shift(const double *EL, int64_t W, double *shift, int *shift_set, hipStream_t st);
hipError_t launch_eval_weights(const double *EL, const double *lnpsi, const double *lnjac,
                               const double *lnpsi0, int64_t W, double *wnorm, double *Ehat, hipStream_t st);
hipError_t launch_energy_cotangents(int64_t W, double gE, const double *EL, const double *wnorm,
                                    const double *Ehat, double *gEL, double *gPsi, double *gJac,
                                    hipStream_t st);
hipError_t launch_combine(const double *acc, const double *comp, int64_t n, double *out, hipStream_t st);
hipError_t launch_matvec(const double *H, const double *x, double *y, int64_t d, hipStream_t st);
hipError_t launch_dot(const double *a, const double *b, int64_t d, double *part, int n_part, double *out,
                      hipStream_t st);
hipError_t launch_cg_init(double *x, double *r, double *p, const double *b, int64_t d, hipStream_t st);
hipError_t launch_cg_update_xr(double *x, double *r, const double *p, const double *Hp, int64_t d,
                               const double *rr, const double *pHp, hipStream_t st);
hipError_t launch_cg_update_p(double *p, const double *r, int64_t d, const double *rr_new, const double *rr,
                              hipStream_t st);

}  // namespace vmcx
