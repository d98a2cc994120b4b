/*
 * vmc.h -- C ABI of the MI355X VMC force hot path.
 *
 * The library evaluates, for a Jastrow-correlated Slater determinant in a
 * cartesian Gaussian-type-orbital basis (Nakano, Battaglia, Hutter,
 * arXiv:2511.05222, Appendix A "Wavefunction Ansatz"), the quantities whose
 * Monte Carlo averages give
 *   E      = <E_L>                               (Appendix A, eq. eval-observable)
 *   F_bare = Hellmann-Feynman + Pulay force with the space-warp transformation
 *            (Appendix A, "Computing derivatives"; Sec. I, eqs. hf and pulay)
 *   dE/dC  = 2 (<E_L O> - <E_L><O>),  O = d ln|Psi| / dC
 *            (eq. fc-vmc-eval; B = dE/dC is the right-hand side of the
 *            Z-vector equations, eq. AZ_eq_B_elements)
 * and, optionally, solves H z = -b for a caller-supplied SPD orbital Hessian
 * (Z-vector equations, Sec. II).
 *
 * Conventions
 *   - All floating point arguments are IEEE double.  Lengths in bohr, energies
 *     in hartree, forces in hartree/bohr.
 *   - "host" pointers are read during the call only; "device" pointers are
 *     device memory of the context's GPU, owned by the caller, and must stay
 *     valid until the work queued on `stream` has completed.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call queues
 *     its kernels on that stream and returns without synchronising, except
 *     vmc_accumulate, vmc_jackknife and zvector_solve, which synchronise it.
 *   - Every function returns VMC_OK (0) or a negative status; none aborts,
 *     throws or prints.  vmc_last_error(ctx) gives a human-readable detail.
 *   - A context is not thread-safe; distinct contexts are independent.
 *
 * Wavefunction (Appendix A):
 *   psi_mu(r) = eta(a,b,c) x^a y^b z^c sum_k c'_k exp(-alpha_k |r-R_A|^2),
 *     cartesian components, order s; x,y,z; xx,xy,xz,yy,yz,zz; contraction
 *     coefficients multiply unit-normalised primitives and each cartesian
 *     component is renormalised to unit norm (the library folds all norms).
 *   phi_i = sum_mu C[mu][i] psi_mu                  (eq. restricted-C)
 *   Psi   = det[phi_i(r_e)]_up * det[phi_i(r_e)]_dn * exp(sum_{i<j} u(r_ij)),
 *           u(r) = a r / (1 + F r)                  (eqs. twobody_jastrow, twobody_v)
 *   electrons 0..n_up-1 are spin up, n_up..N-1 spin down.
 */
#ifndef VMC_H
#define VMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define VMC_OK           0
#define VMC_EINVAL      -1   /* invalid argument or unsupported size            */
#define VMC_ENOMEM      -2   /* device or host allocation failed                */
#define VMC_EDEVICE     -3   /* HIP runtime error                               */
#define VMC_ESINGULAR   -4   /* a Slater block singular to working precision    */
#define VMC_ENOTCONV    -5   /* iterative solver hit maxit                      */
#define VMC_ENONFINITE  -6   /* non-finite value in an input or a result        */
#define VMC_ECAPACITY   -7   /* a per-walker capacity was exceeded              */

/* ---- precision modes ------------------------------------------------------ */
#define VMC_FP64   0         /* every step in FP64                              */
#define VMC_MIXED  1         /* FP32 AO values (the measurement's value,
                                gradient and Laplacian components formed in
                                FP64 around an FP32 exponential and rounded
                                once), MO products on FP32 MFMA, FP32
                                Sherman-Morrison, acceptance ratio (its
                                Jastrow difference included) and
                                back-projection; FP64 inverse refresh,
                                determinants, E_L assembly with its Jastrow
                                terms and every sum over walkers              */

/* ---- flags ---------------------------------------------------------------- */
#define VMC_SWEEP_MEASURE   1u   /* measure + accumulate after every sweep      */
#define VMC_ACCUM_RESET     1u   /* clear the accumulators after reading them   */

/* ---- limits (compile-time sizes of the kernels) --------------------------- */
#define VMC_MAX_OCC      64      /* max orbitals per spin                        */
#define VMC_MAX_ELEC    128      /* max electrons                                */
#define VMC_MAX_AO     1024      /* max atomic orbitals                          */
#define VMC_MAX_ATOMS    64      /* max nuclei                                   */
#define VMC_MAX_L         2      /* max shell angular momentum (d)               */

typedef struct vmc_ctx vmc_ctx;

/* Basis set (host arrays, all of length n_shells unless noted).
 * shell_atom[s] : index of the nucleus the shell sits on
 * shell_l[s]    : angular momentum, 0..VMC_MAX_L
 * shell_nprim[s]: primitives of shell s; they occupy prim_exp/prim_coef
 *                 [sum_{t<s} shell_nprim[t], ... + shell_nprim[s])
 * prim_exp      : exponents alpha_k > 0 (length sum shell_nprim)
 * prim_coef     : contraction coefficients of unit-normalised primitives     */
typedef struct {
    int32_t n_shells;
    const int32_t *shell_atom;
    const int32_t *shell_l;
    const int32_t *shell_nprim;
    const double  *prim_exp;
    const double  *prim_coef;
} vmc_basis;

/* Nuclei (host): xyz[A][3] bohr, Z[A] charges. */
typedef struct {
    int32_t n_atoms;
    const double *xyz;
    const double *Z;
} vmc_nuclei;

/* Occupied MO coefficients (host): C[n_ao][n_occ] row-major, restricted
 * (both spins use the same C).  n_up == n_dn == n_occ is required.          */
typedef struct {
    int32_t n_ao;
    int32_t n_occ;
    int32_t n_up;
    int32_t n_dn;
    const double *C;
} vmc_mo;

/* Jastrow factor, spin independent (Appendix A, "Wavefunction Ansatz"),
 * J = exp(U), U = sum_{i<j} u(r_ij) + U1 + U3:
 * two-body term
 *   ee_form = VMC_JASTROW_PADE: u(r) = ee_a r / (1 + ee_F r)      (eq. twobody_v)
 *   ee_form = VMC_JASTROW_EXP : u(r) = ee_a (1 - exp(-ee_F r)) / ee_F
 *                                                         (eq. twobody_v_exp)
 * (the paper's forms have ee_a = 1/2, the electron-electron cusp; the
 * exponential form needs ee_F > 0);
 * optional one-body and three/four-body terms on a Jastrow GTO basis chi_mu
 * (jas_basis, same conventions and limits as the determinant's basis, at
 * most VMC_MAX_JAS cartesian functions, each atom of jas_basis->shell_atom
 * an index into the nuclei):
 *   U1 = sum_i sum_mu xi1[mu] chi_mu(r_i)                (eq. onebody_J_inhom)
 *   U3 = sum_{i<j} sum_{mu,nu} xi3[mu][nu] chi_mu(r_i) chi_nu(r_j)
 *                                                        (eq. threebody_jas)
 * xi1[M_J], xi3[M_J][M_J] row-major and exactly symmetric (host arrays,
 * copied; NULL = zero); all atom pairs may be coupled (four-body elements).
 * jas_basis = NULL: two-body term only. */
#define VMC_JASTROW_PADE 0
#define VMC_JASTROW_EXP  1
#define VMC_MAX_JAS    256       /* max Jastrow basis functions                  */
typedef struct {
    double ee_a;
    double ee_F;
    int32_t ee_form;
    const vmc_basis *jas_basis;
    const double *xi1;
    const double *xi3;
} vmc_jastrow;

/* Semilocal pseudopotential (the paper's VMC uses ccECP pseudopotentials,
 * Sec. III and Sec. IV "computational details"; the paper does not restate
 * their form, so the standard semilocal one is taken: Mitas, Shirley and
 * Ceperley, J. Chem. Phys. 95, 3467 (1991)).  On nucleus a, for an electron
 * at distance d = |r_i - R_a| with direction u_i:
 *   V_loc(d) + sum_l V_l(d) sum_m |l m><l m|,
 *   V(d) = sum_t term_coef[t] d^(term_n[t] - 2) exp(-term_exp[t] d^2)
 * over the terms t of the channel (term_l[t] = -1: the local part; 0 ..
 * VMC_MAX_ECP_L: the projector on l).  The projectors enter E_L as
 *   sum_l V_l(d) (2l + 1) sum_q (1/12) P_l(u_i . v_q) Psi(.., R_a + d v_q, ..) / Psi
 * over the 12 vertices v_q of an icosahedron, turned by one random rotation
 * per (walker, electron): Shoemake's unit quaternion from the first three
 * 32-bit words (u = w 2^-32) of Philox4x32-10 with key rot_seed and counter
 * (walker id, rotation index, electron | 2 << 16, 0); the rotation index is
 * the sweep index for the measurement after each sweep of vmc_sweep and 0
 * for every other call; the walker id is the row of the positions passed.
 * Only electrons with d < rcut[a] see the projectors of nucleus a; the local
 * part acts at every distance.  The charges of vmc_nuclei are the effective
 * ones (the removed core's charge subtracted).
 * term_n in 1..4, term_exp > 0; rcut[n_atoms] >= 0 (host arrays, copied).
 * max_pairs: (electron, nucleus) pairs inside the cutoffs a measurement
 * launch holds, per walker of the launch (the pairs of a launch's walkers are
 * packed together, so it bounds their average; 0 = N times the number of
 * nuclei with a projector, which cannot overflow; smaller values allow more
 * walkers per launch); a launch with more pairs drops those past the
 * capacity and reports VMC_ECAPACITY at vmc_accumulate.  Not combined with
 * the one-/three-body Jastrow terms. */
#define VMC_MAX_ECP_L      3
#define VMC_MAX_ECP_TERMS  256
typedef struct {
    int32_t n_terms;
    const int32_t *term_atom;
    const int32_t *term_l;
    const int32_t *term_n;
    const double  *term_exp;
    const double  *term_coef;
    const double  *rcut;
    uint64_t rot_seed;
    int32_t max_pairs;
} vmc_ecp;

/* Run options.
 * precision      : VMC_FP64 or VMC_MIXED
 * refresh_period : each spin block's inverse (kept in device memory between
 *                  its blocks of moves and between sweeps) is rebuilt from
 *                  scratch (FP64 Gauss-Jordan, partial pivoting) from the
 *                  walker's MO matrix after every refresh_period-th proposed
 *                  move of that block's electrons (block move index
 *                  sweep * n_occ + j for its j-th electron), at the start of
 *                  every vmc_sweep call, and after an accepted move of the
 *                  block with |ratio| < forced_refresh_ratio; Sherman-Morrison
 *                  updates in between
 * block_sweeps   : sweeps per block of the blocked energy error bar
 * max_walkers    : largest n_walkers any call on this context will pass
 * staging_walkers: most walkers measured per launch (per-walker staging
 *                  buffers); 0 = as many as fit in 16 GiB of staging.  A
 *                  call on n walkers measures them in the fewest launches
 *                  of at most this many, of equal size (up to one walker)
 * step_sigma     : proposal r' = r + step_sigma * N(0, I_3)
 * promote_fraction: VMC_MIXED only, in [0, 1]: the share of each measurement
 *                  launch's walkers that is measured again in FP64, its FP64
 *                  results replacing the mixed ones (ceil(fraction * walkers)
 *                  walkers; 0 disables).  The walkers taken are those with
 *                  the largest max|Abar| (ties to the lower index), where
 *                  Abar = (K X K)^T / 2 is formed per spin block in FP64
 *                  (K = A^-1 from the FP32 orbital values; X[e][i] =
 *                  lap phi_i(r_e) + 2 grad J . grad phi_i(r_e)): the
 *                  sensitivity of E_L to errors in the orbital values, so
 *                  the walkers whose FP32 rounding would dominate the
 *                  walker-averaged error.  Non-finite keys rank first.
 * jackknife_blocks: number of blocks (of block_sweeps sweeps) whose sums of
 *                  every estimator element are kept for vmc_jackknife
 *                  (at most 65535; 0 = none; (2 + 9A + 3 M n_occ) doubles of
 *                  device memory per block).
 * forced_refresh_ratio: an accepted move whose determinant ratio has
 *                  |ratio| below this value rebuilds its block's inverse
 *                  before the block's next move (the Sherman-Morrison update
 *                  divides by the ratio); 0 selects the default 1e-8, larger
 *                  values force more rebuilds (>= 0, finite).
 * ecp            : a semilocal pseudopotential in E_L (NULL = none; see
 *                  vmc_ecp).
 * jastrow_gradient: with the one-/three-body Jastrow terms, nonzero adds to
 *                  every accumulated batch the sums that vmc_jastrow_gradient
 *                  reads (their cost grows as M_J^2 N per walker). */
typedef struct {
    int32_t precision;
    int32_t refresh_period;
    int32_t block_sweeps;
    int32_t max_walkers;
    int32_t staging_walkers;
    double  step_sigma;
    double  promote_fraction;
    int32_t jackknife_blocks;
    double  forced_refresh_ratio;
    const vmc_ecp *ecp;
    int32_t jastrow_gradient;
} vmc_options;

/* Per-walker outputs of one measurement (device arrays, any may be NULL).
 * EL[W], lnpsi[W] (ln|Psi|), lnjac[W] (ln of the warp Jacobian),
 * dEL_dR[W][A][3], dlnpsi_dR[W][A][3], dlnjac_dR[W][A][3]: derivatives with
 *   respect to the nuclei of E_L, ln|Psi| and ln Jac of the warped
 *   configuration (space-warp transformation, Appendix A, kappa = d^-4);
 * O[W][n_ao][n_occ] = d ln|Psi| / dC, G[W][n_ao][n_occ] = d E_L / dC.        */
typedef struct {
    double *EL;
    double *lnpsi;
    double *lnjac;
    double *dEL_dR;
    double *dlnpsi_dR;
    double *dlnjac_dR;
    double *O;
    double *G;
} vmc_walker_out;

/* Create a context on HIP device `device` for the Jastrow-Slater wavefunction
 * of Appendix A, "Wavefunction Ansatz": the determinant part expanded over
 * the occupied MOs of the frozen coefficients C (eq. agp_expansion with
 * p = N/2 MOs, i.e. eq. restricted-C), the two-body Jastrow of eqs.
 * twobody_jastrow / twobody_v / twobody_v_exp.  Validates and deep-copies the
 * host inputs (the caller may free them on return), folds the GTO
 * normalisation, and allocates device state for opt->max_walkers walkers.
 * Errors: VMC_EINVAL (l > 2, alpha <= 0, non-finite input, n_up != n_dn,
 * n_occ != n_up, sizes beyond the VMC_MAX_* limits), VMC_ENOMEM, VMC_EDEVICE. */
int vmc_init(const vmc_basis *basis, const vmc_nuclei *nuclei, const vmc_mo *mo,
             const vmc_jastrow *jastrow, const vmc_options *opt, int32_t device,
             vmc_ctx **out);

/* Advance n_walkers independent Markov chains by nsteps sweeps (Appendix A,
 * "Variational Monte Carlo Methods": MCMC sampling of |Psi|^2).
 * walkers_dev  : device [n_walkers][N][3] positions, updated in place.
 * A sweep proposes r'_e = r_e + step_sigma z for e = 0..N-1 in order and
 * accepts iff u < |Psi'/Psi|^2; z and u come from Philox4x32-10 with key
 * `seed` and counter (walker id, sweep index, electron | purpose << 16, 0),
 * sweep index = sweep_offset + t, walker id = row of walkers_dev.  The MO
 * matrix of every walker is built from walkers_dev at the start of the call
 * and kept current by the moves (row e rewritten on each accepted move).
 * flags & VMC_SWEEP_MEASURE: after every sweep measure every walker and add
 *   the samples to the context's accumulators (read by vmc_accumulate) and,
 *   with jackknife_blocks > 0, to the running block's sums (vmc_jackknife).
 * accept_dev   : optional device uint8 [nsteps][N][n_walkers], 1 = accepted.
 * Errors: VMC_EINVAL (n_walkers > max_walkers or < 1, nsteps < 0),
 * VMC_EDEVICE. */
int vmc_sweep(vmc_ctx *ctx, double *walkers_dev, int64_t n_walkers, int32_t nsteps,
              uint64_t seed, uint64_t sweep_offset, uint32_t flags, uint8_t *accept_dev,
              void *stream);

/* Read the estimators accumulated since the last reset (host outputs):
 *   E[0] = <E_L>, E[1] = blocked error bar (NaN with < 2 blocks),
 *   F_bare[A][3], dE_dC[n_ao][n_occ] (covariance form, eq. fc-vmc-eval with
 *   B = dE/dC), dEL_dC_mean[n_ao][n_occ] = <dE_L/dC> (may be NULL),
 *   n_samples (may be NULL).
 * All sums are FP64, shifted by the mean E_L of the first measured batch and
 * compensated (Neumaier); every sample carries its weight (1 for the sweeps'
 * own measurements, see vmc_accumulate_walkers) and the averages divide by
 * the sum of the weights.  Synchronises `stream`.
 * flags & VMC_ACCUM_RESET clears the accumulators afterwards.
 * Errors: VMC_EINVAL (no samples); VMC_ESINGULAR if, since the last reset,
 * an inverse rebuild of the sweeps or of a measurement met a Slater block
 * that is singular to working precision (a pivot of at most 2^-40 times the
 * block's largest orbital value: e.g. two same-spin electrons at one point,
 * or an electron where every orbital vanishes); otherwise
 * VMC_ENONFINITE if a measured E_L, ln|Psi| or log|det| was not finite (e.g.
 * a walker with a NaN coordinate); otherwise VMC_ECAPACITY if a measurement
 * launch had more pseudopotential pairs than its capacity (vmc_ecp.max_pairs;
 * the pairs beyond it were left out).  On these errors the outputs are
 * still written (they include the offending samples) and VMC_ACCUM_RESET
 * still clears the accumulators and the error state. */
int vmc_accumulate(vmc_ctx *ctx, double *E, double *F_bare, double *dE_dC,
                   double *dEL_dC_mean, int64_t *n_samples, uint32_t flags, void *stream);

/* Gradient of the energy in the one- and three/four-body Jastrow parameters
 * over the samples accumulated since the last reset (the covariance form of
 * eq. fc-vmc-eval applied to the Jastrow parameters of App. A, eqs.
 * onebody_J_inhom and threebody_jas; the gradient the paper's stochastic
 * reconfiguration of the Jastrow works with):
 *   dE/dxi = 2 (<E_L O_xi> - <E_L><O_xi>),  O_xi = dln|Psi|/dxi,
 *   O_xi1 = sum_i chi(r_i),  O_xi3 = (s s^T - sum_i chi(r_i) chi(r_i)^T) / 2
 * (s = sum_i chi(r_i); xi3 as a symmetric matrix: for a symmetric change D
 * the energy changes by sum_{mu,nu} dE_dxi3[mu][nu] D[mu][nu]), with the
 * weights and shifted FP64 sums of vmc_accumulate.  Host outputs
 * dE_dxi1[M_J], dE_dxi3[M_J][M_J]; read before vmc_accumulate resets.
 * Synchronises `stream`.
 * Errors: VMC_EINVAL (no one-/three-body terms, options.jastrow_gradient
 * off, or no samples), VMC_EDEVICE. */
int vmc_jastrow_gradient(vmc_ctx *ctx, double *dE_dxi1, double *dE_dxi3, void *stream);

/* Measure n_walkers given configurations (device [n_walkers][N][3]) at the
 * context's MO coefficients and nuclei and add them to the accumulators as
 * one measured batch (one sweep of the blocking), each with the weight
 * weights_dev[k] (device [n_walkers], NULL = all 1): the reweighting of
 * Appendix A (reweighting equation), <O> = <O W> / <W> with
 * W = |Psi / Psi_G|^2 for configurations drawn from a guiding distribution
 * Psi_G^2 (the paper names the Attaccalite-Sorella guiding function without
 * defining it, so the weights are the caller's; samples of Psi^2 itself have
 * W = 1).  vmc_accumulate then normalises every sum by the sum of the
 * weights and forms the blocked error bar from weighted block means;
 * vmc_jackknife likewise.  Weights must be finite and >= 0 with a positive
 * sum (else vmc_accumulate returns VMC_EINVAL).  Queued on `stream`.
 * Errors: VMC_EINVAL (NULL walkers, n_walkers < 1 or > max_walkers),
 * VMC_EDEVICE. */
int vmc_accumulate_walkers(vmc_ctx *ctx, const double *walkers_dev, int64_t n_walkers, const double *weights_dev,
                           void *stream);

/* Jackknife replicas of the estimators (Sec. II: the statistical error of B
 * carried through the Z-vector equations by resampling; App. A blocking):
 * for each of the nb complete blocks accumulated since the last reset (at
 * most jackknife_blocks), the estimate from all other blocks,
 *   E_jk_dev[nb]                 E^(-b)
 *   F_jk_dev[nb][n_atoms][3]     F_bare^(-b)
 *   dEdC_jk_dev[nb][n_ao][n_occ] dE/dC^(-b)
 * (device, caller-owned, any may be NULL; all NULL = only report nb).  The
 * jackknife mean and error of any quantity computed from the replicas follow
 * from zvector_jackknife.  *n_blocks (host, may be NULL) = nb.  Call before
 * the vmc_accumulate that resets.  Synchronises `stream`.
 * Errors: VMC_EINVAL (jackknife_blocks = 0, or fewer than two complete
 * blocks when an output is requested), VMC_EDEVICE. */
int vmc_jackknife(vmc_ctx *ctx, double *E_jk_dev, double *F_jk_dev, double *dEdC_jk_dev, int64_t *n_blocks,
                  void *stream);

/* Per-walker measurement at fixed configurations for arbitrary MO
 * coefficients C_dev[n_ao][n_occ] and nuclei R_dev[A][3] (device): electrons
 * are warped r' = r + sum_a omega_a(r; R0) (R_a - R0_a) with weights taken at
 * the sampling geometry R0_dev[A][3].  Fills the non-NULL fields of *out. */
int vmc_measure(vmc_ctx *ctx, const double *walkers_dev, int64_t n_walkers,
                const double *C_dev, const double *R_dev, const double *R0_dev,
                const vmc_walker_out *out, void *stream);

/* Forward of the fixed-sample reweighted energy (reweighting, Appendix A):
 *   E_hat = sum_k w_k E_L,k / sum_k w_k,
 *   w_k = exp(2 (ln|Psi_k| - lnpsi0_dev[k])) * Jac_k,
 * evaluated with vmc_measure's conventions.  Outputs (device): EL[W],
 * lnpsi[W], lnjac[W], wnorm[W] = w_k / sum w, Ehat[1]. */
int vmc_eval(vmc_ctx *ctx, const double *walkers_dev, int64_t n_walkers,
             const double *C_dev, const double *R_dev, const double *R0_dev,
             const double *lnpsi0_dev, double *EL_dev, double *lnpsi_dev, double *lnjac_dev,
             double *wnorm_dev, double *Ehat_dev, void *stream);

/* Cotangents of E_hat with respect to the per-walker (E_L, ln|Psi|, ln Jac),
 * scaled by the upstream gradient gE (host scalar):
 *   gEL[k] = gE w_k,  gPsi[k] = 2 gE w_k (E_L,k - E_hat),
 *   gJac[k] = gE w_k (E_L,k - E_hat),   w = wnorm (device arrays). */
int vmc_energy_cotangents(vmc_ctx *ctx, int64_t n_walkers, double gE, const double *EL_dev,
                          const double *wnorm_dev, const double *Ehat_dev, double *gEL_dev,
                          double *gPsi_dev, double *gJac_dev, void *stream);

/* Vector-Jacobian product of the per-walker map (C, R) -> (E_L, ln|Psi|, ln Jac)
 * (the derivatives the paper takes by algorithmic differentiation, Appendix A
 * "Computing derivatives": the dE_L/dC and O = dln|Psi|/dC of eq.
 * fc-vmc-eval, and the space-warp force terms) with per-walker cotangents
 * gEL, gPsi, gJac (device [W]):
 *   dC_dev[n_ao][n_occ] = sum_k gEL_k dE_L,k/dC + gPsi_k dln|Psi_k|/dC
 *   dR_dev[A][3]        = sum_k gEL_k dE_L,k/dR + gPsi_k dln|Psi_k|/dR + gJac_k dlnJac_k/dR
 * (hand-written reverse mode; forward intermediates are recomputed, not
 * stored).  Outputs are overwritten. */
int vmc_adjoint(vmc_ctx *ctx, const double *walkers_dev, int64_t n_walkers,
                const double *C_dev, const double *R_dev, const double *R0_dev,
                const double *gEL_dev, const double *gPsi_dev, const double *gJac_dev,
                double *dC_dev, double *dR_dev, void *stream);

/* ---- Z-vector step (Sec. II, eq. AZ_eq_B_elements: A Z = -B) ----------------
 * The orbital rotation z lives in the virtual-occupied block: z[a][i], a over
 * the n_virt virtual orbitals, i over the n_occ occupied ones, flattened
 * row-major to d = n_virt * n_occ.  The orbital Hessian H over that index is
 * the caller's (its CPKS integrals are outside this library).  Every call
 * takes a batch of right-hand sides (n_batch / n_rhs >= 1, stored one after
 * another), e.g. the jackknife replicas of dE/dC.
 *
 * zvector_rhs: b[k][a][i] = sum_mu Cv[mu][a] dEdC[k][mu][i], the
 * virtual-occupied block of C^T dE/dC (the occupied-occupied block
 * C_occ^T dE/dC vanishes, so this is the whole projection of B onto orbital
 * rotations).
 *   Cv_dev[n_ao][n_virt]: the virtual MO coefficients (columns of the full,
 *   S-orthonormal C after the occupied ones), row-major;
 *   dEdC_dev[n_batch][n_ao][n_occ]; b_dev[n_batch][n_virt][n_occ].
 * zvector_backmap: Z[k][mu][i] = sum_a Cv[mu][a] z[k][a][i], the AO-basis
 * response (Z^T S C_occ = 0 follows from the S-orthonormality of C).
 *   z_dev[n_batch][n_virt][n_occ] in, Z_dev[n_batch][n_ao][n_occ] out.
 * zvector_jackknife: over n_blocks replicas x_jk_dev[n_blocks][len], the
 * jackknife mean[len] = sum_b x_b / nb and standard error
 * sigma[len] = sqrt((nb - 1)/nb sum_b (x_b - mean)^2) (either may be NULL).
 * These three are queued on `stream` (no synchronisation); all pointers are
 * device memory owned by the caller; outputs are overwritten.  Errors:
 * VMC_EINVAL (NULL pointer, a size < 1, n_batch > 65535, n_blocks < 2),
 * VMC_EDEVICE (launch failure).
 *
 * zvector_solve: H z_k = -b_k for k < n_rhs by conjugate gradients in FP64
 * from z = 0 (Hestenes-Stiefel; with flags & ZVECTOR_JACOBI, preconditioned
 * by diag H) until ||H z + b|| <= rtol ||b|| (the true residual norm, not the
 * preconditioned one), at most maxit iterations each.
 *   H_dev[d][d] symmetric positive definite, row-major; b_dev[n_rhs][d];
 *   z_dev[n_rhs][d] (device, caller-owned; z is overwritten).  The iteration
 *   state stays on the device; the host reads it once every 8 iterations.
 *   Several right-hand sides run in lockstep in groups of up to 64, every
 *   read of H shared by the group (an FP64 matrix-core product); each keeps
 *   its own step lengths and stopping test.  Host output: iters[n_rhs] =
 *   iterations used (may be NULL).  Synchronises `stream`; allocates device
 *   scratch for the call: about 4.2 d doubles for one right-hand side,
 *   (3 + s) * g * d doubles for a group of g (s <= 16 column splits).
 * Errors (the first failing right-hand side decides): VMC_EINVAL (NULL
 * pointer, d < 1, n_rhs < 1, rtol <= 0, maxit < 1, unknown flag),
 * VMC_ENOTCONV (maxit reached; z holds the last iterate), VMC_ENONFINITE (a
 * non-finite residual or curvature; z unspecified), VMC_ENOMEM, VMC_EDEVICE. */
#define ZVECTOR_JACOBI 1u
int zvector_rhs(const double *Cv_dev, int64_t n_ao, int64_t n_virt, int64_t n_occ, int64_t n_batch,
                const double *dEdC_dev, double *b_dev, void *stream);
int zvector_backmap(const double *Cv_dev, int64_t n_ao, int64_t n_virt, int64_t n_occ, int64_t n_batch,
                    const double *z_dev, double *Z_dev, void *stream);
int zvector_jackknife(const double *x_jk_dev, int64_t n_blocks, int64_t len, double *mean_dev,
                      double *sigma_dev, void *stream);
int zvector_solve(const double *H_dev, int64_t d, int64_t n_rhs, const double *b_dev, double *z_dev,
                  double rtol, int32_t maxit, uint32_t flags, int32_t *iters, void *stream);

/* zvector_solve_noalloc: zvector_solve with no device allocation, for
 * callers that cannot allocate device memory (code between the steps of a
 * captured or replayed sequence, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as zvector_solve, except
 * that the right-hand sides are solved one after another (no batch shares
 * the reads of H) and d <= ZVECTOR_NOALLOC_MAX_D (VMC_EINVAL beyond).  The
 * CG state (about 4.1 d doubles) lives in a library-owned device array of
 * 2.5 MiB on each GPU, taken on the first call on that GPU and kept until
 * the process ends; it allocates nothing else (no hipMalloc, hipFree or
 * allocating library call).  All calls on one GPU share that array: calls
 * that overlap in time on one GPU (two host threads, or two streams without
 * synchronisation between them) race and give undefined results.  Every
 * value of the array is written before it is read, so what an earlier call
 * left there does not matter.  Synchronises `stream`. */
#define ZVECTOR_NOALLOC_MAX_D 65536
int zvector_solve_noalloc(const double *H_dev, int64_t d, int64_t n_rhs, const double *b_dev, double *z_dev,
                          double rtol, int32_t maxit, uint32_t flags, int32_t *iters, void *stream);

/* Most walkers processed per measurement launch (size of the per-walker
 * staging); returns -1 for a NULL context. */
int64_t vmc_staging_walkers(const vmc_ctx *ctx);

/* ---- kernel timing --------------------------------------------------------
 * vmc_profile(ctx, enable): while enabled, every launch of the kernels named
 * below (in the context's own precision; not the FP64 re-measurement of
 * promoted walkers) is bracketed by HIP events recorded on its launch stream,
 * and their elapsed times accumulate.  Enabling clears the totals.
 * vmc_profile_read(ctx, kernel, ms, launches, walkers): waits for the recorded
 * events and returns the summed elapsed milliseconds, the number of launches
 * and the walkers they processed (any output pointer may be NULL).
 * Returns VMC_EINVAL for an unknown kernel, VMC_EDEVICE on HIP errors.     */
#define VMC_K_ADJOINT   0    /* k_adjoint_mfma: back-projection, outer products */
#define VMC_K_DENSE     1    /* k_dense: inverses, E_L, (K X K)^T / 2           */
#define VMC_K_MO_ROWS   2    /* k_mo_rows_mfma (value, gradient, Laplacian)      */
#define VMC_K_SWEEP     3    /* k_sweep_r: the moves of one sweep of all walkers */
#define VMC_K_PROPOSALS 4    /* k_propose + k_mo_rows_mfma (values): a sweep's
                                proposals and their MO rows                      */
#define VMC_K_ECP_POINTS  5  /* k_ecp_pairs + k_mo_rows_mfma at the quadrature
                                points of the pseudopotential                    */
#define VMC_K_ECP_ENERGY  6  /* k_ecp_energy                                     */
#define VMC_K_ECP_ADJOINT 7  /* k_ecp_adjoint                                    */
#define VMC_K_JAS_GEMM  8    /* k_jas_gemm: the one-/three-body Jastrow's products
                                with [xi3 | xi1] (the values' and xi3 h per
                                measurement launch, the moves' differences per
                                sweep)                                           */
#define VMC_N_PROFILED  9
int vmc_profile(vmc_ctx *ctx, int32_t enable);
int vmc_profile_read(vmc_ctx *ctx, int32_t kernel, double *ms, int64_t *launches, int64_t *walkers);

/* Release the context and its device memory (NULL is ignored). */
void vmc_free(vmc_ctx *ctx);

/* Detail of the last error on ctx (never NULL; "" if none). */
const char *vmc_last_error(const vmc_ctx *ctx);

/* Detail of the last failed vmc_init in the calling thread (never NULL). */
const char *vmc_init_error(void);

/* Name of a status code. */
const char *vmc_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* VMC_H */
