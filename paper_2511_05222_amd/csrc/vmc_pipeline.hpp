// vmc_pipeline.hpp -- argument structs and launchers of vmc_pipeline.hip (internal).
#pragma once

#include "vmc_kernels.hpp"

namespace vmcx {

// AO tiles: consecutive whole shells (at most 16 AOs each for k_mo_rows_mfma).
struct AoTiles {
    const int *s0, *s1, *mu0, *mu1;
    int n_tiles;
};

// LDS layout of k_sweep_r (bytes): wpb wavefront regions of two broadcast
// vectors each.
struct SweepLayout {
    int off_phin, off_colj;                         // within a wavefront region
    int wave_bytes;
    int wpb;                                        // walkers (wavefronts) per block
    size_t bytes;                                   // per block
};

// LDS layout of k_dense (bytes).
struct DenseLayout {
    int ldk;                 // row stride (doubles, odd) of K, X and T
    int off_p, off_g, off_k, off_x, off_perm, off_red, off_jas;
    size_t bytes;
};

// LDS layout of k_adjoint_mfma (bytes).
struct AdjLayout {
    int ldk;                         // row stride (elements, odd) of K~ and Abar
    int rt;                          // 16-electron row tiles
    int off_k, off_a, off_p, off_g, off_d;
    int waves;                       // wavefronts per block
    size_t bytes;
};

// Per-walker staging of one measurement launch (chunk of walkers).
template <typename T>
struct MeasBufs {
    const double *pos;    // [W][N][3] evaluation (possibly warped) positions
    const double *pos0;   // [W][N][3] sampling positions
    T *phi;               // [W][N][5][n]   MO value, gradient, Laplacian rows
    T *ktil;              // [W][N][n]      K[i][e] of the electron's spin block
    T *abar;              // [W][N][n]      dE_L / dA[e][i]
    double *gb;           // [W][N][6]      Jastrow gradient (0..2), det gradient (3..5)
    double *dedr_part;    // [W][N][3]      dE_L/dr_e, determinant part
    double *tao;          // [W][M][6]      per-AO electron sums of t_k, s_k
    // per walker, max|Abar| over both spin blocks (Abar = (K X K)^T / 2, the
    // sensitivity of E_L to the orbital values; +inf if not finite): the key
    // that picks the walkers measured again in FP64; null = not needed
    double *promote_key;
    // the sweep's persistent inverses of these walkers (KState layout); when
    // set, a block whose inverse is not stale starts from it and one FP64
    // Newton step instead of a Gauss-Jordan inversion (no ln|det| then)
    const T *kst;
    const uint8_t *ksig;
    const int *kstale;
    // one-/three-body Jastrow terms (null: none): grad_e U, lap_e U per
    // electron [W][N][4] and U [W], added to the two-body terms
    const double *jg = nullptr, *ju = nullptr;
};

struct MeasBufsD {
    const double *pos, *pos0;
    const double *gb, *dedr_part, *tao;
    // one-/three-body Jastrow (null: none): per-function electron sums
    // jtao[W][MJ][6] of its dE_L/dr and dlnPsi/dr terms; jb its basis
    const double *jtao = nullptr;
    BasisDev jb{};
    // pseudopotential (null: none): its explicit derivative in each nucleus,
    // ecp_dR[W][A][3]
    const double *ecp_dR = nullptr;
};

// Semilocal pseudopotential (vmc_ecp.hip): radial terms sorted by nucleus,
// beta d^(n - 2) e^{-alpha d^2} in channel l (-1: local).
struct EcpDev {
    int n_nl;                  // nuclei with projectors
    const int *nl_atom;        // [n_nl]
    const int *t0;             // [A + 1]: the terms of nucleus a are t0[a] .. t0[a + 1]
    const int *t_l, *t_n;
    const double *t_alpha, *t_beta;
    const double *rcut;        // [A]
    int lmax;                  // largest projector l
    uint64_t seed;             // key of the quadrature rotations
    int pcap;                  // (electron, nucleus) pairs per walker
};

// Staging of the pseudopotential terms of one measurement launch of W
// walkers, packed over the walkers (capacity W * pcap pairs): walker w's
// pairs are pairs[off[w] .. off[w] + npairs[w]) (electron | nucleus << 8),
// its points qpos[12 off[w] ..][3], the MO rows there phiq[12 off[w] ..][nc][n]
// (type T) and per point rows[12 off[w] ..][ECP_ROW]; *nrows = 12 * the
// pairs of the launch; ecp_dR[W][A][3]; per AO the sums over the points
// tc[W][M][3] of kappa grad psi.  rows[10..12]: the gradient at the point of
// the one-/three-body Jastrow change (with those terms).
constexpr int ECP_ROW = 13;
template <typename T>
struct EcpBufs {
    int *pairs, *npairs, *off, *nrows;
    double *qpos;
    T *phiq;
    double *rows;
    double *ecp_dR;
    double *tc;
};
// The one-/three-body Jastrow in the pseudopotential's ratios (X null:
// none): chi at the electrons X[W N][MJ], their gradients and Laplacians
// D[W N][4][MJ] and the value products V with [xi3 | xi1] (the
// measurement's, nq blocks of [W N][64]), xi1 and the FP64 column blocks of
// [xi3 | xi1]; jg[W][N][4] the electrons' gradients of U1 + U3; jtao the
// per-function sums the measurement subtracts per nucleus.
template <typename T>
struct EcpJas {
    BasisDev jb{};
    int MJ = 0;
    int64_t rows = 0;
    const T *X = nullptr, *D = nullptr, *V = nullptr;
    const double *xi1 = nullptr, *xiblk = nullptr, *jg = nullptr;
    double *jtao = nullptr;
};
// Pairs and points of the W walkers (walker id id0 + w, or id0 + idlist[w]).
hipError_t launch_ecp_pairs(const SysDev &S, const EcpDev &E, const double *R, const double *pos, int W,
                            int64_t id0, const int *idlist, uint32_t rot, int *pairs, int *npairs, int *off,
                            int *nrows, double *qpos, int *status, hipStream_t st);
// LDS the energy kernel needs (bytes), and raising the limits to it
size_t ecp_energy_lds(int N, int n, int MJ);
hipError_t configure_ecp(size_t lds);
// E_loc + E_nl added to EL[w]; with abar: dE/dA through the inverses added.
template <typename T>
hipError_t launch_ecp_energy(const SysDev &S, const EcpDev &E, const double *R, const double *pos, int W,
                             const EcpBufs<T> &eb, int nc, const T *ktil, T *abar, double *EL, int *status,
                             const EcpJas<T> &J, hipStream_t st);
// The derivatives through the points: G (or Gf) += sum psi(r_q) y_q^T,
// dedr[w][e] += ..., ecp_dR[w][a] = ...
template <typename T>
hipError_t launch_ecp_adjoint(const SysDev &S, const EcpDev &E, const T *C, const double *R, const double *pos,
                              int W, const EcpBufs<T> &eb, const T *ktil, double *G, float *Gf, double *dedr,
                              const EcpJas<T> &J, hipStream_t st);

// cpad: scratch of (M + 16) * 64 elements for the padded copy of C (n_occ <= 64);
// rows_dev (optional): a device count that caps n_rows
template <typename T>
hipError_t launch_mo_rows_mfma(const SysDev &S, const T *C, const double *R, const double *pos, int64_t n_rows,
                               const AoTiles &tiles16, T *out, int nc, T *cpad, hipStream_t st,
                               const int *rows_dev = nullptr);
// One-/three-body Jastrow terms (vmc_jastrow.hip).  jas_values: out[row][mu]
// = chi_mu(pos[row]) and, with der, der[row][c][mu] its gradient (c < 3) and
// Laplacian (c = 3) (in FP32 over the tiles of <= 32 functions jt32 when
// given, else jt's of <= 16).  jas_vprod: the products of the rows of X (of X - X0
// when X0 is given) with [xi3 | xi1] ([nq][MJ][64] in xiblk), MJ + 1 columns:
// in blocks of 64, V[q][row][64] (X), or row by row with a row stride of
// MJ + 1 rounded up to a multiple of 4 (X - X0).
// jas_assemble: grad_e U, lap_e U, U from the values, their derivatives and
// the value products.  jas_hxi: Q[row] = xi3 h_row (h = grad chi abar -
// lap chi / 2, abar from gb).  jas_adjoint: its terms of dE_L/dr_e (added to
// dedr) and the per-function sums jtao.
template <typename T>
hipError_t launch_jas_values(const BasisDev &JB, const AoTiles &jt, const double *R, const double *pos, int64_t rows,
                             T *out, hipStream_t st, T *der = nullptr, const AoTiles *jt32 = nullptr);
template <typename T>
hipError_t launch_jas_vprod(int MJ, int nq, int64_t rows, const T *X, const T *X0, const T *xiblk, T *V,
                            hipStream_t st);
template <typename T>
hipError_t launch_jas_assemble(int N, int MJ, int nq, int64_t rows, int64_t row0, int W, const T *X, const T *D,
                               const T *V, const double *xi1, double *jg, double *ju, hipStream_t st);
template <typename T>
hipError_t launch_jas_hxi(int MJ, int nq, int64_t rows, const T *D, const double *gb, const T *xiblk, T *Q,
                          hipStream_t st);
template <typename T>
hipError_t launch_jas_adjoint(const BasisDev &JB, const double *R, int N, int64_t rows, int64_t row0, int W,
                              const double *pos, const T *V, const T *Q, const double *gb, const double *xi1,
                              double *dedr, double *jtao, hipStream_t st);
// The launch's sums of the Jastrow-parameter log-derivatives (weights wt,
// null = 1; E_L - shift) added into acc/comp: [s | (E-s) s | O3 | (E-s) O3];
// scratch of xi_scratch_doubles(W, MJ) doubles.
size_t xi_scratch_doubles(int W, int MJ);
hipError_t launch_xi_sums(const double *X, int N, int MJ, int W, const double *EL, const double *shift,
                          const double *wt, double *part, double *scratch, double *acc, double *comp,
                          hipStream_t st);
// The sweep's one-/three-body terms (null Xp: none): chi at the proposals and
// at the positions of the sweep's start ([W N][MJ]) and the [xi3 | xi1]
// products of their difference (rows of MJ + 1 rounded up to a multiple of 4).
template <typename T>
struct JasSweep {
    const T *Xp = nullptr, *X0 = nullptr, *Pd = nullptr;
    int MJ = 0, nq = 0;
    int64_t rows = 0;
};

// Persistent inverses of the two spin blocks of every walker, in the
// register layout of the sweep: K[w][b][r][lane] (KN x KN, type T), the
// permutation sig[w][b][lane] and stale[w][b] = a rebuild is due.
template <typename T>
struct KState {
    T *K;
    uint8_t *sig;
    int *stale;
};

int sweep_kn(int n_occ);
// prop[w][e] = walkers[w][e] + sigma z_e for the W walkers (Philox normals of
// the sweep)
hipError_t launch_propose(const double *walkers, int64_t W, int N, uint32_t sweep, uint64_t seed, double sigma,
                          double *prop, hipStream_t st);
// The moves of one sweep; Phip[w][e][n] = the MO row at the proposal prop[w][e]
template <typename T>
hipError_t launch_sweep(const SysDev &S, const T *Phip, const double *prop, double *walkers, int W, T *Amo,
                        const KState<T> &ks, int fresh, uint32_t sweep, uint64_t seed, int refresh_period,
                        uint8_t *accept, int *status, const SweepLayout &L, const JasSweep<T> &js, hipStream_t st);
hipError_t launch_warp(const SysDev &S, const double *R, const double *R0, const double *pos0, double *posw,
                       double *lnjac, int W, hipStream_t st);
template <typename T>
hipError_t launch_dense(const SysDev &S, const double *R, const MeasBufs<T> &mb, const WalkerOut &out, int *status,
                        const DenseLayout &L, int W, hipStream_t st);
template <typename T>
hipError_t configure_dense(size_t lds);
template <typename T>
hipError_t launch_adjoint(const SysDev &S, const T *C, const double *R, const MeasBufs<T> &mb,
                          const WalkerOut &out, const AdjLayout &L, int W, hipStream_t st);
template <typename T>
hipError_t configure_adjoint(size_t lds);
hipError_t launch_finalize(const SysDev &S, const double *R, const double *R0, const MeasBufsD &mb,
                           const WalkerOut &out, int warp, int W, hipStream_t st);
template <typename T>
hipError_t configure_sweep(size_t lds);
// resident blocks of k_sweep_r per CU for blocks of wpb walkers and lds bytes
// (0 when the runtime cannot tell)
template <typename T>
int sweep_blocks_per_cu(int n_occ, int wpb, size_t lds);

// list[0..k) = the k walkers of W with the largest keys (ties to the lower
// index), in index order
hipError_t launch_promote_select(const double *key, int W, int k, int *list, hipStream_t st);
hipError_t launch_round_f32(const double *x, float *y, int64_t n, hipStream_t st);

hipError_t launch_gather_rows(const double *src, const int *list, int64_t kc, int64_t len, double *dst,
                              hipStream_t st);
hipError_t launch_scatter_rows(const double *src, const int *list, int64_t kc, int64_t len, double *dst,
                               hipStream_t st);
hipError_t launch_scatter_rows_f32(const double *src, const int *list, int64_t kc, int64_t len, float *dst,
                                   hipStream_t st);

}  // namespace vmcx
