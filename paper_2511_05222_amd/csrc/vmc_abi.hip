// vmc_abi.hip -- host side of the C ABI declared in include/vmc.h.
//
// Owns the context (validated inputs, folded GTO normalisation, device
// buffers), sequences the kernels of the vmc_*.hip sources on the caller's
// stream, and finishes the estimators in FP64 on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "vmc.h"
#include "vmc_kernels.hpp"
#include "vmc_pipeline.hpp"

using vmcx::AdjLayout;
using vmcx::AoTiles;
using vmcx::DenseLayout;
using vmcx::MeasBufs;
using vmcx::MeasBufsD;
using vmcx::SweepLayout;
using vmcx::EstArgs;
using vmcx::SysDev;
using vmcx::WalkerOut;

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr int64_t MAX_SEG = 256;
constexpr int64_t MAX_BLOCKS = 1 << 16;
constexpr size_t STAGING_BUDGET = size_t(1) << 34;   // bytes of per-walker staging (16 GiB)

int dfact(int n) {
    int r = 1;
    while (n > 1) {
        r *= n;
        n -= 2;
    }
    return r;
}

bool all_finite(const double *p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

struct vmc_ctx {
    int device = 0;
    int N = 0, n_up = 0, n_dn = 0, n_occ = 0, M = 0, A = 0, S = 0, P = 0;
    vmc_options opt{};
    double ee_a = 0.5, ee_F = 1.0;
    int ee_form = VMC_JASTROW_PADE;
    std::string err;

    std::vector<void *> allocs;
    double *d_C = nullptr, *d_R = nullptr, *d_Z = nullptr;
    vmcx::BasisDev bdev{};   // the determinant's basis tables
    AoTiles tiles16{};       // its AO tiles: whole shells, <= 16 AOs
    // one- and three/four-body Jastrow (MJ = 0: absent): the Jastrow basis,
    // [xi3 | xi1] in column blocks of 64 ([nq][MJ][64], FP64 and FP32), xi1
    int MJ = 0, nq = 0;
    vmcx::BasisDev jdev{};
    AoTiles jtiles16{}, jtiles32{};   // the Jastrow basis in tiles of <= 16 and <= 32 functions
    double *d_xiblk = nullptr, *d_xi1 = nullptr;
    // the Jastrow-parameter gradient's sums (jastrow_gradient): per launch
    // the FP64 basis values at the electrons and the partial sums, and the
    // compensated accumulators [s | (E-s) s | O3 | (E-s) O3]
    double *xg_X = nullptr, *xg_part = nullptr, *xg_acc = nullptr, *xg_comp = nullptr, *xg_scr = nullptr;
    int64_t xg_n = 0;
    float *d_xiblk_f = nullptr;
    // staging of the Jastrow terms: sweeps ([W][N] rows) and measurements
    // ([chunk][N] rows); element sizes of the arithmetic type
    void *js_Xp = nullptr, *js_X0 = nullptr, *js_Pd = nullptr;
    double *jm_X = nullptr, *jm_D = nullptr, *jm_V = nullptr, *jm_Q = nullptr, *jm_g = nullptr, *jm_u = nullptr,
           *jm_tao = nullptr;
    // semilocal pseudopotential (has_ecp false: none): device tables, the
    // staging of one measurement launch (EcpBufs) and the frame of its
    // quadrature rotations for the next measurement: walker id of the
    // launch's first walker (or of the listed walkers) and rotation index
    bool has_ecp = false;
    vmcx::EcpDev edev{};
    int *e_pairs = nullptr, *e_npairs = nullptr, *e_off = nullptr, *e_nrows = nullptr;
    double *e_qpos = nullptr, *e_phiq = nullptr, *e_rows = nullptr, *e_dR = nullptr, *e_tc = nullptr;
    int64_t ecp_id0 = 0;
    uint32_t ecp_rot = 0;
    const int *ecp_idlist = nullptr;
    SysDev sys{};
    SweepLayout swl{};   // k_sweep_r in the arithmetic type of the precision
    DenseLayout dl{};
    AdjLayout al{};      // k_adjoint_mfma in the arithmetic type of the precision

    int64_t chunk = 0;
    double *st_EL = nullptr, *st_lnpsi = nullptr, *st_lnjac = nullptr, *st_dEdR = nullptr, *st_dPdR = nullptr,
           *st_dJdR = nullptr, *st_O = nullptr, *st_G = nullptr;
    // measurement pipeline staging (chunk walkers)
    double *mb_phi = nullptr, *mb_ktil = nullptr, *mb_abar = nullptr, *mb_gb = nullptr, *mb_dpart = nullptr,
           *mb_tao = nullptr, *mb_posw = nullptr;
    void *Amo = nullptr;     // [max_walkers][N][n] MO matrix maintained by the sweep (type T)
    void *Phip = nullptr;    // [max_walkers][N][n] MO rows at the sweep's proposals (type T)
    double *prop = nullptr;  // [max_walkers][N][3] the sweep's proposals
    void *Kst = nullptr;     // [max_walkers][2][KN][KN] persistent inverses (type T)
    uint8_t *Ksig = nullptr; // [max_walkers][2][KN]
    int *Kstale = nullptr;   // [max_walkers][2]
    float *d_Cf = nullptr;   // C in FP32 (mixed precision)
    float *d_Cm = nullptr;   // FP32 copy of a caller's C (mixed precision)
    double *d_cpad = nullptr;   // C padded for the MO-row kernel ((M + 16) x 64, either type)
    // FP64 re-measurement of the walkers whose E_L is most sensitive to the
    // FP32 orbital values (mixed precision)
    AdjLayout al64{};
    int *plist = nullptr;
    double *pkey = nullptr;
    int64_t pcap = 0;
    double *cp_pos = nullptr, *cp_pos0 = nullptr, *cp_EL = nullptr, *cp_lnpsi = nullptr, *cp_dEdR = nullptr,
           *cp_dPdR = nullptr, *cp_dJdR = nullptr, *cp_O = nullptr, *cp_G = nullptr;

    // kernel timing (vmc_profile): event pairs per kernel id
    struct ProfRec {
        hipEvent_t a, b;
        int64_t walkers;
    };
    bool prof = false;
    std::vector<ProfRec> prof_recs[VMC_N_PROFILED];

    int64_t n_est = 0;
    double *acc = nullptr, *comp = nullptr, *partial = nullptr;
    // per-block sums of every estimator element (jackknife), jk_cap blocks
    double *blk_all = nullptr;
    int64_t jk_cap = 0;
    double *shift = nullptr;
    int *shift_set = nullptr;
    int *status = nullptr;
    double *blocks = nullptr;    // [MAX_BLOCKS] per-block sums of w (E_L - s)
    double *blocks_w = nullptr;  // [MAX_BLOCKS] per-block sums of w
    std::vector<int64_t> block_counts;   // walkers per block
    int64_t n_samples = 0;
    int64_t sweeps_since_reset = 0;
    double *vjp_acc = nullptr, *vjp_comp = nullptr, *vjp_out = nullptr;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }

    template <class T>
    int dalloc(T **p, size_t n) {
        void *q = nullptr;
        if (hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(VMC_ENOMEM, "hipMalloc of %zu bytes failed", n * sizeof(T));
        }
        allocs.push_back(q);
        *p = (T *)q;
        return VMC_OK;
    }

    template <class T>
    int upload(T **p, const T *h, size_t n) {
        int rc = dalloc(p, n);
        if (rc) return rc;
        if (hipMemcpy(*p, h, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return fail(VMC_EDEVICE, "hipMemcpy to device failed");
        return VMC_OK;
    }
};

#define HIP_OK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return (ctx)->fail(VMC_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Kernel timing: prof_begin records the start event of kernel id k (or does
// nothing when profiling is off or !on); prof_end the stop event.
static void prof_clear(vmc_ctx *c) {
    for (auto &v : c->prof_recs) {
        for (auto &r : v) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        v.clear();
    }
}

static int prof_begin(vmc_ctx *c, int k, bool on, int64_t walkers, hipStream_t st) {
    if (!c->prof || !on) return -1;
    vmc_ctx::ProfRec r{};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess ||
        hipEventRecord(r.a, st) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    r.walkers = walkers;
    c->prof_recs[k].push_back(r);
    return (int)c->prof_recs[k].size() - 1;
}

static void prof_end(vmc_ctx *c, int k, int idx, hipStream_t st) {
    if (idx >= 0 && hipEventRecord(c->prof_recs[k][idx].b, st) != hipSuccess) (void)hipGetLastError();
}

// LDS layout of the sweep for an arithmetic type of ts bytes and blocks of
// wpb walkers: two broadcast vectors per wavefront.
static SweepLayout sweep_layout(const vmc_ctx *c, size_t ts, int wpb) {
    SweepLayout s{};
    auto al = [](size_t b) { return (int)((b + 15) & ~(size_t)15); };
    const int kn = vmcx::sweep_kn(c->n_occ);
    size_t w = 0;
    s.off_phin = (int)w;
    w += al((size_t)kn * ts);
    s.off_colj = (int)w;
    w += al((size_t)kn * ts);
    s.wave_bytes = (int)w;
    s.wpb = wpb;
    s.bytes = (size_t)wpb * w;
    return s;
}

// The block size that keeps the most walkers resident on a CU (ties go to
// the larger block).
static SweepLayout sweep_layout(const vmc_ctx *c, size_t ts) {
    SweepLayout best = sweep_layout(c, ts, 1);
    int best_res = -1;
    for (int wpb : {8, 4, 2}) {
        const SweepLayout s = sweep_layout(c, ts, wpb);
        const int nb = ts == sizeof(float) ? vmcx::sweep_blocks_per_cu<float>(c->n_occ, wpb, s.bytes)
                                           : vmcx::sweep_blocks_per_cu<double>(c->n_occ, wpb, s.bytes);
        if (nb * wpb > best_res) {
            best = s;
            best_res = nb * wpb;
        }
    }
    return best;
}

// LDS layout of the adjoint for an arithmetic type of ts bytes.
static AdjLayout adjoint_layout(const vmc_ctx *c, size_t ts) {
    AdjLayout a{};
    auto al = [](size_t b) { return (int)((b + 15) & ~(size_t)15); };
    const int nt = (c->n_occ + 15) / 16, N = c->N;
    a.ldk = 16 * nt + 1;
    a.rt = (N + 15) / 16;
    const int kb = al((size_t)a.rt * 16 * a.ldk * ts);
    a.off_k = 0;
    a.off_a = kb;
    a.off_p = 2 * kb;
    a.off_g = a.off_p + al((size_t)3 * N * 8);
    a.off_d = a.off_g + al((size_t)3 * N * 8);
    // FP32 needs about 140 registers (three wavefronts per SIMD): blocks of
    // four wavefronts let three walkers share a CU; FP64 (about 250) runs two
    // per SIMD, one block of eight
    a.waves = ts == sizeof(float) ? 4 : 8;
    while (a.waves > 1 && (size_t)a.off_d + (size_t)a.waves * 3 * N * 8 > 160 * 1024) a.waves /= 2;
    a.bytes = (size_t)a.off_d + (size_t)a.waves * 3 * N * 8;
    return a;
}

// LDS layout of k_dense.
static void layouts(vmc_ctx *c) {
    auto al = [](size_t b) { return (int)((b + 15) & ~(size_t)15); };
    const int N = c->N, kn = vmcx::sweep_kn(c->n_occ);
    DenseLayout &d = c->dl;
    d.ldk = kn + 1;
    d.off_p = 0;
    d.off_g = d.off_p + al((size_t)3 * N * 8);
    d.off_k = d.off_g + al((size_t)3 * N * 8);
    d.off_x = d.off_k + al((size_t)2 * kn * d.ldk * 8);
    d.off_perm = d.off_x + al((size_t)kn * d.ldk * 8);
    d.off_red = d.off_perm + al(128 * 4);
    d.off_jas = d.off_red + al(16 * 8);
    d.bytes = (size_t)d.off_jas + (size_t)(2 + 4) * N * 3 * 8;
}

// Walkers per measurement launch: W split into the fewest chunks that fit
// the staging, of equal length (up to one), so that no launch is a small
// tail (the FP64 re-measurement of each launch included).
static int64_t chunk_len(const vmc_ctx *c, int64_t W) {
    const int64_t nch = (W + c->chunk - 1) / c->chunk;
    return nch > 0 ? (W + nch - 1) / nch : c->chunk;
}

// The measurement kernels on cw walkers at (possibly warped) positions pos
// with sampling positions pos0.  plist: promotion list for the dense kernel.
// Chunk offsets into the sweep's persistent inverses (null: none).
// [xi3 | xi1] column blocks in the arithmetic type
template <typename T>
static const T *xi_blocks(const vmc_ctx *c);
template <>
const float *xi_blocks<float>(const vmc_ctx *c) { return c->d_xiblk_f; }
template <>
const double *xi_blocks<double>(const vmc_ctx *c) { return c->d_xiblk; }

struct KStateRef {
    const void *K = nullptr;
    const uint8_t *sig = nullptr;
    const int *stale = nullptr;
};

template <typename T>
static int measure_core(vmc_ctx *c, const double *pos, const double *pos0, int64_t cw, const T *C, const double *R,
                        const double *R0, int warp, int full, const WalkerOut &o, const AdjLayout &al, double *pkey,
                        bool prof, const KStateRef &ks, hipStream_t st) {
    const SysDev &S = c->sys;
    T *phi = (T *)c->mb_phi;
    MeasBufs<T> mb{pos,         pos0,       phi,       (full || c->has_ecp) ? (T *)c->mb_ktil : nullptr,
                   (T *)c->mb_abar, c->mb_gb,   c->mb_dpart, c->mb_tao,
                   pkey,      (const T *)ks.K,                  ks.sig,
                   ks.stale};
    int pi = prof_begin(c, VMC_K_MO_ROWS, prof, cw, st);
    HIP_OK(c, vmcx::launch_mo_rows_mfma<T>(S, C, R, pos, cw * c->N, c->tiles16, phi, 5, (T *)c->d_cpad, st));
    prof_end(c, VMC_K_MO_ROWS, pi, st);
    // pseudopotential: the pairs inside the cutoffs, their points and the
    // MO rows there (values; with the adjoint also gradients)
    const vmcx::EcpBufs<T> eb{c->e_pairs, c->e_npairs, c->e_off,  c->e_nrows, c->e_qpos,
                              (T *)c->e_phiq, c->e_rows, c->e_dR,    c->e_tc};
    const int enc = full ? 5 : 1;
    if (c->has_ecp) {
        pi = prof_begin(c, VMC_K_ECP_POINTS, prof, cw, st);
        HIP_OK(c, vmcx::launch_ecp_pairs(S, c->edev, R, pos, (int)cw, c->ecp_id0, c->ecp_idlist, c->ecp_rot,
                                         c->e_pairs, c->e_npairs, c->e_off, c->e_nrows, c->e_qpos, c->status, st));
        HIP_OK(c, vmcx::launch_mo_rows_mfma<T>(S, C, R, c->e_qpos, cw * c->edev.pcap * 12, c->tiles16,
                                               (T *)c->e_phiq, enc, (T *)c->d_cpad, st, c->e_nrows));
        prof_end(c, VMC_K_ECP_POINTS, pi, st);
    }
    const int64_t jrows = cw * c->N;
    T *jX = (T *)c->jm_X, *jD = (T *)c->jm_D, *jV = (T *)c->jm_V, *jQ = (T *)c->jm_Q;
    if (c->MJ > 0) {
        // one-/three-body Jastrow: chi with its gradients and Laplacians, the
        // value products with [xi3 | xi1]; gradient, Laplacian and value per
        // walker (the dense kernel adds them)
        HIP_OK(c, vmcx::launch_jas_values<T>(c->jdev, c->jtiles16, R, pos, jrows, jX, st, jD, &c->jtiles32));
        const int pg = prof_begin(c, VMC_K_JAS_GEMM, prof, cw, st);
        HIP_OK(c, vmcx::launch_jas_vprod<T>(c->MJ, c->nq, jrows, jX, (const T *)nullptr, xi_blocks<T>(c), jV, st));
        prof_end(c, VMC_K_JAS_GEMM, pg, st);
        HIP_OK(c, vmcx::launch_jas_assemble<T>(c->N, c->MJ, c->nq, jrows, 0, (int)cw, jX, jD, jV, c->d_xi1, c->jm_g,
                                               c->jm_u, st));
        mb.jg = c->jm_g;
        mb.ju = c->jm_u;
    }
    // the same terms in the pseudopotential's ratios
    vmcx::EcpJas<T> ej;
    if (c->MJ > 0) {
        ej.jb = c->jdev;
        ej.MJ = c->MJ;
        ej.rows = jrows;
        ej.X = jX;
        ej.D = jD;
        ej.V = jV;
        ej.xi1 = c->d_xi1;
        ej.xiblk = c->d_xiblk;
        ej.jg = c->jm_g;
        ej.jtao = c->jm_tao;
    }
    pi = prof_begin(c, VMC_K_DENSE, prof, cw, st);
    HIP_OK(c, vmcx::launch_dense<T>(S, R, mb, o, c->status, c->dl, (int)cw, st));
    prof_end(c, VMC_K_DENSE, pi, st);
    if (c->has_ecp) {
        pi = prof_begin(c, VMC_K_ECP_ENERGY, prof, cw, st);
        HIP_OK(c, vmcx::launch_ecp_energy<T>(S, c->edev, R, pos, (int)cw, eb, enc, mb.ktil, full ? mb.abar : nullptr,
                                             o.EL, c->status, ej, st));
        prof_end(c, VMC_K_ECP_ENERGY, pi, st);
    }
    if (!full) return VMC_OK;
    pi = prof_begin(c, VMC_K_ADJOINT, prof, cw, st);
    HIP_OK(c, vmcx::launch_adjoint<T>(S, C, R, mb, o, al, (int)cw, st));
    prof_end(c, VMC_K_ADJOINT, pi, st);
    MeasBufsD md{pos, pos0, c->mb_gb, c->mb_dpart, c->mb_tao};
    if (c->MJ > 0) {
        // (writes the per-function sums jtao that the pseudopotential's
        // one-/three-body terms then add to)
        const int pg = prof_begin(c, VMC_K_JAS_GEMM, prof, cw, st);
        HIP_OK(c, vmcx::launch_jas_hxi<T>(c->MJ, c->nq, jrows, jD, c->mb_gb, xi_blocks<T>(c), jQ, st));
        prof_end(c, VMC_K_JAS_GEMM, pg, st);
        HIP_OK(c, vmcx::launch_jas_adjoint<T>(c->jdev, R, c->N, jrows, 0, (int)cw, pos, jV, jQ, c->mb_gb, c->d_xi1,
                                              c->mb_dpart, c->jm_tao, st));
        md.jtao = c->jm_tao;
        md.jb = c->jdev;
    }
    if (c->has_ecp) {
        pi = prof_begin(c, VMC_K_ECP_ADJOINT, prof, cw, st);
        HIP_OK(c, vmcx::launch_ecp_adjoint<T>(S, c->edev, C, R, pos, (int)cw, eb, mb.ktil, o.G, o.Gf, c->mb_dpart,
                                              ej, st));
        prof_end(c, VMC_K_ECP_ADJOINT, pi, st);
        md.ecp_dR = c->e_dR;
    }
    HIP_OK(c, vmcx::launch_finalize(S, R, R0, md, o, warp, (int)cw, st));
    return VMC_OK;
}

// One measurement of `cw` walkers at positions pos0 (device [cw][N][3]) with
// the caller's FP64 C: forward always; adjoint when `full`.  Outputs already
// offset to the chunk.  In mixed precision C is rounded to FP32, and the
// walkers the dense kernel flags as sensitive are measured again in
// FP64 (gathered, measured, scattered over their mixed results).
static int run_measure(vmc_ctx *c, const double *pos0, int64_t cw, const double *C, const double *R,
                       const double *R0, int warp, int full, const WalkerOut &o, hipStream_t st,
                       const KStateRef &ks = KStateRef()) {
    const SysDev &S = c->sys;
    const double *pos = pos0;
    if (warp) {
        HIP_OK(c, vmcx::launch_warp(S, R, R0, pos0, c->mb_posw, o.lnjac ? o.lnjac : c->st_lnjac, (int)cw, st));
        pos = c->mb_posw;
    } else if (o.lnjac) {
        HIP_OK(c, hipMemsetAsync(o.lnjac, 0, cw * sizeof(double), st));
    }
    if (c->opt.precision != VMC_MIXED)
        return measure_core<double>(c, pos, pos0, cw, C, R, R0, warp, full, o, c->al, nullptr, true, ks, st);
    const float *Cf = c->d_Cf;
    if (C != c->d_C) {
        HIP_OK(c, vmcx::launch_round_f32(C, c->d_Cm, (int64_t)c->M * c->n_occ, st));
        Cf = c->d_Cm;
    }
    // the walkers re-measured in FP64: a fixed share of the launch, those
    // with the largest max|Abar| (known count: no host round trip)
    const int64_t cnt = c->opt.promote_fraction > 0.0
                            ? std::min<int64_t>(cw, (int64_t)std::ceil(c->opt.promote_fraction * (double)cw))
                            : 0;
    int rc = measure_core<float>(c, pos, pos0, cw, Cf, R, R0, warp, full, o, c->al, cnt ? c->pkey : nullptr, true,
                                 ks, st);
    if (rc || !cnt) return rc;
    HIP_OK(c, vmcx::launch_promote_select(c->pkey, (int)cw, (int)cnt, c->plist, st));
    const int64_t N3 = 3 * (int64_t)c->N, A3 = 3 * (int64_t)c->A, Mn = (int64_t)c->M * c->n_occ;
    for (int64_t k0 = 0; k0 < cnt; k0 += c->pcap) {
        const int64_t kc = std::min<int64_t>(c->pcap, cnt - k0);
        const int *lst = c->plist + k0;
        HIP_OK(c, vmcx::launch_gather_rows(pos, lst, kc, N3, c->cp_pos, st));
        HIP_OK(c, vmcx::launch_gather_rows(pos0, lst, kc, N3, c->cp_pos0, st));
        WalkerOut oc{o.EL ? c->cp_EL : nullptr,        o.lnpsi ? c->cp_lnpsi : nullptr,  nullptr,
                     o.dEL_dR ? c->cp_dEdR : nullptr, o.dlnpsi_dR ? c->cp_dPdR : nullptr,
                     o.dlnjac_dR ? c->cp_dJdR : nullptr, (o.O || o.Of) ? c->cp_O : nullptr,
                     (o.G || o.Gf) ? c->cp_G : nullptr};
        c->ecp_idlist = lst;
        rc = measure_core<double>(c, c->cp_pos, c->cp_pos0, kc, C, R, R0, warp, full, oc, c->al64, nullptr, false,
                                  KStateRef(), st);
        c->ecp_idlist = nullptr;
        if (rc) return rc;
        const std::pair<double *, double *> rows[] = {{oc.EL, o.EL},         {oc.lnpsi, o.lnpsi},
                                                      {oc.dEL_dR, o.dEL_dR}, {oc.dlnpsi_dR, o.dlnpsi_dR},
                                                      {oc.dlnjac_dR, o.dlnjac_dR}, {oc.O, o.O},
                                                      {oc.G, o.G}};
        const int64_t lens[] = {1, 1, A3, A3, A3, Mn, Mn};
        for (int k = 0; k < 7; ++k)
            if (rows[k].first && rows[k].second && (full || k < 2))
                HIP_OK(c, vmcx::launch_scatter_rows(rows[k].first, lst, kc, lens[k], rows[k].second, st));
        if (full && o.Of) HIP_OK(c, vmcx::launch_scatter_rows_f32(oc.O, lst, kc, Mn, o.Of, st));
        if (full && o.Gf) HIP_OK(c, vmcx::launch_scatter_rows_f32(oc.G, lst, kc, Mn, o.Gf, st));
    }
    return VMC_OK;
}

// One sweep of W walkers: the proposals of every electron with their MO rows
// (and Jastrow terms) -- independent of the moves' outcomes -- then the moves.
template <typename T>
static int sweep_once(vmc_ctx *c, double *walkers, int64_t W, int t, uint32_t sidx, uint64_t seed, uint8_t *acc_t,
                      const T *C, hipStream_t st) {
    const int64_t rows = W * c->N;
    T *Amo = (T *)c->Amo;
    const int pp = prof_begin(c, VMC_K_PROPOSALS, true, W, st);
    HIP_OK(c, vmcx::launch_propose(walkers, W, c->N, sidx, seed, c->opt.step_sigma, c->prop, st));
    HIP_OK(c, vmcx::launch_mo_rows_mfma<T>(c->sys, C, c->d_R, c->prop, rows, c->tiles16, (T *)c->Phip, 1,
                                          (T *)c->d_cpad, st));
    vmcx::JasSweep<T> js;
    if (c->MJ > 0) {
        T *Xp = (T *)c->js_Xp, *X0 = (T *)c->js_X0, *Pd = (T *)c->js_Pd;
        HIP_OK(c, vmcx::launch_jas_values<T>(c->jdev, c->jtiles16, c->d_R, c->prop, rows, Xp, st));
        HIP_OK(c, vmcx::launch_jas_values<T>(c->jdev, c->jtiles16, c->d_R, walkers, rows, X0, st));
        const int pg = prof_begin(c, VMC_K_JAS_GEMM, true, W, st);
        HIP_OK(c, vmcx::launch_jas_vprod<T>(c->MJ, c->nq, rows, Xp, X0, xi_blocks<T>(c), Pd, st));
        prof_end(c, VMC_K_JAS_GEMM, pg, st);
        js.Xp = Xp;
        js.X0 = X0;
        js.Pd = Pd;
        js.MJ = c->MJ;
        js.nq = c->nq;
        js.rows = rows;
    }
    prof_end(c, VMC_K_PROPOSALS, pp, st);
    // the MO matrix of every walker from the caller's positions; the sweeps
    // keep it current (row e rewritten on each accepted move)
    if (t == 0)
        HIP_OK(c, vmcx::launch_mo_rows_mfma<T>(c->sys, C, c->d_R, walkers, rows, c->tiles16, Amo, 1, (T *)c->d_cpad,
                                              st));
    const int pi = prof_begin(c, VMC_K_SWEEP, true, W, st);
    const vmcx::KState<T> ks{(T *)c->Kst, c->Ksig, c->Kstale};
    HIP_OK(c, vmcx::launch_sweep<T>(c->sys, (const T *)c->Phip, c->prop, walkers, (int)W, Amo, ks, t == 0, sidx, seed,
                                    c->opt.refresh_period, acc_t, c->status, c->swl, js, st));
    prof_end(c, VMC_K_SWEEP, pi, st);
    return VMC_OK;
}

// Measure W walkers at the context's C and nuclei and add them, with weights
// wt (null: 1), to the accumulators as one measured batch (one sweep of the
// blocking).  from_sweep: the walkers are those of the last sweep, whose
// persistent inverses the measurement may start from.
static int measure_accumulate(vmc_ctx *c, const double *walkers, int64_t W, const double *wt, bool from_sweep,
                              hipStream_t st) {
    int rc;
    const int64_t Mn = (int64_t)c->M * c->n_occ, A3 = 3 * c->A;
    const int64_t blk_idx = c->sweeps_since_reset / c->opt.block_sweeps;
    double *blk = blk_idx < MAX_BLOCKS ? c->blocks + blk_idx : nullptr;
    double *blkw = blk_idx < MAX_BLOCKS ? c->blocks_w + blk_idx : nullptr;
    double *blk_all = blk_idx < c->jk_cap ? c->blk_all + blk_idx * c->n_est : nullptr;
    const int64_t step = chunk_len(c, W);
    for (int64_t c0 = 0; c0 < W; c0 += step) {
        const int64_t cw = std::min(step, W - c0);
        // ln|Psi| is not an estimator input: the dense kernel may start
        // from the sweep's inverses
        // (in mixed precision O and G are staged in FP32: the estimator
        // reduction reads them once per launch)
        const bool f32 = c->opt.precision == VMC_MIXED;
        WalkerOut o{c->st_EL, nullptr, nullptr, c->st_dEdR, c->st_dPdR, c->st_dJdR, f32 ? nullptr : c->st_O,
                    f32 ? nullptr : c->st_G};
        if (f32) {
            o.Of = (float *)c->st_O;
            o.Gf = (float *)c->st_G;
        }
        KStateRef ks;
        if (from_sweep) {
            const int kn = vmcx::sweep_kn(c->n_occ);
            const size_t tsz = f32 ? sizeof(float) : sizeof(double);
            ks.K = (const char *)c->Kst + (size_t)c0 * 2 * kn * kn * tsz;
            ks.sig = c->Ksig + (size_t)c0 * 2 * kn;
            ks.stale = c->Kstale + 2 * c0;
        }
        c->ecp_id0 = c0;
        if ((rc = run_measure(c, walkers + c0 * c->N * 3, cw, c->d_C, c->d_R, c->d_R, 0, 1, o, st, ks))) return rc;
        HIP_OK(c, vmcx::launch_set_shift(c->st_EL, cw, c->shift, c->shift_set, st));
        EstArgs a{c->st_EL, c->st_dEdR, c->st_dPdR, c->st_dJdR, c->st_O, c->st_G, c->shift,
                  nullptr,  nullptr,    nullptr,    A3,         Mn};
        if (f32) {
            a.Of = o.Of;
            a.Gf = o.Gf;
        }
        a.wt = wt ? wt + c0 : nullptr;
        if (c->xg_n > 0) {
            // the Jastrow-parameter sums of this launch (basis values again in
            // FP64: the measurement's may have been replaced by a promoted subset)
            HIP_OK(c, vmcx::launch_jas_values<double>(c->jdev, c->jtiles16, c->d_R, walkers + c0 * c->N * 3,
                                                      cw * c->N, c->xg_X, st));
            HIP_OK(c, vmcx::launch_xi_sums(c->xg_X, c->N, c->MJ, (int)cw, c->st_EL, c->shift, a.wt, c->xg_part,
                                           c->xg_scr, c->xg_acc, c->xg_comp, st));
        }
        HIP_OK(c, vmcx::launch_reduce(a, 0, c->n_est, cw, c->partial, MAX_SEG, c->acc, c->comp, blk, blkw, blk_all,
                                      st));
    }
    if (blk_idx < MAX_BLOCKS) {
        if ((int64_t)c->block_counts.size() <= blk_idx) c->block_counts.resize(blk_idx + 1, 0);
        c->block_counts[blk_idx] += W;
    }
    c->n_samples += W;
    c->sweeps_since_reset += 1;
    return VMC_OK;
}

// Device scratch of zvector_solve_noalloc: one copy of this array per GPU,
// held until the process ends.  Its name is a host-side stand-in; the device
// address of each GPU's copy comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is used.
constexpr int64_t NOALLOC_DOUBLES = int64_t(5) << 16;   // 2.5 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Address of the current device's copy of `scratch` (nullptr on failure).
static double *noalloc_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = (double *)ptr;
    }
    return g_scratch_ptr[dev];
}

static size_t ts_of(int precision) { return precision == VMC_MIXED ? sizeof(float) : sizeof(double); }

// Fold the GTO normalisation of a basis (coefficients of unit-normalised
// primitives; every cartesian component renormalised to unit norm) and upload
// its tables and AO tiles (whole shells of at most 16 AOs).  Shell counts,
// angular momenta and exponents have been validated.
static int upload_basis(vmc_ctx *c, const vmc_basis *basis, int A, vmcx::BasisDev &bd, AoTiles &tiles,
                        AoTiles *tiles32 = nullptr) {
    const int S = basis->n_shells;
    int P = 0;
    for (int s = 0; s < S; ++s) P += basis->shell_nprim[s];
    std::vector<int> ao_shell, ao_pow, shell_p0(S), shell_mu0(S);
    std::vector<double> ao_eta, cp(P);
    int p0 = 0;
    for (int s = 0; s < S; ++s) {
        const int l = basis->shell_l[s], np = basis->shell_nprim[s];
        shell_p0[s] = p0;
        shell_mu0[s] = (int)ao_shell.size();
        std::vector<double> cn(np);
        for (int k = 0; k < np; ++k) {
            const double al = basis->prim_exp[p0 + k];
            cn[k] = basis->prim_coef[p0 + k] * std::pow(2.0 * al / PI, 0.75) * std::pow(4.0 * al, 0.5 * l);
        }
        double ov = 0.0;
        for (int k = 0; k < np; ++k)
            for (int q = 0; q < np; ++q) {
                const double pp = basis->prim_exp[p0 + k] + basis->prim_exp[p0 + q];
                ov += cn[k] * cn[q] * std::pow(PI / pp, 1.5) / std::pow(2.0 * pp, l);
            }
        if (!(ov > 0.0)) return c->fail(VMC_EINVAL, "shell %d has zero norm", s);
        for (int k = 0; k < np; ++k) cp[p0 + k] = cn[k] / std::sqrt(ov);
        p0 += np;
        // cartesian components in order s; x,y,z; xx,xy,xz,yy,yz,zz
        static const int comps[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                         {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
        const int first = l == 0 ? 0 : (l == 1 ? 1 : 4);
        const int cnt = (l + 1) * (l + 2) / 2;
        for (int q = 0; q < cnt; ++q) {
            const int *cc = comps[first + q];
            ao_shell.push_back(s);
            ao_pow.push_back(cc[0] | (cc[1] << 4) | (cc[2] << 8));
            ao_eta.push_back(1.0 / std::sqrt((double)(dfact(2 * cc[0] - 1) * dfact(2 * cc[1] - 1) * dfact(2 * cc[2] - 1))));
        }
    }
    const int M = (int)ao_shell.size();
    // AO tiles: consecutive whole shells with at most mt AOs, as four arrays
    // (first shell, end shell, first AO, end AO)
    auto make_tiles = [&](int mt) {
        std::vector<int> tl;
        for (int s = 0; s < S;) {
            int s1 = s, cnt = 0;
            while (s1 < S && cnt + (basis->shell_l[s1] + 1) * (basis->shell_l[s1] + 2) / 2 <= mt) {
                cnt += (basis->shell_l[s1] + 1) * (basis->shell_l[s1] + 2) / 2;
                ++s1;
            }
            tl.push_back(s);
            tl.push_back(s1);
            tl.push_back(shell_mu0[s]);
            tl.push_back(s1 < S ? shell_mu0[s1] : M);
            s = s1;
        }
        const int n = (int)tl.size() / 4;
        std::vector<int> soa(4 * n);
        for (int t = 0; t < n; ++t)
            for (int k = 0; k < 4; ++k) soa[k * n + t] = tl[4 * t + k];
        return soa;
    };
    const std::vector<int> soa = make_tiles(16);
    const int nt = (int)soa.size() / 4;
    // the AOs of each atom (any shell order), for per-nucleus sums
    std::vector<int> atom_ao_ptr(A + 1, 0), atom_ao(M);
    for (int m = 0; m < M; ++m) ++atom_ao_ptr[basis->shell_atom[ao_shell[m]] + 1];
    for (int a = 0; a < A; ++a) atom_ao_ptr[a + 1] += atom_ao_ptr[a];
    {
        std::vector<int> fill(atom_ao_ptr.begin(), atom_ao_ptr.end() - 1);
        for (int m = 0; m < M; ++m) atom_ao[fill[basis->shell_atom[ao_shell[m]]]++] = m;
    }
    int *d_ao_shell, *d_ao_pow, *d_shell_atom, *d_shell_p0, *d_shell_np, *d_shell_l, *d_shell_mu0, *d_ptr, *d_aa,
        *d_tiles;
    double *d_eta, *d_exp, *d_cp;
    int rc;
    if ((rc = c->upload(&d_shell_l, (const int *)basis->shell_l, S)) ||
        (rc = c->upload(&d_shell_mu0, shell_mu0.data(), S)) || (rc = c->upload(&d_tiles, soa.data(), 4 * nt)) ||
        (rc = c->upload(&d_ptr, atom_ao_ptr.data(), A + 1)) || (rc = c->upload(&d_aa, atom_ao.data(), M)) ||
        (rc = c->upload(&d_ao_shell, ao_shell.data(), M)) || (rc = c->upload(&d_ao_pow, ao_pow.data(), M)) ||
        (rc = c->upload(&d_eta, ao_eta.data(), M)) ||
        (rc = c->upload(&d_shell_atom, (const int *)basis->shell_atom, S)) ||
        (rc = c->upload(&d_shell_p0, shell_p0.data(), S)) ||
        (rc = c->upload(&d_shell_np, (const int *)basis->shell_nprim, S)) ||
        (rc = c->upload(&d_exp, basis->prim_exp, P)) || (rc = c->upload(&d_cp, cp.data(), P)))
        return rc;
    bd = vmcx::BasisDev{M,           S,         d_ao_shell, d_ao_pow, d_eta,       d_shell_atom, d_shell_p0,
                        d_shell_np, d_exp,     d_cp,       d_shell_l, d_shell_mu0, d_ptr,        d_aa};
    tiles = AoTiles{d_tiles, d_tiles + nt, d_tiles + 2 * nt, d_tiles + 3 * nt, nt};
    if (tiles32) {
        const std::vector<int> s32 = make_tiles(32);
        const int n32 = (int)s32.size() / 4;
        int *d32;
        if ((rc = c->upload(&d32, s32.data(), 4 * n32))) return rc;
        *tiles32 = AoTiles{d32, d32 + n32, d32 + 2 * n32, d32 + 3 * n32, n32};
    }
    return VMC_OK;
}

// Validate a basis: shells on existing atoms, l <= VMC_MAX_L, >= 1
// primitive, finite exponents > 0 and finite coefficients.  Returns the
// number of cartesian functions (or a negative status).
static int check_basis(vmc_ctx *c, const vmc_basis *basis, int A, const char *what) {
    if (!basis || basis->n_shells < 1 || !basis->shell_atom || !basis->shell_l || !basis->shell_nprim ||
        !basis->prim_exp || !basis->prim_coef)
        return c->fail(VMC_EINVAL, "%s: missing arrays or no shells", what);
    int P = 0, M = 0;
    for (int s = 0; s < basis->n_shells; ++s) {
        const int l = basis->shell_l[s], np = basis->shell_nprim[s], at = basis->shell_atom[s];
        if (l < 0 || l > VMC_MAX_L) return c->fail(VMC_EINVAL, "%s shell %d: l = %d not supported", what, s, l);
        if (np < 1) return c->fail(VMC_EINVAL, "%s shell %d: %d primitives", what, s, np);
        if (at < 0 || at >= A) return c->fail(VMC_EINVAL, "%s shell %d: atom %d out of range", what, s, at);
        P += np;
        M += (l + 1) * (l + 2) / 2;
    }
    for (int k = 0; k < P; ++k) {
        if (!(basis->prim_exp[k] > 0.0) || !std::isfinite(basis->prim_exp[k]))
            return c->fail(VMC_EINVAL, "%s primitive %d: exponent %g must be finite and > 0", what, k,
                           basis->prim_exp[k]);
        if (!std::isfinite(basis->prim_coef[k]))
            return c->fail(VMC_EINVAL, "%s primitive %d: non-finite coefficient", what, k);
    }
    if (P >= 32768) return c->fail(VMC_EINVAL, "%s: %d primitives exceed 32767", what, P);
    return M;
}

// The one- and three/four-body Jastrow: its basis tables and [xi3 | xi1] in
// column blocks of 64 (block q holds columns 64 q .. 64 q + 63 of the
// MJ x (MJ + 1) matrix whose last column is xi1), FP64 and FP32.
// Pseudopotential: validation (host only), then the terms sorted by nucleus
// and uploaded (the staging is sized with the rest of the measurement's).
static int check_ecp(vmc_ctx *c, const vmc_ecp *e, int A) {
    const int T = e->n_terms;
    if (T < 1 || T > VMC_MAX_ECP_TERMS || !e->term_atom || !e->term_l || !e->term_n || !e->term_exp ||
        !e->term_coef || !e->rcut || e->max_pairs < 0)
        return c->fail(VMC_EINVAL, "pseudopotential: bad counts or missing arrays (%d terms)", T);
    for (int t = 0; t < T; ++t) {
        const int a = e->term_atom[t], l = e->term_l[t], n = e->term_n[t];
        if (a < 0 || a >= A || l < -1 || l > VMC_MAX_ECP_L || n < 1 || n > 4 || !(e->term_exp[t] > 0.0) ||
            !std::isfinite(e->term_exp[t]) || !std::isfinite(e->term_coef[t]))
            return c->fail(VMC_EINVAL, "pseudopotential term %d: nucleus %d, l %d, n %d, exponent %g", t, a, l, n,
                           e->term_exp[t]);
    }
    for (int a = 0; a < A; ++a)
        if (!(e->rcut[a] >= 0.0) || !std::isfinite(e->rcut[a]))
            return c->fail(VMC_EINVAL, "pseudopotential: bad cutoff %g of nucleus %d", e->rcut[a], a);
    return VMC_OK;
}

static int setup_ecp(vmc_ctx *c, const vmc_ecp *e, int A) {
    const int T = e->n_terms;
    int lmax = -1;
    for (int t = 0; t < T; ++t) lmax = std::max(lmax, (int)e->term_l[t]);
    std::vector<int> t0(A + 1, 0), tl, tn, nl;
    std::vector<double> ta, tb;
    for (int a = 0; a < A; ++a) {
        t0[a] = (int)tl.size();
        bool proj = false;
        for (int t = 0; t < T; ++t)
            if (e->term_atom[t] == a) {
                tl.push_back(e->term_l[t]);
                tn.push_back(e->term_n[t]);
                ta.push_back(e->term_exp[t]);
                tb.push_back(e->term_coef[t]);
                proj = proj || e->term_l[t] >= 0;
            }
        if (proj && e->rcut[a] > 0.0) nl.push_back(a);
    }
    t0[A] = (int)tl.size();
    if (nl.empty()) nl.push_back(0);   // (a valid pointer; n_nl below stays exact)
    vmcx::EcpDev &E = c->edev;
    int rc;
    int *d_t0 = nullptr, *d_tl = nullptr, *d_tn = nullptr, *d_nl = nullptr;
    double *d_ta = nullptr, *d_tb = nullptr, *d_rc = nullptr;
    if ((rc = c->upload(&d_t0, t0.data(), t0.size())) || (rc = c->upload(&d_tl, tl.data(), tl.size())) ||
        (rc = c->upload(&d_tn, tn.data(), tn.size())) || (rc = c->upload(&d_ta, ta.data(), ta.size())) ||
        (rc = c->upload(&d_tb, tb.data(), tb.size())) || (rc = c->upload(&d_rc, e->rcut, (size_t)A)) ||
        (rc = c->upload(&d_nl, nl.data(), nl.size())))
        return rc;
    int n_nl = 0;
    for (int a = 0; a < A; ++a) {
        bool proj = false;
        for (int t = 0; t < T; ++t) proj = proj || (e->term_atom[t] == a && e->term_l[t] >= 0);
        n_nl += (proj && e->rcut[a] > 0.0) ? 1 : 0;
    }
    E.n_nl = n_nl;
    E.nl_atom = d_nl;
    E.t0 = d_t0;
    E.t_l = d_tl;
    E.t_n = d_tn;
    E.t_alpha = d_ta;
    E.t_beta = d_tb;
    E.rcut = d_rc;
    E.lmax = lmax;
    E.seed = e->rot_seed;
    E.pcap = e->max_pairs > 0 ? e->max_pairs : std::max(1, c->N * n_nl);
    c->has_ecp = true;
    return VMC_OK;
}

static int setup_body_jastrow(vmc_ctx *c, const vmc_jastrow *jas, int A) {
    int rc;
    if ((rc = upload_basis(c, jas->jas_basis, A, c->jdev, c->jtiles16, &c->jtiles32))) return rc;
    const int MJ = c->MJ, nq = c->nq;
    std::vector<double> blk((size_t)nq * MJ * 64, 0.0);
    for (int q = 0; q < nq; ++q)
        for (int mu = 0; mu < MJ; ++mu)
            for (int i = 0; i < 64; ++i) {
                const int col = 64 * q + i;
                double v = 0.0;
                if (col < MJ)
                    v = jas->xi3 ? jas->xi3[(size_t)mu * MJ + col] : 0.0;
                else if (col == MJ)
                    v = jas->xi1 ? jas->xi1[mu] : 0.0;
                blk[((size_t)q * MJ + mu) * 64 + i] = v;
            }
    std::vector<float> blkf(blk.size());
    for (size_t k = 0; k < blk.size(); ++k) blkf[k] = (float)blk[k];
    std::vector<double> x1(MJ, 0.0);
    for (int mu = 0; mu < MJ; ++mu) x1[mu] = jas->xi1 ? jas->xi1[mu] : 0.0;
    if ((rc = c->upload(&c->d_xiblk, blk.data(), blk.size())) ||
        (rc = c->upload(&c->d_xiblk_f, blkf.data(), blkf.size())) || (rc = c->upload(&c->d_xi1, x1.data(), MJ)))
        return rc;
    return VMC_OK;
}

static int set_device(vmc_ctx *c) {
    HIP_OK(c, hipSetDevice(c->device));
    return VMC_OK;
}

extern "C" {

const char *vmc_strerror(int s) {
    switch (s) {
        case VMC_OK: return "VMC_OK";
        case VMC_EINVAL: return "VMC_EINVAL";
        case VMC_ENOMEM: return "VMC_ENOMEM";
        case VMC_EDEVICE: return "VMC_EDEVICE";
        case VMC_ESINGULAR: return "VMC_ESINGULAR";
        case VMC_ENOTCONV: return "VMC_ENOTCONV";
        case VMC_ENONFINITE: return "VMC_ENONFINITE";
        case VMC_ECAPACITY: return "VMC_ECAPACITY";
        default: return "VMC_UNKNOWN";
    }
}

const char *vmc_last_error(const vmc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void vmc_free(vmc_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    prof_clear(ctx);
    if (!ctx->allocs.empty()) {
        for (void *p : ctx->allocs) (void)hipFree(p);
    }
    delete ctx;
}

static thread_local std::string g_init_err;

int vmc_init(const vmc_basis *basis, const vmc_nuclei *nuclei, const vmc_mo *mo, const vmc_jastrow *jas,
             const vmc_options *opt, int32_t device, vmc_ctx **out) {
    if (!out) return VMC_EINVAL;
    *out = nullptr;
    if (!basis || !nuclei || !mo || !jas || !opt) return VMC_EINVAL;
    vmc_ctx *c = new (std::nothrow) vmc_ctx();
    if (!c) return VMC_ENOMEM;
    auto bail = [&](int rc) {
        *out = nullptr;
        g_init_err = c->err;
        vmc_free(c);
        return rc;
    };
    c->device = device;
    c->opt = *opt;
    const int S = basis ? basis->n_shells : 0, A = nuclei->n_atoms;
    if (A < 1 || A > VMC_MAX_ATOMS || !nuclei->xyz || !nuclei->Z || !mo->C)
        return bail(c->fail(VMC_EINVAL, "missing arrays or bad counts (atoms %d)", A));
    const int M = check_basis(c, basis, A, "basis");
    if (M < 0) return bail(M);
    int P = 0;
    for (int s = 0; s < S; ++s) P += basis->shell_nprim[s];
    if (M != mo->n_ao) return bail(c->fail(VMC_EINVAL, "n_ao = %d but the shells give %d AOs", mo->n_ao, M));
    if (M > VMC_MAX_AO) return bail(c->fail(VMC_EINVAL, "n_ao = %d exceeds %d", M, VMC_MAX_AO));
    if (mo->n_up != mo->n_dn || mo->n_up < 1 || mo->n_occ != mo->n_up)
        return bail(c->fail(VMC_EINVAL, "need a closed shell with n_up = n_dn = n_occ >= 1 (got %d, %d, %d)",
                            mo->n_up, mo->n_dn, mo->n_occ));
    if (mo->n_occ > VMC_MAX_OCC || mo->n_up + mo->n_dn > VMC_MAX_ELEC)
        return bail(c->fail(VMC_EINVAL, "n_occ = %d / N = %d exceed the limits", mo->n_occ, mo->n_up + mo->n_dn));
    if (!all_finite(nuclei->xyz, 3 * A) || !all_finite(nuclei->Z, A) || !all_finite(mo->C, (int64_t)M * mo->n_occ))
        return bail(c->fail(VMC_EINVAL, "non-finite nuclei or MO coefficients"));
    if (!std::isfinite(jas->ee_a) || !std::isfinite(jas->ee_F) || jas->ee_F < 0.0 ||
        (jas->ee_form != VMC_JASTROW_PADE && jas->ee_form != VMC_JASTROW_EXP) ||
        (jas->ee_form == VMC_JASTROW_EXP && !(jas->ee_F > 0.0)))
        return bail(c->fail(VMC_EINVAL, "bad Jastrow parameters"));
    if (jas->jas_basis) {
        const int MJ = check_basis(c, jas->jas_basis, A, "Jastrow basis");
        if (MJ < 0) return bail(MJ);
        if (MJ > VMC_MAX_JAS)
            return bail(c->fail(VMC_EINVAL, "%d Jastrow basis functions exceed %d", MJ, VMC_MAX_JAS));
        if ((jas->xi1 && !all_finite(jas->xi1, MJ)) || (jas->xi3 && !all_finite(jas->xi3, (int64_t)MJ * MJ)))
            return bail(c->fail(VMC_EINVAL, "non-finite Jastrow parameters"));
        if (jas->xi3)
            for (int a = 0; a < MJ; ++a)
                for (int b = 0; b < a; ++b)
                    if (jas->xi3[(size_t)a * MJ + b] != jas->xi3[(size_t)b * MJ + a])
                        return bail(c->fail(VMC_EINVAL, "xi3 is not symmetric (%d, %d)", a, b));
        c->MJ = MJ;
        c->nq = (MJ + 1 + 63) / 64;
    }
    if (opt->precision != VMC_FP64 && opt->precision != VMC_MIXED)
        return bail(c->fail(VMC_EINVAL, "precision %d not available (VMC_FP64 or VMC_MIXED)", opt->precision));
    if (opt->refresh_period < 1 || opt->block_sweeps < 1 || opt->max_walkers < 1 || opt->staging_walkers < 0 ||
        !(opt->step_sigma > 0.0) || !std::isfinite(opt->step_sigma) || !(opt->promote_fraction >= 0.0 && opt->promote_fraction <= 1.0) || opt->jackknife_blocks < 0 ||
        !(opt->forced_refresh_ratio >= 0.0) || !std::isfinite(opt->forced_refresh_ratio))
        return bail(c->fail(VMC_EINVAL, "bad options"));
    if (opt->ecp) {
        const int rc0 = check_ecp(c, opt->ecp, A);
        if (rc0) return bail(rc0);
    }
    double Zsum = 0.0;
    for (int a = 0; a < A; ++a) Zsum += nuclei->Z[a];
    c->N = mo->n_up + mo->n_dn;
    c->n_up = mo->n_up;
    c->n_dn = mo->n_dn;
    c->n_occ = mo->n_occ;
    c->M = M;
    c->A = A;
    c->S = S;
    c->P = P;
    c->ee_a = jas->ee_a;
    c->ee_F = jas->ee_F;
    c->ee_form = jas->ee_form;
    (void)Zsum;

    // ---- fold normalisation, upload the basis tables -----------------------
    int rc;
    if ((rc = set_device(c))) return bail(rc);
    if ((rc = upload_basis(c, basis, A, c->bdev, c->tiles16))) return bail(rc);
    if ((rc = c->upload(&c->d_C, mo->C, (size_t)M * c->n_occ)) || (rc = c->upload(&c->d_R, nuclei->xyz, 3 * A)) ||
        (rc = c->upload(&c->d_Z, nuclei->Z, A)))
        return bail(rc);
    if (opt->precision == VMC_MIXED) {
        std::vector<float> cf((size_t)M * c->n_occ);
        for (size_t k = 0; k < cf.size(); ++k) cf[k] = (float)mo->C[k];
        if ((rc = c->upload(&c->d_Cf, cf.data(), cf.size())) || (rc = c->dalloc(&c->d_Cm, cf.size())))
            return bail(rc);
    }
    if ((rc = c->dalloc(&c->d_cpad, (size_t)(std::max(M, c->MJ) + 16) * 64))) return bail(rc);
    if (c->MJ > 0 && (rc = setup_body_jastrow(c, jas, A))) return bail(rc);
    if (opt->ecp && (rc = setup_ecp(c, opt->ecp, A))) return bail(rc);

    SysDev &sd = c->sys;
    sd.N = c->N;
    sd.n_up = c->n_up;
    sd.n_dn = c->n_dn;
    sd.n_occ = c->n_occ;
    sd.M = M;
    sd.A = A;
    sd.ee_a = c->ee_a;
    sd.ee_F = c->ee_F;
    sd.ee_form = c->ee_form;
    sd.forced_ratio = opt->forced_refresh_ratio > 0.0 ? opt->forced_refresh_ratio : vmcx::FORCED_REFRESH_RATIO;
    sd.basis = c->bdev;
    sd.Z = c->d_Z;
    layouts(c);
    const bool mixed = opt->precision == VMC_MIXED;
    const size_t ts = mixed ? sizeof(float) : sizeof(double);
    // the occupancy query behind the sweep's block size needs the LDS limit
    // raised first
    if (vmcx::configure_sweep<double>(160 * 1024) != hipSuccess ||
        (mixed && vmcx::configure_sweep<float>(160 * 1024) != hipSuccess))
        return bail(c->fail(VMC_EDEVICE, "cannot raise the LDS limit of the sweep"));
    c->swl = sweep_layout(c, ts);
    c->al = adjoint_layout(c, ts);
    if (c->swl.bytes > 160 * 1024 || c->dl.bytes > 160 * 1024 || c->al.bytes > 160 * 1024)
        return bail(c->fail(VMC_EINVAL, "system too large for the LDS of one workgroup (%zu / %zu / %zu bytes)",
                            c->swl.bytes, c->dl.bytes, c->al.bytes));
    c->al64 = adjoint_layout(c, sizeof(double));
    if (c->al64.bytes > 160 * 1024)
        return bail(c->fail(VMC_EINVAL, "system too large for the LDS of one workgroup (%zu bytes)", c->al64.bytes));
    // the FP64 kernels are also the fallback of the mixed path.  Limits are
    // only raised (the largest size any context of the process has asked for),
    // so that contexts of different sizes in one process never lower each
    // other's; every launch passes its own size.
    bool cfg_ok;
    {
        static std::mutex mu;
        static size_t lim[7] = {0, 0, 0, 0, 0, 0, 0};
        std::lock_guard<std::mutex> lock(mu);
        const size_t need[7] = {c->dl.bytes, sweep_layout(c, sizeof(double)).bytes, c->al64.bytes,
                                c->dl.bytes, c->swl.bytes, c->al.bytes,
                                c->has_ecp ? vmcx::ecp_energy_lds(c->N, c->n_occ, c->MJ) : 0};
        for (int q = 0; q < 7; ++q) lim[q] = std::max(lim[q], need[q]);
        cfg_ok = vmcx::configure_dense<double>(lim[0]) == hipSuccess &&
                 vmcx::configure_sweep<double>(lim[1]) == hipSuccess &&
                 vmcx::configure_adjoint<double>(lim[2]) == hipSuccess &&
                 (lim[6] == 0 || vmcx::configure_ecp(lim[6]) == hipSuccess);
        if (mixed)
            cfg_ok = cfg_ok && vmcx::configure_dense<float>(lim[3]) == hipSuccess &&
                     vmcx::configure_sweep<float>(lim[4]) == hipSuccess &&
                     vmcx::configure_adjoint<float>(lim[5]) == hipSuccess;
    }
    if (!cfg_ok)
        return bail(c->fail(VMC_EDEVICE, "cannot raise the LDS limit of the kernels"));

    // ---- staging and accumulators -------------------------------------------
    const int64_t Mn = (int64_t)M * c->n_occ, A3 = 3 * A;
    const int64_t Nn = (int64_t)c->N * c->n_occ;
    // (with the one-/three-body Jastrow: its basis values with their
    // gradients and Laplacians, the value products with [xi3 | xi1], xi3 h,
    // gradient + Laplacian, per-function sums)
    const int64_t jas_pw = c->MJ > 0 ? 6 * (int64_t)c->N * c->MJ + (int64_t)c->nq * c->N * 64 + 4 * (int64_t)c->N +
                                           1 + 6 * (int64_t)c->MJ
                                     : 0;
    // (with a pseudopotential: its pairs, points, the MO rows and values kept
    // per point, and the per-nucleus derivative)
    const int64_t eq = c->has_ecp ? (int64_t)c->edev.pcap * 12 : 0;
    const int64_t ecp_pw = c->has_ecp ? eq * (3 + 5 * (int64_t)c->n_occ + vmcx::ECP_ROW) + A3 + 3 * M + c->edev.pcap + 2
                                      : 0;
    const int64_t xg_pw = (opt->jastrow_gradient && c->MJ > 0) ? (int64_t)(c->N + 1) * c->MJ : 0;
    const size_t per_walker = sizeof(double) * (size_t)(3 + 3 * A3 + 2 * Mn + 5 * Nn + 2 * Nn + 6 * c->N +
                                                        3 * (int64_t)c->N + 6 * M + 3 * c->N + jas_pw + ecp_pw +
                                                        xg_pw);
    int64_t chunk = (int64_t)(STAGING_BUDGET / per_walker);
    chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, opt->max_walkers));
    if (opt->staging_walkers > 0) chunk = std::min<int64_t>(chunk, opt->staging_walkers);
    c->chunk = chunk;
    if ((rc = c->dalloc(&c->st_EL, chunk)) || (rc = c->dalloc(&c->st_lnpsi, chunk)) ||
        (rc = c->dalloc(&c->st_lnjac, chunk)) || (rc = c->dalloc(&c->st_dEdR, chunk * A3)) ||
        (rc = c->dalloc(&c->st_dPdR, chunk * A3)) || (rc = c->dalloc(&c->st_dJdR, chunk * A3)) ||
        (rc = c->dalloc(&c->st_O, chunk * Mn)) || (rc = c->dalloc(&c->st_G, chunk * Mn)) ||
        (rc = c->dalloc(&c->mb_phi, chunk * 5 * Nn)) || (rc = c->dalloc(&c->mb_ktil, chunk * Nn)) ||
        (rc = c->dalloc(&c->mb_abar, chunk * Nn)) || (rc = c->dalloc(&c->mb_gb, chunk * 6 * c->N)) ||
        (rc = c->dalloc(&c->mb_dpart, chunk * 3 * (int64_t)c->N)) ||
        (rc = c->dalloc(&c->mb_tao, chunk * 6 * M)) || (rc = c->dalloc(&c->mb_posw, chunk * 3 * c->N)) ||
        (rc = c->dalloc((double **)&c->Amo, (size_t)opt->max_walkers * Nn)) ||
        (rc = c->dalloc((double **)&c->Phip, (size_t)opt->max_walkers * Nn * (opt->precision == VMC_MIXED ? 4 : 8) /
                                                 8 + 1)) ||
        (rc = c->dalloc(&c->prop, (size_t)opt->max_walkers * 3 * c->N)) ||
        (rc = c->dalloc((double **)&c->Kst, (size_t)opt->max_walkers * 2 * vmcx::sweep_kn(c->n_occ) *
                                                vmcx::sweep_kn(c->n_occ))) ||
        (rc = c->dalloc(&c->Ksig, (size_t)opt->max_walkers * 2 * vmcx::sweep_kn(c->n_occ))) ||
        (rc = c->dalloc(&c->Kstale, (size_t)opt->max_walkers * 2)))
        return bail(rc);
    if (c->MJ > 0) {
        // sweeps: values at the proposals and the current positions and the
        // [xi3 | xi1] products of their difference, in the arithmetic type;
        // measurements: FP64 sizes (the mixed path's FP64 re-measurement
        // reuses them)
        const size_t rows = (size_t)opt->max_walkers * c->N, tsz = ts_of(opt->precision);
        const size_t nx = (rows * c->MJ * tsz + 7) / 8, np = (rows * c->nq * 64 * tsz + 7) / 8;
        if ((rc = c->dalloc((double **)&c->js_Xp, nx)) || (rc = c->dalloc((double **)&c->js_X0, nx)) ||
            (rc = c->dalloc((double **)&c->js_Pd, np)) ||
            (rc = c->dalloc(&c->jm_X, (size_t)chunk * c->N * c->MJ)) ||
            (rc = c->dalloc(&c->jm_D, (size_t)chunk * c->N * 4 * c->MJ)) ||
            (rc = c->dalloc(&c->jm_V, (size_t)c->nq * chunk * c->N * 64)) ||
            (rc = c->dalloc(&c->jm_Q, (size_t)chunk * c->N * c->MJ)) ||
            (rc = c->dalloc(&c->jm_g, (size_t)chunk * c->N * 4)) || (rc = c->dalloc(&c->jm_u, (size_t)chunk)) ||
            (rc = c->dalloc(&c->jm_tao, (size_t)chunk * c->MJ * 6)))
            return bail(rc);
    }
    if (opt->jastrow_gradient && c->MJ > 0) {
        c->xg_n = 2 * (int64_t)c->MJ + 2 * (int64_t)c->MJ * c->MJ;
        if ((rc = c->dalloc(&c->xg_X, (size_t)chunk * c->N * c->MJ)) || (rc = c->dalloc(&c->xg_part, c->xg_n)) ||
            (rc = c->dalloc(&c->xg_scr, vmcx::xi_scratch_doubles((int)chunk, c->MJ))) ||
            (rc = c->dalloc(&c->xg_acc, c->xg_n)) || (rc = c->dalloc(&c->xg_comp, c->xg_n)))
            return bail(rc);
        if (hipMemset(c->xg_acc, 0, c->xg_n * 8) != hipSuccess || hipMemset(c->xg_comp, 0, c->xg_n * 8) != hipSuccess)
            return bail(c->fail(VMC_EDEVICE, "hipMemset failed"));
    }
    if (c->has_ecp) {
        if ((rc = c->dalloc(&c->e_pairs, (size_t)chunk * c->edev.pcap)) ||
            (rc = c->dalloc(&c->e_npairs, (size_t)chunk)) || (rc = c->dalloc(&c->e_off, (size_t)chunk)) ||
            (rc = c->dalloc(&c->e_nrows, 1)) || (rc = c->dalloc(&c->e_qpos, (size_t)chunk * eq * 3)) ||
            (rc = c->dalloc(&c->e_phiq, (size_t)chunk * eq * 5 * c->n_occ)) ||
            (rc = c->dalloc(&c->e_rows, (size_t)chunk * eq * vmcx::ECP_ROW)) ||
            (rc = c->dalloc(&c->e_dR, (size_t)chunk * A3)) || (rc = c->dalloc(&c->e_tc, (size_t)chunk * 3 * M)))
            return bail(rc);
    }
    if (opt->precision == VMC_MIXED && opt->promote_fraction > 0.0) {
        c->pcap = std::max<int64_t>(1, std::min<int64_t>(chunk, (int64_t)std::ceil(opt->promote_fraction * chunk)));
        const int64_t p = c->pcap;
        if ((rc = c->dalloc(&c->plist, chunk)) || (rc = c->dalloc(&c->pkey, chunk)) ||
            (rc = c->dalloc(&c->cp_pos, p * 3 * c->N)) || (rc = c->dalloc(&c->cp_pos0, p * 3 * c->N)) ||
            (rc = c->dalloc(&c->cp_EL, p)) || (rc = c->dalloc(&c->cp_lnpsi, p)) ||
            (rc = c->dalloc(&c->cp_dEdR, p * A3)) || (rc = c->dalloc(&c->cp_dPdR, p * A3)) ||
            (rc = c->dalloc(&c->cp_dJdR, p * A3)) || (rc = c->dalloc(&c->cp_O, p * Mn)) ||
            (rc = c->dalloc(&c->cp_G, p * Mn)))
            return bail(rc);
    }
    c->n_est = 3 + 3 * A3 + 3 * Mn;   // the last element: the sum of the weights
    const int64_t n_vjp = Mn + A3;
    if ((rc = c->dalloc(&c->acc, c->n_est)) || (rc = c->dalloc(&c->comp, c->n_est)) ||
        (rc = c->dalloc(&c->partial, MAX_SEG * std::max(c->n_est, n_vjp))) || (rc = c->dalloc(&c->shift, 1)) ||
        (rc = c->dalloc(&c->shift_set, 1)) || (rc = c->dalloc(&c->status, 1)) ||
        (rc = c->dalloc(&c->blocks, MAX_BLOCKS)) || (rc = c->dalloc(&c->blocks_w, MAX_BLOCKS)) || (rc = c->dalloc(&c->vjp_acc, n_vjp)) ||
        (rc = c->dalloc(&c->vjp_comp, n_vjp)) || (rc = c->dalloc(&c->vjp_out, n_vjp)))
        return bail(rc);
    if (opt->jackknife_blocks > 0) {
        c->jk_cap = std::min<int64_t>(opt->jackknife_blocks, 65535);
        if ((rc = c->dalloc(&c->blk_all, c->jk_cap * c->n_est)))
            return bail(rc);
        if (hipMemset(c->blk_all, 0, c->jk_cap * c->n_est * 8) != hipSuccess)
            return bail(c->fail(VMC_EDEVICE, "hipMemset failed"));
    }
    if (hipMemset(c->acc, 0, c->n_est * 8) != hipSuccess || hipMemset(c->comp, 0, c->n_est * 8) != hipSuccess ||
        hipMemset(c->shift, 0, 8) != hipSuccess || hipMemset(c->shift_set, 0, 4) != hipSuccess ||
        hipMemset(c->status, 0, 4) != hipSuccess || hipMemset(c->blocks, 0, MAX_BLOCKS * 8) != hipSuccess ||
        hipMemset(c->blocks_w, 0, MAX_BLOCKS * 8) != hipSuccess)
        return bail(c->fail(VMC_EDEVICE, "hipMemset failed"));
    *out = c;
    return VMC_OK;
}

int vmc_sweep(vmc_ctx *c, double *walkers, int64_t W, int32_t nsteps, uint64_t seed, uint64_t sweep_offset,
              uint32_t flags, uint8_t *accept, void *stream) {
    if (!c) return VMC_EINVAL;
    if (!walkers || W < 1 || W > c->opt.max_walkers || nsteps < 0)
        return c->fail(VMC_EINVAL, "bad arguments: walkers=%p n_walkers=%lld (max %d) nsteps=%d", (void *)walkers,
                       (long long)W, c->opt.max_walkers, nsteps);
    if (sweep_offset + (uint64_t)nsteps > 0xFFFFFFFFull)
        return c->fail(VMC_EINVAL, "sweep index beyond 2^32");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int t = 0; t < nsteps; ++t) {
        const uint32_t sidx = (uint32_t)(sweep_offset + t);
        uint8_t *acc_t = accept ? accept + (size_t)t * c->N * W : nullptr;
        if ((rc = c->opt.precision == VMC_MIXED
                      ? sweep_once<float>(c, walkers, W, t, sidx, seed, acc_t, c->d_Cf, st)
                      : sweep_once<double>(c, walkers, W, t, sidx, seed, acc_t, c->d_C, st)))
            return rc;
        if (!(flags & VMC_SWEEP_MEASURE)) continue;
        c->ecp_rot = sidx;
        rc = measure_accumulate(c, walkers, W, nullptr, true, st);
        c->ecp_rot = 0;
        if (rc) return rc;
    }
    return VMC_OK;
}

int vmc_jastrow_gradient(vmc_ctx *c, double *dE_dxi1, double *dE_dxi3, void *stream) {
    if (!c) return VMC_EINVAL;
    if (c->xg_n == 0)
        return c->fail(VMC_EINVAL, "no one-/three-body Jastrow terms, or options.jastrow_gradient off");
    if (c->n_samples < 1) return c->fail(VMC_EINVAL, "no samples accumulated");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = c->n_est, m = c->xg_n, MJ = c->MJ;
    std::vector<double> a(m), q(m);
    double e[2], ec[2], K[2];
    HIP_OK(c, hipMemcpyAsync(a.data(), c->xg_acc, m * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(q.data(), c->xg_comp, m * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(e, c->acc, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(ec, c->comp, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(K, c->acc + n - 1, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(K + 1, c->comp + n - 1, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
    // (element 0 of the estimator vector: the weighted sum of E_L - shift;
    // the last: the sum of the weights)
    const double W = K[0] + K[1];
    if (!(W > 0.0) || !std::isfinite(W)) return c->fail(VMC_EINVAL, "the sum of the weights is %g", W);
    const double vE = (e[0] + ec[0]) / W;
    auto v = [&](int64_t k) { return (a[k] + q[k]) / W; };
    if (dE_dxi1)
        for (int64_t mu = 0; mu < MJ; ++mu) dE_dxi1[mu] = 2.0 * (v(MJ + mu) - vE * v(mu));
    if (dE_dxi3)
        for (int64_t k = 0; k < MJ * MJ; ++k) dE_dxi3[k] = 2.0 * (v(2 * MJ + MJ * MJ + k) - vE * v(2 * MJ + k));
    return VMC_OK;
}

int vmc_accumulate(vmc_ctx *c, double *E, double *F, double *dEdC, double *dELdC, int64_t *n_samples,
                   uint32_t flags, void *stream) {
    if (!c) return VMC_EINVAL;
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (c->n_samples < 1) return c->fail(VMC_EINVAL, "no samples accumulated");
    const int64_t n = c->n_est, Mn = (int64_t)c->M * c->n_occ, A3 = 3 * c->A;
    std::vector<double> acc(n), comp(n);
    double shift = 0.0;
    int status = 0;
    const int64_t nb = std::min<int64_t>((int64_t)c->block_counts.size(), MAX_BLOCKS);
    std::vector<double> blocks(std::max<int64_t>(nb, 1)), blocks_w(std::max<int64_t>(nb, 1));
    HIP_OK(c, hipMemcpyAsync(acc.data(), c->acc, n * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(comp.data(), c->comp, n * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(&shift, c->shift, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(&status, c->status, 4, hipMemcpyDeviceToHost, st));
    if (nb > 0) HIP_OK(c, hipMemcpyAsync(blocks.data(), c->blocks, nb * 8, hipMemcpyDeviceToHost, st));
    if (nb > 0) HIP_OK(c, hipMemcpyAsync(blocks_w.data(), c->blocks_w, nb * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
    // normalisation: the sum of the weights (the sample count when all are 1)
    const double K = acc[n - 1] + comp[n - 1];
    if (!(K > 0.0) || !std::isfinite(K)) return c->fail(VMC_EINVAL, "the sum of the weights is %g", K);
    std::vector<double> v(n);
    for (int64_t i = 0; i < n; ++i) v[i] = (acc[i] + comp[i]) / K;
    const double vE = v[0];
    const double *vH = &v[2], *vP = &v[2 + A3], *vEP = &v[2 + 2 * A3];
    const double *vO = &v[2 + 3 * A3], *vEO = &v[2 + 3 * A3 + Mn], *vG = &v[2 + 3 * A3 + 2 * Mn];
    if (E) {
        E[0] = shift + vE;
        // blocked error bar over complete blocks
        int64_t full = (c->sweeps_since_reset / c->opt.block_sweeps);
        full = std::min(full, nb);
        if (full >= 2) {
            double mean = 0.0;
            std::vector<double> bm(full);
            for (int64_t b = 0; b < full; ++b) {
                bm[b] = blocks[b] / blocks_w[b];
                mean += bm[b];
            }
            mean /= (double)full;
            double var = 0.0;
            for (int64_t b = 0; b < full; ++b) var += (bm[b] - mean) * (bm[b] - mean);
            var /= (double)(full - 1);
            E[1] = std::sqrt(var / (double)full);
        } else {
            E[1] = std::nan("");
        }
    }
    if (F)
        for (int64_t i = 0; i < A3; ++i) F[i] = -vH[i] - 2.0 * (vEP[i] - vE * vP[i]);
    if (dEdC)
        for (int64_t i = 0; i < Mn; ++i) dEdC[i] = 2.0 * (vEO[i] - vE * vO[i]);
    if (dELdC)
        for (int64_t i = 0; i < Mn; ++i) dELdC[i] = vG[i];
    if (n_samples) *n_samples = c->n_samples;
    if (flags & VMC_ACCUM_RESET) {
        HIP_OK(c, hipMemsetAsync(c->acc, 0, n * 8, st));
        HIP_OK(c, hipMemsetAsync(c->comp, 0, n * 8, st));
        HIP_OK(c, hipMemsetAsync(c->shift_set, 0, 4, st));
        HIP_OK(c, hipMemsetAsync(c->status, 0, 4, st));
        HIP_OK(c, hipMemsetAsync(c->blocks, 0, MAX_BLOCKS * 8, st));
        HIP_OK(c, hipMemsetAsync(c->blocks_w, 0, MAX_BLOCKS * 8, st));
        if (c->jk_cap) HIP_OK(c, hipMemsetAsync(c->blk_all, 0, c->jk_cap * n * 8, st));
        if (c->xg_n) {
            HIP_OK(c, hipMemsetAsync(c->xg_acc, 0, c->xg_n * 8, st));
            HIP_OK(c, hipMemsetAsync(c->xg_comp, 0, c->xg_n * 8, st));
        }
        HIP_OK(c, hipStreamSynchronize(st));
        c->block_counts.clear();
        c->n_samples = 0;
        c->sweeps_since_reset = 0;
    }
    if (status & vmcx::STATUS_SINGULAR) return c->fail(VMC_ESINGULAR, "a Slater block was singular to working precision");
    if (status & vmcx::STATUS_NONFINITE) return c->fail(VMC_ENONFINITE, "non-finite local energy or ln|Psi|");
    if (status & vmcx::STATUS_CAPACITY)
        return c->fail(VMC_ECAPACITY, "a measurement launch had more pseudopotential pairs than its capacity (%d per "
                                      "walker)", c->edev.pcap);
    return VMC_OK;
}

int vmc_accumulate_walkers(vmc_ctx *c, const double *walkers, int64_t W, const double *weights, void *stream) {
    if (!c) return VMC_EINVAL;
    if (!walkers || W < 1 || W > c->opt.max_walkers)
        return c->fail(VMC_EINVAL, "bad arguments: walkers=%p n_walkers=%lld (max %d)", (void *)walkers,
                       (long long)W, c->opt.max_walkers);
    int rc;
    if ((rc = set_device(c))) return rc;
    return measure_accumulate(c, walkers, W, weights, false, (hipStream_t)stream);
}

int vmc_jackknife(vmc_ctx *c, double *E_jk, double *F_jk, double *dEdC_jk, int64_t *n_blocks, void *stream) {
    if (!c) return VMC_EINVAL;
    if (!c->jk_cap) return c->fail(VMC_EINVAL, "vmc_jackknife: the context keeps no block sums (jackknife_blocks = 0)");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    int64_t nb = std::min<int64_t>(c->sweeps_since_reset / c->opt.block_sweeps, c->jk_cap);
    nb = std::min<int64_t>(nb, (int64_t)c->block_counts.size());
    if (n_blocks) *n_blocks = nb;
    if (!E_jk && !F_jk && !dEdC_jk) return VMC_OK;
    if (nb < 2) return c->fail(VMC_EINVAL, "vmc_jackknife: %lld complete blocks (need 2)", (long long)nb);
    HIP_OK(c, vmcx::launch_jackknife(c->blk_all, (int)nb, c->n_est, 3 * c->A, (int64_t)c->M * c->n_occ, c->shift,
                                     E_jk, F_jk, dEdC_jk, st));
    HIP_OK(c, hipStreamSynchronize(st));
    return VMC_OK;
}

int vmc_measure(vmc_ctx *c, const double *walkers, int64_t W, const double *C, const double *R, const double *R0,
                const vmc_walker_out *out, void *stream) {
    if (!c) return VMC_EINVAL;
    if (!walkers || !C || !R || !R0 || !out || W < 1)
        return c->fail(VMC_EINVAL, "vmc_measure: null argument or n_walkers < 1");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int full = (out->dEL_dR || out->dlnpsi_dR || out->dlnjac_dR || out->O || out->G) ? 1 : 0;
    const int warp = (R != R0) ? 1 : 0;
    const int64_t Mn = (int64_t)c->M * c->n_occ, A3 = 3 * c->A;
    const int64_t step = chunk_len(c, W);
    for (int64_t c0 = 0; c0 < W; c0 += step) {
        const int64_t cw = std::min(step, W - c0);
        auto off = [&](double *p, int64_t stride) { return p ? p + c0 * stride : nullptr; };
        WalkerOut o{off(out->EL, 1),      off(out->lnpsi, 1),  off(out->lnjac, 1),
                    off(out->dEL_dR, A3), off(out->dlnpsi_dR, A3), off(out->dlnjac_dR, A3),
                    off(out->O, Mn),      off(out->G, Mn)};
        c->ecp_id0 = c0;
        if ((rc = run_measure(c, walkers + c0 * c->N * 3, cw, C, R, R0, warp, full, o, st))) return rc;
    }
    return VMC_OK;
}

int vmc_eval(vmc_ctx *c, const double *walkers, int64_t W, const double *C, const double *R, const double *R0,
             const double *lnpsi0, double *EL, double *lnpsi, double *lnjac, double *wnorm, double *Ehat,
             void *stream) {
    if (!c) return VMC_EINVAL;
    if (!EL || !lnpsi || !lnjac) return c->fail(VMC_EINVAL, "vmc_eval: EL, lnpsi and lnjac are required");
    vmc_walker_out o{EL, lnpsi, lnjac, nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = vmc_measure(c, walkers, W, C, R, R0, &o, stream);
    if (rc) return rc;
    if (lnpsi0) {
        if (!wnorm || !Ehat) return c->fail(VMC_EINVAL, "vmc_eval: wnorm and Ehat are required with lnpsi0");
        HIP_OK(c, vmcx::launch_eval_weights(EL, lnpsi, lnjac, lnpsi0, W, wnorm, Ehat, (hipStream_t)stream));
    }
    return VMC_OK;
}

int vmc_energy_cotangents(vmc_ctx *c, int64_t W, double gE, const double *EL, const double *wnorm,
                          const double *Ehat, double *gEL, double *gPsi, double *gJac, void *stream) {
    if (!c) return VMC_EINVAL;
    if (W < 1 || !EL || !wnorm || !Ehat || !gEL || !gPsi || !gJac)
        return c->fail(VMC_EINVAL, "vmc_energy_cotangents: bad arguments");
    int rc;
    if ((rc = set_device(c))) return rc;
    HIP_OK(c, vmcx::launch_energy_cotangents(W, gE, EL, wnorm, Ehat, gEL, gPsi, gJac, (hipStream_t)stream));
    return VMC_OK;
}

int vmc_adjoint(vmc_ctx *c, const double *walkers, int64_t W, const double *C, const double *R, const double *R0,
                const double *gEL, const double *gPsi, const double *gJac, double *dC, double *dR, void *stream) {
    if (!c) return VMC_EINVAL;
    if (!walkers || !C || !R || !R0 || !gEL || !gPsi || !gJac || !dC || !dR || W < 1)
        return c->fail(VMC_EINVAL, "vmc_adjoint: null argument or n_walkers < 1");
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t Mn = (int64_t)c->M * c->n_occ, A3 = 3 * c->A, nv = Mn + A3;
    HIP_OK(c, hipMemsetAsync(c->vjp_acc, 0, nv * 8, st));
    HIP_OK(c, hipMemsetAsync(c->vjp_comp, 0, nv * 8, st));
    const int warp = (R != R0) ? 1 : 0;
    const int64_t step = chunk_len(c, W);
    for (int64_t c0 = 0; c0 < W; c0 += step) {
        const int64_t cw = std::min(step, W - c0);
        WalkerOut o{c->st_EL, c->st_lnpsi, c->st_lnjac, c->st_dEdR, c->st_dPdR, c->st_dJdR, c->st_O, c->st_G};
        c->ecp_id0 = c0;
        if ((rc = run_measure(c, walkers + c0 * c->N * 3, cw, C, R, R0, warp, 1, o, st))) return rc;
        EstArgs a{c->st_EL, c->st_dEdR, c->st_dPdR, c->st_dJdR, c->st_O, c->st_G, nullptr,
                  gEL + c0, gPsi + c0,  gJac + c0,  A3,         Mn};
        HIP_OK(c, vmcx::launch_reduce(a, 1, nv, cw, c->partial, MAX_SEG, c->vjp_acc, c->vjp_comp, nullptr, nullptr,
                                      nullptr,
                                      st));
    }
    HIP_OK(c, vmcx::launch_combine(c->vjp_acc, c->vjp_comp, nv, c->vjp_out, st));
    HIP_OK(c, hipMemcpyAsync(dC, c->vjp_out, Mn * 8, hipMemcpyDeviceToDevice, st));
    HIP_OK(c, hipMemcpyAsync(dR, c->vjp_out + Mn, A3 * 8, hipMemcpyDeviceToDevice, st));
    return VMC_OK;
}

// One CG solve (device state; batches of iterations between host reads).
static int cg_one(const double *H, int64_t d, const double *b, double *z, double rtol, int32_t maxit, uint32_t flags,
                  int32_t *iters, double *work, hipStream_t st) {
    const int nb = vmcx::cg_matvec_blocks(d);
    double *r = work, *p = r + d, *Hp = p + d, *dinv = Hp + d, *part = dinv + d;
    vmcx::CgState *cs = (vmcx::CgState *)(part + nb);
    vmcx::CgState hs{};
    bool ok = vmcx::launch_cg_setup(H, b, d, 1, (flags & ZVECTOR_JACOBI) ? 1 : 0, rtol, maxit, z, r, p, dinv, cs,
                                    st) == hipSuccess;
    const int batch = 8;
    while (ok) {
        ok = hipMemcpyAsync(&hs, cs, sizeof(hs), hipMemcpyDeviceToHost, st) == hipSuccess &&
             hipStreamSynchronize(st) == hipSuccess;
        if (!ok || hs.done) break;
        for (int k = 0; ok && k < batch; ++k)
            ok = vmcx::launch_cg_iteration(H, d, z, r, p, Hp, dinv, part, cs, st) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        return VMC_EDEVICE;
    }
    if (iters) *iters = hs.it;
    if (hs.done == vmcx::CG_NONFINITE) return VMC_ENONFINITE;
    return hs.done == vmcx::CG_CONVERGED ? VMC_OK : VMC_ENOTCONV;
}

// Up to 64 CG solves in lockstep, every read of H shared by all of them; each
// right-hand side keeps its own step lengths and stopping test.
static int cg_batch(const double *H, int64_t d, int nrhs, const double *b, double *z, double rtol, int32_t maxit,
                    uint32_t flags, int32_t *iters, hipStream_t st) {
    const size_t vec = (size_t)nrhs * d;
    const size_t n = 3 * vec + (size_t)vmcx::cgb_ksplit(d) * vec;
    void *work = nullptr;
    if (hipMalloc(&work, n * sizeof(double) + nrhs * sizeof(vmcx::CgState)) != hipSuccess) {
        (void)hipGetLastError();
        return VMC_ENOMEM;
    }
    double *R = (double *)work, *P = R + vec, *Dinv = P + vec, *HPp = Dinv + vec;
    vmcx::CgState *cs = (vmcx::CgState *)(HPp + (size_t)vmcx::cgb_ksplit(d) * vec);
    std::vector<vmcx::CgState> hs(nrhs);
    bool ok = vmcx::launch_cg_setup(H, b, d, nrhs, (flags & ZVECTOR_JACOBI) ? 1 : 0, rtol, maxit, z, R, P, Dinv, cs,
                                    st) == hipSuccess;
    const int batch = 8;
    while (ok) {
        ok = hipMemcpyAsync(hs.data(), cs, nrhs * sizeof(vmcx::CgState), hipMemcpyDeviceToHost, st) == hipSuccess &&
             hipStreamSynchronize(st) == hipSuccess;
        bool all = true;
        for (const auto &h : hs) all = all && h.done;
        if (!ok || all) break;
        for (int k = 0; ok && k < batch; ++k)
            ok = vmcx::launch_cgb_iteration(H, d, nrhs, z, R, P, HPp, Dinv, cs, st) == hipSuccess;
    }
    if (!ok) (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    (void)hipFree(work);
    if (!ok) return VMC_EDEVICE;
    int status = VMC_OK;
    for (int k = 0; k < nrhs; ++k) {
        if (iters) iters[k] = hs[k].it;
        const int rc = hs[k].done == vmcx::CG_NONFINITE ? VMC_ENONFINITE
                       : hs[k].done == vmcx::CG_CONVERGED ? VMC_OK
                                                          : VMC_ENOTCONV;
        if (rc != VMC_OK && status == VMC_OK) status = rc;
    }
    return status;
}

int zvector_solve(const double *H, int64_t d, int64_t n_rhs, const double *b, double *z, double rtol, int32_t maxit,
                  uint32_t flags, int32_t *iters, void *stream) {
    if (!H || !b || !z || d < 1 || n_rhs < 1 || !(rtol > 0.0) || maxit < 1 || (flags & ~(uint32_t)ZVECTOR_JACOBI))
        return VMC_EINVAL;
    if (iters)
        for (int64_t k = 0; k < n_rhs; ++k) iters[k] = 0;
    hipStream_t st = (hipStream_t)stream;
    if (n_rhs > 1) {
        // groups of up to 64 right-hand sides share the reads of H
        int status = VMC_OK;
        for (int64_t k0 = 0; k0 < n_rhs; k0 += 64) {
            const int g = (int)std::min<int64_t>(64, n_rhs - k0);
            const int rc = cg_batch(H, d, g, b + k0 * d, z + k0 * d, rtol, maxit, flags, iters ? iters + k0 : nullptr,
                                    st);
            if (rc != VMC_OK && status == VMC_OK) status = rc;
            if (rc == VMC_EDEVICE || rc == VMC_ENOMEM) break;
        }
        return status;
    }
    // r, p, Hp, dinv, the matvec partials, then the iteration state
    const size_t nwork = 4 * (size_t)d + (size_t)vmcx::cg_matvec_blocks(d);
    void *work = nullptr;
    if (hipMalloc(&work, nwork * sizeof(double) + sizeof(vmcx::CgState)) != hipSuccess) {
        (void)hipGetLastError();
        return VMC_ENOMEM;
    }
    int status = VMC_OK;
    for (int64_t k = 0; k < n_rhs; ++k) {
        const int rc = cg_one(H, d, b + k * d, z + k * d, rtol, maxit, flags, iters ? iters + k : nullptr,
                              (double *)work, st);
        // the first failure decides the status; a device error stops at once
        if (rc != VMC_OK && status == VMC_OK) status = rc;
        if (rc == VMC_EDEVICE) break;
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(work);
    return status;
}

int zvector_solve_noalloc(const double *H, int64_t d, int64_t n_rhs, const double *b, double *z, double rtol,
                          int32_t maxit, uint32_t flags, int32_t *iters, void *stream) {
    if (!H || !b || !z || d < 1 || n_rhs < 1 || !(rtol > 0.0) || maxit < 1 || (flags & ~(uint32_t)ZVECTOR_JACOBI))
        return VMC_EINVAL;
    // r, p, Hp, dinv, the matvec partials, then the iteration state
    const int64_t need = 4 * d + vmcx::cg_matvec_blocks(d) +
                         (int64_t)((sizeof(vmcx::CgState) + sizeof(double) - 1) / sizeof(double));
    if (d > ZVECTOR_NOALLOC_MAX_D || need > NOALLOC_DOUBLES) return VMC_EINVAL;
    if (iters)
        for (int64_t k = 0; k < n_rhs; ++k) iters[k] = 0;
    double *work = noalloc_scratch();
    if (!work) return VMC_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    // every scratch value is written by the setup kernel before it is read,
    // so what the last call left there does not matter
    int status = VMC_OK;
    for (int64_t k = 0; k < n_rhs; ++k) {
        const int rc = cg_one(H, d, b + k * d, z + k * d, rtol, maxit, flags, iters ? iters + k : nullptr, work, st);
        if (rc != VMC_OK && status == VMC_OK) status = rc;
        if (rc == VMC_EDEVICE) break;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return VMC_EDEVICE;
    }
    return status;
}

int zvector_rhs(const double *Cv, int64_t n_ao, int64_t n_virt, int64_t n_occ, int64_t n_batch, const double *dEdC,
                double *b, void *stream) {
    if (!Cv || !dEdC || !b || n_ao < 1 || n_virt < 1 || n_occ < 1 || n_batch < 1 || n_batch > 65535)
        return VMC_EINVAL;
    if (vmcx::launch_zv_rhs(Cv, dEdC, n_ao, n_virt, n_occ, n_batch, b, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return VMC_EDEVICE;
    }
    return VMC_OK;
}

int zvector_backmap(const double *Cv, int64_t n_ao, int64_t n_virt, int64_t n_occ, int64_t n_batch, const double *z,
                    double *Z, void *stream) {
    if (!Cv || !z || !Z || n_ao < 1 || n_virt < 1 || n_occ < 1 || n_batch < 1 || n_batch > 65535)
        return VMC_EINVAL;
    if (vmcx::launch_zv_backmap(Cv, z, n_ao, n_virt, n_occ, n_batch, Z, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return VMC_EDEVICE;
    }
    return VMC_OK;
}

int zvector_jackknife(const double *x_jk, int64_t n_blocks, int64_t len, double *mean, double *sigma, void *stream) {
    if (!x_jk || n_blocks < 2 || len < 1 || (!mean && !sigma)) return VMC_EINVAL;
    if (vmcx::launch_jackknife_stats(x_jk, n_blocks, len, mean, sigma, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return VMC_EDEVICE;
    }
    return VMC_OK;
}

int vmc_profile(vmc_ctx *c, int32_t enable) {
    if (!c) return VMC_EINVAL;
    int rc;
    if ((rc = set_device(c))) return rc;
    prof_clear(c);
    c->prof = enable != 0;
    return VMC_OK;
}

int vmc_profile_read(vmc_ctx *c, int32_t kernel, double *ms, int64_t *launches, int64_t *walkers) {
    if (!c) return VMC_EINVAL;
    if (kernel < 0 || kernel >= VMC_N_PROFILED)
        return c->fail(VMC_EINVAL, "vmc_profile_read: unknown kernel %d", kernel);
    int rc;
    if ((rc = set_device(c))) return rc;
    double tot = 0.0;
    int64_t nw = 0;
    for (const auto &r : c->prof_recs[kernel]) {
        float e = 0.f;
        HIP_OK(c, hipEventSynchronize(r.b));
        HIP_OK(c, hipEventElapsedTime(&e, r.a, r.b));
        tot += e;
        nw += r.walkers;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (int64_t)c->prof_recs[kernel].size();
    if (walkers) *walkers = nw;
    return VMC_OK;
}

const char *vmc_init_error(void) { return g_init_err.c_str(); }

int64_t vmc_staging_walkers(const vmc_ctx *c) { return c ? c->chunk : -1; }

}  // extern "C"
