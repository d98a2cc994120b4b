// vmc_jastrow.hip -- one-body and three/four-body Jastrow terms on a Jastrow
// GTO basis chi_mu (gfx950).
//
//   U1 = sum_i xi1 . chi(r_i)                            (eq. onebody_J_inhom)
//   U3 = sum_{i<j} chi(r_i)^T xi3 chi(r_j)               (eq. threebody_jas)
//
// With s = sum_i chi(r_i) and the [xi3 | xi1] products of the derivative
// components D_c of chi at each electron, O_c[e] = D_c chi(r_e)^T [xi3 | xi1]
// (MJ + 1 columns, formed on the matrix cores by k_mo_rows_mfma with the
// Jastrow basis in column blocks of 64; xi3 is symmetric):
//   grad_e U = O_grad[e] . (s - chi_e)  + O_grad[e][MJ],
//   lap_e U  = O_lap[e]  . (s - chi_e)  + O_lap[e][MJ],
//   U        = sum_e [ O_val[e] . (s - chi_e) / 2 + O_val[e][MJ] ],
// where a . b runs over the MJ basis functions.
//
// Reverse mode (forces): with the total Jastrow gradient G_e and the
// determinant gradient b_e, E_L depends on grad_e U through
// abar_e = -(G_e + b_e) and on lap_e U through -1/2.  With
//   g_e = xi1 + xi3 (s - chi_e)               (the coefficient vector of e),
//   h_e = grad chi_e abar_e - lap chi_e / 2   (dE_L / dg_e),
//   q_e = xi3 (sum_j h_j - h_e)               (dE_L / dchi_e through the g_j),
// where xi3 h_e = sum_d abar_e,d O_d[e] - O_lap[e] / 2 comes from the same
// products, the explicit dependence on r_e is
//   dE_L/dr_e = sum_mu [ q_e,mu grad chi_mu + g_e,mu (hess chi_mu) abar_e
//                        - g_e,mu grad(lap chi_mu) / 2 ](r_e),
//   dlnPsi/dr_e (Jastrow) = sum_mu g_e,mu grad chi_mu(r_e),
// and a function centred on nucleus alpha moves with it, so its terms enter
// dE_L/dR_alpha and dlnPsi/dR_alpha with the opposite sign (per-function
// sums over electrons, added per nucleus by k_finalize).
#include "vmc_pipeline.hpp"

namespace vmcx {

constexpr int JAS_MAX = 256;   // Jastrow basis functions
constexpr int JAS_ELEC = 128;  // electrons

// out[row][mu] = chi_mu(pos[row]) for the rows' positions; one block per
// (64 rows, shell): the shell index is uniform over the block.
template <typename T>
__global__ __launch_bounds__(64) void k_jas_values(BasisDev JB, const double *__restrict__ R,
                                                   const double *__restrict__ pos, int64_t rows,
                                                   T *__restrict__ out) {
    const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int s = blockIdx.y;
    if (row >= rows) return;
    const double *p = pos + 3 * row;
    T v[6];
    const int cnt = shell_eval_to<1, T>(JB, R, s, p[0], p[1], p[2], v);
    T *o = out + row * JB.n_ao + ldc(JB.shell_mu0 + s);
    for (int q = 0; q < cnt; ++q) o[q] = v[q];
}

// Per walker: grad_e U, lap_e U (jg[w][e][0..3]) and U (ju[w]), FP64 sums.
// X[row][MJ]: chi values; O: nq blocks of [rows][5][64] (value, gradient,
// Laplacian products with [xi3 | xi1]).
template <typename T>
__global__ __launch_bounds__(256) void k_jas_assemble(int N, int MJ, int nq, int64_t rows, int64_t row0,
                                                      const T *__restrict__ X, const T *__restrict__ O,
                                                      double *__restrict__ jg, double *__restrict__ ju) {
    __shared__ double sv[JAS_MAX];
    __shared__ double ue[JAS_ELEC];
    const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T *Xw = X + (size_t)w * N * MJ;
    for (int mu = tid; mu < MJ; mu += 256) {
        double a = 0.0;
        for (int e = 0; e < N; ++e) a += (double)Xw[(size_t)e * MJ + mu];
        sv[mu] = a;
    }
    __syncthreads();
    for (int e = wave; e < N; e += 4) {
        const int64_t row = row0 + (int64_t)w * N + e;
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < nq; ++q) {
            const int mu = 64 * q + lane;
            // weights of the products: s - chi_e for the xi3 columns, 1 for
            // the xi1 column, 0 past it (zero columns of the block)
            const double d = mu < MJ ? sv[mu] - (double)Xw[(size_t)e * MJ + mu] : (mu == MJ ? 1.0 : 0.0);
            const double dv = mu < MJ ? 0.5 * d : d;
            const T *o = O + ((size_t)q * rows + row) * 5 * 64 + lane;
            acc[0] += (double)o[0] * dv;
#pragma unroll
            for (int c = 1; c < 5; ++c) acc[c] += (double)o[c * 64] * d;
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) acc[c] = wave_sum_dpp(acc[c]);
        if (lane == 0) {
            double *g = jg + ((size_t)w * N + e) * 4;
            g[0] = acc[1];
            g[1] = acc[2];
            g[2] = acc[3];
            g[3] = acc[4];
            ue[e] = acc[0];
        }
    }
    __syncthreads();
    if (tid == 0) {
        double u = 0.0;
        for (int e = 0; e < N; ++e) u += ue[e];
        ju[w] = u;
    }
}

// The 14 derivative components (value, gradient, Laplacian, Hessian,
// gradient of the Laplacian) of Jastrow function mu at (x, y, z).
template <typename T>
__device__ inline void jas_function14(const BasisDev &JB, const double *R, int mu, double x, double y, double z,
                                      T *c) {
    const int s = JB.ao_shell[mu];
    const int atom = JB.shell_atom[s];
    const double dx = x - R[3 * atom], dy = y - R[3 * atom + 1], dz = z - R[3 * atom + 2];
    const double rho_d = dx * dx + dy * dy + dz * dz;
    const int p0 = JB.shell_p0[s], np = JB.shell_np[s];
    T R0 = T(0), R1 = T(0), R2 = T(0), R3 = T(0);
    for (int k = 0; k < np; ++k) {
        const T al = (T)JB.prim_exp[p0 + k];
        const T e = (T)JB.prim_cp[p0 + k] * exp_neg((double)al, rho_d, T(0));
        R0 += e;
        R1 -= al * e;
        R2 += al * al * e;
        R3 -= al * al * al * e;
    }
    ao_components<14, T>((T)dx, (T)dy, (T)dz, (T)rho_d, R0, R1, R2, R3, JB.ao_pow[mu], (T)JB.ao_eta[mu], c);
}

// dE_L/dr_e and dlnPsi/dr_e contributions of function mu at electron e.
struct JasTerm {
    double f[3], p[3];
};

template <typename T>
__device__ inline JasTerm jas_term(const BasisDev &JB, const double *R, int mu, const double *pe, const double *ab,
                                   double g, double q) {
    T c[14];
    jas_function14<T>(JB, R, mu, pe[0], pe[1], pe[2], c);
    JasTerm o;
    const double hs[3][3] = {{(double)c[5], (double)c[6], (double)c[7]},
                             {(double)c[6], (double)c[8], (double)c[9]},
                             {(double)c[7], (double)c[9], (double)c[10]}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double ha = hs[k][0] * ab[0] + hs[k][1] * ab[1] + hs[k][2] * ab[2];
        o.f[k] = q * (double)c[1 + k] + g * ha - 0.5 * g * (double)c[11 + k];
        o.p[k] = g * (double)c[1 + k];
    }
    return o;
}

// Per walker: adds the Jastrow terms' dE_L/dr_e to dedr[w][e] and writes the
// per-function electron sums jtao[w][mu] = (sum_e f, sum_e p).  pos: the
// evaluation positions; gb[w][e]: total Jastrow gradient (0..2) and
// determinant gradient (3..5).
template <typename T>
__global__ __launch_bounds__(256) void k_jas_adjoint(BasisDev JB, const double *__restrict__ R, int N, int MJ, int nq,
                                                     int64_t rows, int64_t row0, const double *__restrict__ pos,
                                                     const T *__restrict__ X, const T *__restrict__ O,
                                                     const double *__restrict__ gb, const double *__restrict__ xi1,
                                                     double *__restrict__ dedr, double *__restrict__ jtao) {
    __shared__ double tv[JAS_MAX], xh[JAS_MAX];
    __shared__ double ab[JAS_ELEC * 3], pe[JAS_ELEC * 3];
    __shared__ double half0[JAS_ELEC * 3], half1[JAS_ELEC * 3];
    const int w = blockIdx.x, tid = threadIdx.x;
    const T *Xw = X + (size_t)w * N * MJ;
    // element (e, c, mu) of the products
    auto Oat = [&](int e, int c, int mu) -> double {
        const int q = mu >> 6;
        return (double)O[(((size_t)q * rows + row0 + (size_t)w * N + e) * 5 + c) * 64 + (mu & 63)];
    };
    for (int i = tid; i < 3 * N; i += 256) {
        const int e = i / 3, d = i - 3 * (i / 3);
        ab[i] = -(gb[((size_t)w * N + e) * 6 + d] + gb[((size_t)w * N + e) * 6 + 3 + d]);
        pe[i] = pos[(size_t)w * N * 3 + i];
    }
    __syncthreads();
    (void)Xw;
    // t = xi3 s (the value products summed over electrons) and xi3 H
    for (int mu = tid; mu < MJ; mu += 256) {
        double t = 0.0, h = 0.0;
        for (int e = 0; e < N; ++e) {
            t += Oat(e, 0, mu);
            h += ab[3 * e] * Oat(e, 1, mu) + ab[3 * e + 1] * Oat(e, 2, mu) + ab[3 * e + 2] * Oat(e, 3, mu) -
                 0.5 * Oat(e, 4, mu);
        }
        tv[mu] = t;
        xh[mu] = h;
    }
    __syncthreads();
    (void)nq;
    // per function: sums over electrons
    for (int mu = tid; mu < MJ; mu += 256) {
        double f[3] = {0.0, 0.0, 0.0}, p[3] = {0.0, 0.0, 0.0};
        const double x1 = xi1[mu];
        for (int e = 0; e < N; ++e) {
            const double *a = ab + 3 * e;
            const double g = x1 + tv[mu] - Oat(e, 0, mu);
            const double hq = a[0] * Oat(e, 1, mu) + a[1] * Oat(e, 2, mu) + a[2] * Oat(e, 3, mu) - 0.5 * Oat(e, 4, mu);
            const JasTerm o = jas_term<T>(JB, R, mu, pe + 3 * e, a, g, xh[mu] - hq);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                f[k] += o.f[k];
                p[k] += o.p[k];
            }
        }
        double *jt = jtao + ((size_t)w * MJ + mu) * 6;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            jt[k] = f[k];
            jt[3 + k] = p[k];
        }
    }
    // per electron: sums over functions, in two halves (threads e and e + 128)
    for (int i = tid; i < 2 * JAS_ELEC; i += 256) {
        const int e = i & (JAS_ELEC - 1), hh = i >> 7;
        if (e >= N) continue;
        const double *a = ab + 3 * e;
        double f[3] = {0.0, 0.0, 0.0};
        const int m0 = hh ? MJ / 2 : 0, m1 = hh ? MJ : MJ / 2;
        for (int mu = m0; mu < m1; ++mu) {
            const double g = xi1[mu] + tv[mu] - Oat(e, 0, mu);
            const double hq = a[0] * Oat(e, 1, mu) + a[1] * Oat(e, 2, mu) + a[2] * Oat(e, 3, mu) - 0.5 * Oat(e, 4, mu);
            const JasTerm o = jas_term<T>(JB, R, mu, pe + 3 * e, a, g, xh[mu] - hq);
#pragma unroll
            for (int k = 0; k < 3; ++k) f[k] += o.f[k];
        }
        double *hv = hh ? half1 : half0;
#pragma unroll
        for (int k = 0; k < 3; ++k) hv[3 * e + k] = f[k];
    }
    __syncthreads();
    for (int i = tid; i < 3 * N; i += 256) dedr[(size_t)w * N * 3 + i] += half0[i] + half1[i];
}

template <typename T>
hipError_t launch_jas_values(const BasisDev &JB, const double *R, const double *pos, int64_t rows, T *out,
                             hipStream_t st) {
    const dim3 g((unsigned)((rows + 63) / 64), (unsigned)JB.n_shells);
    hipLaunchKernelGGL(k_jas_values<T>, g, dim3(64), 0, st, JB, R, pos, rows, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jas_products(const SysDev &S, const BasisDev &JB, const AoTiles &jt, int nq, const T *xiblk,
                               const double *R, const double *pos, int64_t rows, int nc, T *out, T *cpad,
                               hipStream_t st) {
    SysDev J = S;
    J.basis = JB;
    J.M = JB.n_ao;
    J.n_occ = 64;
    for (int q = 0; q < nq; ++q) {
        const hipError_t e = launch_mo_rows_mfma<T>(J, xiblk + (size_t)q * JB.n_ao * 64, R, pos, rows, jt,
                                                    out + (size_t)q * rows * nc * 64, nc, cpad, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_jas_assemble(int N, int MJ, int nq, int64_t rows, int64_t row0, int W, const T *X, const T *O,
                               double *jg, double *ju, hipStream_t st) {
    hipLaunchKernelGGL(k_jas_assemble<T>, dim3((unsigned)W), dim3(256), 0, st, N, MJ, nq, rows, row0, X, O, jg, ju);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jas_adjoint(const BasisDev &JB, const double *R, int N, int nq, int64_t rows, int64_t row0, int W,
                              const double *pos, const T *X, const T *O, const double *gb, const double *xi1,
                              double *dedr, double *jtao, hipStream_t st) {
    hipLaunchKernelGGL(k_jas_adjoint<T>, dim3((unsigned)W), dim3(256), 0, st, JB, R, N, JB.n_ao, nq, rows, row0, pos,
                       X, O, gb, xi1, dedr, jtao);
    return hipGetLastError();
}

#define JAS_INST(T)                                                                                               \
    template hipError_t launch_jas_values<T>(const BasisDev &, const double *, const double *, int64_t, T *,       \
                                             hipStream_t);                                                         \
    template hipError_t launch_jas_products<T>(const SysDev &, const BasisDev &, const AoTiles &, int, const T *, \
                                               const double *, const double *, int64_t, int, T *, T *,            \
                                               hipStream_t);                                                       \
    template hipError_t launch_jas_assemble<T>(int, int, int, int64_t, int64_t, int, const T *, const T *,        \
                                               double *, double *, hipStream_t);                                   \
    template hipError_t launch_jas_adjoint<T>(const BasisDev &, const double *, int, int, int64_t, int64_t, int,  \
                                              const double *, const T *, const T *, const double *,               \
                                              const double *, double *, double *, hipStream_t);
JAS_INST(float)
JAS_INST(double)

}  // namespace vmcx

namespace vmcx {

// ---------------------------------------------------------------------------
// Sums of the Jastrow-parameter log-derivatives over one measurement launch,
// for dE/dxi = 2 (<E_L O_xi> - <E_L><O_xi>):
//   O_xi1 = s = sum_i chi(r_i),  O_xi3 = (s s^T - sum_i chi(r_i) chi(r_i)^T) / 2
// (the gradient of U3 with respect to the symmetric xi3).  With a_w the
// walker's weight and b_w = a_w (E_L,w - shift), the launch's partial sums
//   part = [sum a s | sum b s | sum a O_xi3 | sum b O_xi3]   (MJ, MJ, MJ^2, MJ^2)
// one block per 16 x 16 tile (mu, nu) of O_xi3, walkers in order; the tiles
// of the first column also form the O_xi1 sums.  X[w][i][mu] = chi_mu(r_i) in
// FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_xi_sums(const double *__restrict__ X, int N, int MJ, int W,
                                                 const double *__restrict__ EL, const double *__restrict__ shift,
                                                 const double *__restrict__ wt, double *part) {
    __shared__ double xm[128 * 16], xn[128 * 16];
    const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
    const int mu0 = 16 * blockIdx.x, nu0 = 16 * blockIdx.y;
    const int mu = mu0 + ti, nu = nu0 + tj;
    double s3a = 0.0, s3b = 0.0, s1a = 0.0, s1b = 0.0;
    const double sh = *shift;
    for (int w = 0; w < W; ++w) {
        __syncthreads();
        const double *xw = X + (size_t)w * N * MJ;
        for (int k = tid; k < N * 16; k += 256) {
            const int i = k >> 4, q = k & 15;
            xm[k] = mu0 + q < MJ ? xw[(size_t)i * MJ + mu0 + q] : 0.0;
            xn[k] = nu0 + q < MJ ? xw[(size_t)i * MJ + nu0 + q] : 0.0;
        }
        __syncthreads();
        double sm = 0.0, sn = 0.0, p = 0.0;
        for (int i = 0; i < N; ++i) {
            const double a = xm[16 * i + ti], b = xn[16 * i + tj];
            sm += a;
            sn += b;
            p += a * b;
        }
        const double aw = wt ? wt[w] : 1.0, bw = aw * (EL[w] - sh);
        const double o3 = 0.5 * (sm * sn - p);
        s3a += aw * o3;
        s3b += bw * o3;
        s1a += aw * sm;
        s1b += bw * sm;
    }
    if (mu < MJ && nu < MJ) {
        part[2 * MJ + (size_t)mu * MJ + nu] = s3a;
        part[2 * MJ + (size_t)MJ * MJ + (size_t)mu * MJ + nu] = s3b;
        if (blockIdx.y == 0 && tj == 0) {
            part[mu] = s1a;
            part[MJ + mu] = s1b;
        }
    }
}

// acc + comp += part (Neumaier), element by element.
__global__ void k_add_compensated(const double *__restrict__ part, int64_t n, double *acc, double *comp) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double s = acc[k], x = part[k], t = s + x;
    comp[k] += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    acc[k] = t;
}

hipError_t launch_xi_sums(const double *X, int N, int MJ, int W, const double *EL, const double *shift,
                          const double *wt, double *part, double *acc, double *comp, hipStream_t st) {
    if (N > 128) return hipErrorInvalidValue;
    const int nt = (MJ + 15) / 16;
    hipLaunchKernelGGL(k_xi_sums, dim3(nt, nt), dim3(256), 0, st, X, N, MJ, W, EL, shift, wt, part);
    const int64_t n = 2 * (int64_t)MJ + 2 * (int64_t)MJ * MJ;
    hipLaunchKernelGGL(k_add_compensated, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, n, acc, comp);
    return hipGetLastError();
}

}  // namespace vmcx
