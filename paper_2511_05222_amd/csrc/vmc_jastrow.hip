// vmc_jastrow.hip -- one-body and three/four-body Jastrow terms on a Jastrow
// GTO basis chi_mu (gfx950).
//
//   U1 = sum_i xi1 . chi(r_i)                            (eq. onebody_J_inhom)
//   U3 = sum_{i<j} chi(r_i)^T xi3 chi(r_j)               (eq. threebody_jas)
//
// With s = sum_i chi(r_i), the value products V[e] = chi(r_e)^T [xi3 | xi1]
// (MJ + 1 columns, formed on the matrix cores by k_jas_gemm; xi3 is
// symmetric), t = xi3 s = sum_e V[e] and the coefficient vector of electron e
//   g_e = xi1 + xi3 (s - chi_e) = xi1 + t - V[e]          (first MJ columns),
// the terms of E_L are dot products with the basis derivatives at r_e:
//   grad_e U = grad chi(r_e) . g_e,   lap_e U = lap chi(r_e) . g_e,
//   U = sum_e [ V[e] . (s - chi_e) / 2 + V[e][MJ] ].
// A move of electron e to r' changes U by (xi3 d) . (s - chi_e) + xi1 . d,
// d = chi(r') - chi_e; a sweep's proposals start from the positions of its
// start, so their d rows form one product (k_sweep_r adds the terms).
//
// Reverse mode (forces): with the total Jastrow gradient G_e and the
// determinant gradient b_e, E_L depends on grad_e U through
// abar_e = -(G_e + b_e) and on lap_e U through -1/2.  With
//   h_e = grad chi_e abar_e - lap chi_e / 2   (dE_L / dg_e),
//   Q[e] = xi3 h_e                            (one more product, k_jas_gemm),
//   q_e = xi3 (sum_j h_j - h_e) = sum_j Q[j] - Q[e]   (dE_L / dchi_e through the g_j),
// the explicit dependence on r_e is
//   dE_L/dr_e = sum_mu [ q_e,mu grad chi_mu + g_e,mu (hess chi_mu) abar_e
//                        - g_e,mu grad(lap chi_mu) / 2 ](r_e),
//   dlnPsi/dr_e (Jastrow) = sum_mu g_e,mu grad chi_mu(r_e),
// and a function centred on nucleus alpha moves with it, so its terms enter
// dE_L/dR_alpha and dlnPsi/dR_alpha with the opposite sign (per-function
// sums over electrons, added per nucleus by k_finalize).
#include <type_traits>

#include "vmc_mfma.hpp"

#include "vmc_pipeline.hpp"

namespace vmcx {

constexpr int JAS_MAX = 256;   // Jastrow basis functions
constexpr int JAS_ELEC = 128;  // electrons

// out[row][mu] = chi_mu(pos[row]) for the rows' positions and, with NC = 5,
// der[row][c][mu] = (d/dx, d/dy, d/dz, Laplacian)_c chi_mu(pos[row]); one
// block per 64 rows.  Per tile of whole shells (<= MT functions) a wavefront
// evaluates one shell at 64 rows (uniform angular momentum) into an LDS
// tile, which the block then writes row by row (consecutive threads,
// consecutive functions).
template <typename T, int NC, int MT>
__global__ __launch_bounds__(256) void k_jas_values(BasisDev JB, AoTiles tiles, const double *__restrict__ R,
                                                    const double *__restrict__ pos, int64_t rows,
                                                    T *__restrict__ out, T *__restrict__ der) {
    constexpr int RB = 64, TS = MT * NC + 1;
    __shared__ double sp[RB * 3];
    __shared__ T tv[RB * TS];
    const int tid = threadIdx.x, MJ = JB.n_ao;
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    for (int k = tid; k < RB * 3; k += 256) sp[k] = (row0 + k / 3) < rows ? pos[row0 * 3 + k] : 0.0;
    for (int tile = 0; tile < tiles.n_tiles; ++tile) {
        const int s0 = tiles.s0[tile], s1 = tiles.s1[tile], mu0 = tiles.mu0[tile], nmu = tiles.mu1[tile] - mu0;
        __syncthreads();
        for (int p = tid; p < RB * (s1 - s0); p += 256) {
            const int s = __builtin_amdgcn_readfirstlane(s0 + p / RB), r = p % RB;
            shell_eval_to<NC, T>(JB, R, s, sp[3 * r], sp[3 * r + 1], sp[3 * r + 2],
                                 tv + r * TS + (ldc(JB.shell_mu0 + s) - mu0) * NC);
        }
        __syncthreads();
        for (int p = tid; p < RB * nmu; p += 256) {
            const int r = p / nmu, c = p - (p / nmu) * nmu;
            if (row0 + r >= rows) continue;
            const T *t = tv + r * TS + c * NC;
            out[(row0 + r) * MJ + mu0 + c] = t[0];
            if constexpr (NC == 5)
#pragma unroll
                for (int k = 0; k < 4; ++k) der[((row0 + r) * 4 + k) * MJ + mu0 + c] = t[1 + k];
        }
    }
}

// Per walker: grad_e U, lap_e U (jg[w][e][0..3]) and U (ju[w]), FP64 sums.
// X[row][MJ]: chi values; D[row][4][MJ]: their gradients and Laplacians;
// V: nq blocks of [rows][64] (value products with [xi3 | xi1]).
template <typename T>
__global__ __launch_bounds__(256) void k_jas_assemble(int N, int MJ, int64_t rows, int64_t row0,
                                                      const T *__restrict__ X, const T *__restrict__ D,
                                                      const T *__restrict__ V, const double *__restrict__ xi1,
                                                      double *__restrict__ jg, double *__restrict__ ju) {
    __shared__ double sv[JAS_MAX], tv[JAS_MAX];
    __shared__ double uw[4];
    const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const T *Xw = X + (size_t)w * N * MJ;
    auto Vat = [&](int e, int mu) -> double {
        return (double)V[((size_t)(mu >> 6) * rows + row0 + (size_t)w * N + e) * 64 + (mu & 63)];
    };
    // s, t = xi3 s and sum_e V[e] . chi_e: wavefront v sums the electrons
    // e = v mod 4 for the functions mu = lane + 64 k (independent chains per
    // lane), then the wavefronts' partials of s and t are added in wavefront
    // order.  U = t . s / 2 - sum_e V[e] . chi_e / 2 + xi1 . s.
    double dvl = 0.0;
    {
        double pa[4] = {0.0, 0.0, 0.0, 0.0}, pt[4] = {0.0, 0.0, 0.0, 0.0};
        for (int e = wave; e < N; e += 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int mu = lane + 64 * k;
                if (mu < MJ) {
                    const double x = (double)Xw[(size_t)e * MJ + mu], v = Vat(e, mu);
                    pa[k] += x;
                    pt[k] += v;
                    dvl += v * x;
                }
            }
        }
        for (int v = 0; v < 4; ++v) {
            if (wave == v)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int mu = lane + 64 * k;
                    if (mu < MJ) {
                        sv[mu] = (v ? sv[mu] : 0.0) + pa[k];
                        tv[mu] = (v ? tv[mu] : 0.0) + pt[k];
                    }
                }
            __syncthreads();
        }
    }
    {
        // (MJ <= 256: one function per thread)
        const double q = tid < MJ ? (0.5 * tv[tid] + xi1[tid]) * sv[tid] : 0.0;
        const double u = wave_sum_dpp(q - 0.5 * dvl);
        if (lane == 0) uw[wave] = u;
    }
    // per electron: grad_e U and lap_e U, dot products of the basis
    // derivatives with g_e = xi1 + t - V[e]
    for (int e = wave; e < N; e += 4) {
        const size_t row = row0 + (size_t)w * N + e;
        const T *de = D + row * 4 * MJ;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        // (the slots k = 0..3 cover mu < MJ <= 256: their loads are issued
        // together)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int mu = lane + 64 * k;
            if (mu >= MJ) continue;
            const double g = xi1[mu] + tv[mu] - Vat(e, mu);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += (double)de[(size_t)c * MJ + mu] * g;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = wave_sum_dpp(acc[c]);
        if (lane == 0) {
            double *g = jg + ((size_t)w * N + e) * 4;
            g[0] = acc[0];
            g[1] = acc[1];
            g[2] = acc[2];
            g[3] = acc[3];
        }
    }
    __syncthreads();
    if (tid == 0) ju[w] = (uw[0] + uw[1]) + (uw[2] + uw[3]);
}

// out = A [xi3 | xi1] over the Jastrow basis (k < MJ), for three kinds of
// rows of A:
//   AM = 0: A = X                   (chi at the rows' positions),
//   AM = 1: A = X - X0              (a proposal's change chi(r') - chi(r)),
//   AM = 2: A = h = grad chi abar - lap chi / 2 at the row's electron, from
//           D = [rows][4][MJ] (gradient, Laplacian) and abar = -(Jastrow +
//           determinant gradient) from gb.
// AM 0 writes the MJ + 1 columns in blocks of 64 ([nq][rows][64]); AM 1 row
// by row with a row stride of MJ + 1 rounded up to a multiple of 4, the xi1
// column at MJ; AM 2 writes xi3 h, MJ columns row by row ([rows][MJ]).
// The xi3 columns on the matrix cores: 64 rows per block, 16 per wavefront;
// the columns in groups of NTL tiles of 16 whose accumulators stay in
// registers; k in chunks of 16 with the chunk of xi3 staged in LDS (two
// buffers, one barrier per chunk; thread i stages column i mod 16 NTL) and
// each lane's A entries read from memory directly, both loaded one chunk
// ahead.  In a chunk, lane (m, g) of the 16x16x4 product takes k = 4 g + j at
// step j: a permutation of k that the A entries and the LDS reads share.
// The LDS chunk is laid out [k][m][tile] (rows of NTL + 16 bytes), so that a
// lane reads its NTL B entries of a step as 16-byte vectors without bank
// conflicts.  The xi1 column (AM 0, 1) is a dot product per row: lane
// partial sums over its k, added over the four lanes of the row.
template <typename T, int NTL, int AM, bool VA>
__global__ __launch_bounds__(256) void k_jas_gemm(int MJ, int64_t rows, const T *__restrict__ A0,
                                                  const T *__restrict__ A1, const double *__restrict__ gb,
                                                  const T *__restrict__ xiblk, T *__restrict__ out) {
    typedef Mfma<T> MF;
    constexpr int CW = 16 * NTL, KPT = CW / 16, NA = AM == 2 ? 16 : (AM == 1 ? 8 : 4);
    constexpr int VL = 16 / sizeof(T), PS = NTL + VL, KS = 16 * PS;   // vector length, row and k strides
    static_assert(256 % CW == 0 && 16 % (256 / CW) == 0 && NTL % VL == 0, "column group");
    typedef T V16 __attribute__((ext_vector_type(VL)));
    __shared__ __align__(16) T xs[2][16 * KS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ml = lane & 15, kg = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * 64, arow = row0 + 16 * wave + ml;
    const bool rok = arow < rows;
    double ab[3] = {0.0, 0.0, 0.0};
    if (AM == 2 && rok)
        for (int d = 0; d < 3; ++d) ab[d] = -(gb[arow * 6 + d] + gb[arow * 6 + 3 + d]);
    const T *x1 = xiblk + (size_t)(MJ >> 6) * MJ * 64 + (MJ & 63);   // the xi1 column
    const int nt = (MJ + 15) / 16, nk = (MJ + 15) / 16;
    // (loads read clamped, in-bounds addresses unconditionally; the entries
    // outside the matrices are then replaced by zeros)
    const int64_t arc = min(arow, rows - 1);
    // the staging thread's column of the group and its first k in a chunk
    const int scol = tid % CW, sk = (tid / CW) * KPT;
    for (int t0 = 0; t0 < nt; t0 += NTL) {
        const int ntg = min(NTL, nt - t0), col = 16 * t0 + scol, colc = min(col, MJ - 1);
        const bool cok = col < MJ;
        const T *xcol = xiblk + (size_t)(colc >> 6) * MJ * 64 + (colc & 63);
        typename MF::acc_t acc[NTL];
#pragma unroll
        for (int t = 0; t < NTL; ++t) acc[t] = MF::zero();
        T ra[NA], rb[KPT], p1 = T(0);
        // a lane's four entries k0 + 4 g + (0..3) of a row of A (of A0 and
        // A1; of the four components of D): VA (MJ a multiple of 4) as 16-byte
        // vectors, else one by one; a chunk inside the basis (full) needs no
        // clamping
        auto load4 = [&](const T *src, T *dst, int k0, bool full) {
            const int k = k0 + 4 * kg;
            if constexpr (VA) {
                typedef T V4 __attribute__((ext_vector_type(4)));
                const V4 v = *(const V4 *)(src + (full ? k : min(k, MJ - 4)));
                const bool ok = rok && (full || k < MJ);
#pragma unroll
                for (int j = 0; j < 4; ++j) dst[j] = ok ? v[j] : T(0);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const T v = src[full ? k + j : min(k + j, MJ - 1)];
                    dst[j] = (rok && (full || k + j < MJ)) ? v : T(0);
                }
            }
        };
        auto load = [&](int k0) {
            const bool full = k0 + 16 <= MJ;
            if constexpr (AM == 2) {
#pragma unroll
                for (int c = 0; c < 4; ++c) load4(A0 + (arc * 4 + c) * MJ, ra + 4 * c, k0, full);
            } else {
                load4(A0 + arc * MJ, ra, k0, full);
                if constexpr (AM == 1) load4(A1 + arc * MJ, ra + 4, k0, full);
            }
            if (full) {
                const T *p = xcol + (size_t)(k0 + sk) * 64;
#pragma unroll
                for (int m = 0; m < KPT; ++m) {
                    const T v = p[m * 64];
                    rb[m] = cok ? v : T(0);
                }
            } else {
#pragma unroll
                for (int m = 0; m < KPT; ++m) {
                    const int k = k0 + sk + m;
                    const T v = xcol[(size_t)min(k, MJ - 1) * 64];
                    rb[m] = (cok && k < MJ) ? v : T(0);
                }
            }
        };
        auto stage = [&](int buf) {
#pragma unroll
            for (int m = 0; m < KPT; ++m) xs[buf][(sk + m) * KS + (scol & 15) * PS + (scol >> 4)] = rb[m];
        };
        // the chunks; FULL: all NTL tiles of the group hold columns (the
        // last group of a basis of fewer functions may not)
        auto chunks = [&](auto full) {
            load(0);
            stage(0);
            __syncthreads();
            for (int c = 0; c < nk; ++c) {
                T a[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if constexpr (AM == 2)
                        a[j] = (T)(ab[0] * (double)ra[j] + ab[1] * (double)ra[4 + j] + ab[2] * (double)ra[8 + j] -
                                   0.5 * (double)ra[12 + j]);
                    else if constexpr (AM == 1)
                        a[j] = ra[j] - ra[4 + j];
                    else
                        a[j] = ra[j];
                }
                if (AM != 2 && t0 == 0) {
                    // (a[j] is zero past the basis)
#pragma unroll
                    for (int j = 0; j < 4; ++j) p1 += a[j] * x1[(size_t)min(16 * c + 4 * kg + j, MJ - 1) * 64];
                }
                if (c + 1 < nk) load(16 * (c + 1));
                const T *xb = xs[c & 1] + 4 * kg * KS + ml * PS;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    T b[NTL];
#pragma unroll
                    for (int u = 0; u < NTL; u += VL) {
                        const V16 v = *(const V16 *)(xb + j * KS + u);
#pragma unroll
                        for (int i = 0; i < VL; ++i) b[u + i] = v[i];
                    }
#pragma unroll
                    for (int t = 0; t < NTL; ++t)
                        if (decltype(full)::value || t < ntg) acc[t] = MF::fma(a[j], b[t], acc[t]);
                }
                if (c + 1 < nk) stage((c + 1) & 1);
                __syncthreads();
            }
        };
        if (ntg == NTL)
            chunks(std::true_type{});
        else
            chunks(std::false_type{});
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = row0 + 16 * wave + MF::row(lane, v);
            if (row >= rows) continue;
#pragma unroll
            for (int t = 0; t < NTL; ++t) {
                const int oc = 16 * (t0 + t) + ml;
                if (t >= ntg || oc >= MJ) continue;
                if constexpr (AM == 2)
                    out[row * MJ + oc] = acc[t][v];
                else if constexpr (AM == 1)
                    out[row * ((MJ + 4) & ~3) + oc] = acc[t][v];
                else
                    out[((size_t)(oc >> 6) * rows + row) * 64 + (oc & 63)] = acc[t][v];
            }
        }
        if (AM != 2 && t0 == 0) {
            // (the four lanes of row ml: kg = 0..3, 16 apart)
            p1 += __shfl_xor(p1, 16);
            p1 += __shfl_xor(p1, 32);
            if (kg == 0 && rok) {
                if constexpr (AM == 1)
                    out[arow * ((MJ + 4) & ~3) + MJ] = p1;
                else
                    out[((size_t)(MJ >> 6) * rows + arow) * 64 + (MJ & 63)] = p1;
            }
        }
    }
}

// The 14 derivative components (value, gradient, Laplacian, Hessian,
// gradient of the Laplacian) of Jastrow function mu at (x, y, z): the lane's
// function data as in the adjoint's AO lanes (monomial as branch-free
// per-axis quadratics; the first primitive in registers in FP32, the
// Jastrow basis being uncontracted).
template <typename T>
__device__ inline void jas_function14(const BasisDev &JB, const double *R, int mu, double x, double y, double z,
                                      T *c) {
    constexpr int NPR = sizeof(T) == 4 ? 1 : 0;
    AoLane<T, NPR> al;
    ao_lane_load<T, NPR>(JB, mu, al);
    const int atom = JB.shell_atom[JB.ao_shell[mu]];
    const double dx = x - R[3 * atom], dy = y - R[3 * atom + 1], dz = z - R[3 * atom + 2];
    const double rho_d = dx * dx + dy * dy + dz * dz;
    T R0, u1, u2, u3;
    ao_lane_radial<T, NPR>(al, JB, rho_d, R0, u1, u2, u3);
    ao_lane_components<T, NPR>(al, (T)dx, (T)dy, (T)dz, (T)rho_d, R0, u1, u2, u3, c);
}

// dE_L/dr_e and dlnPsi/dr_e contributions of function mu at electron e, in
// the arithmetic type (ab = abar_e).
template <typename T>
struct JasTerm {
    T f[3], p[3];
};

template <typename T>
__device__ inline JasTerm<T> jas_term(const BasisDev &JB, const double *R, int mu, const double *pe, const T *ab, T g,
                                      T q) {
    T c[14];
    jas_function14<T>(JB, R, mu, pe[0], pe[1], pe[2], c);
    JasTerm<T> o;
    const T hs[3][3] = {{c[5], c[6], c[7]}, {c[6], c[8], c[9]}, {c[7], c[9], c[10]}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T ha = hs[k][0] * ab[0] + hs[k][1] * ab[1] + hs[k][2] * ab[2];
        o.f[k] = q * c[1 + k] + g * (ha - T(0.5) * c[11 + k]);
        o.p[k] = g * c[1 + k];
    }
    return o;
}

// Per walker: adds the Jastrow terms' dE_L/dr_e to dedr[w][e] and writes the
// per-function electron sums jtao[w][mu] = (sum_e f, sum_e p).  pos: the
// evaluation positions; gb[w][e]: total Jastrow gradient (0..2) and
// determinant gradient (3..5).  Each (electron, function) term is evaluated
// once: wavefront v takes the electrons e = v mod 4, lanes the functions
// mu = lane + 64 k; per electron the sum over functions by a wavefront sum,
// per function the wavefronts' partial sums added in wavefront order.  The
// terms and the sums inside a wavefront are in the arithmetic type, FP64 from
// the wavefront sums on.
template <typename T>
__global__ __launch_bounds__(256) void k_jas_adjoint(BasisDev JB, const double *__restrict__ R, int N, int MJ,
                                                     int64_t rows, int64_t row0, const double *__restrict__ pos,
                                                     const T *__restrict__ V, const T *__restrict__ Q,
                                                     const double *__restrict__ gb, const double *__restrict__ xi1,
                                                     double *__restrict__ dedr, double *__restrict__ jtao) {
    __shared__ double tv[JAS_MAX], xh[JAS_MAX];
    __shared__ double ab[JAS_ELEC * 3], pe[JAS_ELEC * 3], fe[JAS_ELEC * 3];
    __shared__ double fp[JAS_MAX * 6];
    const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the value products and Q = xi3 h of electron e
    auto Vat = [&](int e, int mu) -> double {
        return (double)V[((size_t)(mu >> 6) * rows + row0 + (size_t)w * N + e) * 64 + (mu & 63)];
    };
    auto Qat = [&](int e, int mu) -> double { return (double)Q[(row0 + (size_t)w * N + e) * MJ + mu]; };
    for (int i = tid; i < 3 * N; i += 256) {
        const int e = i / 3, d = i - 3 * (i / 3);
        ab[i] = -(gb[((size_t)w * N + e) * 6 + d] + gb[((size_t)w * N + e) * 6 + 3 + d]);
        pe[i] = pos[(size_t)w * N * 3 + i];
    }
    __syncthreads();
    // t = xi3 s (the value products summed over electrons) and xi3 H
    for (int mu = tid; mu < MJ; mu += 256) {
        double t = 0.0, h = 0.0;
        for (int e = 0; e < N; ++e) {
            t += Vat(e, mu);
            h += Qat(e, mu);
        }
        tv[mu] = t;
        xh[mu] = h;
    }
    __syncthreads();
    T F[4][3], P[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) F[k][d] = P[k][d] = T(0);
    for (int e = wave; e < N; e += 4) {
        const T a[3] = {(T)ab[3 * e], (T)ab[3 * e + 1], (T)ab[3 * e + 2]};
        T f3[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int mu = lane + 64 * k;
            if (mu >= MJ) continue;
            const T g = (T)(xi1[mu] + tv[mu] - Vat(e, mu)), q = (T)(xh[mu] - Qat(e, mu));
            const JasTerm<T> o = jas_term<T>(JB, R, mu, pe + 3 * e, a, g, q);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                F[k][d] += o.f[d];
                P[k][d] += o.p[d];
                f3[d] += o.f[d];
            }
        }
        double f3d[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) f3d[d] = wave_sum_dpp((double)f3[d]);
        if (lane == 0) {
            fe[3 * e] = f3d[0];
            fe[3 * e + 1] = f3d[1];
            fe[3 * e + 2] = f3d[2];
        }
    }
    // per function: the wavefronts' partials, in wavefront order
    for (int v = 0; v < 4; ++v) {
        if (wave == v)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int mu = lane + 64 * k;
                if (mu >= MJ) continue;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    fp[6 * mu + d] = (v ? fp[6 * mu + d] : 0.0) + (double)F[k][d];
                    fp[6 * mu + 3 + d] = (v ? fp[6 * mu + 3 + d] : 0.0) + (double)P[k][d];
                }
            }
        __syncthreads();
    }
    for (int i = tid; i < 6 * MJ; i += 256) jtao[(size_t)w * MJ * 6 + i] = fp[i];
    for (int i = tid; i < 3 * N; i += 256) dedr[(size_t)w * N * 3 + i] += fe[i];
}

template <typename T>
hipError_t launch_jas_values(const BasisDev &JB, const AoTiles &jt, const double *R, const double *pos, int64_t rows,
                             T *out, hipStream_t st, T *der, const AoTiles *jt32) {
    if (rows < 1) return hipSuccess;
    const dim3 g((unsigned)((rows + 63) / 64));
    // (wider tiles: half the barriers and row segments twice as long; the
    // FP64 tile of 32 functions would not fit the static LDS)
    if constexpr (sizeof(T) == sizeof(float))
        if (der && jt32) {
            hipLaunchKernelGGL((k_jas_values<T, 5, 32>), g, dim3(256), 0, st, JB, *jt32, R, pos, rows, out, der);
            return hipGetLastError();
        }
    if (der)
        hipLaunchKernelGGL((k_jas_values<T, 5, 16>), g, dim3(256), 0, st, JB, jt, R, pos, rows, out, der);
    else
        hipLaunchKernelGGL((k_jas_values<T, 1, 16>), g, dim3(256), 0, st, JB, jt, R, pos, rows, out, der);
    return hipGetLastError();
}

// (a column group's accumulators: 64 registers in either type, the xi3
// columns of MJ <= 256 in one group in FP32)
template <typename T>
constexpr int jas_gemm_ntl() { return sizeof(T) == sizeof(float) ? 16 : 8; }

template <typename T, int AM>
static void launch_jas_gemm(int MJ, int64_t rows, const T *A0, const T *A1, const double *gb, const T *xiblk, T *out,
                            hipStream_t st) {
    const dim3 g((unsigned)((rows + 63) / 64)), b(256);
    if (MJ % 4 == 0)
        hipLaunchKernelGGL((k_jas_gemm<T, jas_gemm_ntl<T>(), AM, true>), g, b, 0, st, MJ, rows, A0, A1, gb, xiblk,
                           out);
    else
        hipLaunchKernelGGL((k_jas_gemm<T, jas_gemm_ntl<T>(), AM, false>), g, b, 0, st, MJ, rows, A0, A1, gb, xiblk,
                           out);
}

template <typename T>
hipError_t launch_jas_vprod(int MJ, int /* nq (implied by MJ) */, int64_t rows, const T *X, const T *X0,
                            const T *xiblk, T *V, hipStream_t st) {
    if (rows < 1) return hipSuccess;
    if (X0)
        launch_jas_gemm<T, 1>(MJ, rows, X, X0, nullptr, xiblk, V, st);
    else
        launch_jas_gemm<T, 0>(MJ, rows, X, nullptr, nullptr, xiblk, V, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jas_assemble(int N, int MJ, int /* nq */, int64_t rows, int64_t row0, int W, const T *X,
                               const T *D, const T *V, const double *xi1, double *jg, double *ju, hipStream_t st) {
    hipLaunchKernelGGL(k_jas_assemble<T>, dim3((unsigned)W), dim3(256), 0, st, N, MJ, rows, row0, X, D, V, xi1, jg,
                       ju);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jas_hxi(int MJ, int /* nq */, int64_t rows, const T *D, const double *gb, const T *xiblk, T *Q,
                          hipStream_t st) {
    if (rows < 1) return hipSuccess;
    launch_jas_gemm<T, 2>(MJ, rows, D, nullptr, gb, xiblk, Q, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jas_adjoint(const BasisDev &JB, const double *R, int N, int64_t rows, int64_t row0, int W,
                              const double *pos, const T *V, const T *Q, const double *gb, const double *xi1,
                              double *dedr, double *jtao, hipStream_t st) {
    hipLaunchKernelGGL(k_jas_adjoint<T>, dim3((unsigned)W), dim3(256), 0, st, JB, R, N, JB.n_ao, rows, row0, pos, V,
                       Q, gb, xi1, dedr, jtao);
    return hipGetLastError();
}

#define JAS_INST(T)                                                                                               \
    template hipError_t launch_jas_values<T>(const BasisDev &, const AoTiles &, const double *, const double *,   \
                                             int64_t, T *, hipStream_t, T *, const AoTiles *);                     \
    template hipError_t launch_jas_vprod<T>(int, int, int64_t, const T *, const T *, const T *, T *,             \
                                            hipStream_t);                                                          \
    template hipError_t launch_jas_assemble<T>(int, int, int, int64_t, int64_t, int, const T *, const T *,        \
                                               const T *, const double *, double *, double *, hipStream_t);        \
    template hipError_t launch_jas_hxi<T>(int, int, int64_t, const T *, const double *, const T *, T *,           \
                                          hipStream_t);                                                            \
    template hipError_t launch_jas_adjoint<T>(const BasisDev &, const double *, int, int64_t, int64_t, int,       \
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
//   part = [sum a s | sum b s | sum a O_xi3 | sum b O_xi3]   (MJ, MJ, MJ^2, MJ^2).
// The O_xi3 sums are weighted Gram matrices, (S^T D S - Y^T D' Y) / 2 with
// Y = [W N x MJ] the basis values of every electron, S = [W x MJ] their
// walker sums and D, D' the walker weights (repeated over the electrons for
// D'), formed on FP64 MFMA: k_wgram computes a 64 x 64 block-tile of both
// weightings over a range of rows, for the block-tiles on and above the
// diagonal (the matrices are symmetric); the row ranges' partials are added
// in order by k_xi_finish, which takes the entries below the diagonal tiles
// from their mirror images.  X[w][i][mu] = chi_mu(r_i) in FP64.
// ---------------------------------------------------------------------------
constexpr int XI_SPLIT_Y = 96, XI_SPLIT_S = 8;   // row ranges of the two products

size_t xi_scratch_doubles(int W, int MJ) {
    return (size_t)W * MJ + (size_t)(XI_SPLIT_Y + XI_SPLIT_S) * 2 * MJ * MJ;
}

// S[w][mu] = sum_i X[w][i][mu]
__global__ __launch_bounds__(256) void k_xi_walker_sums(const double *__restrict__ X, int N, int MJ,
                                                        double *__restrict__ Sm) {
    const int w = blockIdx.x;
    for (int mu = threadIdx.x; mu < MJ; mu += 256) {
        double a = 0.0;
        for (int i = 0; i < N; ++i) a += X[((size_t)w * N + i) * MJ + mu];
        Sm[(size_t)w * MJ + mu] = a;
    }
}

// Block (tile, range): rows [k0, k1) of Z [K][MJ], row k belonging to walker
// k / rpw; alpha_k = wt[w] (1 without weights), beta_k = alpha_k (EL[w] - shift).
// part[range][0 / 1][mu][nu] = sum_k alpha_k / beta_k z_k[mu] z_k[nu] over the
// block-tile's 64 x 64 entries; blockIdx.x enumerates the block-tiles (bi, bj)
// with bi <= bj.  Wavefront v takes the 16 rows mu of sub-tile v and all four
// nu sub-tiles.  The next 16 rows are loaded into registers while the matrix
// cores work on the current ones.
__global__ __launch_bounds__(256) void k_wgram(const double *__restrict__ Z, int64_t K, int MJ, int rpw,
                                               const double *__restrict__ wt, const double *__restrict__ EL,
                                               const double *__restrict__ shift, int64_t per, double *part) {
    typedef Mfma<double> MF;
    __shared__ double zm[16][64], zn[16][64], al[16], be[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ml = lane & 15, kg = lane >> 4;
    const int nbt = (MJ + 63) / 64;
    int bi = 0, bj = blockIdx.x;
    while (bj >= nbt - bi) {
        bj -= nbt - bi;
        ++bi;
    }
    bj += bi;
    const int64_t k0 = (int64_t)blockIdx.y * per, k1 = min(K, k0 + per);
    const double sh = *shift;
    MF::acc_t ga[4], gb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) ga[j] = gb[j] = MF::zero();
    // this thread's staging slots: rows r = idx / 64 of the chunk, column c
    double rm[4], rn[4], ra = 0.0, rb = 0.0;
    auto load = [&](int64_t kb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i, r = idx >> 6, c = idx & 63, cm = 64 * bi + c, cn = 64 * bj + c;
            const int64_t k = kb + r, kc = min(k, K - 1);
            const double vm = Z[kc * MJ + min(cm, MJ - 1)], vn = Z[kc * MJ + min(cn, MJ - 1)];
            rm[i] = (k < k1 && cm < MJ) ? vm : 0.0;
            rn[i] = (k < k1 && cn < MJ) ? vn : 0.0;
        }
        if (tid < 16) {
            const int64_t k = kb + tid;
            ra = rb = 0.0;
            if (k < k1) {
                const int64_t w = k / rpw;
                ra = wt ? wt[w] : 1.0;
                rb = ra * (EL[w] - sh);
            }
        }
    };
    if (k0 < k1) load(k0);
    for (int64_t kb = k0; kb < k1; kb += 16) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i;
            zm[idx >> 6][idx & 63] = rm[i];
            zn[idx >> 6][idx & 63] = rn[i];
        }
        if (tid < 16) {
            al[tid] = ra;
            be[tid] = rb;
        }
        __syncthreads();
        if (kb + 16 < k1) load(kb + 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int r = 4 * ks + kg;
            const double am = zm[r][16 * wave + ml], wa = al[r], wb = be[r];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double z = zn[r][16 * j + ml];
                ga[j] = MF::fma(am, wa * z, ga[j]);
                gb[j] = MF::fma(am, wb * z, gb[j]);
            }
        }
    }
    double *pa = part + (size_t)blockIdx.y * 2 * MJ * MJ, *pb = pa + (size_t)MJ * MJ;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int mu = 64 * bi + 16 * wave + MF::row(lane, v), nu = 64 * bj + 16 * j + ml;
            if (mu < MJ && nu < MJ) {
                pa[(size_t)mu * MJ + nu] = ga[j][v];
                pb[(size_t)mu * MJ + nu] = gb[j][v];
            }
        }
}

// part[mu] = sum_w a_w s_w[mu], part[MJ + mu] = sum_w b_w s_w[mu]: block mu,
// threads over walkers, a fixed-order block sum.
__global__ __launch_bounds__(256) void k_xi_s1(const double *__restrict__ Sm, int W, int MJ,
                                               const double *__restrict__ EL, const double *__restrict__ shift,
                                               const double *__restrict__ wt, double *part) {
    __shared__ double ra[256], rb[256];
    const int mu = blockIdx.x, tid = threadIdx.x;
    const double sh = *shift;
    double a1 = 0.0, b1 = 0.0;
    for (int w = tid; w < W; w += 256) {
        const double aw = wt ? wt[w] : 1.0, sv = Sm[(size_t)w * MJ + mu];
        a1 += aw * sv;
        b1 += aw * (EL[w] - sh) * sv;
    }
    ra[tid] = a1;
    rb[tid] = b1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            ra[tid] += ra[tid + h];
            rb[tid] += rb[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[mu] = ra[0];
        part[MJ + mu] = rb[0];
    }
}

// part[2 MJ ..] = [(G_S - G_Y)_a / 2 | (G_S - G_Y)_b / 2], the ranges'
// partials added in order.
__global__ void k_xi_finish(int MJ, const double *__restrict__ pY, int nY, const double *__restrict__ pS, int nS,
                            double *part) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m2 = (int64_t)MJ * MJ;
    if (t < 2 * m2) {
        // (mu, nu) in a block-tile below the diagonal: its mirror (nu, mu)
        const int64_t h = t / m2, mu = (t - h * m2) / MJ, nu = t - h * m2 - mu * MJ;
        const int64_t src = (mu >> 6) > (nu >> 6) ? h * m2 + nu * MJ + mu : t;
        double y = 0.0, q = 0.0;
        for (int g = 0; g < nY; ++g) y += pY[(size_t)g * 2 * m2 + src];
        for (int g = 0; g < nS; ++g) q += pS[(size_t)g * 2 * m2 + src];
        part[2 * MJ + t] = 0.5 * (q - y);
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
                          const double *wt, double *part, double *scratch, double *acc, double *comp,
                          hipStream_t st) {
    if (W < 1 || MJ < 1) return hipSuccess;
    const size_t m2 = (size_t)MJ * MJ;
    double *Sm = scratch, *pY = Sm + (size_t)W * MJ, *pS = pY + (size_t)XI_SPLIT_Y * 2 * m2;
    hipLaunchKernelGGL(k_xi_walker_sums, dim3((unsigned)W), dim3(256), 0, st, X, N, MJ, Sm);
    const int nbt = (MJ + 63) / 64;
    const int64_t KY = (int64_t)W * N, perY = (KY + XI_SPLIT_Y - 1) / XI_SPLIT_Y;
    const int64_t perS = ((int64_t)W + XI_SPLIT_S - 1) / XI_SPLIT_S;
    const unsigned ntri = (unsigned)(nbt * (nbt + 1) / 2);
    hipLaunchKernelGGL(k_wgram, dim3(ntri, XI_SPLIT_Y), dim3(256), 0, st, X, KY, MJ, N, wt, EL, shift, perY, pY);
    hipLaunchKernelGGL(k_wgram, dim3(ntri, XI_SPLIT_S), dim3(256), 0, st, Sm, (int64_t)W, MJ, 1, wt, EL, shift, perS,
                       pS);
    const int64_t n = 2 * (int64_t)MJ + 2 * (int64_t)m2;
    hipLaunchKernelGGL(k_xi_s1, dim3((unsigned)MJ), dim3(256), 0, st, Sm, W, MJ, EL, shift, wt, part);
    hipLaunchKernelGGL(k_xi_finish, dim3((unsigned)((2 * m2 + 255) / 256)), dim3(256), 0, st, MJ, pY, XI_SPLIT_Y,
                       pS, XI_SPLIT_S, part);
    hipLaunchKernelGGL(k_add_compensated, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, n, acc, comp);
    return hipGetLastError();
}

}  // namespace vmcx
