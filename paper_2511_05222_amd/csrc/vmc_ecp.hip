// vmc_ecp.hip -- semilocal pseudopotential in the local energy (gfx950).
//
// On nucleus a, an electron i at distance d = |r_i - R_a| (direction u) sees
// the local potential V_loc(d) and, for d < rcut[a], the projectors of the
// channels l, which enter E_L as
//   E_nl = sum_(i,a) sum_q c_q rho_q,   c_q = sum_l (2l + 1)/12 V_l(d) P_l(u . v_q),
//   rho_q = Psi(.., r_q, ..) / Psi(.., r_i, ..) = t_q exp(dJ_q),
//   t_q = phi(r_q)^T K e_i (determinant lemma),  r_q = R_a + d v_q,
// over the 12 icosahedron vertices v_q turned by one random rotation per
// (walker, electron), dJ_q the change of the Jastrow: the two-body pair terms
// of electron i and, with the one- and three/four-body terms,
//   (chi(r_q) - chi(r_i)) . h_i,   h_i = xi1 + xi3 sum_{j != i} chi(r_j).
// The kernels around the measurement:
//   k_ecp_count / k_ecp_scan / k_ecp_place
//                  the (electron, nucleus) pairs inside the cutoffs, packed
//                  over the walkers of a launch, and their 12 points each;
//                  the MO rows at the points are then one k_mo_rows_mfma
//                  launch over the packed rows;
//   k_ecp_energy_pts (threads over the points; with the one-/three-body
//   terms k_ecp_energy, a wavefront per electron)
//                  after k_dense: rho_q, E_loc + E_nl added to E_L; and, with
//                  Z[j][i] = sum_q c'_q phi_q[j] (c'_q = c_q exp(dJ_q), the
//                  points of electron i), the derivative through the inverses,
//                  dE/dA_b = -(K~_b Z_b K~_b) with K~[e][j] = K[j][e], added to
//                  Abar, which k_adjoint_mfma carries into G, dE_L/dr and the
//                  AO centres like the kinetic energy's share;
//   k_ecp_adjoint  after k_adjoint_mfma: the derivatives through the points.
//                  With y_q = c'_q K~[i] (dE/dphi(r_q)):  G += sum_q psi(r_q) y_q^T;
//                  g_q = dE/dr_q (orbitals and Jastrow at r_q) carried to r_i
//                  and R_a through r_q = R_a + d v_q; c_q through d and u . v_q;
//                  the Jastrow's dependence on the other electrons; the AOs
//                  at the points moving with their nuclei; V_loc.  With the
//                  one-/three-body terms k_ecp_jas first forms their share:
//                  the gradient at each point, the electrons' terms through
//                  the h_j, and the Jastrow functions' per-nucleus sums.
#include <algorithm>

#include "vmc.h"
#include "vmc_pipeline.hpp"
#include "vmc_regs.hpp"

namespace vmcx {

constexpr uint32_t PURPOSE_ROTATION = 2;

// Quadrature direction q: (0, s1, s2 g), (s1, s2 g, 0), (s2 g, 0, s1) for
// s1, s2 in (+1, -1) in that order (q = 6 i1 + 3 i2 + k), g the golden
// ratio, normalised.
__device__ inline void ico_dir(int q, double v[3]) {
    const double g = 0.5 * (1.0 + sqrt(5.0)), nrm = sqrt(1.0 + g * g);
    const int i1 = q / 6, i2 = (q / 3) & 1, k = q % 3;
    const double s1 = i1 ? -1.0 : 1.0, s2 = i2 ? -g : g;
    const double a[3] = {0.0, s1, s2}, b[3] = {s1, s2, 0.0}, c[3] = {s2, 0.0, s1};
    const double *x = k == 0 ? a : (k == 1 ? b : c);
    v[0] = x[0] / nrm;
    v[1] = x[1] / nrm;
    v[2] = x[2] / nrm;
}

// Rotation of the quadrature of (walker id, rotation index, electron):
// Shoemake's uniform unit quaternion (x, y, z, s) from three uniforms
// u = w 2^-32 of one Philox draw, as a row-major 3 x 3 matrix.
__device__ inline void ecp_rotation(uint64_t seed, uint32_t wid, uint32_t rot, int e, double Rm[9]) {
    const U4 wd = draw_words(seed, wid, rot, (uint32_t)e, PURPOSE_ROTATION);
    const double u1 = (double)wd.x * 2.3283064365386963e-10, u2 = (double)wd.y * 2.3283064365386963e-10,
                 u3 = (double)wd.z * 2.3283064365386963e-10;
    const double a = sqrt(1.0 - u1), b = sqrt(u1);
    const double x = a * sin(6.283185307179586 * u2), y = a * cos(6.283185307179586 * u2);
    const double z = b * sin(6.283185307179586 * u3), s = b * cos(6.283185307179586 * u3);
    Rm[0] = 1.0 - 2.0 * (y * y + z * z);
    Rm[1] = 2.0 * (x * y - z * s);
    Rm[2] = 2.0 * (x * z + y * s);
    Rm[3] = 2.0 * (x * y + z * s);
    Rm[4] = 1.0 - 2.0 * (x * x + z * z);
    Rm[5] = 2.0 * (y * z - x * s);
    Rm[6] = 2.0 * (x * z - y * s);
    Rm[7] = 2.0 * (y * z + x * s);
    Rm[8] = 1.0 - 2.0 * (x * x + y * y);
}

// V_l of nucleus a at d (l = -1: local) and its derivative in d.
__device__ inline void ecp_radial(const EcpDev &E, int a, int l, double d, double &v, double &dv) {
    v = dv = 0.0;
    for (int t = E.t0[a]; t < E.t0[a + 1]; ++t) {
        if (E.t_l[t] != l) continue;
        const int n = E.t_n[t];
        const double al = E.t_alpha[t], b = E.t_beta[t];
        const double ex = exp(-al * d * d);
        const double pw = n == 1 ? 1.0 / d : (n == 2 ? 1.0 : (n == 3 ? d : d * d));     // d^(n-2)
        const double pm = n == 1 ? -1.0 / (d * d) : (n == 2 ? 0.0 : (n == 3 ? 1.0 : 2.0 * d));   // (n-2) d^(n-3)
        v += b * pw * ex;
        dv += b * ex * (pm - 2.0 * al * d * pw);
    }
}

// Components (NC = 1: value; 5: value, gradient, Laplacian) of Jastrow
// function mu at (x, y, z), FP64.
template <int NC>
__device__ inline void jas_fn(const BasisDev &JB, const double *R, int mu, double x, double y, double z, double *c) {
    const int s = JB.ao_shell[mu], atom = JB.shell_atom[s];
    const double dx = x - R[3 * atom], dy = y - R[3 * atom + 1], dz = z - R[3 * atom + 2];
    const double rho = dx * dx + dy * dy + dz * dz;
    double R0, R1, R2, R3;
    shell_radial<NC, double>(JB, s, rho, R0, R1, R2, R3);
    ao_components<NC, double>(dx, dy, dz, rho, R0, R1, R2, R3, JB.ao_pow[mu], JB.ao_eta[mu], c);
}

// The value product of electron e with column mu of [xi3 | xi1]:
// (xi3 chi(r_e))_mu for mu < MJ.
template <typename T>
__device__ inline double ecp_jas_oval(const EcpJas<T> &J, int64_t row, int mu) {
    return (double)J.V[((size_t)(mu >> 6) * J.rows + row) * 64 + (mu & 63)];
}

// The two-body pair term u(r) and u'(r) / r from r^2 > 0, the reciprocal and
// inverse square root from the hardware estimates and Newton steps.
__device__ inline double ecp_u(double r2, const SysDev &S) {
    const double r = r2 * rsqrt_nr(r2);
    if (S.ee_form == 1) return S.ee_a * (1.0 - exp(-S.ee_F * r)) / S.ee_F;
    return S.ee_a * r * rcp_nr(1.0 + S.ee_F * r);
}
__device__ inline double ecp_u1r(double r2, const SysDev &S) {
    const double ir = rsqrt_nr(r2), r = r2 * ir;
    if (S.ee_form == 1) return S.ee_a * exp(-S.ee_F * r) * ir;
    const double q = rcp_nr(1.0 + S.ee_F * r);
    return S.ee_a * q * q * ir;
}

__device__ inline double legendre(int l, double x) {
    return l == 0 ? 1.0 : (l == 1 ? x : (l == 2 ? 1.5 * x * x - 0.5 : (2.5 * x * x - 1.5) * x));
}
__device__ inline double legendre_d(int l, double x) {
    return l == 0 ? 0.0 : (l == 1 ? 1.0 : (l == 2 ? 3.0 * x : 7.5 * x * x - 1.5));
}

// ---------------------------------------------------------------------------
// Pairs inside the cutoffs, packed over the walkers of a launch: the count
// per walker, the offsets (one block, in walker order), then the pairs (in
// electron order, then the order of the nuclei with projectors) and their
// points.
// ---------------------------------------------------------------------------
__device__ inline int ecp_inside(const EcpDev &E, const double *R, int a, double x, double y, double z) {
    const double dx = x - R[3 * a], dy = y - R[3 * a + 1], dz = z - R[3 * a + 2];
    return sqrt(dx * dx + dy * dy + dz * dz) < E.rcut[a] ? 1 : 0;
}

__global__ __launch_bounds__(128) void k_ecp_count(SysDev S, EcpDev E, const double *__restrict__ R,
                                                   const double *__restrict__ pos, int *npairs) {
    __shared__ int cnt[128];
    const int w = blockIdx.x, tid = threadIdx.x, N = S.N;
    const double *p = pos + (size_t)w * N * 3;
    int c = 0;
    if (tid < N)
        for (int k = 0; k < E.n_nl; ++k) c += ecp_inside(E, R, E.nl_atom[k], p[3 * tid], p[3 * tid + 1], p[3 * tid + 2]);
    cnt[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int i = 0; i < N; ++i) s += cnt[i];
        npairs[w] = s;
    }
}

// off[w] = pairs of the walkers before w; a walker's pairs past the
// launch's capacity are dropped (and flagged); *nrows = 12 * the pairs kept.
__global__ __launch_bounds__(1024) void k_ecp_scan(int W, int64_t cap, int *npairs, int *off, int *nrows,
                                                   int *status) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int seg = (W + 1023) / 1024, w0 = tid * seg, w1 = min(W, w0 + seg);
    int64_t s = 0;
    for (int w = w0; w < w1; ++w) s += npairs[w];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t t = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t v = part[i];
            part[i] = t;
            t += v;
        }
        *nrows = (int)(12 * min(t, cap));
        if (t > cap) atomicOr(status, STATUS_CAPACITY);
    }
    __syncthreads();
    int64_t o = part[tid];
    for (int w = w0; w < w1; ++w) {
        const int c = npairs[w];
        off[w] = (int)min(o, cap);
        npairs[w] = (int)max((int64_t)0, min((int64_t)c, cap - o));
        o += c;
    }
}

__global__ __launch_bounds__(128) void k_ecp_place(SysDev S, EcpDev E, const double *__restrict__ R,
                                                   const double *__restrict__ pos, int64_t id0,
                                                   const int *__restrict__ idlist, uint32_t rot,
                                                   const int *__restrict__ npairs, const int *__restrict__ off,
                                                   int *pairs, double *qpos) {
    __shared__ int cnt[128];
    const int w = blockIdx.x, tid = threadIdx.x, N = S.N;
    const double *p = pos + (size_t)w * N * 3;
    int c = 0;
    if (tid < N)
        for (int k = 0; k < E.n_nl; ++k) c += ecp_inside(E, R, E.nl_atom[k], p[3 * tid], p[3 * tid + 1], p[3 * tid + 2]);
    cnt[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int i = 0; i < 128; ++i) {
            const int t = cnt[i];
            cnt[i] = s;
            s += t;
        }
    }
    __syncthreads();
    const int np = npairs[w], o0 = off[w];
    int *pw = pairs + o0;
    if (tid < N) {
        int o = cnt[tid];
        for (int k = 0; k < E.n_nl; ++k) {
            const int a = E.nl_atom[k];
            if (ecp_inside(E, R, a, p[3 * tid], p[3 * tid + 1], p[3 * tid + 2])) {
                if (o < np) pw[o] = tid | (a << 8);
                ++o;
            }
        }
    }
    __syncthreads();
    const uint32_t wid = (uint32_t)(id0 + (idlist ? idlist[w] : w));
    double *qp = qpos + (size_t)o0 * 12 * 3;
    for (int t = tid; t < np * 12; t += 128) {
        const int pi = t / 12, q = t - 12 * (t / 12);
        const int pr = pw[pi], e = pr & 255, a = pr >> 8;
        const double dx = p[3 * e] - R[3 * a], dy = p[3 * e + 1] - R[3 * a + 1], dz = p[3 * e + 2] - R[3 * a + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        double Rm[9], u[3];
        ecp_rotation(E.seed, wid, rot, e, Rm);
        ico_dir(q, u);
        qp[3 * t] = R[3 * a] + d * (Rm[0] * u[0] + Rm[1] * u[1] + Rm[2] * u[2]);
        qp[3 * t + 1] = R[3 * a + 1] + d * (Rm[3] * u[0] + Rm[4] * u[1] + Rm[5] * u[2]);
        qp[3 * t + 2] = R[3 * a + 2] + d * (Rm[6] * u[0] + Rm[7] * u[1] + Rm[8] * u[2]);
    }
}

// ---------------------------------------------------------------------------
// The energy and the derivative through the inverses.  One block per walker;
// wavefront v takes the pairs of the electrons i = v mod 4 (so that Z[.][i]
// has one writer), lanes run over orbitals (ratio) and electrons (Jastrow).
// Per point it keeps rows[.] = (c'_q, t_q, exp(dJ_q), c_q).
// ---------------------------------------------------------------------------
size_t ecp_energy_pts_lds(int N, int n);
// (the larger of the two energy kernels' needs)
size_t ecp_energy_lds(int N, int n, int MJ) {
    return std::max(sizeof(double) * ((size_t)3 * N + (size_t)N * n + (size_t)n * n + 132 + (size_t)MJ),
                    ecp_energy_pts_lds(N, n));
}

template <typename T, bool J13>
__global__ __launch_bounds__(256) void k_ecp_energy(SysDev S, EcpDev E, const double *__restrict__ R,
                                                    const double *__restrict__ pos, EcpBufs<T> eb, int nc,
                                                    const T *__restrict__ ktil, T *abar, double *EL, int *status,
                                                    EcpJas<T> J) {
    extern __shared__ double sm[];
    const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int N = S.N, n = S.n_occ, MJ = J13 ? J.MJ : 0;
    double *sp = sm;               // [N][3]
    double *sz = sp + 3 * N;       // [N][n]: Z^T, row i = sum over the points of electron i
    double *sP = sz + N * n;       // [n][n]
    double *red = sP + n * n;      // [128] local terms, [4] per-wave E_nl
    double *tv = red + 132;        // [MJ] xi3 s (one-/three-body terms)
    for (int i = tid; i < 3 * N; i += 256) sp[i] = pos[(size_t)w * N * 3 + i];
    if (abar)
        for (int i = tid; i < N * n; i += 256) sz[i] = 0.0;
    if constexpr (J13)
        for (int mu = tid; mu < MJ; mu += 256) {
            double t = 0.0;
            for (int e = 0; e < N; ++e) t += ecp_jas_oval(J, (int64_t)w * N + e, mu);
            tv[mu] = t;
        }
    __syncthreads();
    const int np = eb.npairs[w];
    const size_t o0 = (size_t)eb.off[w];
    const int *pw = eb.pairs + o0;
    const T *ph = eb.phiq + o0 * 12 * nc * n;
    const T *kt = ktil + (size_t)w * N * n;
    const double *qp = eb.qpos + o0 * 12 * 3;
    double *rw = eb.rows + o0 * 12 * ECP_ROW;
    double Ew = 0.0;
    for (int pi = 0; pi < np; ++pi) {
        const int pr = pw[pi], e = pr & 255, a = pr >> 8;
        if ((e & 3) != wave) continue;
        const double ex = sp[3 * e], ey = sp[3 * e + 1], ez = sp[3 * e + 2];
        const double dx = ex - R[3 * a], dy = ey - R[3 * a + 1], dz = ez - R[3 * a + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double ux = dx / d, uy = dy / d, uz = dz / d;
        double Vl[VMC_MAX_ECP_L + 1];
        for (int l = 0; l <= E.lmax; ++l) {
            double dv;
            ecp_radial(E, a, l, d, Vl[l], dv);
        }
        const double kte = lane < n ? (double)kt[(size_t)e * n + lane] : 0.0;
        // the electron's own pair terms, sum_{j != e} u(|r_e - r_j|)
        double uo = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            if (j < N && j != e) {
                const double qx = ex - sp[3 * j], qy = ey - sp[3 * j + 1], qz = ez - sp[3 * j + 2];
                uo += ecp_u(qx * qx + qy * qy + qz * qz, S);
            }
        }
        uo = wave_sum_dpp(uo);
        // one-/three-body: h_e and chi(r_e) of the lane's functions
        double hj[4], xe[4];
        if constexpr (J13) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int mu = lane + 64 * k;
                const bool v = mu < MJ;
                hj[k] = v ? J.xi1[mu] + tv[mu] - ecp_jas_oval(J, (int64_t)w * N + e, mu) : 0.0;
                xe[k] = v ? (double)J.X[((size_t)w * N + e) * MJ + mu] : 0.0;
            }
        }
        for (int q = 0; q < 12; ++q) {
            const int row = 12 * pi + q;
            const double px = qp[3 * row], py = qp[3 * row + 1], pz = qp[3 * row + 2];
            const double cs = (ux * (px - R[3 * a]) + uy * (py - R[3 * a + 1]) + uz * (pz - R[3 * a + 2])) / d;
            double c = 0.0;
            for (int l = 0; l <= E.lmax; ++l) c += (double)(2 * l + 1) / 12.0 * Vl[l] * legendre(l, cs);
            const double phj = lane < n ? (double)ph[(size_t)row * nc * n + lane] : 0.0;
            const double t = wave_sum_dpp(phj * kte);
            double un = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = lane + 64 * h;
                if (j < N && j != e) {
                    const double qx = px - sp[3 * j], qy = py - sp[3 * j + 1], qz = pz - sp[3 * j + 2];
                    un += ecp_u(qx * qx + qy * qy + qz * qz, S);
                }
            }
            double d13 = 0.0;
            if constexpr (J13) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int mu = lane + 64 * k;
                    if (mu < MJ) {
                        double cv;
                        jas_fn<1>(J.jb, R, mu, px, py, pz, &cv);
                        d13 += (cv - xe[k]) * hj[k];
                    }
                }
                d13 = wave_sum_dpp(d13);
            }
            const double jr = exp(wave_sum_dpp(un) - uo + d13);
            const double cq = c * jr;
            Ew += cq * t;
            if (abar && lane < n) sz[(size_t)e * n + lane] += cq * phj;
            if (lane == 0) {
                double *o = rw + (size_t)row * ECP_ROW;
                o[0] = cq;
                o[1] = t;
                o[2] = jr;
                o[3] = c;
            }
        }
    }
    // the local part, every electron and nucleus
    double El = 0.0;
    if (tid < N)
        for (int a = 0; a < S.A; ++a) {
            if (E.t0[a] == E.t0[a + 1]) continue;
            const double dx = sp[3 * tid] - R[3 * a], dy = sp[3 * tid + 1] - R[3 * a + 1],
                         dz = sp[3 * tid + 2] - R[3 * a + 2];
            double v, dv;
            ecp_radial(E, a, -1, sqrt(dx * dx + dy * dy + dz * dz), v, dv);
            El += v;
        }
    if (tid < 128) red[tid] = El;
    if (lane == 0) red[128 + wave] = Ew;
    __syncthreads();
    if (tid == 0 && EL) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += red[i];
        const double e_l = EL[w] + (s + ((red[128] + red[129]) + (red[130] + red[131])));
        EL[w] = e_l;
        if (!isfinite(e_l)) atomicOr(status, STATUS_NONFINITE);
    }
    if (!abar) return;
    // dE/dA_b = -(K~_b Z_b K~_b): sP = Z_b K~_b, then Abar_b -= K~_b sP
    for (int b = 0; b < 2; ++b) {
        const int off = b ? S.n_up : 0, nb = b ? S.n_dn : S.n_up;
        __syncthreads();
        for (int idx = tid; idx < n * n; idx += 256) {
            const int a = idx / n, j = idx - (idx / n) * n;
            double s = 0.0;
            for (int i = 0; i < nb; ++i) s += sz[(size_t)(off + i) * n + a] * (double)kt[(size_t)(off + i) * n + j];
            sP[idx] = s;
        }
        __syncthreads();
        for (int idx = tid; idx < nb * n; idx += 256) {
            const int ei = idx / n, j = idx - (idx / n) * n;
            double s = 0.0;
            for (int a = 0; a < n; ++a) s += (double)kt[(size_t)(off + ei) * n + a] * sP[(size_t)a * n + j];
            T *ab = abar + ((size_t)w * N + off + ei) * n + j;
            *ab = (T)((double)*ab - s);
        }
    }
}

// The same without the one-/three-body terms, threads over the points (one
// block per walker): per electron its own pair sum; per point t_q, the pair
// terms at r_q and c_q; E_nl summed over the threads in a fixed order; with
// abar, Z^T[e][j] by threads over (electron, orbital) from the points' rows,
// then dE/dA as above.
size_t ecp_energy_pts_lds(int N, int n) {
    return sizeof(double) * ((size_t)4 * N + (size_t)2 * N * n + (size_t)n * n + 256 + 4) + sizeof(int) * 2 * N;
}

template <typename T>
__global__ __launch_bounds__(256) void k_ecp_energy_pts(SysDev S, EcpDev E, const double *__restrict__ R,
                                                        const double *__restrict__ pos, EcpBufs<T> eb, int nc,
                                                        const T *__restrict__ ktil, T *abar, double *EL,
                                                        int *status) {
    extern __shared__ double sm[];
    const int w = blockIdx.x, tid = threadIdx.x;
    const int N = S.N, n = S.n_occ;
    double *sp = sm;               // [N][3]
    double *suo = sp + 3 * N;      // [N] sum_{j != e} u(r_ej)
    double *sz = suo + N;          // [N][n]: Z^T
    double *sP = sz + N * n;       // [n][n]
    double *red = sP + n * n;      // [256] E_nl partials, then the local terms
    double *skt = red + 260;       // [N][n]: K~ of the walker
    int *pr0 = (int *)(skt + N * n);   // [2][N]: each electron's pairs [pr0, pr1)
    for (int i = tid; i < 3 * N; i += 256) sp[i] = pos[(size_t)w * N * 3 + i];
    __syncthreads();
    for (int e = tid; e < N; e += 256) {
        double uo = 0.0;
        for (int j = 0; j < N; ++j)
            if (j != e) {
                const double qx = sp[3 * e] - sp[3 * j], qy = sp[3 * e + 1] - sp[3 * j + 1],
                             qz = sp[3 * e + 2] - sp[3 * j + 2];
                uo += ecp_u(qx * qx + qy * qy + qz * qz, S);
            }
        suo[e] = uo;
    }
    __syncthreads();
    const int np = eb.npairs[w], nrow = 12 * np;
    const size_t o0 = (size_t)eb.off[w];
    const int *pw = eb.pairs + o0;
    const T *ph = eb.phiq + o0 * 12 * nc * n;
    const T *kt = ktil + (size_t)w * N * n;
    const double *qp = eb.qpos + o0 * 12 * 3;
    double *rw = eb.rows + o0 * 12 * ECP_ROW;
    double Ew = 0.0;
    for (int row = tid; row < nrow; row += 256) {
        const int pr = pw[row / 12], e = pr & 255, a = pr >> 8;
        const double ex = sp[3 * e], ey = sp[3 * e + 1], ez = sp[3 * e + 2];
        const double dx = ex - R[3 * a], dy = ey - R[3 * a + 1], dz = ez - R[3 * a + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double px = qp[3 * row], py = qp[3 * row + 1], pz = qp[3 * row + 2];
        const double cs = (dx * (px - R[3 * a]) + dy * (py - R[3 * a + 1]) + dz * (pz - R[3 * a + 2])) / (d * d);
        double c = 0.0;
        for (int l = 0; l <= E.lmax; ++l) {
            double V, dV;
            ecp_radial(E, a, l, d, V, dV);
            c += (double)(2 * l + 1) / 12.0 * V * legendre(l, cs);
        }
        const T *phr = ph + (size_t)row * nc * n;
        const T *ke = kt + (size_t)e * n;
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += (double)phr[j] * (double)ke[j];
        double un = 0.0;
        for (int j = 0; j < N; ++j)
            if (j != e) {
                const double qx = px - sp[3 * j], qy = py - sp[3 * j + 1], qz = pz - sp[3 * j + 2];
                un += ecp_u(qx * qx + qy * qy + qz * qz, S);
            }
        const double jr = exp(un - suo[e]);
        const double cq = c * jr;
        Ew += cq * t;
        double *o = rw + (size_t)row * ECP_ROW;
        o[0] = cq;
        o[1] = t;
        o[2] = jr;
        o[3] = c;
    }
    red[tid] = Ew;
    __syncthreads();
    // the local part, every electron and nucleus
    double El = 0.0;
    for (int i = tid; i < N; i += 256)
        for (int a = 0; a < S.A; ++a) {
            if (E.t0[a] == E.t0[a + 1]) continue;
            const double dx = sp[3 * i] - R[3 * a], dy = sp[3 * i + 1] - R[3 * a + 1], dz = sp[3 * i + 2] - R[3 * a + 2];
            double v, dv;
            ecp_radial(E, a, -1, sqrt(dx * dx + dy * dy + dz * dz), v, dv);
            El += v;
        }
    if (tid == 0 && EL) {
        double enl = 0.0;
        for (int k = 0; k < 256; ++k) enl += red[k];
        red[256] = enl;
    }
    __syncthreads();
    red[tid] = El;
    __syncthreads();
    if (tid == 0 && EL) {
        double s = 0.0;
        for (int k = 0; k < 256; ++k) s += red[k];
        const double e_l = EL[w] + (s + red[256]);
        EL[w] = e_l;
        if (!isfinite(e_l)) atomicOr(status, STATUS_NONFINITE);
    }
    if (!abar) return;
    // K~ of the walker into LDS; each electron's pairs (the pairs are placed
    // electron by electron, so an electron's pairs are one range)
    for (int i = tid; i < N * n; i += 256) skt[i] = (double)kt[i];
    for (int e = tid; e < N; e += 256) pr0[e] = pr0[N + e] = 0;
    __syncthreads();
    for (int pi = tid; pi < np; pi += 256) {
        const int e = pw[pi] & 255;
        if (pi == 0 || (pw[pi - 1] & 255) != e) pr0[e] = pi;
        if (pi == np - 1 || (pw[pi + 1] & 255) != e) pr0[N + e] = pi + 1;
    }
    __syncthreads();
    // Z^T[e][j] = sum over e's points c'_q phi_q[j] (the rows written above)
    for (int idx = tid; idx < N * n; idx += 256) {
        const int e = idx / n, j = idx - (idx / n) * n;
        double z = 0.0;
        for (int pi = pr0[e]; pi < pr0[N + e]; ++pi) {
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const int row = 12 * pi + q;
                z += rw[(size_t)row * ECP_ROW] * (double)ph[(size_t)row * nc * n + j];
            }
        }
        sz[idx] = z;
    }
    // dE/dA_b = -(K~_b Z_b K~_b): sP = Z_b K~_b, then Abar_b -= K~_b sP
    for (int b = 0; b < 2; ++b) {
        const int off = b ? S.n_up : 0, nb = b ? S.n_dn : S.n_up;
        __syncthreads();
        for (int idx = tid; idx < n * n; idx += 256) {
            const int a = idx / n, j = idx - (idx / n) * n;
            double s = 0.0;
            for (int i = 0; i < nb; ++i) s += sz[(size_t)(off + i) * n + a] * skt[(size_t)(off + i) * n + j];
            sP[idx] = s;
        }
        __syncthreads();
        for (int idx = tid; idx < nb * n; idx += 256) {
            const int ei = idx / n, j = idx - (idx / n) * n;
            double s = 0.0;
            for (int a = 0; a < n; ++a) s += skt[(size_t)(off + ei) * n + a] * sP[(size_t)a * n + j];
            T *ab = abar + ((size_t)w * N + off + ei) * n + j;
            *ab = (T)((double)*ab - s);
        }
    }
}

// ---------------------------------------------------------------------------
// The derivatives through the points, two kernels with one block per walker.
// The value and gradient of the lane's AO at displacement (x, y, z) from the
// radial sums R0 and u1 = 2 R' of ao_lane_radial (the first four of the 14
// components of ao_lane_components).
template <typename T, int NPR>
__device__ inline void ao_lane_value_grad(const AoLane<T, NPR> &L, T x, T y, T z, T R0, T u1, T *d) {
    const T r[3] = {x, y, z};
    T f[3], f1[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const T h = fma(L.c2[q], r[q], L.c1[q]);
        f[q] = fma(h, r[q], L.c0[q]);
        f1[q] = fma(L.c2[q], r[q], h);
    }
    const T fyz = f[1] * f[2];
    const T P = f[0] * fyz, PR1 = P * u1;
    d[0] = P * R0;
    d[1] = fma(f1[0] * fyz, R0, x * PR1);
    d[2] = fma(f1[1] * f[0] * f[2], R0, y * PR1);
    d[3] = fma(f1[2] * f[0] * f[1], R0, z * PR1);
}

// k_ecp_points_ao (threads over (AO mu, slot), the slots splitting the
//   points when the AOs are fewer than the threads): G[mu] += sum_q
//   psi_mu(r_q) y_q and tc[mu] = sum_q kappa_q,mu grad psi_mu(r_q),
//   kappa_q = C y_q, over batches of 32 points staged in LDS; the slots'
//   partials added in slot order.
// k_ecp_chain:
//   phase 0 (threads over electrons): jo[e] = sum_{j != e} u'(r_ej) (r_e - r_j)/r_ej;
//            (threads over pairs) es[e] = the sum of E_q = c'_q t_q over e's
//            points, by pair sums added in pair order;
//   phase 2 (threads over points): the chain through r_q = R_a + d v_q, the
//            weights c_q and the Jastrow at r_q, into rows[4..9];
//   phase 3 (threads over (electron, slot)): per electron its own points'
//            terms and the other points' Jastrow terms; (threads over pairs)
//            per nucleus its pairs' point terms in pair order, then V_loc and
//            the AOs at the points (tc; fixed order).
// The pair sums go through LDS in chunks of 256 pairs.
// ---------------------------------------------------------------------------

constexpr int ECP_AO_ROWS = 64;   // points staged per batch

template <typename T, int NT>
__global__ __launch_bounds__(256) void k_ecp_points_ao(SysDev S, const T *__restrict__ C,
                                                       const double *__restrict__ R, EcpBufs<T> eb,
                                                       const T *__restrict__ ktil, double *G, float *Gf) {
    constexpr int NW = 16 * NT, RB = ECP_AO_ROWS;
    extern __shared__ double sm[];
    const int w = blockIdx.x, tid = threadIdx.x;
    const int N = S.N, n = S.n_occ, M = S.M;
    const BasisDev &B = S.basis;
    double *sq = sm;               // [RB][3]
    double *part = sq + 3 * RB;    // [256][16]
    T *sy = (T *)(part + 256 * 16);   // [RB][n]
    const int np = eb.npairs[w], nrow = 12 * np;
    const size_t o0 = (size_t)eb.off[w];
    const int *pw = eb.pairs + o0;
    const T *kt = ktil + (size_t)w * N * n;
    const double *qp = eb.qpos + o0 * 12 * 3;
    const double *rw = eb.rows + o0 * 12 * ECP_ROW;
    double *stc = eb.tc + (size_t)w * M * 3;
    const int nsl = M < 256 ? 256 / M : 1;
    const int per = 256 / nsl;
    constexpr int NPR = sizeof(T) == 4 ? 3 : 0;   // primitives held in registers (FP32)
    for (int mu0 = 0; mu0 < M; mu0 += per) {
        const int mu = mu0 + tid / nsl, slot = tid - (tid / nsl) * nsl;
        const bool vm = tid < per * nsl && mu < M;
        const int mm = vm ? mu : M - 1;
        const int atom = B.shell_atom[B.ao_shell[mm]];
        const double Rx = R[3 * atom], Ry = R[3 * atom + 1], Rz = R[3 * atom + 2];
        // the thread's AO for all points: monomial and primitives in registers
        AoLane<T, NPR> al;
        ao_lane_load<T, NPR>(B, mm, al);
        // (sums over the points in the arithmetic type: in FP32 the mixed
        // measurement's G rows are FP32 too)
        T cr[NW], g[NW];
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            cr[j] = j < n ? C[(size_t)mm * n + j] : T(0);
            g[j] = T(0);
        }
        T tcx = T(0), tcy = T(0), tcz = T(0);
        for (int r0 = 0; r0 < nrow; r0 += RB) {
            __syncthreads();
            for (int idx = tid; idx < RB * n; idx += 256) {
                const int r = idx / n, j = idx - (idx / n) * n, row = r0 + r;
                double y = 0.0;
                if (row < nrow) {
                    const int e = pw[row / 12] & 255;
                    y = rw[(size_t)row * ECP_ROW] * (double)kt[(size_t)e * n + j];
                }
                sy[idx] = (T)y;
            }
            for (int idx = tid; idx < 3 * RB; idx += 256) {
                const int row = r0 + idx / 3;
                sq[idx] = row < nrow ? qp[(size_t)3 * r0 + idx] : 0.0;
            }
            __syncthreads();
            const int nr = min(RB, nrow - r0);
            if (!vm) continue;
            for (int r = slot; r < nr; r += nsl) {
                const double dx = sq[3 * r] - Rx, dy = sq[3 * r + 1] - Ry, dz = sq[3 * r + 2] - Rz;
                const double rho = dx * dx + dy * dy + dz * dz;
                // the AO and its gradient in the arithmetic type (FP32: the
                // split exponential, as in the measurement's adjoint)
                T R0, u1, u2, u3, o[4];
                ao_lane_radial<T, NPR>(al, B, rho, R0, u1, u2, u3);
                ao_lane_value_grad<T, NPR>(al, (T)dx, (T)dy, (T)dz, R0, u1, o);
                T kap = T(0);
                const T *y = sy + (size_t)r * n;
#pragma unroll
                for (int j = 0; j < NW; ++j) {
                    const T yj = j < n ? y[j] : T(0);
                    kap += cr[j] * yj;
                    g[j] += o[0] * yj;
                }
                tcx += kap * o[1];
                tcy += kap * o[2];
                tcz += kap * o[3];
            }
        }
        // the slots' partials, added in slot order (16 columns at a time)
#pragma unroll
        for (int c0 = 0; c0 < NW; c0 += 16) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; ++j) part[tid * 16 + j] = (double)g[c0 + j];
            __syncthreads();
            if (vm && slot == 0)
                for (int j = c0; j < min(n, c0 + 16); ++j) {
                    double t = 0.0;
                    for (int q = 0; q < nsl; ++q) t += part[(tid + q) * 16 + (j - c0)];
                    const size_t o = ((size_t)w * M + mu) * n + j;
                    if (G)
                        G[o] += t;
                    else if (Gf)
                        Gf[o] = (float)((double)Gf[o] + t);
                }
        }
        __syncthreads();
        part[3 * tid] = (double)tcx;
        part[3 * tid + 1] = (double)tcy;
        part[3 * tid + 2] = (double)tcz;
        __syncthreads();
        if (vm && slot == 0)
            for (int k = 0; k < 3; ++k) {
                double t = 0.0;
                for (int q = 0; q < nsl; ++q) t += part[3 * (tid + q) + k];
                stc[3 * mu + k] = t;
            }
    }
}

// ---------------------------------------------------------------------------
// The one-/three-body share of the derivatives through the ratios, one block
// per walker.  With E_q = c'_q t_q, h_e = xi1 + xi3 (s - chi(r_e)) and
// D_e = sum over e's points E_q (chi(r_q) - chi(r_e)), D = sum_e D_e:
//   at each point       g13_q = grad chi(r_q)^T h_e           (rows[10..12]);
//   at electron j       grad chi(r_j)^T xi3 (D - D_j)          (dedr; the
//                       -grad chi(r_e)^T h_e of e's own points is the
//                       electron's Jastrow gradient, taken by k_ecp_chain);
//   per function mu     P_mu = sum_q E_q h_e,mu (grad chi_mu(r_q) - grad chi_mu(r_e))
//                              + sum_j grad chi_mu(r_j) (xi3 (D - D_j))_mu,
//                       added to jtao (the nucleus of mu gets -P_mu).
// Wavefront v takes the electrons e = v mod 4 (e's points are consecutive
// rows), lanes the functions mu = lane + 64 k; the wavefronts' per-function
// partials are added in wavefront order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ecp_jas(int N, EcpJas<T> J, const double *__restrict__ R,
                                                 const double *__restrict__ pos, EcpBufs<T> eb, double *dedr) {
    __shared__ double tv[256], sDs[256];
    __shared__ double sD[4][256], sDt[4][256];
    __shared__ double sPp[4][3][256];
    __shared__ double sel[128 * 3];
    const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, MJ = J.MJ;
    const double *p = pos + (size_t)w * N * 3;
    const int np = eb.npairs[w];
    const size_t o0 = (size_t)eb.off[w];
    const int *pw = eb.pairs + o0;
    const double *qp = eb.qpos + o0 * 12 * 3;
    double *rw = eb.rows + o0 * 12 * ECP_ROW;
    for (int mu = tid; mu < MJ; mu += 256) {
        double t = 0.0;
        for (int e = 0; e < N; ++e) t += ecp_jas_oval(J, (int64_t)w * N + e, mu);
        tv[mu] = t;
    }
    for (int i = tid; i < 3 * N; i += 256) sel[i] = 0.0;
    __syncthreads();
    double Pk[4][3], Dt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Dt[k] = 0.0;
        Pk[k][0] = Pk[k][1] = Pk[k][2] = 0.0;
    }
    int pi = 0;
    for (int e = wave; e < N; e += 4) {
        while (pi < np && (pw[pi] & 255) < e) ++pi;
        int pe = pi;
        while (pe < np && (pw[pe] & 255) == e) ++pe;
        if (pe == pi) continue;
        double hj[4], xe[4], Da[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int mu = lane + 64 * k;
            const bool v = mu < MJ;
            hj[k] = v ? J.xi1[mu] + tv[mu] - ecp_jas_oval(J, (int64_t)w * N + e, mu) : 0.0;
            xe[k] = v ? (double)J.X[((size_t)w * N + e) * MJ + mu] : 0.0;
            Da[k] = 0.0;
        }
        double es = 0.0;
        for (int row = 12 * pi; row < 12 * pe; ++row) {
            double *o = rw + (size_t)row * ECP_ROW;
            const double Eq = o[0] * o[1];
            const double px = qp[3 * row], py = qp[3 * row + 1], pz = qp[3 * row + 2];
            double g3[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int mu = lane + 64 * k;
                if (mu < MJ) {
                    double c5[5];
                    jas_fn<5>(J.jb, R, mu, px, py, pz, c5);
                    Da[k] += Eq * (c5[0] - xe[k]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        g3[d] += c5[1 + d] * hj[k];
                        Pk[k][d] += Eq * hj[k] * c5[1 + d];
                    }
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) g3[d] = wave_sum_dpp(g3[d]);
            if (lane == 0) {
                o[10] = g3[0];
                o[11] = g3[1];
                o[12] = g3[2];
            }
            es += Eq;
        }
        // the electron's own functions, D_e staged for xi3 D_e
        double ge[4][3];
        wave_sync_s();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int mu = lane + 64 * k;
            ge[k][0] = ge[k][1] = ge[k][2] = 0.0;
            if (mu < MJ) {
                double c5[5];
                jas_fn<5>(J.jb, R, mu, p[3 * e], p[3 * e + 1], p[3 * e + 2], c5);
                ge[k][0] = c5[1];
                ge[k][1] = c5[2];
                ge[k][2] = c5[3];
                sD[wave][mu] = Da[k];
            }
            Dt[k] += Da[k];
#pragma unroll
            for (int d = 0; d < 3; ++d) Pk[k][d] -= es * hj[k] * ge[k][d];
        }
        wave_sync_s();
        double el[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int mu = lane + 64 * k;
            if (mu >= MJ) continue;
            // (xi3 D_e)_mu; xi3 symmetric: row nu of column block k
            const double *xb = J.xiblk + (size_t)k * MJ * 64 + lane;
            double x3 = 0.0;
            for (int nu = 0; nu < MJ; ++nu) x3 += xb[(size_t)nu * 64] * sD[wave][nu];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Pk[k][d] -= ge[k][d] * x3;
                el[d] -= ge[k][d] * x3;
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) el[d] = wave_sum_dpp(el[d]);
        if (lane == 0) {
            sel[3 * e] = el[0];
            sel[3 * e + 1] = el[1];
            sel[3 * e + 2] = el[2];
        }
        pi = pe;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int mu = lane + 64 * k;
        if (mu < MJ) {
            sDt[wave][mu] = Dt[k];
            for (int d = 0; d < 3; ++d) sPp[wave][d][mu] = Pk[k][d];
        }
    }
    __syncthreads();
    for (int mu = tid; mu < MJ; mu += 256) sDs[mu] = (sDt[0][mu] + sDt[1][mu]) + (sDt[2][mu] + sDt[3][mu]);
    __syncthreads();
    // per function: the partials, and (xi3 D)_mu sum_j grad chi_mu(r_j)
    // (x3 = (xi3 D)_mu kept in sDt[0] for the electrons' terms)
    const T *Dw = J.D + (size_t)w * N * 4 * MJ;
    for (int mu = tid; mu < MJ; mu += 256) {
        const double *xb = J.xiblk + (size_t)(mu >> 6) * MJ * 64 + (mu & 63);
        double x3 = 0.0;
        for (int nu = 0; nu < MJ; ++nu) x3 += xb[(size_t)nu * 64] * sDs[nu];
        double gs[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < N; ++j)
            for (int d = 0; d < 3; ++d) gs[d] += (double)Dw[((size_t)j * 4 + d) * MJ + mu];
        double *jt = J.jtao + ((size_t)w * MJ + mu) * 6;
        for (int d = 0; d < 3; ++d)
            jt[d] += ((sPp[0][d][mu] + sPp[1][d][mu]) + (sPp[2][d][mu] + sPp[3][d][mu])) + x3 * gs[d];
        sDt[0][mu] = x3;
    }
    __syncthreads();
    // per electron: grad chi(r_j)^T xi3 D, and -grad chi(r_j)^T xi3 D_j
    if (tid < N) {
        const int j = tid;
        double s3[3] = {sel[3 * j], sel[3 * j + 1], sel[3 * j + 2]};
        for (int mu = 0; mu < MJ; ++mu) {
            const double x3 = sDt[0][mu];
            for (int d = 0; d < 3; ++d) s3[d] += (double)Dw[((size_t)j * 4 + d) * MJ + mu] * x3;
        }
        double *de = dedr + ((size_t)w * N + j) * 3;
        de[0] += s3[0];
        de[1] += s3[1];
        de[2] += s3[2];
    }
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ecp_chain(SysDev S, EcpDev E, const double *__restrict__ R,
                                                   const double *__restrict__ pos, EcpBufs<T> eb,
                                                   const T *__restrict__ ktil, double *dedr,
                                                   const double *__restrict__ jg) {
    extern __shared__ double sm[];
    __shared__ int cpi[256];       // a chunk's pairs: electron or nucleus (-1: none)
    const int w = blockIdx.x, tid = threadIdx.x;
    const int N = S.N, n = S.n_occ, M = S.M, A = S.A;
    const BasisDev &B = S.basis;
    double *sp = sm;               // [N][3]
    double *sjo = sp + 3 * N;      // [N][3]
    double *ses = sjo + 3 * N;     // [N]
    double *part = ses + N;        // [256][3] (also a chunk's pair sums)
    const double *stc = eb.tc + (size_t)w * M * 3;
    for (int i = tid; i < 3 * N; i += 256) sp[i] = pos[(size_t)w * N * 3 + i];
    const int np = eb.npairs[w], nrow = 12 * np;
    const size_t o0 = (size_t)eb.off[w];
    const int *pw = eb.pairs + o0;
    const T *ph = eb.phiq + o0 * 12 * 5 * n;
    const T *kt = ktil + (size_t)w * N * n;
    const double *qp = eb.qpos + o0 * 12 * 3;
    double *rw = eb.rows + o0 * 12 * ECP_ROW;
    __syncthreads();
    // ---- phase 0 ----
    if (tid < N) {
        const int e = tid;
        double jx = 0.0, jy = 0.0, jz = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == e) continue;
            const double sx = sp[3 * e] - sp[3 * j], sy_ = sp[3 * e + 1] - sp[3 * j + 1],
                         sz_ = sp[3 * e + 2] - sp[3 * j + 2];
            const double f = ecp_u1r(sx * sx + sy_ * sy_ + sz_ * sz_, S);
            jx += f * sx;
            jy += f * sy_;
            jz += f * sz_;
        }
        if (jg) {
            // the one-/three-body terms: grad_e (U1 + U3) = grad chi(r_e)^T h_e
            const double *g = jg + ((size_t)w * N + e) * 4;
            jx += g[0];
            jy += g[1];
            jz += g[2];
        }
        sjo[3 * e] = jx;
        sjo[3 * e + 1] = jy;
        sjo[3 * e + 2] = jz;
        ses[e] = 0.0;
    }
    for (int p0 = 0; p0 < np; p0 += 256) {
        __syncthreads();
        const int pi = p0 + tid;
        double sq = 0.0;
        if (pi < np)
            for (int q = 0; q < 12; ++q) {
                const double *o = rw + (size_t)(12 * pi + q) * ECP_ROW;
                sq += o[0] * o[1];
            }
        part[tid] = sq;
        cpi[tid] = pi < np ? (pw[pi] & 255) : -1;
        __syncthreads();
        if (tid < N) {
            double es = ses[tid];
            for (int k = 0; k < min(256, np - p0); ++k)
                if (cpi[k] == tid) es += part[k];
            ses[tid] = es;
        }
    }
    __syncthreads();
    // ---- phase 2 ----
    for (int row = tid; row < nrow; row += 256) {
        const int pr = pw[row / 12], e = pr & 255, a = pr >> 8;
        const double ex = sp[3 * e], ey = sp[3 * e + 1], ez = sp[3 * e + 2];
        const double dx = ex - R[3 * a], dy = ey - R[3 * a + 1], dz = ez - R[3 * a + 2];
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double u[3] = {dx / d, dy / d, dz / d};
        const double px = qp[3 * row], py = qp[3 * row + 1], pz = qp[3 * row + 2];
        const double v[3] = {(px - R[3 * a]) / d, (py - R[3 * a + 1]) / d, (pz - R[3 * a + 2]) / d};
        const double cs = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
        double *o = rw + (size_t)row * ECP_ROW;
        const double cq = o[0], t = o[1], jr = o[2];
        const double Eq = cq * t, hq = jr * t;
        // dE/dr_q through the orbitals: cq sum_j K~[e][j] grad phi_j(r_q)
        double g[3] = {0.0, 0.0, 0.0};
        const T *pr5 = ph + (size_t)row * 5 * n;
        // (unrolled: the loads of several orbitals in flight together)
#pragma unroll 4
        for (int j = 0; j < n; ++j) {
            const double kj = (double)kt[(size_t)e * n + j];
            g[0] += kj * (double)pr5[n + j];
            g[1] += kj * (double)pr5[2 * n + j];
            g[2] += kj * (double)pr5[3 * n + j];
        }
        // through the Jastrow at r_q
        double gj[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < N; ++j) {
            if (j == e) continue;
            const double qx = px - sp[3 * j], qy = py - sp[3 * j + 1], qz = pz - sp[3 * j + 2];
            const double fq = ecp_u1r(qx * qx + qy * qy + qz * qz, S);
            gj[0] += fq * qx;
            gj[1] += fq * qy;
            gj[2] += fq * qz;
        }
        if (jg)
#pragma unroll
            for (int k = 0; k < 3; ++k) gj[k] += o[10 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = cq * g[k] + Eq * gj[k];
        // c_q through d and u . v
        double dc[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l <= E.lmax; ++l) {
            double V, dV;
            ecp_radial(E, a, l, d, V, dV);
            const double wl = (double)(2 * l + 1) / 12.0;
            const double f1 = wl * dV * legendre(l, cs), f2 = wl * V * legendre_d(l, cs) / d;
#pragma unroll
            for (int k = 0; k < 3; ++k) dc[k] += f1 * u[k] + f2 * (v[k] - cs * u[k]);
        }
        const double gv = g[0] * v[0] + g[1] * v[1] + g[2] * v[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[4 + k] = gv * u[k] + hq * dc[k] - Eq * sjo[3 * e + k];   // to r_e
            o[7 + k] = g[k] - gv * u[k] - hq * dc[k];                  // to R_a
        }
    }
    __syncthreads();
    // ---- phase 3: electrons, (electron, slot) over the points ----
    const int esl = 256 / N;
    {
        const int j = tid / esl, slot = tid - (tid / esl) * esl;
        double s3[3] = {0.0, 0.0, 0.0};
        if (j < N) {
            const double xj = sp[3 * j], yj = sp[3 * j + 1], zj = sp[3 * j + 2];
#pragma unroll 4
            for (int row = slot; row < nrow; row += esl) {
                const double *o = rw + (size_t)row * ECP_ROW;
                if ((pw[row / 12] & 255) == j) {
                    s3[0] += o[4];
                    s3[1] += o[5];
                    s3[2] += o[6];
                    continue;
                }
                // the Jastrow change of another electron's point, through r_j
                const double Eq = o[0] * o[1];
                const double qx = qp[3 * row] - xj, qy = qp[3 * row + 1] - yj, qz = qp[3 * row + 2] - zj;
                const double fq = Eq * ecp_u1r(qx * qx + qy * qy + qz * qz, S);
                s3[0] -= fq * qx;
                s3[1] -= fq * qy;
                s3[2] -= fq * qz;
            }
        }
        part[3 * tid] = s3[0];
        part[3 * tid + 1] = s3[1];
        part[3 * tid + 2] = s3[2];
    }
    __syncthreads();
    if (tid < N) {
        const int j = tid;
        double s3[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < esl; ++q)
            for (int k = 0; k < 3; ++k) s3[k] += part[3 * (j * esl + q) + k];
        const double xj = sp[3 * j], yj = sp[3 * j + 1], zj = sp[3 * j + 2];
        // ... and through r_j in the pair terms at the other electrons' own positions
        for (int e = 0; e < N; ++e) {
            if (e == j || ses[e] == 0.0) continue;
            const double sx = sp[3 * e] - xj, sy_ = sp[3 * e + 1] - yj, sz_ = sp[3 * e + 2] - zj;
            const double fe = ses[e] * ecp_u1r(sx * sx + sy_ * sy_ + sz_ * sz_, S);
            s3[0] += fe * sx;
            s3[1] += fe * sy_;
            s3[2] += fe * sz_;
        }
        for (int a = 0; a < A; ++a) {
            if (E.t0[a] == E.t0[a + 1]) continue;
            const double dx = xj - R[3 * a], dy = yj - R[3 * a + 1], dz = zj - R[3 * a + 2];
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            double v, dv;
            ecp_radial(E, a, -1, d, v, dv);
            s3[0] += dv * dx / d;
            s3[1] += dv * dy / d;
            s3[2] += dv * dz / d;
        }
        double *de = dedr + ((size_t)w * N + j) * 3;
        de[0] += s3[0];
        de[1] += s3[1];
        de[2] += s3[2];
    }
    // per nucleus: its pairs' point terms
    double sa[3] = {0.0, 0.0, 0.0};
    for (int p0 = 0; p0 < np; p0 += 256) {
        __syncthreads();
        const int pi = p0 + tid;
        double s3[3] = {0.0, 0.0, 0.0};
        if (pi < np)
            for (int q = 0; q < 12; ++q) {
                const double *o = rw + (size_t)(12 * pi + q) * ECP_ROW;
                s3[0] += o[7];
                s3[1] += o[8];
                s3[2] += o[9];
            }
        part[3 * tid] = s3[0];
        part[3 * tid + 1] = s3[1];
        part[3 * tid + 2] = s3[2];
        cpi[tid] = pi < np ? (pw[pi] >> 8) : -1;
        __syncthreads();
        if (tid < A)
            for (int k = 0; k < min(256, np - p0); ++k)
                if (cpi[k] == tid) {
                    sa[0] += part[3 * k];
                    sa[1] += part[3 * k + 1];
                    sa[2] += part[3 * k + 2];
                }
    }
    if (tid < A) {
        const int a = tid;
        double s3[3] = {sa[0], sa[1], sa[2]};
        if (E.t0[a] != E.t0[a + 1])
            for (int j = 0; j < N; ++j) {
                const double dx = sp[3 * j] - R[3 * a], dy = sp[3 * j + 1] - R[3 * a + 1], dz = sp[3 * j + 2] - R[3 * a + 2];
                const double d = sqrt(dx * dx + dy * dy + dz * dz);
                double v, dv;
                ecp_radial(E, a, -1, d, v, dv);
                s3[0] -= dv * dx / d;
                s3[1] -= dv * dy / d;
                s3[2] -= dv * dz / d;
            }
        // the AOs at the points move with their nuclei
        for (int q = B.atom_ao_ptr[a]; q < B.atom_ao_ptr[a + 1]; ++q) {
            const int mu = B.atom_ao[q];
            s3[0] -= stc[3 * mu];
            s3[1] -= stc[3 * mu + 1];
            s3[2] -= stc[3 * mu + 2];
        }
        double *o = eb.ecp_dR + ((size_t)w * A + a) * 3;
        o[0] = s3[0];
        o[1] = s3[1];
        o[2] = s3[2];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_ecp_pairs(const SysDev &S, const EcpDev &E, const double *R, const double *pos, int W,
                            int64_t id0, const int *idlist, uint32_t rot, int *pairs, int *npairs, int *off,
                            int *nrows, double *qpos, int *status, hipStream_t st) {
    if (S.N > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ecp_count, dim3(W), dim3(128), 0, st, S, E, R, pos, npairs);
    hipLaunchKernelGGL(k_ecp_scan, dim3(1), dim3(1024), 0, st, W, (int64_t)W * E.pcap, npairs, off, nrows, status);
    hipLaunchKernelGGL(k_ecp_place, dim3(W), dim3(128), 0, st, S, E, R, pos, id0, idlist, rot, npairs, off, pairs,
                       qpos);
    return hipGetLastError();
}

static size_t ecp_points_ao_lds(int n) { return sizeof(double) * ((size_t)ECP_AO_ROWS * n + 3 * ECP_AO_ROWS + 256 * 16); }
static size_t ecp_chain_lds(int N) { return sizeof(double) * ((size_t)7 * N + 256 * 3); }

hipError_t configure_ecp(size_t lds) {
    const void *f[4] = {(const void *)k_ecp_energy_pts<double>, (const void *)k_ecp_energy_pts<float>,
                        (const void *)k_ecp_energy<double, true>, (const void *)k_ecp_energy<float, true>};
    for (const void *g : f) {
        const hipError_t e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_ecp_energy(const SysDev &S, const EcpDev &E, const double *R, const double *pos, int W,
                             const EcpBufs<T> &eb, int nc, const T *ktil, T *abar, double *EL, int *status,
                             const EcpJas<T> &J, hipStream_t st) {
    if (J.X && (J.MJ > 256 || S.N > 128)) return hipErrorInvalidValue;
    if (J.X)
        hipLaunchKernelGGL((k_ecp_energy<T, true>), dim3(W), dim3(256),
                           sizeof(double) * ((size_t)3 * S.N + (size_t)S.N * S.n_occ + (size_t)S.n_occ * S.n_occ +
                                             132 + (size_t)J.MJ),
                           st, S, E,
                           R, pos, eb, nc, ktil, abar, EL, status, J);
    else
        hipLaunchKernelGGL((k_ecp_energy_pts<T>), dim3(W), dim3(256), ecp_energy_pts_lds(S.N, S.n_occ), st, S, E, R,
                           pos, eb, nc, ktil, abar, EL, status);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ecp_adjoint(const SysDev &S, const EcpDev &E, const T *C, const double *R, const double *pos,
                              int W, const EcpBufs<T> &eb, const T *ktil, double *G, float *Gf, double *dedr,
                              const EcpJas<T> &J, hipStream_t st) {
    if (J.X) {
        if (J.MJ > 256 || S.N > 128) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_ecp_jas<T>), dim3(W), dim3(256), 0, st, S.N, J, R, pos, eb, dedr);
    }
    const size_t lds = ecp_points_ao_lds(S.n_occ);
    const int nt = (S.n_occ + 15) / 16;
    if (nt == 1)
        hipLaunchKernelGGL((k_ecp_points_ao<T, 1>), dim3(W), dim3(256), lds, st, S, C, R, eb, ktil, G, Gf);
    else if (nt == 2)
        hipLaunchKernelGGL((k_ecp_points_ao<T, 2>), dim3(W), dim3(256), lds, st, S, C, R, eb, ktil, G, Gf);
    else if (nt == 3)
        hipLaunchKernelGGL((k_ecp_points_ao<T, 3>), dim3(W), dim3(256), lds, st, S, C, R, eb, ktil, G, Gf);
    else
        hipLaunchKernelGGL((k_ecp_points_ao<T, 4>), dim3(W), dim3(256), lds, st, S, C, R, eb, ktil, G, Gf);
    hipLaunchKernelGGL((k_ecp_chain<T>), dim3(W), dim3(256), ecp_chain_lds(S.N), st, S, E, R, pos, eb, ktil, dedr,
                       J.X ? J.jg : nullptr);
    return hipGetLastError();
}

#define ECP_INST(T)                                                                                                \
    template hipError_t launch_ecp_energy<T>(const SysDev &, const EcpDev &, const double *, const double *, int,     \
                                             const EcpBufs<T> &, int, const T *, T *, double *, int *,               \
                                             const EcpJas<T> &, hipStream_t);                                        \
    template hipError_t launch_ecp_adjoint<T>(const SysDev &, const EcpDev &, const T *, const double *,             \
                                              const double *, int, const EcpBufs<T> &, const T *, double *, float *, \
                                              double *, const EcpJas<T> &, hipStream_t);
ECP_INST(double)
ECP_INST(float)

}  // namespace vmcx
