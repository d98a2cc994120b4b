// vmc_device.hpp -- device math of the VMC hot path (gfx950).
//
// The random numbers, tables and Jastrow value are __host__ __device__ (plain
// arithmetic); the AO evaluation, reciprocals and wavefront sums use device
// builtins and are device-only.  The kernels live in the vmc_*.hip sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmcx {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit
// multiplies with xor of the key; key advanced by the Weyl constants.
// Counter layout of the Markov-chain draws: (walker, sweep, electron |
// purpose << 16, 0), key = (seed lo, seed hi).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

enum : uint32_t { PURPOSE_NORMAL = 0, PURPOSE_UNIFORM = 1 };

__host__ __device__ inline U4 draw_words(uint64_t seed, uint32_t walker, uint32_t sweep,
                                         uint32_t electron, uint32_t purpose) {
    return philox4x32_10(U4{walker, sweep, (electron & 0xFFFFu) | (purpose << 16), 0u},
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Box-Muller from two words: u1 in (0,1], u2 in [0,1).
__host__ __device__ inline void box_muller(uint32_t a, uint32_t b, double &z0, double &z1) {
    const double u1 = ((double)a + 1.0) * 2.3283064365386963e-10;   // 2^-32
    const double u2 = (double)b * 2.3283064365386963e-10;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;
    z0 = rad * cos(ang);
    z1 = rad * sin(ang);
}

// Three proposal normals and the accept uniform of one move.
// The proposal's three normals z of one move.
__host__ __device__ inline void move_normals(uint64_t seed, uint32_t walker, uint32_t sweep,
                                             uint32_t electron, double z[3]) {
    const U4 a = draw_words(seed, walker, sweep, electron, PURPOSE_NORMAL);
    double t;
    box_muller(a.x, a.y, z[0], z[1]);
    box_muller(a.z, a.w, z[2], t);
}

// The accept test's uniform u in [0, 1) of one move (53 random bits).
__host__ __device__ inline double move_uniform(uint64_t seed, uint32_t walker, uint32_t sweep, uint32_t electron) {
    const U4 b = draw_words(seed, walker, sweep, electron, PURPOSE_UNIFORM);
    const uint64_t bits = ((uint64_t)b.x << 21) | ((uint64_t)b.y >> 11);
    return (double)bits * 1.1102230246251565e-16;                   // 2^-53
}

// ---------------------------------------------------------------------------
// Basis tables (device pointers), normalisation folded in by the host.
// AO mu: shell ao_shell[mu], monomial exponents ao_pow[mu] = a | b<<4 | c<<8,
// component factor ao_eta[mu]; shell s: atom, first primitive, count.
// ---------------------------------------------------------------------------
struct BasisDev {
    int n_ao;
    int n_shells;
    const int *ao_shell;
    const int *ao_pow;
    const double *ao_eta;
    const int *shell_atom;
    const int *shell_p0;
    const int *shell_np;
    const double *prim_exp;
    const double *prim_cp;   // radial coefficient incl. all norms
    const int *shell_l;
    const int *shell_mu0;    // first AO of the shell
    const int *atom_ao_ptr;  // [A + 1]: the AOs of atom a are atom_ao[ptr[a] .. ptr[a + 1])
    const int *atom_ao;      // [M]
};

// Monomial exponents of cartesian component q of a shell with angular
// momentum l, in the order s; x,y,z; xx,xy,xz,yy,yz,zz (packed a | b<<4 | c<<8).
__host__ __device__ inline int cart_pow(int l, int q) {
    const int first = l == 0 ? 0 : (l == 1 ? 1 : 4);
    const int tab[10] = {0x000, 0x001, 0x010, 0x100, 0x002, 0x011, 0x101, 0x020, 0x110, 0x200};
    return tab[first + q];
}

__host__ __device__ inline int n_cart(int l) { return (l + 1) * (l + 2) / 2; }

template <typename T>
__host__ __device__ inline T tpow(T x, int k) {
    return k <= 0 ? (k == 0 ? T(1) : T(0)) : (k == 1 ? x : x * x);
}

// e^{-x} for x = a rho >= 0 in the arithmetic type T.  In FP32 the exponent
// is formed in FP64 and split into FP32 parts before the exponential
// (exp2_neg_split): rounding x itself to FP32 would cost a relative error of
// x 2^-24 in the result (1e-6 at x = 20).
__device__ inline float exp2_neg_split(double t);
__host__ __device__ inline double exp_neg(double a, double rho, double) { return exp(-a * rho); }
__device__ inline float exp_neg(double a, double rho, float) {
    return exp2_neg_split(a * rho * 1.4426950408889634);
}

// Entry of an array that the running kernel does not write (tables, or data
// of earlier kernels), read through the constant address space: with a
// wavefront-uniform index it becomes a scalar load.
template <typename T>
__device__ inline T ldc(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// Radial sums of shell s at rho = |r - R_A|^2 (formed in FP64):
// R0 = sum c' e^{-a rho} and its first three rho-derivatives (NC > 5 needs R3).
template <int NC, typename T>
__device__ inline void shell_radial(const BasisDev &B, int s, double rho, T &R0, T &R1, T &R2, T &R3) {
    const int p0 = ldc(B.shell_p0 + s), np = ldc(B.shell_np + s);
    R0 = R1 = R2 = R3 = T(0);
    for (int k = 0; k < np; ++k) {
        // the exponent in the arithmetic type, used alike in the exponential
        // and in the derivative factors, so that value and derivatives belong
        // to one function
        const T al = (T)ldc(B.prim_exp + p0 + k);
        const T e = (T)ldc(B.prim_cp + p0 + k) * exp_neg((double)al, rho, T(0));
        R0 += e;
        if (NC > 1) {
            R1 -= al * e;
            R2 += al * al * e;
            if (NC > 5) R3 -= al * al * al * e;
        }
    }
}

// Derivative components of one cartesian AO eta x^a y^b z^c R(rho) (x,y,z
// relative to the centre), written to out[0..NC):
//   NC = 1  : value
//   NC = 5  : value, d/dx, d/dy, d/dz, laplacian
//   NC = 14 : + hessian xx,xy,xz,yy,yz,zz (5..10), d(lap)/dx,dy,dz (11..13)
// Monomials have l <= 2, so their laplacian is constant.
template <int NC, typename T>
__host__ __device__ inline void ao_components(T x, T y, T z, T rho, T R0, T R1, T R2, T R3, int pw, T eta,
                                              T *out) {
    const int a = pw & 15, b = (pw >> 4) & 15, c = (pw >> 8) & 15;
    const int l = a + b + c;
    const T xa = tpow(x, a), yb = tpow(y, b), zc = tpow(z, c);
    const T P = xa * yb * zc;
    out[0] = eta * P * R0;
    if (NC == 1) return;
    const T Px = T(a) * tpow(x, a - 1) * yb * zc;
    const T Py = T(b) * xa * tpow(y, b - 1) * zc;
    const T Pz = T(c) * xa * yb * tpow(z, c - 1);
    const T Pxx = T(a * (a - 1)) * tpow(x, a - 2) * yb * zc;
    const T Pyy = T(b * (b - 1)) * xa * tpow(y, b - 2) * zc;
    const T Pzz = T(c * (c - 1)) * xa * yb * tpow(z, c - 2);
    const T lapP = Pxx + Pyy + Pzz;
    const T two = T(2);
    out[1] = eta * (Px * R0 + two * x * P * R1);
    out[2] = eta * (Py * R0 + two * y * P * R1);
    out[3] = eta * (Pz * R0 + two * z * P * R1);
    // lap[P R(rho)] = lapP R + 4 (x.gradP) R' + P (6 R' + 4 rho R''), x.gradP = l P
    out[4] = eta * (lapP * R0 + T(4 * l + 6) * P * R1 + T(4) * rho * P * R2);
    if (NC == 5) return;
    const T Pxy = T(a * b) * tpow(x, a - 1) * tpow(y, b - 1) * zc;
    const T Pxz = T(a * c) * tpow(x, a - 1) * yb * tpow(z, c - 1);
    const T Pyz = T(b * c) * xa * tpow(y, b - 1) * tpow(z, c - 1);
    const T four = T(4);
    // d_i d_j [P R] = P_ij R + 2 (x_j P_i + x_i P_j) R' + 2 delta_ij P R' + 4 x_i x_j P R''
    out[5] = eta * (Pxx * R0 + four * x * Px * R1 + two * P * R1 + four * x * x * P * R2);
    out[6] = eta * (Pxy * R0 + two * (y * Px + x * Py) * R1 + four * x * y * P * R2);
    out[7] = eta * (Pxz * R0 + two * (z * Px + x * Pz) * R1 + four * x * z * P * R2);
    out[8] = eta * (Pyy * R0 + four * y * Py * R1 + two * P * R1 + four * y * y * P * R2);
    out[9] = eta * (Pyz * R0 + two * (z * Py + y * Pz) * R1 + four * y * z * P * R2);
    out[10] = eta * (Pzz * R0 + four * z * Pz * R1 + two * P * R1 + four * z * z * P * R2);
    // d_k lap[P R]: (2 x_k lapP + (4l+6) P_k) R' + ((8l+20) x_k P + 4 rho P_k) R'' + 8 rho x_k P R'''
    const T c1 = T(4 * l + 6), c2 = T(8 * l + 20), eight = T(8);
    out[11] = eta * ((two * x * lapP + c1 * Px) * R1 + (c2 * x * P + four * rho * Px) * R2 + eight * rho * x * P * R3);
    out[12] = eta * ((two * y * lapP + c1 * Py) * R1 + (c2 * y * P + four * rho * Py) * R2 + eight * rho * y * P * R3);
    out[13] = eta * ((two * z * lapP + c1 * Pz) * R1 + (c2 * z * P + four * rho * Pz) * R2 + eight * rho * z * P * R3);
}

// ---------------------------------------------------------------------------
// One AO held by one lane across many electrons (the adjoint's layout): the
// shell's primitives and the monomial are loaded once into registers.
//
// FP32 exponential of the primitives: t = a rho log2(e) is formed in FP64 and
// split as t = th + tl (th = fp32(t)); 2^-t = 2^-th (1 - tl ln 2) up to
// (tl ln 2)^2 / 2 < 1e-10 relative for t < 150, with 2^-th from the hardware
// base-2 exponential.  The FP64 path calls exp.
// ---------------------------------------------------------------------------
__device__ inline float exp2_neg_split(double t) {
    const float th = (float)t;
    const float tl = (float)(t - (double)th);
    return __builtin_amdgcn_exp2f(-th) * fmaf(-tl, 0.69314718055994531f, 1.0f);
}

template <typename T, int NPR>
struct AoLane {
    // monomial eta x^a y^b z^c as a product of per-axis quadratics
    // f_q(t) = c0 + c1 t + c2 t^2 with one-hot coefficients (eta folded into
    // the x axis), so that f, f' = c1 + 2 c2 t and f'' = 2 c2 need no branch
    T c0[3], c1[3], c2[3], c22[3];   // c22 = 2 c2
    T h46, h820;               // (4l + 6) / 2 and (8l + 20) / 4
    int np, p0;                // primitives of the shell
    T al[NPR], al2[NPR], al3[NPR], cp[NPR];   // first NPR exponents (in T), their powers, coefficients
    double alt[NPR];           // al * log2(e) in FP64 (FP32 exponential)
};

template <typename T, int NPR>
__device__ inline void ao_lane_load(const BasisDev &B, int mu, AoLane<T, NPR> &L) {
    const int s = B.ao_shell[mu], pw = B.ao_pow[mu];
    const T eta = (T)B.ao_eta[mu];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int p = (pw >> (4 * q)) & 15;
        const T sc = q == 0 ? eta : T(1);
        L.c0[q] = p == 0 ? sc : T(0);
        L.c1[q] = p == 1 ? sc : T(0);
        L.c2[q] = p == 2 ? sc : T(0);
        L.c22[q] = L.c2[q] + L.c2[q];
    }
    const int l = B.shell_l[s];
    L.h46 = T(2 * l + 3);
    L.h820 = T(2 * l + 5);
    L.np = B.shell_np[s];
    L.p0 = B.shell_p0[s];
#pragma unroll
    for (int k = 0; k < NPR; ++k) {
        const int p = L.p0 + max(min(k, L.np - 1), 0);
        L.al[k] = (T)B.prim_exp[p];
        L.al2[k] = L.al[k] * L.al[k];
        L.al3[k] = L.al2[k] * L.al[k];
        L.cp[k] = k < L.np ? (T)B.prim_cp[p] : T(0);
        L.alt[k] = (double)L.al[k] * 1.4426950408889634;
    }
}

template <typename T>
__device__ inline T prim_exp_neg(T al, double alt, double rho);
template <>
__device__ inline float prim_exp_neg<float>(float, double alt, double rho) {
    return exp2_neg_split(alt * rho);
}
template <>
__device__ inline double prim_exp_neg<double>(double al, double, double rho) {
    return exp(-al * rho);
}

// Radial sums of the lane's shell at rho (FP64): R0 = sum c' e^{-a rho} and
// u1 = 2 R0', u2 = 4 R0'', u3 = 8 R0''' (derivatives in rho).
template <typename T, int NPR>
__device__ inline void ao_lane_radial(const AoLane<T, NPR> &L, const BasisDev &B, double rho, T &R0, T &u1,
                                      T &u2, T &u3) {
    T r0 = T(0), r1 = T(0), r2 = T(0), r3 = T(0);
#pragma unroll
    for (int k = 0; k < NPR; ++k) {
        // padded primitives carry cp = 0
        const T e = L.cp[k] * prim_exp_neg<T>(L.al[k], L.alt[k], rho);
        r0 += e;
        r1 = fma(-L.al[k], e, r1);
        r2 = fma(L.al2[k], e, r2);
        r3 = fma(-L.al3[k], e, r3);
    }
    for (int k = NPR; k < L.np; ++k) {
        const T al = (T)B.prim_exp[L.p0 + k];
        const T e = (T)B.prim_cp[L.p0 + k] * prim_exp_neg<T>(al, (double)al * 1.4426950408889634, rho);
        r0 += e;
        r1 = fma(-al, e, r1);
        r2 = fma(al * al, e, r2);
        r3 = fma(-(al * al * al), e, r3);
    }
    R0 = r0;
    u1 = T(2) * r1;
    u2 = T(4) * r2;
    u3 = T(8) * r3;
}

// The 14 components of ao_components<14> for the lane's AO at displacement
// (x, y, z), rho = x^2 + y^2 + z^2, from R0, u1, u2, u3 of ao_lane_radial.
template <typename T, int NPR>
__device__ inline void ao_lane_components(const AoLane<T, NPR> &L, T x, T y, T z, T rho, T R0, T u1, T u2, T u3,
                                          T *d) {
    const T r[3] = {x, y, z};
    T f[3], f1[3], f2[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const T h = fma(L.c2[q], r[q], L.c1[q]);
        f[q] = fma(h, r[q], L.c0[q]);
        f1[q] = fma(L.c2[q], r[q], h);
        f2[q] = L.c22[q];
    }
    const T fyz = f[1] * f[2], fxz = f[0] * f[2], fxy = f[0] * f[1];
    const T P = f[0] * fyz;
    const T Px = f1[0] * fyz, Py = f1[1] * fxz, Pz = f1[2] * fxy;
    const T Pxx = f2[0] * fyz, Pyy = f2[1] * fxz, Pzz = f2[2] * fxy;
    const T Pxy = f1[0] * f1[1] * f[2], Pxz = f1[0] * f1[2] * f[1], Pyz = f1[1] * f1[2] * f[0];
    const T lapP = Pxx + Pyy + Pzz;
    const T PR1 = P * u1, PR2 = P * u2;                   // 2 P R', 4 P R''
    const T Pxu = Px * u1, Pyu = Py * u1, Pzu = Pz * u1;  // 2 P_k R'
    d[0] = P * R0;
    d[1] = fma(Px, R0, x * PR1);
    d[2] = fma(Py, R0, y * PR1);
    d[3] = fma(Pz, R0, z * PR1);
    // lapP R + (4l + 6) P R' + 4 rho P R''
    d[4] = fma(lapP, R0, fma(L.h46, PR1, rho * PR2));
    // P_kk R + 4 x_k P_k R' + 2 P R' + 4 x_k^2 P R''
    const T xP2 = x * PR2, yP2 = y * PR2, zP2 = z * PR2;
    d[5] = fma(Pxx, R0, fma(x + x, Pxu, fma(x, xP2, PR1)));
    d[8] = fma(Pyy, R0, fma(y + y, Pyu, fma(y, yP2, PR1)));
    d[10] = fma(Pzz, R0, fma(z + z, Pzu, fma(z, zP2, PR1)));
    // P_kj R + 2 (x_j P_k + x_k P_j) R' + 4 x_k x_j P R''
    d[6] = fma(Pxy, R0, fma(y, Pxu, fma(x, Pyu, x * yP2)));
    d[7] = fma(Pxz, R0, fma(z, Pxu, fma(x, Pzu, x * zP2)));
    d[9] = fma(Pyz, R0, fma(z, Pyu, fma(y, Pzu, y * zP2)));
    // d_k lap = x_k (2 lapP R' + (8l + 20) P R'' + 8 rho P R''') + P_k ((4l + 6) R' + 4 rho R'')
    const T S1 = fma(lapP, u1, fma(L.h820, PR2, rho * P * u3));
    const T S2 = fma(L.h46, u1, rho * u2);
    d[11] = fma(x, S1, Px * S2);
    d[12] = fma(y, S1, Py * S2);
    d[13] = fma(z, S1, Pz * S2);
}

// Sum over the 16 lanes of each DPP row, left in the row's last lane (lane
// 15 of the row; the other lanes hold partial sums): an inclusive scan with
// row shifts 1, 2, 4, 8, lanes shifted in from outside the row reading 0.
template <int K>
__device__ inline double dpp_row_shr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x110 + K, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x110 + K, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int K>
__device__ inline float dpp_row_shr(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x110 + K, 0xF, 0xF, true));
}

template <typename T>
__device__ inline T row16_sum_last(T v) {
    v += dpp_row_shr<1>(v);
    v += dpp_row_shr<2>(v);
    v += dpp_row_shr<4>(v);
    v += dpp_row_shr<8>(v);
    return v;
}

// Sum over the wavefront (all 64 lanes active), the same in every lane: the
// four DPP row sums, then their totals by lane reads, in a fixed order.
__device__ inline double wave_sum_dpp(double v) {
    v = row16_sum_last<double>(v);
    const long long b = __double_as_longlong(v);
    double r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lo = __builtin_amdgcn_readlane((int)b, 16 * q + 15);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * q + 15);
        r[q] = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    }
    return (r[0] + r[1]) + (r[2] + r[3]);
}

// All cartesian components of shell s at an electron, with the angular
// momentum fixed at compile time so that every component index is a constant
// and nothing lands in per-lane scratch: stored straight to dst[q*NC + k] (LDS
// or registers).  The displacement is formed in FP64 and rounded to T.
template <int NC, typename T, int L>
__device__ inline void shell_components(const BasisDev &B, int mu0, T x, T y, T z, T rho, T R0, T R1, T R2, T R3,
                                        T *dst) {
#pragma unroll
    for (int q = 0; q < (L + 1) * (L + 2) / 2; ++q) {
        T o[NC];
        ao_components<NC, T>(x, y, z, rho, R0, R1, R2, R3, cart_pow(L, q), (T)ldc(B.ao_eta + mu0 + q), o);
#pragma unroll
        for (int k = 0; k < NC; ++k) dst[q * NC + k] = o[k];
    }
}

// Shell s (uniform over the wavefront in the callers) at one electron per
// lane; the basis tables and R are read with ldc.
template <int NC, typename T>
__device__ inline int shell_eval_to(const BasisDev &B, const double *R, int s, double rx, double ry, double rz,
                                    T *dst) {
    const int atom = ldc(B.shell_atom + s);
    const double dx = rx - ldc(R + 3 * atom), dy = ry - ldc(R + 3 * atom + 1), dz = rz - ldc(R + 3 * atom + 2);
    const double rho_d = dx * dx + dy * dy + dz * dz;
    const T x = (T)dx, y = (T)dy, z = (T)dz;
    const T rho = (T)rho_d;
    T R0, R1, R2, R3;
    shell_radial<NC, T>(B, s, rho_d, R0, R1, R2, R3);
    const int l = ldc(B.shell_l + s), mu0 = ldc(B.shell_mu0 + s);
    if (l == 0) {
        shell_components<NC, T, 0>(B, mu0, x, y, z, rho, R0, R1, R2, R3, dst);
        return 1;
    }
    if (l == 1) {
        shell_components<NC, T, 1>(B, mu0, x, y, z, rho, R0, R1, R2, R3, dst);
        return 3;
    }
    shell_components<NC, T, 2>(B, mu0, x, y, z, rho, R0, R1, R2, R3, dst);
    return 6;
}

// 1/sqrt(x) and 1/x (x > 0) in FP64: the hardware estimate refined by two
// Newton-Raphson steps, y <- y (3 - x y^2) / 2 and y <- y (2 - x y).
__device__ inline double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    return y * (1.5 - 0.5 * x * y * y);
}

__device__ inline double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * (2.0 - x * y);
    return y * (2.0 - x * y);
}

// ---------------------------------------------------------------------------
// Two-body Jastrow function u(r) and its derivatives:
//   form 0 (Pade)       u = a r / (1 + F r)
//   form 1 (exponential) u = a (1 - e^{-F r}) / F
// ---------------------------------------------------------------------------
__host__ __device__ inline double jas_u(double r, double a, double F, int form) {
    return form == 1 ? a * (1.0 - exp(-F * r)) / F : a * r / (1.0 + F * r);
}

struct JasD {
    double u, u1, u2, u3;
};

__device__ inline JasD jas_all(double r, double a, double F, int form) {
    if (form == 1) {
        const double e = exp(-F * r), ae = a * e;
        return JasD{a * (1.0 - e) / F, ae, -F * ae, F * F * ae};
    }
    const double q = rcp_nr(1.0 + F * r);
    const double q2 = q * q;
    return JasD{a * r * q, a * q2, -2.0 * a * F * q2 * q, 6.0 * a * F * F * q2 * q2};
}

}  // namespace vmcx
