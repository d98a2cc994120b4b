"""Cartesian contracted Gaussian-type orbitals (oracle).

The paper expands the pairing function, hence the molecular orbitals, over
GTOs psi_mu (Appendix A, eq. agp_expansion and eq. restricted-C).  Its
Sec. III notes that codes differ in cartesian vs spherical GTOs and in where
normalisation is applied.  Reading used here:
  * cartesian components, order  s;  x, y, z;  xx, xy, xz, yy, yz, zz;
  * contraction coefficients multiply unit-normalised primitives;
  * the contracted function is renormalised so that every cartesian
    component has unit norm.

With x = r - R_A and rho = |x|^2 a component is
    psi(r) = eta(a,b,c) x^a y^b z^c R(rho),   R(rho) = sum_k c'_k exp(-alpha_k rho),
eta = ((2a-1)!!(2b-1)!!(2c-1)!!)^(-1/2); c'_k folds the primitive radial norm
(2 alpha/pi)^(3/4) (4 alpha)^(l/2) and the shell renormalisation.

Every expression is complex-analytic in r and R_A (no abs, no branch on the
perturbed part), so the complex-step method can differentiate through it.
"""
from math import pi, sqrt

import numpy as np

CART = {
    0: [(0, 0, 0)],
    1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}


def dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def radial_prim_norm(alpha, l):
    """(2 alpha/pi)^(3/4) (4 alpha)^(l/2): norm of x^l exp(-alpha r^2) up to eta."""
    return (2.0 * alpha / pi) ** 0.75 * (4.0 * alpha) ** (0.5 * l)


def shell_radial_coefficients(exps, coefs, l):
    """c'_k such that every cartesian component of the shell has unit norm.

    The self-overlap of eta x^a.. sum_k c_k n_k exp(-alpha_k r^2) is
    sum_kl c_k c_l n_k n_l (pi/p)^(3/2) / (2p)^l with p = alpha_k + alpha_l,
    independent of the component once eta is applied.
    """
    n = np.array([radial_prim_norm(a, l) for a in exps])
    c = np.asarray(coefs, dtype=np.float64) * n
    s = 0.0
    for k in range(len(exps)):
        for m in range(len(exps)):
            p = exps[k] + exps[m]
            s += c[k] * c[m] * (pi / p) ** 1.5 / (2.0 * p) ** l
    return c / sqrt(s)


class ShellTable:
    """Per-shell data with normalisation folded in."""

    def __init__(self, basis):
        off = basis.prim_offsets()
        self.shells = []
        for s in range(basis.n_shells):
            l = int(basis.shell_l[s])
            sl = slice(int(off[s]), int(off[s] + basis.shell_nprim[s]))
            exps = np.array(basis.prim_exp[sl], dtype=np.float64)
            cp = shell_radial_coefficients(exps, basis.prim_coef[sl], l)
            comps = [(c, 1.0 / sqrt(dfact(2 * c[0] - 1) * dfact(2 * c[1] - 1) * dfact(2 * c[2] - 1)))
                     for c in CART[l]]
            self.shells.append((int(basis.shell_atom[s]), l, exps, cp, comps))
        self.n_ao = sum(len(sh[4]) for sh in self.shells)
        self.ao_atom = np.array([sh[0] for sh in self.shells for _ in sh[4]], dtype=np.int64)


def _pow(x, k):
    if k < 0:
        return np.zeros_like(x)
    if k == 0:
        return np.ones_like(x)
    out = x
    for _ in range(k - 1):
        out = out * x
    return out


def eval_aos(table, centres, r):
    """AO value, gradient and Laplacian at positions r.

    table   : ShellTable
    centres : [A][3] nuclear positions (real or complex)
    r       : [..., 3] electron positions (real or complex)
    returns val [..., M], grad [..., M, 3], lap [..., M]
    """
    r = np.asarray(r)
    dtype = np.result_type(r.dtype, np.asarray(centres).dtype, np.float64)
    shape = r.shape[:-1]
    M = table.n_ao
    val = np.zeros(shape + (M,), dtype=dtype)
    grad = np.zeros(shape + (M, 3), dtype=dtype)
    lap = np.zeros(shape + (M,), dtype=dtype)
    mu = 0
    for atom, l, exps, cp, comps in table.shells:
        d = r - centres[atom]
        x, y, z = d[..., 0], d[..., 1], d[..., 2]
        rho = x * x + y * y + z * z
        R0 = np.zeros(shape, dtype=dtype)
        R1 = np.zeros(shape, dtype=dtype)   # dR/drho
        R2 = np.zeros(shape, dtype=dtype)   # d2R/drho2
        for a, c in zip(exps, cp):
            e = c * np.exp(-a * rho)
            R0 = R0 + e
            R1 = R1 - a * e
            R2 = R2 + a * a * e
        for (ax, ay, az), eta in comps:
            P = _pow(x, ax) * _pow(y, ay) * _pow(z, az)
            dP = [ax * _pow(x, ax - 1) * _pow(y, ay) * _pow(z, az),
                  ay * _pow(x, ax) * _pow(y, ay - 1) * _pow(z, az),
                  az * _pow(x, ax) * _pow(y, ay) * _pow(z, az - 1)]
            lapP = (ax * (ax - 1) * _pow(x, ax - 2) * _pow(y, ay) * _pow(z, az)
                    + ay * (ay - 1) * _pow(x, ax) * _pow(y, ay - 2) * _pow(z, az)
                    + az * (az - 1) * _pow(x, ax) * _pow(y, ay) * _pow(z, az - 2))
            xdP = x * dP[0] + y * dP[1] + z * dP[2]
            val[..., mu] = eta * P * R0
            for k, xk in enumerate((x, y, z)):
                # d/dx_k [P R(rho)] = dP/dx_k R + P R' 2 x_k
                grad[..., mu, k] = eta * (dP[k] * R0 + 2.0 * xk * P * R1)
            # lap[P R] = lapP R + 2 grad P . grad R + P lap R,
            # grad R = 2 x R', lap R = 6 R' + 4 rho R''
            lap[..., mu] = eta * (lapP * R0 + 4.0 * xdP * R1 + P * (6.0 * R1 + 4.0 * rho * R2))
            mu += 1
    return val, grad, lap
