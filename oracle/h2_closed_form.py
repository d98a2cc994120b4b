"""Closed-form RHF energy of H2 in a contracted s-Gaussian basis (oracle pin).

With the Jastrow switched off the two-electron Jastrow-Slater wavefunction of
H2 is the closed-shell determinant phi(r1) phi(r2) of the bonding MO, so its
exact energy expectation is the RHF energy
    E = 2 h_pp + (pp|pp) + 1/R,
which needs only the textbook one- and two-electron integrals over
normalised s Gaussians (Boys function F0(t) = sqrt(pi/t) erf(sqrt t) / 2);
see Szabo & Ostlund, Modern Quantum Chemistry, Appendix A.  Being a
stationary-state expectation value of a fixed-shape MO (symmetry fixes the
bonding combination), dE/dR at fixed MO shape is the exact force, and the
bare VMC force estimator must reproduce -dE/dR.
"""
from math import erf, exp, pi, sqrt

import numpy as np


def _boys0(t):
    if t < 1e-12:
        return 1.0 - t / 3.0
    return 0.5 * sqrt(pi / t) * erf(sqrt(t))


def _prims(exps, coefs):
    """(alpha, c * (2 alpha/pi)^(3/4)) renormalised to a unit-norm contraction."""
    c = [ck * (2 * a / pi) ** 0.75 for a, ck in zip(exps, coefs)]
    s = sum(ci * cj * (pi / (ai + aj)) ** 1.5 for ai, ci in zip(exps, c) for aj, cj in zip(exps, c))
    return [(a, ci / sqrt(s)) for a, ci in zip(exps, c)]


def integrals(R, exps, coefs):
    centres = [np.array([0.0, 0.0, 0.0]), np.array([R, 0.0, 0.0])]
    pr = _prims(exps, coefs)
    S = np.zeros((2, 2)); T = np.zeros((2, 2)); V = np.zeros((2, 2)); G = np.zeros((2, 2, 2, 2))
    for m in range(2):
        for n in range(2):
            A, B = centres[m], centres[n]
            AB2 = float(np.sum((A - B) ** 2))
            for a, ca in pr:
                for b, cb in pr:
                    p = a + b
                    mu = a * b / p
                    Pc = (a * A + b * B) / p
                    s = (pi / p) ** 1.5 * exp(-mu * AB2)
                    S[m, n] += ca * cb * s
                    T[m, n] += ca * cb * mu * (3.0 - 2.0 * mu * AB2) * s
                    for Cn in centres:
                        V[m, n] -= ca * cb * 2.0 * pi / p * exp(-mu * AB2) * _boys0(p * float(np.sum((Pc - Cn) ** 2)))
    for m in range(2):
        for n in range(2):
            for k in range(2):
                for l in range(2):
                    A, B, C, D = centres[m], centres[n], centres[k], centres[l]
                    v = 0.0
                    for a, ca in pr:
                        for b, cb in pr:
                            p = a + b
                            P = (a * A + b * B) / p
                            eab = exp(-a * b / p * float(np.sum((A - B) ** 2)))
                            for c, cc in pr:
                                for d, cd in pr:
                                    q = c + d
                                    Q = (c * C + d * D) / q
                                    ecd = exp(-c * d / q * float(np.sum((C - D) ** 2)))
                                    t = p * q / (p + q) * float(np.sum((P - Q) ** 2))
                                    v += ca * cb * cc * cd * 2.0 * pi ** 2.5 / (p * q * sqrt(p + q)) * eab * ecd * _boys0(t)
                    G[m, n, k, l] = v
    return S, T, V, G


def rhf_energy(R, exps, coefs):
    S, T, V, G = integrals(R, exps, coefs)
    c = np.array([1.0, 1.0]) / sqrt(2.0 + 2.0 * S[0, 1])
    h = T + V
    return float(2.0 * c @ h @ c + np.einsum("m,n,k,l,mnkl->", c, c, c, c, G) + 1.0 / R)


def rhf_force(R, exps, coefs, h=1e-4):
    """-dE/dR of the nucleus at +R (central difference of the closed form)."""
    return -(rhf_energy(R + h, exps, coefs) - rhf_energy(R - h, exps, coefs)) / (2 * h)
