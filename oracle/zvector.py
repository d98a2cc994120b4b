"""Z-vector solve H z = -b (oracle).

The Z-vector equations A Z = -B (eq. AZ_eq_B_elements) are linear in Z with
the VMC derivative B on the right-hand side.  The orbital Hessian is supplied
by the caller (the CPKS integrals are outside this path); for a symmetric
positive definite H the solution is unique.

Two solutions are given: a dense Cholesky solve (library routine) and
conjugate gradients with the stopping rule of the GPU path,
||r_k|| <= rtol ||b||, x_0 = 0 (Hestenes & Stiefel, 1952), optionally
preconditioned by diag H.

The unknowns are rotations of the occupied orbitals into the virtual ones,
C_occ -> C_occ + C_virt kappa (kappa[a][i], virtual a, occupied i): the
right-hand side is the derivative of E along them and the solution maps back
to a change of the occupied AO coefficients.
"""
import numpy as np


def cholesky_solve(H, b):
    L = np.linalg.cholesky(H)
    y = np.linalg.solve(L, -b)
    return np.linalg.solve(L.T, y)


def cg_solve(H, b, rtol=1e-12, maxit=10000, jacobi=False):
    """Returns (z, iterations, converged)."""
    rhs = -np.asarray(b, dtype=np.float64)
    x = np.zeros_like(rhs)
    r = rhs.copy()
    Minv = 1.0 / np.diag(H) if jacobi else np.ones_like(rhs)
    zr = Minv * r
    p = zr.copy()
    rz = float(r @ zr)
    bn = float(np.linalg.norm(rhs))
    if bn == 0.0:
        return x, 0, True
    for it in range(1, maxit + 1):
        Hp = H @ p
        alpha = rz / float(p @ Hp)
        x += alpha * p
        r -= alpha * Hp
        if np.linalg.norm(r) <= rtol * bn:
            return x, it, True
        zr = Minv * r
        rz_new = float(r @ zr)
        p = zr + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, False



def rhs(C_virt, dE_dC):
    """b[a][i] = dE/dkappa_ai = sum_mu C_virt[mu][a] dE/dC[mu][i] (chain rule
    through C_occ + C_virt kappa; the virtual orbitals do not enter E)."""
    return np.asarray(C_virt).T @ np.asarray(dE_dC)


def backmap(C_virt, z):
    """Z[mu][i] = sum_a C_virt[mu][a] z[a][i]: the rotation z as a change of the
    occupied AO coefficients."""
    return np.asarray(C_virt) @ np.asarray(z)
