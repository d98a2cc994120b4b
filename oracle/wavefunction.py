"""Jastrow-Slater determinant, log|Psi| and the local energy (oracle).

Follows Appendix A of the paper:
  * Psi = J * det, with the determinant part the JAGP restricted to the
    occupied MOs (eq. occ-expansion), i.e. det A_up * det A_dn with
    A_sigma[e, i] = phi_i(r_e),  phi_i = sum_mu C_mu,i psi_mu (eq. restricted-C);
    restricted closed shell: electrons 0..n_up-1 are spin up and the rest spin
    down, both spins use the same C (Sec. II, restricted case).
  * Two-body Pade Jastrow J2 = exp(sum_{i<j} v(r_ij)), v(r) = a r / (1 + F r)
    (eq. twobody_v with a = 1/2); spin independent.
  * Optional one-body and three/four-body terms on a Jastrow GTO basis
    psi^Jas_mu (Appendix A, eqs. onebody_J_inhom and threebody_jas):
      J1 = exp(sum_i sum_mu xi1_mu psi^Jas_mu(r_i)),
      J3 = exp(sum_{i<j} Xi(r_i, r_j)),
      Xi(r_i, r_j) = sum_{mu,nu} xi3_mu,nu psi^Jas_mu(r_i) psi^Jas_nu(r_j).
    Readings: the one-body factor, printed without an exponential, enters as
    exp(.) like the two- and three-body ones (the total J = J1 J2 J3 is a
    product of exponentials); xi3 is symmetric (a sum over i < j of a
    non-symmetric Xi would depend on the electrons' labels); all atom pairs
    are coupled (the four-body elements are kept, as in the paper's runs);
    the Jastrow basis functions follow the GTO conventions of gto.py.
  * Optional electron-nucleus cusp factor exp(sum_{e,alpha} -Z r/(1 + b r)):
    the paper omits it because its ECPs remove the singularity; here it is used
    only for the hydrogen-atom check.
  * E_L = H Psi / Psi (Appendix A) with H the all-electron molecular
    Hamiltonian, including the nuclear repulsion.

The kinetic term uses
    lap Psi / Psi |_e = lapD/D + 2 gradD/D . gradJ + lap J + |grad J|^2,
with gradD/D|_e = sum_i Kinv[i,e] grad phi_i(r_e) and lapD/D likewise from the
explicit inverse (for any invertible A, d det / det = tr(A^-1 dA)).

All routines accept complex arrays and stay complex-analytic, so derivatives
can be taken by the complex-step method (Squire & Trapp, SIAM Rev. 1998).
"""
import numpy as np

from . import ecp as ecp_mod
from . import gto


class System:
    """Molecule + wavefunction parameters in the oracle's own layout."""

    def __init__(self, mol, C=None):
        self.xyz = np.array(mol.xyz, dtype=np.float64)
        self.Z = np.array(mol.Z, dtype=np.float64)
        self.table = gto.ShellTable(mol.basis)
        self.C = np.array(mol.C if C is None else C)
        self.n_up = int(mol.n_up)
        self.n_dn = int(mol.n_dn)
        self.N = self.n_up + self.n_dn
        jas = mol.jastrow
        self.a = float(jas.ee_a)
        self.F = float(jas.ee_F)
        self.ee_form = int(getattr(jas, "ee_form", 0))
        self.en_on = int(jas.en_on)
        self.en_b = float(jas.en_b)
        jb = getattr(jas, "jas_basis", None)
        self.jas_table = gto.ShellTable(jb) if jb is not None else None
        self.xi1 = None if jb is None else np.array(jas.xi1, dtype=np.float64)
        self.xi3 = None if jb is None else np.array(jas.xi3, dtype=np.float64)
        self.A = self.xyz.shape[0]
        self.M = self.table.n_ao
        e = getattr(mol, "ecp", None)
        self.pp = ecp_mod.Pseudo(e, self.A) if e is not None else None
        assert self.C.shape == (self.M, max(self.n_up, self.n_dn))

    def spin_blocks(self):
        """[(electron slice, number of orbitals)] for the up and down blocks."""
        out = []
        if self.n_up:
            out.append((slice(0, self.n_up), self.n_up))
        if self.n_dn:
            out.append((slice(self.n_up, self.N), self.n_dn))
        return out


# --------------------------------------------------------------------------
# determinants
# --------------------------------------------------------------------------

def lu_logdet(A):
    """log|det A| and sign(det A) by LU with partial pivoting.

    A: [W, n, n], real or complex.  Pivot rows are chosen by the largest
    |Re|; the log is taken as 1/2 log(pivot^2) so that it stays analytic for
    the complex step.  Returns (sign [W] real, logabs [W]).
    """
    A = np.array(A, copy=True)
    W, n, _ = A.shape
    sign = np.ones(W)
    logabs = np.zeros(W, dtype=A.dtype)
    w = np.arange(W)
    for k in range(n):
        p = k + np.argmax(np.abs(A[:, k:, k].real), axis=1)
        swap = p != k
        if np.any(swap):
            rows_k = A[w, k, :].copy()
            A[w, k, :] = A[w, p, :]
            A[w, p, :] = rows_k
            sign = np.where(swap, -sign, sign)
        piv = A[:, k, k]
        sign = sign * np.sign(piv.real)
        logabs = logabs + 0.5 * np.log(piv * piv)
        if k + 1 < n:
            A[:, k + 1:, k] = A[:, k + 1:, k] / piv[:, None]
            A[:, k + 1:, k + 1:] -= A[:, k + 1:, k, None] * A[:, k, None, k + 1:]
    return sign, logabs


def mo_matrices(system, R, r, C=None):
    """AOs and MOs (value, gradient, Laplacian) at all electrons.

    r: [W, N, 3].  Returns dict with ao_val [W,N,M], ao_grad [W,N,M,3],
    ao_lap [W,N,M], phi [W,N,n], gphi [W,N,3,n], lphi [W,N,n].
    """
    C = system.C if C is None else C
    ao_val, ao_grad, ao_lap = gto.eval_aos(system.table, R, r)
    phi = ao_val @ C
    gphi = np.einsum("wemk,mi->weki", ao_grad, C)
    lphi = ao_lap @ C
    return dict(ao_val=ao_val, ao_grad=ao_grad, ao_lap=ao_lap, phi=phi, gphi=gphi, lphi=lphi)


# --------------------------------------------------------------------------
# Jastrow and potential
# --------------------------------------------------------------------------

def pade(r, a, F):
    """u, u', u'' of u(r) = a r / (1 + F r)  (eq. twobody_v, a = 1/2)."""
    q = 1.0 / (1.0 + F * r)
    return a * r * q, a * q * q, -2.0 * a * F * q * q * q


def expo(r, a, F):
    """u, u', u'' of u(r) = a (1 - exp(-F r)) / F  (eq. twobody_v_exp, a = 1/2)."""
    e = np.exp(-F * r)
    return a * (1.0 - e) / F, a * e, -a * F * e


def ee_pair(system, r):
    """The electron-electron Jastrow function of the system and its first two
    derivatives at distances r."""
    return (expo if system.ee_form == 1 else pade)(r, system.a, system.F)


def _pairs(r):
    """All ordered pairs: d[w,i,j] = r_i - r_j, r_ij, and the off-diagonal mask.

    The diagonal distance is set to 1 (then masked) so that no sqrt(0) enters
    the complex-step derivative.
    """
    N = r.shape[1]
    d = r[:, :, None, :] - r[:, None, :, :]
    eye = np.eye(N)
    rij = np.sqrt(np.sum(d * d, axis=-1) + eye)
    return d, rij, 1.0 - eye


def jastrow_terms(system, R, r):
    """J [W], grad_e J [W,N,3], lap_e J [W,N]."""
    W, N, _ = r.shape
    dtype = np.result_type(r.dtype, np.asarray(R).dtype)
    J = np.zeros(W, dtype=dtype)
    g = np.zeros((W, N, 3), dtype=dtype)
    h = np.zeros((W, N), dtype=dtype)
    if N > 1:
        d, rij, off = _pairs(r)                         # [W,N,N,3], [W,N,N], [N,N]
        u, u1, u2 = ee_pair(system, rij)
        J = J + 0.5 * np.sum(u * off, axis=(1, 2))
        g = g + np.sum((off * u1 / rij)[..., None] * d, axis=2)
        h = h + np.sum(off * (u2 + 2.0 * u1 / rij), axis=2)
    if system.jas_table is not None:
        J1, g1, h1, J3, g3, h3 = body_jastrow_terms(system, R, r)
        J = J + J1 + J3
        g = g + g1 + g3
        h = h + h1 + h3
    if system.en_on:
        for al in range(system.A):
            d = r - R[al]                                # [W, N, 3]
            rr = np.sqrt(np.sum(d * d, axis=-1))
            u, u1, u2 = pade(rr, -system.Z[al], system.en_b)
            J = J + u.sum(axis=1)
            g = g + (u1 / rr)[..., None] * d
            h = h + u2 + 2.0 * u1 / rr
    return J, g, h


def body_jastrow_terms(system, R, r):
    """One-body and three/four-body terms (eqs. onebody_J_inhom, threebody_jas):
    J1 [W], grad_e J1 [W,N,3], lap_e J1 [W,N] and the same for J3.

    J1 = sum_i sum_mu xi1_mu chi_mu(r_i); J3 = sum_{i<j} Xi(r_i, r_j) with the
    pair matrix P[i, j] = Xi(r_i, r_j) = chi(r_i)^T xi3 chi(r_j) summed over
    i < j.  r_e enters J3 through the pairs (e, j), j != e, so
    grad_e J3 = sum_{j != e} grad chi(r_e)^T xi3 chi(r_j) and the Laplacian
    likewise with lap chi(r_e).
    """
    chi, gchi, lchi = gto.eval_aos(system.jas_table, R, r)    # [W,N,MJ], [W,N,MJ,3], [W,N,MJ]
    N = r.shape[1]
    xi1, xi3 = system.xi1, system.xi3
    J1 = np.einsum("wim,m->w", chi, xi1)
    g1 = np.einsum("wimk,m->wik", gchi, xi1)
    h1 = np.einsum("wim,m->wi", lchi, xi1)
    T = np.einsum("wjn,mn->wjm", chi, xi3)                  # T[w, j] = xi3 chi(r_j)
    P = np.einsum("wim,wjm->wij", chi, T)                   # P[w, i, j] = Xi(r_i, r_j)
    upper = np.triu(np.ones((N, N)), k=1)
    J3 = np.einsum("wij,ij->w", P, upper)
    off = 1.0 - np.eye(N)
    Tsum = np.einsum("wjm,ej->wem", T, off)                 # sum_{j != e} xi3 chi(r_j)
    g3 = np.einsum("wemk,wem->wek", gchi, Tsum)
    h3 = np.einsum("wem,wem->we", lchi, Tsum)
    return J1, g1, h1, J3, g3, h3


def jastrow_parameter_derivatives(system, R, r):
    """O_xi = dln|Psi|/dxi of the one- and three/four-body parameters:
    O_xi1 [W, MJ] = s = sum_i chi(r_i) (eq. onebody_J_inhom is linear in xi1);
    O_xi3 [W, MJ, MJ] = (s s^T - sum_i chi(r_i) chi(r_i)^T) / 2, the gradient
    of U3 = sum_{i<j} chi(r_i)^T xi3 chi(r_j) (eq. threebody_jas) with respect
    to the symmetric matrix xi3: for a symmetric change D,
    dU3 = sum_{mu,nu} O_xi3[mu, nu] D[mu, nu]."""
    chi, _, _ = gto.eval_aos(system.jas_table, R, r)            # [W, N, MJ]
    s = chi.sum(axis=1)
    return s, 0.5 * (s[:, :, None] * s[:, None, :] - np.einsum("wim,win->wmn", chi, chi))


def potential(system, R, r):
    """V = -sum Z/|r-R| + sum_{i<j} 1/r_ij + sum_{a<b} Z_a Z_b / R_ab  [W]."""
    W, N, _ = r.shape
    V = np.zeros(W, dtype=np.result_type(r.dtype, np.asarray(R).dtype))
    for al in range(system.A):
        d = r - R[al]
        V = V - system.Z[al] * np.sum(1.0 / np.sqrt(np.sum(d * d, axis=-1)), axis=1)
    if N > 1:
        _, rij, off = _pairs(r)
        V = V + 0.5 * np.sum(off / rij, axis=(1, 2))
    for al in range(system.A):
        for be in range(al + 1, system.A):
            d = R[al] - R[be]
            V = V + system.Z[al] * system.Z[be] / np.sqrt(np.sum(d * d))
    return V


# --------------------------------------------------------------------------
# local energy
# --------------------------------------------------------------------------

def evaluate(system, R, r, C=None, keep=False, frame=None):
    """Per-walker E_L, log|Psi| and sign at nuclei R [A,3], electrons r [W,N,3].

    With keep=True the intermediates needed for derivatives are returned too.
    With a pseudopotential, E_L includes its local and non-local parts
    (ecp.py); frame = (walker ids, rotation index) of its quadrature.
    """
    r = np.asarray(r)
    W, N, _ = r.shape
    mo = mo_matrices(system, R, r, C)
    J, g, h = jastrow_terms(system, R, r)
    dtype = np.result_type(mo["phi"].dtype, J.dtype)
    b = np.zeros((W, N, 3), dtype=dtype)       # gradD/D at each electron
    lapD = np.zeros((W, N), dtype=dtype)       # lapD/D at each electron
    logdet = np.zeros(W, dtype=dtype)
    sign = np.ones(W)
    Kinv = []
    for sl, n in system.spin_blocks():
        A = mo["phi"][:, sl, :n]                         # [W, e, i]
        s_, la = lu_logdet(A)
        sign = sign * s_
        logdet = logdet + la
        K = np.linalg.inv(A)                             # K[w, i, e]
        Kinv.append(K)
        b[:, sl, :] = np.einsum("wie,weki->wek", K, mo["gphi"][:, sl, :, :n])
        lapD[:, sl] = np.einsum("wie,wei->we", K, mo["lphi"][:, sl, :n])
    kin_e = lapD + 2.0 * np.sum(b * g, axis=-1) + h + np.sum(g * g, axis=-1)
    E_kin = -0.5 * kin_e.sum(axis=1)
    V = potential(system, R, r)
    E_L = E_kin + V
    t = None
    if system.pp is not None:
        t = ecp_mod.terms(system, R, r, C, Kinv, frame)
        E_L = E_L + t["E_loc"] + t["E_nl"]
    out = dict(E_L=E_L, lnpsi=logdet + J, sign=sign)
    if keep:
        out["ecp"] = t
        out.update(mo)
        out.update(Kinv=Kinv, b=b, lapD=lapD, g=g, h=h, J=J, V=V)
    return out
