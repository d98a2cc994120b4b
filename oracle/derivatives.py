"""Per-walker derivatives for the force and dE/dC estimators (oracle).

Nuclear derivatives with the space-warp coordinate transformation (Appendix A,
"Computing derivatives"): when nucleus alpha moves by dR, every electron
moves with it by omega_alpha(r_i) dR, with
    omega_alpha(r) = kappa(|r - R_alpha|) / sum_beta kappa(|r - R_beta|),
    kappa(d) = d^-4.
The HF+Pulay force with warp is the derivative of the reweighted energy of
warped configurations; the Jacobian of the warp contributes
1/2 d ln det(dr'/dr) per electron to the Pulay term.

Reading used for a fixed-sample estimator at nuclei R with sampling geometry
R0: electrons are warped with weights taken at (r, R0),
    r'_i = r_i + sum_alpha omega_alpha(r_i; R0) (R_alpha - R0_alpha),
    ln Jac = sum_i ln det(I + sum_alpha (R_alpha - R0_alpha) grad omega_alpha(r_i; R0)^T).
At R = R0 the derivatives below reduce to the paper's estimator terms
dE_L/dR_alpha + sum_i omega dE_L/dr_i and
dlnPsi/dR_alpha + sum_i [omega dlnPsi/dr_i + 1/2 grad_i omega].

Derivatives in R are taken by the complex step: f(x + i h)/h has imaginary
part f'(x) + O(h^2) with no subtractive cancellation, so h = 1e-30 gives
the derivative to rounding (Squire & Trapp, SIAM Rev. 40, 1998).

Derivatives in C (the MO coefficients; B = dE/dC, eq. fc-vmc-eval) use
matrix calculus on the same wavefunction: for the Slater matrix A and its
inverse K, d ln det A = tr(K dA) and dK = -K dA K.
"""
import numpy as np

from . import ecp as ecp_mod
from . import wavefunction as wf

H_CS = 1e-30


def swct_weights(R0, r):
    """omega[w, i, alpha] at electrons r [W,N,3] for nuclei R0 [A,3].

    Written as 1 / (1 + sum_{beta != alpha} (d_alpha/d_beta)^4), which equals
    kappa_alpha / sum kappa and stays finite as d_alpha -> 0.  An electron
    within 1e-12 bohr of a nucleus gets omega = 1 for that nucleus.
    """
    d = r[:, :, None, :] - R0[None, None, :, :]
    dist2 = np.sum(d * d, axis=-1)                       # [W,N,A]
    A = R0.shape[0]
    om = np.zeros_like(dist2)
    for al in range(A):
        s = 1.0
        for be in range(A):
            if be != al:
                q = dist2[..., al] / dist2[..., be]
                s = s + q * q
        om[..., al] = 1.0 / s
    near = np.sqrt(np.abs(dist2.real)) < 1e-12
    if np.any(near):
        hit = np.any(near, axis=-1)
        om = np.where(hit[..., None], near.astype(float), om)
    return om


def swct_weight_gradients(R0, r):
    """grad_r omega[w, i, alpha, k] by complex step in each electron coordinate."""
    W, N, _ = r.shape
    A = R0.shape[0]
    out = np.zeros((W, N, A, 3))
    for k in range(3):
        rc = r.astype(np.complex128)
        rc[..., k] += 1j * H_CS
        out[..., k] = swct_weights(R0, rc).imag / H_CS
    return out


def warp(R, R0, r):
    """Warped electrons r' and ln Jacobian for nuclei R (sampled at R0)."""
    om = swct_weights(R0, r)                              # [W,N,A]
    gom = swct_weight_gradients(R0, r)                    # [W,N,A,3]
    dR = np.asarray(R) - R0                               # [A,3]
    rp = r + np.einsum("wna,ak->wnk", om, dR)
    Mj = np.eye(3) + np.einsum("ak,wnal->wnkl", dR, gom)  # dr'_k / dr_l
    lnjac = np.sum(np.log(np.linalg.det(Mj)), axis=1)
    return rp, lnjac


def warped_values(system, R, R0, r, C=None, frame=None):
    """E_L, ln|Psi| and ln Jac of the warped configuration (real or complex R)."""
    rp, lnjac = warp(R, R0, r)
    out = wf.evaluate(system, R, rp, C, frame=frame)
    return out["E_L"], out["lnpsi"], lnjac


def nuclear_derivatives(system, R, R0, r, C=None, frame=None):
    """d/dR of (E_L, ln|Psi|, ln Jac) of warped configurations.

    Returns dE [W,A,3], dlnpsi [W,A,3], dlnjac [W,A,3] (complex step,
    3A evaluations).  The SWCT force terms per walker are
    H = dE and P = dlnpsi + dlnjac / 2.
    """
    R = np.asarray(R, dtype=np.float64)
    W = r.shape[0]
    A = R.shape[0]
    dE = np.zeros((W, A, 3))
    dP = np.zeros((W, A, 3))
    dJ = np.zeros((W, A, 3))
    for al in range(A):
        for k in range(3):
            Rc = R.astype(np.complex128)
            Rc[al, k] += 1j * H_CS
            e, p, j = warped_values(system, Rc, R0, r, C, frame)
            dE[:, al, k] = e.imag / H_CS
            dP[:, al, k] = p.imag / H_CS
            dJ[:, al, k] = np.asarray(j).imag / H_CS
    return dE, dP, dJ


def coefficient_derivatives(system, R, r, C=None, frame=None):
    """O = d ln|Psi| / dC and G = dE_L / dC per walker, each [W, M, n_occ].

    With K = A^-1 per spin (K[i,e]), b_e = sum_i K[i,e] grad phi_i(r_e),
    X[e,i] = lap phi_i(r_e) + 2 grad J_e . grad phi_i(r_e), the determinant part
    of the kinetic energy is -1/2 tr(K X) summed over spins, so
      dE_L/dA[e,i]       =  1/2 (K X K)[i,e]
      dE_L/d(grad phi)   = -grad J_e K[i,e]
      dE_L/d(lap phi)    = -1/2 K[i,e]
      d ln|Psi|/dA[e,i]  =  K[i,e]
    and each MO matrix is AO matrix times C, so dX/dC = AO^T dX/d(MO).
    """
    ev = wf.evaluate(system, R, r, C, keep=True, frame=frame)
    W, N, _ = r.shape
    n_occ = system.C.shape[1]
    O = np.zeros((W, system.M, n_occ), dtype=ev["phi"].dtype)
    G = np.zeros_like(O)
    g = ev["g"]
    for (sl, n), K in zip(system.spin_blocks(), ev["Kinv"]):
        KT = np.swapaxes(K, 1, 2)                          # [W, e, i]
        X = ev["lphi"][:, sl, :n] + 2.0 * np.einsum("wek,weki->wei", g[:, sl], ev["gphi"][:, sl, :, :n])
        Abar = 0.5 * np.swapaxes(K @ X @ K, 1, 2)          # [W, e, i]
        Gbar = -g[:, sl, :, None] * KT[:, :, None, :]      # [W, e, k, i]
        Lbar = -0.5 * KT
        O[:, :, :n] += np.einsum("wem,wei->wmi", ev["ao_val"][:, sl], KT)
        G[:, :, :n] += (np.einsum("wem,wei->wmi", ev["ao_val"][:, sl], Abar)
                        + np.einsum("wemk,weki->wmi", ev["ao_grad"][:, sl], Gbar)
                        + np.einsum("wem,wei->wmi", ev["ao_lap"][:, sl], Lbar))
    if system.pp is not None:
        G = G + ecp_mod.coefficient_terms(system, ev["ecp"], ev["Kinv"], ev["ao_val"], C)
    return O, G, ev


def measure(system, R0, r, C=None, frame=None):
    """All per-walker quantities of one measurement at the sampling geometry.

    Returns dict: E_L, lnpsi [W]; H, P [W,A,3] (SWCT force terms); O, G [W,M,n];
    with one-/three-body Jastrow terms also Oxi1 [W,MJ], Oxi3 [W,MJ,MJ]
    (dln|Psi| / dxi).  frame: (walker ids, rotation index) of a
    pseudopotential's quadrature.
    """
    dE, dP, dJ = nuclear_derivatives(system, R0, R0, r, C, frame)
    O, G, ev = coefficient_derivatives(system, R0, r, C, frame)
    out = dict(E_L=ev["E_L"], lnpsi=ev["lnpsi"], H=dE, P=dP + 0.5 * dJ,
               dlnpsi_dR=dP, dlnjac_dR=dJ, O=O, G=G)
    if system.jas_table is not None:
        out["Oxi1"], out["Oxi3"] = wf.jastrow_parameter_derivatives(system, R0, r)
    return out
