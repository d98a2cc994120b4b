"""Semilocal pseudopotential in the local energy (oracle; test infrastructure).

The paper runs its VMC with ccECP pseudopotentials (Sec. III and the
computational details of Sec. IV); it does not restate how a pseudopotential
enters E_L, so the standard semilocal form is taken (Mitas, Shirley and
Ceperley, J. Chem. Phys. 95, 3467 (1991)).  On nucleus a, with d = |r_i - R_a|
and u_i = (r_i - R_a) / d, electron i sees
    V_loc(d) + sum_l V_l(d) sum_m |l m><l m|,
    V(d) = sum_t beta_t d^(n_t - 2) exp(-alpha_t d^2)   (per channel),
and the projectors enter the local energy through the ratio of the
wavefunction with electron i moved on its sphere around R_a:
    V_nl = sum_l V_l(d) (2l + 1) / (4 pi) int dOmega P_l(u_i . Omega)
           Psi(.., R_a + d Omega, ..) / Psi(.., r_i, ..).
Readings (the paper gives none of this):
  * the sphere integral is the 12-point rule on the vertices of an
    icosahedron, weight 1/12 each (exact for spherical harmonics up to degree
    5), turned by a random rotation per (walker, electron);
  * the rotation comes from Shoemake's uniform random unit quaternion
    (Graphics Gems III, 1992) on three uniforms u = w * 2^-32 of one
    Philox4x32-10 draw: key = the pseudopotential's rot_seed, counter =
    (walker id, rotation index, electron | 2 << 16, 0); the rotation index is
    the sweep index for the measurement that follows a sweep, else 0;
  * the non-local channels of nucleus a act only on electrons with
    d < rcut[a] (the input recipe puts rcut where every channel is below
    1e-12 hartree); the local part acts everywhere;
  * Psi'/Psi = [phi(r')^T K e_i] exp(J(r') - J(r)) (determinant lemma, the
    ratio a single-electron move uses), with the whole Jastrow: the two-body
    change sum_{j != i} u(|r' - r_j|) - u(|r_i - r_j|) and, with the one- and
    three/four-body terms, (chi(r') - chi(r_i))^T (xi1 + xi3 sum_{j != i} chi(r_j)).

Every routine stays complex-analytic in R, r and C (the cutoff is tested on
the real part), so the complex-step derivatives of the local energy include
the pseudopotential.
"""
import numpy as np

from . import gto
from . import philox

PURPOSE_ROTATION = 2


def icosahedron():
    """The 12 quadrature directions: (0, s1, s2 g), (s1, s2 g, 0), (s2 g, 0, s1)
    for s1, s2 in (+1, -1), g the golden ratio, normalised."""
    g = 0.5 * (1.0 + np.sqrt(5.0))
    v = []
    for s1 in (1.0, -1.0):
        for s2 in (1.0, -1.0):
            v += [(0.0, s1, s2 * g), (s1, s2 * g, 0.0), (s2 * g, 0.0, s1)]
    return np.array(v) / np.sqrt(1.0 + g * g)


def rotations(seed, walker_ids, rot_index, N):
    """Rotation matrices [W, N, 3, 3] of the quadrature, one per (walker, electron)."""
    W = len(walker_ids)
    out = np.zeros((W, N, 3, 3))
    for e in range(N):
        w0, w1, w2, _ = philox._words(seed, walker_ids, rot_index, e, PURPOSE_ROTATION)
        u1, u2, u3 = (x.astype(np.float64) * 2.0 ** -32 for x in (w0, w1, w2))
        a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
        x, y = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
        z, s = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
        out[:, e] = np.stack([
            np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * s), 2 * (x * z + y * s)], -1),
            np.stack([2 * (x * y + z * s), 1 - 2 * (x * x + z * z), 2 * (y * z - x * s)], -1),
            np.stack([2 * (x * z - y * s), 2 * (y * z + x * s), 1 - 2 * (x * x + y * y)], -1)], -2)
    return out


def legendre(l, x):
    if l == 0:
        return np.ones_like(x)
    if l == 1:
        return x
    if l == 2:
        return 1.5 * x * x - 0.5
    if l == 3:
        return 2.5 * x * x * x - 1.5 * x
    raise ValueError(l)


class Pseudo:
    """The pseudopotential of a system in the oracle's layout."""

    def __init__(self, ecp, n_atoms):
        self.atom = np.asarray(ecp.term_atom, int)
        self.l = np.asarray(ecp.term_l, int)
        self.n = np.asarray(ecp.term_n, int)
        self.alpha = np.asarray(ecp.term_exp, float)
        self.beta = np.asarray(ecp.term_coef, float)
        self.rcut = np.asarray(ecp.rcut, float)
        self.seed = int(ecp.rot_seed)
        self.A = n_atoms
        self.lmax = int(self.l.max()) if len(self.l) else -1
        self.nl_atoms = [a for a in range(n_atoms) if self.rcut[a] > 0 and np.any((self.atom == a) & (self.l >= 0))]

    def radial(self, a, l, d):
        """V_l of nucleus a at distances d (l = -1: the local part)."""
        v = np.zeros_like(d)
        for t in np.nonzero((self.atom == a) & (self.l == l))[0]:
            v = v + self.beta[t] * d ** (self.n[t] - 2) * np.exp(-self.alpha[t] * d * d)
        return v


def _u(system, d):
    from .wavefunction import ee_pair
    return ee_pair(system, d)[0]


def terms(system, R, r, C, Kinv, frame=None):
    """The pseudopotential's part of E_L and what its derivatives need.

    Kinv: the inverses K[w, i, e] of the spin blocks (wavefunction.evaluate).
    frame: (walker ids, rotation index); default (0..W-1, 0).
    Returns dict: E_loc [W], E_nl [W]; for each non-local nucleus in
    pp.nl_atoms: pts [W, N, 12, 3], cq [W, N, 12] = mask * (quadrature weight
    sum over l of (2l+1) V_l P_l) * exp(J' - J), ratio [W, N, 12] (determinant
    part), jratio [W, N, 12] = exp(J' - J), mask [W, N], ao [W, N*12, M] (AO
    values at the points).
    """
    pp = system.pp
    W, N, _ = r.shape
    C = system.C if C is None else C
    ids, rot_index = frame if frame is not None else (np.arange(W, dtype=np.uint64), 0)
    rot = rotations(pp.seed, ids, rot_index, N)                      # [W, N, 3, 3]
    vq = np.einsum("wnkl,ql->wnqk", rot, icosahedron())             # [W, N, 12, 3]
    dtype = np.result_type(r.dtype, np.asarray(R).dtype, np.asarray(C).dtype, Kinv[0].dtype)
    E_loc = np.zeros(W, dtype=dtype)
    E_nl = np.zeros(W, dtype=dtype)
    # pair terms of the two-body Jastrow at the electrons' own positions
    dij = r[:, :, None, :] - r[:, None, :, :]
    rij = np.sqrt(np.sum(dij * dij, axis=-1) + np.eye(N))
    u_old = _u(system, rij) * (1.0 - np.eye(N))                     # [W, i, j]
    if system.jas_table is not None:
        chi, _, _ = gto.eval_aos(system.jas_table, R, r)                # [W, N, MJ]
        # h_i = xi1 + xi3 sum_{j != i} chi(r_j): the one-/three-body change
        # of a move of electron i from r_i to r' is (chi(r') - chi(r_i)) . h_i
        h13 = system.xi1 + np.einsum("mn,win->wim", system.xi3, chi.sum(axis=1)[:, None, :] - chi)
    per_atom = {}
    for a in range(pp.A):
        if not np.any(pp.atom == a):
            continue
        dv = r - R[a]                                                # [W, N, 3]
        d = np.sqrt(np.sum(dv * dv, axis=-1))                        # [W, N]
        E_loc = E_loc + np.sum(pp.radial(a, -1, d), axis=1)
        if a not in pp.nl_atoms:
            continue
        mask = (d.real < pp.rcut[a]).astype(float)
        ui = dv / d[..., None]
        cos = np.einsum("wnk,wnqk->wnq", ui, vq)                     # [W, N, 12]
        c = np.zeros(cos.shape, dtype=dtype)
        for l in range(pp.lmax + 1):
            c = c + (2 * l + 1) / 12.0 * pp.radial(a, l, d)[..., None] * legendre(l, cos)
        pts = R[a] + d[..., None, None] * vq                         # [W, N, 12, 3]
        ao, _, _ = gto.eval_aos(system.table, R, pts.reshape(W, N * 12, 3))
        phi = (ao @ C).reshape(W, N, 12, -1)
        ratio = np.zeros(cos.shape, dtype=dtype)
        for b, (sl, n) in enumerate(system.spin_blocks()):
            K = Kinv[b]                                              # [W, i, e]
            ratio[:, sl] = np.einsum("weqi,wie->weq", phi[:, sl, :, :n], K)
        # Jastrow: J' - J = sum_{j != i} u(|r_q - r_j|) - u(|r_i - r_j|)
        dq = pts[:, :, :, None, :] - r[:, None, None, :, :]          # [W, i, q, j, 3]
        self_ = np.eye(N)[None, :, None, :]
        rq = np.sqrt(np.sum(dq * dq, axis=-1) + self_)
        dJ = np.sum(_u(system, rq) * (1.0 - self_), axis=-1) - np.sum(u_old, axis=-1)[:, :, None]
        if system.jas_table is not None:
            chq, _, _ = gto.eval_aos(system.jas_table, R, pts.reshape(W, N * 12, 3))
            chq = chq.reshape(W, N, 12, -1)
            dJ = dJ + np.einsum("wiqm,wim->wiq", chq - chi[:, :, None, :], h13)
        jr = np.exp(dJ)
        cq = mask[..., None] * c * jr
        E_nl = E_nl + np.einsum("wnq,wnq->w", cq, ratio)
        per_atom[a] = dict(pts=pts, cq=cq, ratio=ratio, jratio=jr, mask=mask, ao=ao)
    return dict(E_loc=E_loc, E_nl=E_nl, atoms=per_atom)


def coefficient_terms(system, t, Kinv, ao_el, C=None):
    """d(E_loc + E_nl)/dC [W, M, n] from terms(): each ratio phi(r')^T K e_i
    depends on C through phi(r') = psi(r')^T C and through K = A^-1, so with
    t_q[e] = (phi(r')^T K)[e] over the block of i and dK = -K dA K,
      d ratio / dC[mu, j] = K[j, i] (psi_mu(r') - sum_e t_q[e] psi_mu(r_e)).
    ao_el: AO values at the electrons [W, N, M]."""
    W, N, M = ao_el.shape
    C = system.C if C is None else C
    G = None
    for a, p in t["atoms"].items():
        ao = p["ao"].reshape(W, N, 12, M)
        for b, (sl, n) in enumerate(system.spin_blocks()):
            K = Kinv[b]                                              # [W, j, e]
            cq = p["cq"][:, sl]                                      # [W, i, q]
            phi = np.einsum("wiqm,mj->wiqj", ao[:, sl], C[:, :n])
            tq = np.einsum("wiqj,wje->wiqe", phi, K)                 # [W, i, q, e]
            # psi(r') - sum_e t_q[e] psi(r_e)
            dpsi = ao[:, sl] - np.einsum("wiqe,wem->wiqm", tq, ao_el[:, sl])
            g = np.einsum("wiq,wiqm,wji->wmj", cq, dpsi, K)
            if G is None:
                G = np.zeros((W, M, system.C.shape[1]), dtype=g.dtype)
            G[:, :, :n] += g
    if G is None:
        G = np.zeros((W, M, system.C.shape[1]))
    return G
