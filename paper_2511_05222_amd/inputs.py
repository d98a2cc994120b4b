"""Seeded synthetic inputs for the VMC force hot path.

This module only *generates* inputs: geometries, cartesian GTO shell tables,
molecular-orbital coefficient matrices and walker counts.  It evaluates no
part of the Monte Carlo method (no orbitals at electron positions, no
determinants, no Jastrow, no local energy); both the HIP path and the oracle
consume what it returns, and neither's arithmetic lives here.

The one piece of integral arithmetic here is the AO overlap matrix S, used
only to make the random MO coefficients orthonormal in the S metric (the
orthonormality constraint S_kl = delta_kl of the paper's Lagrangian, Sec. II).
The hot path itself never forms S.

Workload recipe (synthetic stand-ins for the paper's rMD17 molecules, Sec. IV):
  * geometry: random sequential addition, uniform in a sphere of radius
    1.74 * A**(1/3) bohr, rejecting any atom closer than 1.8 bohr to another;
  * basis: cartesian shells, heavy atoms 3s2p1d and H 2s1p, three primitives
    per shell with exponents log-uniform in [0.1, 50] (sorted descending) and
    contraction coefficients uniform in [0.2, 1.0];
  * MO coefficients: X ~ N(0,1)^{M x M}, C = X L^-T with L L^T = X^T S X, the
    first n columns occupied;
  * Jastrow: two-body Pade u(r) = a r / (1 + F r), a = 1/2, F = 1; for the
    one-/three-body terms (with_body_jastrow), a Jastrow basis of
    uncontracted cartesian primitives, [3s1p] on H and [4s2p1d] on C and O
    (the paper's basis sizes), exponents log-uniform in [0.2, 4] sorted
    descending, and seeded parameters xi1 ~ N(0, s1^2), xi3 = (G + G^T) / 2
    with G ~ N(0, s3^2);
  * pseudopotential (with_ecp): a seeded semilocal potential on C and O
    (local part and l = 0, 1 projectors of Gaussian radial terms), the two
    core electrons of each removed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache
from math import comb, pi, sqrt

import numpy as np

Z_OF = {"H": 1, "C": 6, "O": 8}

# Shell recipe per element: list of angular momenta.
SHELLS_OF = {
    "H": [0, 0, 1],
    "C": [0, 0, 0, 1, 1, 2],
    "O": [0, 0, 0, 1, 1, 2],
}

N_CART = {0: 1, 1: 3, 2: 6}

STO3G_H_EXP = (3.42525, 0.62391, 0.16886)
STO3G_H_COEF = (0.15433, 0.53533, 0.44463)


@dataclass
class Basis:
    """Cartesian contracted GTO shells.

    shell_atom[s], shell_l[s], shell_nprim[s]; primitives of shell s occupy
    prim_exp/prim_coef[off[s] : off[s] + shell_nprim[s]].  Coefficients
    multiply unit-normalised primitives.
    """

    shell_atom: np.ndarray
    shell_l: np.ndarray
    shell_nprim: np.ndarray
    prim_exp: np.ndarray
    prim_coef: np.ndarray

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_ao(self) -> int:
        return int(sum(N_CART[int(l)] for l in self.shell_l))

    @property
    def n_prim(self) -> int:
        return int(self.prim_exp.shape[0])

    def prim_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.shell_nprim)[:-1]]).astype(np.int64)


@dataclass
class Jastrow:
    ee_a: float = 0.5
    ee_F: float = 1.0
    en_on: int = 0
    en_b: float = 0.0
    ee_form: int = 0   # 0: a r / (1 + F r); 1: a (1 - exp(-F r)) / F
    # one- and three/four-body terms on a Jastrow GTO basis (None: absent):
    # jas_basis has M_J functions, xi1[M_J], xi3[M_J][M_J] symmetric
    jas_basis: "Basis | None" = None
    xi1: "np.ndarray | None" = None
    xi3: "np.ndarray | None" = None


@dataclass
class Ecp:
    """Semilocal pseudopotential: one radial term per entry,
    beta r^(n - 2) exp(-alpha r^2) on nucleus atom[t] in channel l[t]
    (-1 = the local part, l >= 0 the projector on angular momentum l);
    rcut[A] bohr: the non-local channels of nucleus a act on electrons
    closer than rcut[a] (0: none); rot_seed keys the random orientation of
    the quadrature on the sphere."""

    term_atom: np.ndarray
    term_l: np.ndarray
    term_n: np.ndarray
    term_exp: np.ndarray
    term_coef: np.ndarray
    rcut: np.ndarray
    rot_seed: int = 0


@dataclass
class Molecule:
    name: str
    symbols: list
    xyz: np.ndarray          # [A][3] bohr
    Z: np.ndarray            # [A] (effective charges with a pseudopotential)
    basis: Basis
    C_full: np.ndarray       # [M][M]; first n_occ columns occupied
    n_up: int
    n_dn: int
    jastrow: Jastrow = field(default_factory=Jastrow)
    ecp: "Ecp | None" = None

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_occ(self) -> int:
        return max(self.n_up, self.n_dn)

    @property
    def C(self) -> np.ndarray:
        return np.ascontiguousarray(self.C_full[:, : self.n_occ])

    @property
    def n_atoms(self) -> int:
        return int(self.Z.shape[0])


# ----------------------------------------------------------------------------
# AO overlap (input preparation only)
# ----------------------------------------------------------------------------

def _cart_components(l):
    if l == 0:
        return [(0, 0, 0)]
    if l == 1:
        return [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    return [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def _gauss_moment(m, p):
    """integral of t^m exp(-p t^2) over the real line."""
    if m % 2:
        return 0.0
    k = m // 2
    return _dfact(2 * k - 1) / (2.0 * p) ** k * sqrt(pi / p)


def _overlap_1d(a, b, A, B, alpha, beta):
    p = alpha + beta
    P = (alpha * A + beta * B) / p
    pre = np.exp(-alpha * beta / p * (A - B) ** 2)
    s = 0.0
    for i in range(a + 1):
        for j in range(b + 1):
            s += comb(a, i) * comb(b, j) * (P - A) ** (a - i) * (P - B) ** (b - j) * _gauss_moment(i + j, p)
    return pre * s


def _prim_norm(alpha, comp):
    a, b, c = comp
    l = a + b + c
    return sqrt((2 * alpha / pi) ** 1.5 * (4 * alpha) ** l / (_dfact(2 * a - 1) * _dfact(2 * b - 1) * _dfact(2 * c - 1)))


def overlap_matrix(xyz: np.ndarray, basis: Basis) -> np.ndarray:
    """AO overlap for cartesian components renormalised to unit self-overlap."""
    off = basis.prim_offsets()
    aos = []  # (centre, comp, exps, coefs)
    for s in range(basis.n_shells):
        l = int(basis.shell_l[s])
        sl = slice(off[s], off[s] + basis.shell_nprim[s])
        for comp in _cart_components(l):
            aos.append((xyz[basis.shell_atom[s]], comp, basis.prim_exp[sl], basis.prim_coef[sl]))
    M = len(aos)
    raw = np.zeros((M, M))
    for m in range(M):
        Am, cm, em, km = aos[m]
        for n in range(m, M):
            Bn, cn, en, kn = aos[n]
            v = 0.0
            for a1, c1 in zip(em, km):
                n1 = _prim_norm(a1, cm)
                for a2, c2 in zip(en, kn):
                    n2 = _prim_norm(a2, cn)
                    v += c1 * c2 * n1 * n2 * (
                        _overlap_1d(cm[0], cn[0], Am[0], Bn[0], a1, a2)
                        * _overlap_1d(cm[1], cn[1], Am[1], Bn[1], a1, a2)
                        * _overlap_1d(cm[2], cn[2], Am[2], Bn[2], a1, a2)
                    )
            raw[m, n] = raw[n, m] = v
    d = 1.0 / np.sqrt(np.diag(raw))
    return raw * d[:, None] * d[None, :]


# ----------------------------------------------------------------------------
# Generators
# ----------------------------------------------------------------------------

def random_geometry(symbols, seed, min_dist=1.8, density_radius=1.74):
    """Random sequential addition in a sphere of radius 1.74 A^(1/3) bohr."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = len(symbols)
    Rs = density_radius * A ** (1.0 / 3.0)
    pts = []
    while len(pts) < A:
        p = rng.uniform(-Rs, Rs, size=3)
        if np.dot(p, p) > Rs * Rs:
            continue
        if all(np.linalg.norm(p - q) >= min_dist for q in pts):
            pts.append(p)
    return np.array(pts, dtype=np.float64)


def random_basis(symbols, seed, nprim=3, exp_lo=0.1, exp_hi=50.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    sa, sl, sn, pe, pc = [], [], [], [], []
    for a, sym in enumerate(symbols):
        for l in SHELLS_OF[sym]:
            e = np.exp(rng.uniform(np.log(exp_lo), np.log(exp_hi), size=nprim))
            e = np.sort(e)[::-1]
            c = rng.uniform(0.2, 1.0, size=nprim)
            sa.append(a)
            sl.append(l)
            sn.append(nprim)
            pe.extend(e)
            pc.extend(c)
    return Basis(np.array(sa, np.int32), np.array(sl, np.int32), np.array(sn, np.int32),
                 np.array(pe, np.float64), np.array(pc, np.float64))


def s_orthonormal_coefficients(S, seed):
    """C = X L^-T with L L^T = X^T S X, so that C^T S C = I."""
    M = S.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((M, M))
    L = np.linalg.cholesky(X.T @ S @ X)
    return np.linalg.solve(L, X.T).T


def composition(n_atoms):
    """Heavy/H counts for a molecule of n_atoms in the 9-21 atom family."""
    n_c = int(round(2 + 7 * (n_atoms - 9) / 12))
    n_o = int(round(1 + 3 * (n_atoms - 9) / 12))
    n_h = n_atoms - n_c - n_o
    if n_h % 2:
        n_h -= 1
        n_c += 1
    return ["C"] * n_c + ["O"] * n_o + ["H"] * n_h


def make_molecule(symbols, geom_seed, basis_seed, c_seed, name="molecule"):
    xyz = random_geometry(symbols, geom_seed)
    Z = np.array([Z_OF[s] for s in symbols], dtype=np.float64)
    basis = random_basis(symbols, basis_seed)
    S = overlap_matrix(xyz, basis)
    C_full = s_orthonormal_coefficients(S, c_seed)
    n_el = int(Z.sum())
    assert n_el % 2 == 0
    return Molecule(name, list(symbols), xyz, Z, basis, C_full, n_el // 2, n_el // 2)


def make_h2(R=1.4, jastrow=None):
    """H2 with one STO-3G s shell per atom and the bonding MO (1,1)/norm."""
    xyz = np.array([[0.0, 0.0, 0.0], [R, 0.0, 0.0]])
    basis = Basis(np.array([0, 1], np.int32), np.array([0, 0], np.int32), np.array([3, 3], np.int32),
                  np.array(STO3G_H_EXP * 2, np.float64), np.array(STO3G_H_COEF * 2, np.float64))
    S = overlap_matrix(xyz, basis)
    s12 = S[0, 1]
    C_full = np.array([[1.0, 1.0], [1.0, -1.0]])
    C_full[:, 0] /= sqrt(2 + 2 * s12)
    C_full[:, 1] /= sqrt(2 - 2 * s12)
    return Molecule("H2", ["H", "H"], xyz, np.array([1.0, 1.0]), basis, C_full, 1, 1,
                    jastrow if jastrow is not None else Jastrow())


@dataclass
class RunSpec:
    """One benchmark/parity workload."""

    molecule: Molecule
    n_walkers: int
    n_sweeps: int
    seed: int
    step_sigma: float = 0.5
    precision: str = "fp64"


JAS_SHELLS_OF = {
    "H": [0, 0, 0, 1],
    "C": [0, 0, 0, 0, 1, 1, 2],
    "O": [0, 0, 0, 0, 1, 1, 2],
}


def make_jastrow_basis(symbols, seed: int) -> Basis:
    """Uncontracted cartesian primitives on every atom ([3s1p] H, [4s2p1d]
    C, O), exponents log-uniform in [0.2, 4] sorted descending per shell
    type, coefficient 1 (unit-normalised primitives)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sa, sl, ex = [], [], []
    for a, sym in enumerate(symbols):
        ls = JAS_SHELLS_OF[sym]
        for l in sorted(set(ls)):
            k = ls.count(l)
            e = np.sort(np.exp(rng.uniform(np.log(0.2), np.log(4.0), size=k)))[::-1]
            for x in e:
                sa.append(a)
                sl.append(l)
                ex.append(float(x))
    n = len(sa)
    return Basis(np.array(sa, np.int32), np.array(sl, np.int32), np.ones(n, np.int32), np.array(ex),
                 np.ones(n))


def with_body_jastrow(mol: Molecule, seed: int, s1: float = 0.05, s3: float = 0.004) -> Molecule:
    """A copy of mol whose Jastrow has the one- and three/four-body terms:
    a seeded Jastrow basis and seeded parameters (xi3 symmetric, all atom
    pairs coupled)."""
    import dataclasses
    jb = make_jastrow_basis(mol.symbols, seed)
    MJ = jb.n_ao
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    xi1 = rng.normal(0.0, s1, size=MJ)
    G = rng.normal(0.0, s3, size=(MJ, MJ))
    xi3 = 0.5 * (G + G.T)
    jas = dataclasses.replace(mol.jastrow, jas_basis=jb, xi1=xi1, xi3=xi3)
    return dataclasses.replace(mol, jastrow=jas, name=mol.name + " +J1J3")


ECP_CORE = {"C": 2, "O": 2}   # core electrons a pseudopotential removes


def _ecp_radial(r, n, alpha, beta):
    return sum(b * r ** (k - 2) * np.exp(-a * r * r) for k, a, b in zip(n, alpha, beta))


def with_ecp(mol: Molecule, seed: int, tail: float = 1e-12) -> Molecule:
    """A valence-only copy of mol with a seeded semilocal pseudopotential on
    its C and O atoms (synthetic stand-in for the paper's ccECP, whose
    parameters are not available here).  Each such atom loses ECP_CORE
    electrons (its charge becomes Z_eff = Z - core; one electron of each spin
    per atom); the MO coefficients keep their first n_occ columns.  Per
    element, with exponents log-uniform in the ranges given:
      local   Z_eff r^-1 e^{-a1 r^2} (cancels -Z_eff/r at the nucleus),
              b2 e^{-a2 r^2},  a1 in [3, 8], a2 in [1.5, 4], b2 ~ U(-2, 2);
      l = 0   b e^{-a r^2}, a in [2, 5], b ~ U(4, 12);
      l = 1   b e^{-a r^2}, a in [2, 5], b ~ U(-6, 6).
    rcut: the radius beyond which every non-local channel of the atom stays
    below `tail` hartree."""
    import dataclasses
    rng = np.random.Generator(np.random.PCG64(seed))
    par = {}
    for el in sorted(ECP_CORE):
        zeff = Z_OF[el] - ECP_CORE[el]
        lu = lambda lo, hi: float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        a1, a2, b2 = lu(3.0, 8.0), lu(1.5, 4.0), float(rng.uniform(-2.0, 2.0))
        s_a, s_b = lu(2.0, 5.0), float(rng.uniform(4.0, 12.0))
        p_a, p_b = lu(2.0, 5.0), float(rng.uniform(-6.0, 6.0))
        terms = [(-1, 1, a1, float(zeff)), (-1, 2, a2, b2), (0, 2, s_a, s_b), (1, 2, p_a, p_b)]
        rg = np.arange(0.0, 20.0, 1e-3)
        v = np.zeros_like(rg)
        for l, n, a, b in terms:
            if l >= 0:
                v = np.maximum(v, np.abs(_ecp_radial(rg, [n], [a], [b])))
        rc = float(rg[np.nonzero(v > tail)[0][-1] + 1])
        par[el] = (terms, rc)
    ta, tl, tn, te, tc = [], [], [], [], []
    Z = np.array(mol.Z, dtype=np.float64).copy()
    rcut = np.zeros(len(mol.symbols))
    removed = 0
    for a, sym in enumerate(mol.symbols):
        if sym not in par:
            continue
        terms, rc = par[sym]
        for l, n, ex, b in terms:
            ta.append(a)
            tl.append(l)
            tn.append(n)
            te.append(ex)
            tc.append(b)
        rcut[a] = rc
        Z[a] -= ECP_CORE[sym]
        removed += ECP_CORE[sym]
    ecp = Ecp(np.array(ta, np.int32), np.array(tl, np.int32), np.array(tn, np.int32), np.array(te),
              np.array(tc), rcut, rot_seed=seed + 17)
    return dataclasses.replace(mol, Z=Z, n_up=mol.n_up - removed // 2, n_dn=mol.n_dn - removed // 2, ecp=ecp,
                               name=mol.name + " +ECP")


@lru_cache(maxsize=None)
def make_config(i: int) -> RunSpec:
    """The five workloads: 0 = H2, 1 = 9 atoms, 2 = 21 atoms, 3 = 21 atoms
    (differentiation, 256 walkers), 4 = first of the mixed-size family.

    Results are cached; callers must not modify the returned arrays."""
    if i == 0:
        return RunSpec(make_h2(), 1024, 200, 0)
    if i == 1:
        mol = make_molecule(composition(9), 1, 11, 101, "9-atom C2OH6")
        return RunSpec(mol, 16384, 100, 1)
    if i == 2:
        mol = make_molecule(composition(21), 2, 12, 102, "21-atom C9O4H8")
        return RunSpec(mol, 65536, 10, 2, precision="mixed")
    if i == 3:
        mol = make_molecule(composition(21), 2, 12, 102, "21-atom C9O4H8")
        return RunSpec(mol, 256, 50, 3)
    if i == 4:
        return family_member(0)
    raise ValueError(i)


FAMILY_SIZE = 64


def family_sizes():
    """Atom counts of the 64-geometry mixed-size family, A ~ U{9..21} (PCG64 seed 4)."""
    rng = np.random.Generator(np.random.PCG64(4))
    return [int(a) for a in rng.integers(9, 22, size=FAMILY_SIZE)]


@lru_cache(maxsize=None)
def family_member(g: int) -> RunSpec:
    """Geometry g of the mixed-size family: composition of its atom count,
    geometry / basis / C seeds 1000 + g, 2000 + g, 3000 + g; 8192 walkers,
    mixed precision."""
    if not 0 <= g < FAMILY_SIZE:
        raise ValueError(g)
    A = family_sizes()[g]
    mol = make_molecule(composition(A), 1000 + g, 2000 + g, 3000 + g, f"{A}-atom mixed-family g{g}")
    return RunSpec(mol, 8192, 10, 4, precision="mixed")


def init_atom_of_electron(Z, n_up, n_dn):
    """Atom index each electron starts at.

    Atoms in input order each contribute Z electrons to a list; list entries
    alternate spin up/down.  Electron e < n_up is the e-th up entry, electron
    n_up + j the j-th down entry.
    """
    lst = []
    for a, z in enumerate(Z):
        lst.extend([a] * int(round(z)))
    ups = lst[0::2]
    dns = lst[1::2]
    # polarised systems: surplus entries go to the majority spin
    while len(ups) < n_up and dns:
        ups.append(dns.pop())
    while len(dns) < n_dn and ups:
        dns.append(ups.pop())
    out = np.array(ups[:n_up] + dns[:n_dn], dtype=np.int32)
    assert out.shape[0] == n_up + n_dn
    return out


def initial_walkers(mol: Molecule, n_walkers: int, seed: int, sigma: float = 0.5) -> np.ndarray:
    """Start positions [W][N][3]: each electron at its atom plus N(0, sigma^2)
    per cartesian component (numpy PCG64, seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    atom = init_atom_of_electron(mol.Z, mol.n_up, mol.n_dn)
    base = mol.xyz[atom]                                   # [N][3]
    return base[None, :, :] + sigma * rng.standard_normal((n_walkers, mol.n_elec, 3))


def seeded_spd(dim: int, seed: int, rank: int = 64) -> np.ndarray:
    """Synthetic orbital Hessian H = diag(d) + G G^T / rank (SPD), with d
    log-uniform in [0.5, 5] and G ~ N(0,1)^{dim x rank}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = np.exp(rng.uniform(np.log(0.5), np.log(5.0), size=dim))
    G = rng.standard_normal((dim, rank))
    return np.diag(d) + G @ G.T / rank
