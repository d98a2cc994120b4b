"""Python binding of the C ABI in include/vmc.h (argument marshalling only).

Every step of the path runs in the HIP library ``libvmcx.so``; this module
passes device pointers of torch tensors and the current HIP stream.  Loading
fails loudly if the library has not been built (``python -m
paper_2511_05222_amd.build`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmcx.so")

VMC_OK, VMC_EINVAL, VMC_ENOMEM, VMC_EDEVICE, VMC_ESINGULAR, VMC_ENOTCONV, VMC_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
VMC_ECAPACITY = -7
VMC_FP64 = 0
VMC_MIXED = 1
# mixed precision: share of each measurement launch re-measured in FP64 (the
# walkers with the largest max|Abar|, the sensitivity of E_L to the orbital
# values); a few such walkers would otherwise dominate the walker-averaged error
PROMOTE_FRACTION = 0.02
VMC_SWEEP_MEASURE = 1
VMC_ACCUM_RESET = 1

EXPORTED = ["vmc_init", "vmc_sweep", "vmc_accumulate", "vmc_measure", "vmc_eval", "vmc_energy_cotangents",
            "vmc_adjoint", "vmc_jackknife", "zvector_solve", "zvector_rhs", "zvector_backmap", "zvector_jackknife",
            "vmc_staging_walkers", "vmc_free", "vmc_last_error", "vmc_init_error", "vmc_strerror", "vmc_profile",
            "vmc_profile_read", "zvector_solve_noalloc", "vmc_accumulate_walkers", "vmc_jastrow_gradient"]


class VmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class _Basis(ct.Structure):
    _fields_ = [("n_shells", ct.c_int32), ("shell_atom", ct.POINTER(ct.c_int32)),
                ("shell_l", ct.POINTER(ct.c_int32)), ("shell_nprim", ct.POINTER(ct.c_int32)),
                ("prim_exp", ct.POINTER(ct.c_double)), ("prim_coef", ct.POINTER(ct.c_double))]


class _Nuclei(ct.Structure):
    _fields_ = [("n_atoms", ct.c_int32), ("xyz", ct.POINTER(ct.c_double)), ("Z", ct.POINTER(ct.c_double))]


class _MO(ct.Structure):
    _fields_ = [("n_ao", ct.c_int32), ("n_occ", ct.c_int32), ("n_up", ct.c_int32), ("n_dn", ct.c_int32),
                ("C", ct.POINTER(ct.c_double))]


class _Jastrow(ct.Structure):
    _fields_ = [("ee_a", ct.c_double), ("ee_F", ct.c_double), ("ee_form", ct.c_int32),
                ("jas_basis", ct.POINTER(_Basis)), ("xi1", ct.POINTER(ct.c_double)),
                ("xi3", ct.POINTER(ct.c_double))]


class _Ecp(ct.Structure):
    _fields_ = [("n_terms", ct.c_int32), ("term_atom", ct.POINTER(ct.c_int32)), ("term_l", ct.POINTER(ct.c_int32)),
                ("term_n", ct.POINTER(ct.c_int32)), ("term_exp", ct.POINTER(ct.c_double)),
                ("term_coef", ct.POINTER(ct.c_double)), ("rcut", ct.POINTER(ct.c_double)),
                ("rot_seed", ct.c_uint64), ("max_pairs", ct.c_int32)]


class _Options(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("refresh_period", ct.c_int32), ("block_sweeps", ct.c_int32),
                ("max_walkers", ct.c_int32), ("staging_walkers", ct.c_int32), ("step_sigma", ct.c_double),
                ("promote_fraction", ct.c_double), ("jackknife_blocks", ct.c_int32),
                ("forced_refresh_ratio", ct.c_double), ("ecp", ct.POINTER(_Ecp)), ("jastrow_gradient", ct.c_int32)]


class _WalkerOut(ct.Structure):
    _fields_ = [(k, ct.c_void_p) for k in ("EL", "lnpsi", "lnjac", "dEL_dR", "dlnpsi_dR", "dlnjac_dR", "O", "G")]


_lib = None


def lib():
    """Load libvmcx.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing; run paper_2511_05222_amd/build.py")
    L = ct.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, dbl = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_uint64, ct.c_double
    L.vmc_init.argtypes = [ct.POINTER(_Basis), ct.POINTER(_Nuclei), ct.POINTER(_MO), ct.POINTER(_Jastrow),
                           ct.POINTER(_Options), i32, ct.POINTER(vp)]
    L.vmc_sweep.argtypes = [vp, vp, i64, i32, u64, u64, u32, vp, vp]
    L.vmc_accumulate.argtypes = [vp, vp, vp, vp, vp, vp, u32, vp]
    L.vmc_accumulate_walkers.argtypes = [vp, vp, i64, vp, vp]
    L.vmc_jastrow_gradient.argtypes = [vp, vp, vp, vp]
    L.vmc_measure.argtypes = [vp, vp, i64, vp, vp, vp, ct.POINTER(_WalkerOut), vp]
    L.vmc_eval.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.vmc_energy_cotangents.argtypes = [vp, i64, dbl, vp, vp, vp, vp, vp, vp, vp]
    L.vmc_adjoint.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.vmc_jackknife.argtypes = [vp, vp, vp, vp, ct.POINTER(i64), vp]
    L.zvector_solve.argtypes = [vp, i64, i64, vp, vp, dbl, i32, u32, vp, vp]
    L.zvector_solve_noalloc.argtypes = [vp, i64, i64, vp, vp, dbl, i32, u32, vp, vp]
    L.zvector_rhs.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp]
    L.zvector_backmap.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp]
    L.zvector_jackknife.argtypes = [vp, i64, i64, vp, vp, vp]
    L.vmc_profile.argtypes = [vp, i32]
    L.vmc_profile_read.argtypes = [vp, i32, vp, vp, vp]
    L.vmc_staging_walkers.argtypes = [vp]
    L.vmc_staging_walkers.restype = ct.c_int64
    L.vmc_free.argtypes = [vp]
    L.vmc_free.restype = None
    L.vmc_last_error.argtypes = [vp]
    L.vmc_last_error.restype = ct.c_char_p
    L.vmc_init_error.argtypes = []
    L.vmc_init_error.restype = ct.c_char_p
    L.vmc_strerror.argtypes = [ct.c_int]
    L.vmc_strerror.restype = ct.c_char_p
    for name in ("vmc_init", "vmc_sweep", "vmc_accumulate", "vmc_measure", "vmc_eval", "vmc_energy_cotangents",
                 "vmc_adjoint", "vmc_jackknife", "zvector_solve", "zvector_rhs", "zvector_backmap",
                 "zvector_jackknife", "vmc_profile", "vmc_profile_read", "zvector_solve_noalloc",
                 "vmc_accumulate_walkers", "vmc_jastrow_gradient"):
        getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    return ct.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(t, shape, dtype=None):
    import torch
    dtype = dtype or torch.float64
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"expected a contiguous {dtype} device tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device} (contiguous={t.is_contiguous()})")


class Context:
    """A wavefunction on one GPU plus its estimator accumulators."""

    def __init__(self, mol, max_walkers, precision="fp64", refresh_period=32, block_sweeps=1,
                 step_sigma=0.5, device=0, staging_walkers=0, promote_fraction=PROMOTE_FRACTION,
                 jackknife_blocks=0, forced_refresh_ratio=0.0, ecp_max_pairs=0, jastrow_gradient=False):
        L = lib()
        b = mol.basis
        self._keep = [np.ascontiguousarray(b.shell_atom, np.int32), np.ascontiguousarray(b.shell_l, np.int32),
                      np.ascontiguousarray(b.shell_nprim, np.int32), np.ascontiguousarray(b.prim_exp, np.float64),
                      np.ascontiguousarray(b.prim_coef, np.float64), np.ascontiguousarray(mol.xyz, np.float64),
                      np.ascontiguousarray(mol.Z, np.float64), np.ascontiguousarray(mol.C, np.float64)]
        k = self._keep
        ip = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_int32))
        dp = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_double))
        basis = _Basis(b.n_shells, ip(k[0]), ip(k[1]), ip(k[2]), dp(k[3]), dp(k[4]))
        nuc = _Nuclei(mol.n_atoms, dp(k[5]), dp(k[6]))
        n_ao = int(sum((int(l) + 1) * (int(l) + 2) // 2 for l in b.shell_l))
        mo = _MO(n_ao, mol.n_occ, mol.n_up, mol.n_dn, dp(k[7]))
        jas = _Jastrow(mol.jastrow.ee_a, mol.jastrow.ee_F, int(getattr(mol.jastrow, "ee_form", 0)))
        jb = getattr(mol.jastrow, "jas_basis", None)
        if jb is not None:
            jk = [np.ascontiguousarray(jb.shell_atom, np.int32), np.ascontiguousarray(jb.shell_l, np.int32),
                  np.ascontiguousarray(jb.shell_nprim, np.int32), np.ascontiguousarray(jb.prim_exp, np.float64),
                  np.ascontiguousarray(jb.prim_coef, np.float64),
                  np.ascontiguousarray(mol.jastrow.xi1, np.float64), np.ascontiguousarray(mol.jastrow.xi3, np.float64)]
            self._keep += jk
            self._jbasis = _Basis(jb.n_shells, ip(jk[0]), ip(jk[1]), ip(jk[2]), dp(jk[3]), dp(jk[4]))
            jas.jas_basis = ct.pointer(self._jbasis)
            jas.xi1 = dp(jk[5])
            jas.xi3 = dp(jk[6])
        if getattr(mol.jastrow, "en_on", 0):
            raise VmcError(VMC_EINVAL, "the electron-nucleus Jastrow factor is not part of the HIP path")
        prec = {"fp64": VMC_FP64, "mixed": VMC_MIXED}.get(precision)
        if prec is None:
            raise VmcError(VMC_EINVAL, f"precision {precision!r} is not available")
        opt = _Options(prec, refresh_period, block_sweeps, int(max_walkers), int(staging_walkers), step_sigma,
                       float(promote_fraction), int(jackknife_blocks), float(forced_refresh_ratio))
        opt.jastrow_gradient = 1 if jastrow_gradient else 0
        e = getattr(mol, "ecp", None)
        if e is not None:
            ek = [np.ascontiguousarray(e.term_atom, np.int32), np.ascontiguousarray(e.term_l, np.int32),
                  np.ascontiguousarray(e.term_n, np.int32), np.ascontiguousarray(e.term_exp, np.float64),
                  np.ascontiguousarray(e.term_coef, np.float64), np.ascontiguousarray(e.rcut, np.float64)]
            self._keep += ek
            self._ecp = _Ecp(len(ek[0]), ip(ek[0]), ip(ek[1]), ip(ek[2]), dp(ek[3]), dp(ek[4]), dp(ek[5]),
                             ct.c_uint64(int(e.rot_seed)), int(ecp_max_pairs))
            opt.ecp = ct.pointer(self._ecp)
        h = ct.c_void_p()
        rc = L.vmc_init(ct.byref(basis), ct.byref(nuc), ct.byref(mo), ct.byref(jas), ct.byref(opt), device,
                        ct.byref(h))
        if rc != VMC_OK:
            raise VmcError(rc, L.vmc_init_error().decode())
        self._h = h
        self.mol = mol
        self.N, self.A, self.M, self.n_occ = mol.n_elec, mol.n_atoms, n_ao, mol.n_occ
        self.max_walkers = int(max_walkers)
        self.device = device

    # ------------------------------------------------------------------
    def _rc(self, rc):
        if rc != VMC_OK:
            raise VmcError(rc, lib().vmc_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().vmc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def sweep(self, walkers, nsteps, seed, sweep_offset=0, measure=True, accept=None):
        import torch
        W = walkers.shape[0]
        _check_dev(walkers, (W, self.N, 3))
        if accept is not None:
            _check_dev(accept, (nsteps, self.N, W), torch.uint8)
        self._rc(lib().vmc_sweep(self._h, _ptr(walkers), W, nsteps, ct.c_uint64(seed), ct.c_uint64(sweep_offset),
                                 VMC_SWEEP_MEASURE if measure else 0, _ptr(accept), _stream()))

    def accumulate_walkers(self, walkers, weights=None):
        """Measure the given configurations and add them to the accumulators
        with per-walker weights |Psi/Psi_G|^2 (device FP64 [W]; None = 1)."""
        W = walkers.shape[0]
        _check_dev(walkers, (W, self.N, 3))
        if weights is not None:
            _check_dev(weights, (W,))
        self._rc(lib().vmc_accumulate_walkers(self._h, _ptr(walkers), W, _ptr(weights), _stream()))

    def jastrow_gradient(self):
        """dE/dxi1 [MJ] and dE/dxi3 [MJ][MJ] over the samples since the last
        reset (read before accumulate(reset=True))."""
        MJ = self.mol.jastrow.jas_basis.n_ao
        g1 = np.zeros(MJ)
        g3 = np.zeros((MJ, MJ))
        dpn = lambda a: a.ctypes.data_as(ct.c_void_p)
        self._rc(lib().vmc_jastrow_gradient(self._h, dpn(g1), dpn(g3), _stream()))
        return g1, g3

    def accumulate(self, reset=True):
        E = np.zeros(2)
        F = np.zeros((self.A, 3))
        dEdC = np.zeros((self.M, self.n_occ))
        dELdC = np.zeros((self.M, self.n_occ))
        ns = ct.c_int64(0)
        dpn = lambda a: a.ctypes.data_as(ct.c_void_p)
        self._rc(lib().vmc_accumulate(self._h, dpn(E), dpn(F), dpn(dEdC), dpn(dELdC), ct.byref(ns),
                                      VMC_ACCUM_RESET if reset else 0, _stream()))
        return dict(E=E[0], E_sigma=E[1], F_bare=F, dE_dC=dEdC, dEL_dC_mean=dELdC, n_samples=ns.value)

    def jackknife(self):
        """Leave-one-block-out replicas (E [nb], F_bare [nb][A][3], dE_dC [nb][M][n])
        over the complete blocks since the last reset (device tensors)."""
        import torch
        nb = ct.c_int64(0)
        self._rc(lib().vmc_jackknife(self._h, None, None, None, ct.byref(nb), _stream()))
        dev = torch.device("cuda", self.device)
        E = torch.empty((nb.value,), dtype=torch.float64, device=dev)
        F = torch.empty((nb.value, self.A, 3), dtype=torch.float64, device=dev)
        C = torch.empty((nb.value, self.M, self.n_occ), dtype=torch.float64, device=dev)
        self._rc(lib().vmc_jackknife(self._h, _ptr(E), _ptr(F), _ptr(C), ct.byref(nb), _stream()))
        return dict(E=E, F_bare=F, dE_dC=C)

    def profile(self, enable=True):
        """Start (clearing the totals) or stop HIP-event timing of the kernels."""
        self._rc(lib().vmc_profile(self._h, 1 if enable else 0))

    def profile_read(self, kernel):
        """(total ms, launches, walkers) of a kernel since profile(True);
        kernel in ("adjoint", "dense", "mo_rows", "sweep", "proposals", "ecp_points", "ecp_energy",
        "ecp_adjoint", "jas_gemm")."""
        k = {"adjoint": 0, "dense": 1, "mo_rows": 2, "sweep": 3, "proposals": 4, "ecp_points": 5, "ecp_energy": 6,
             "ecp_adjoint": 7, "jas_gemm": 8}[kernel]
        ms, nl, nw = ct.c_double(0), ct.c_int64(0), ct.c_int64(0)
        self._rc(lib().vmc_profile_read(self._h, k, ct.byref(ms), ct.byref(nl), ct.byref(nw)))
        return ms.value, nl.value, nw.value

    def chunk_walkers(self):
        return int(lib().vmc_staging_walkers(self._h))

    def measure(self, walkers, C=None, R=None, R0=None, outputs=("EL", "lnpsi", "lnjac", "dEL_dR", "dlnpsi_dR",
                                                                  "dlnjac_dR", "O", "G")):
        import torch
        W = walkers.shape[0]
        shapes = dict(EL=(W,), lnpsi=(W,), lnjac=(W,), dEL_dR=(W, self.A, 3), dlnpsi_dR=(W, self.A, 3),
                      dlnjac_dR=(W, self.A, 3), O=(W, self.M, self.n_occ), G=(W, self.M, self.n_occ))
        res = {k: torch.empty(shapes[k], dtype=torch.float64, device=walkers.device) for k in outputs}
        return self.measure_into(walkers, res, C, R, R0)

    def measure_into(self, walkers, res, C=None, R=None, R0=None):
        """Per-walker measurement into the tensors of `res` (keys of vmc_walker_out)."""
        W = walkers.shape[0]
        dev = walkers.device
        _check_dev(walkers, (W, self.N, 3))
        C = self._dev_C(C, dev)
        R, R0 = self._dev_R(R, R0, dev)
        shapes = dict(EL=(W,), lnpsi=(W,), lnjac=(W,), dEL_dR=(W, self.A, 3), dlnpsi_dR=(W, self.A, 3),
                      dlnjac_dR=(W, self.A, 3), O=(W, self.M, self.n_occ), G=(W, self.M, self.n_occ))
        for k, t in res.items():
            _check_dev(t, shapes[k])
        wo = _WalkerOut(*[res[k].data_ptr() if k in res else None for k in
                          ("EL", "lnpsi", "lnjac", "dEL_dR", "dlnpsi_dR", "dlnjac_dR", "O", "G")])
        self._rc(lib().vmc_measure(self._h, _ptr(walkers), W, _ptr(C), _ptr(R), _ptr(R0), ct.byref(wo), _stream()))
        return res

    def _dev_C(self, C, dev):
        import torch
        if C is None:
            C = torch.as_tensor(np.ascontiguousarray(self.mol.C), dtype=torch.float64, device=dev)
        _check_dev(C, (self.M, self.n_occ))
        return C

    def _dev_R(self, R, R0, dev):
        import torch
        if R is None:
            R = torch.as_tensor(np.ascontiguousarray(self.mol.xyz), dtype=torch.float64, device=dev)
        _check_dev(R, (self.A, 3))
        if R0 is None:
            R0 = R
        _check_dev(R0, (self.A, 3))
        return R, R0

    def eval(self, walkers, C, R, R0, lnpsi0):
        import torch
        W = walkers.shape[0]
        dev = walkers.device
        _check_dev(walkers, (W, self.N, 3))
        _check_dev(lnpsi0, (W,))
        out = {k: torch.empty(W, dtype=torch.float64, device=dev) for k in ("EL", "lnpsi", "lnjac", "wnorm")}
        out["Ehat"] = torch.empty(1, dtype=torch.float64, device=dev)
        self._rc(lib().vmc_eval(self._h, _ptr(walkers), W, _ptr(C), _ptr(R), _ptr(R0), _ptr(lnpsi0),
                                _ptr(out["EL"]), _ptr(out["lnpsi"]), _ptr(out["lnjac"]), _ptr(out["wnorm"]),
                                _ptr(out["Ehat"]), _stream()))
        return out

    def energy_cotangents(self, gE, EL, wnorm, Ehat):
        import torch
        W = EL.shape[0]
        g = {k: torch.empty(W, dtype=torch.float64, device=EL.device) for k in ("gEL", "gPsi", "gJac")}
        self._rc(lib().vmc_energy_cotangents(self._h, W, float(gE), _ptr(EL), _ptr(wnorm), _ptr(Ehat),
                                             _ptr(g["gEL"]), _ptr(g["gPsi"]), _ptr(g["gJac"]), _stream()))
        return g

    def adjoint(self, walkers, C, R, R0, gEL, gPsi, gJac):
        import torch
        W = walkers.shape[0]
        dev = walkers.device
        for t in (gEL, gPsi, gJac):
            _check_dev(t, (W,))
        dC = torch.empty((self.M, self.n_occ), dtype=torch.float64, device=dev)
        dR = torch.empty((self.A, 3), dtype=torch.float64, device=dev)
        self._rc(lib().vmc_adjoint(self._h, _ptr(walkers), W, _ptr(C), _ptr(R), _ptr(R0), _ptr(gEL), _ptr(gPsi),
                                   _ptr(gJac), _ptr(dC), _ptr(dR), _stream()))
        return dC, dR


ZVECTOR_JACOBI = 1


def _zv_check(rc):
    if rc != VMC_OK:
        raise VmcError(rc, lib().vmc_strerror(rc).decode())


def zvector_solve(H, b, rtol=1e-12, maxit=1000, jacobi=False):
    """Solve H z = -b by FP64 conjugate gradients on the GPU (optionally
    Jacobi-preconditioned).  b holds one right-hand side of H.shape[0]
    values, or a batch along its first dimension (then shape (n_rhs, ...)).
    Returns (z shaped like b, iterations: an int, or a list for a batch)."""
    import torch
    d = H.shape[0]
    _check_dev(H, (d, d))
    _check_dev(b, tuple(b.shape))
    single = b.numel() == d
    n_rhs = 1 if single else b.shape[0]
    if b.numel() != n_rhs * d:
        raise ValueError(f"b has {b.numel()} values, not a multiple {n_rhs} x {d}")
    z = torch.empty_like(b)
    it = (ct.c_int32 * n_rhs)()
    rc = lib().zvector_solve(_ptr(H), d, n_rhs, _ptr(b), _ptr(z), float(rtol), int(maxit),
                             ZVECTOR_JACOBI if jacobi else 0, ct.cast(it, ct.c_void_p), _stream())
    _zv_check(rc)
    return z, (it[0] if single else list(it))


ZVECTOR_NOALLOC_MAX_D = 65536


def zvector_solve_noalloc(H, b, z, rtol=1e-12, maxit=1000, jacobi=False):
    """zvector_solve into a caller-provided z (same shape as b), with no
    device allocation by the library (its CG state lives in a fixed device
    array; right-hand sides are solved one after another).  Returns the
    iterations (an int, or a list for a batch)."""
    d = H.shape[0]
    _check_dev(H, (d, d))
    _check_dev(b, tuple(b.shape))
    _check_dev(z, tuple(b.shape))
    single = b.numel() == d
    n_rhs = 1 if single else b.shape[0]
    if b.numel() != n_rhs * d:
        raise ValueError(f"b has {b.numel()} values, not a multiple {n_rhs} x {d}")
    it = (ct.c_int32 * n_rhs)()
    rc = lib().zvector_solve_noalloc(_ptr(H), d, n_rhs, _ptr(b), _ptr(z), float(rtol), int(maxit),
                                     ZVECTOR_JACOBI if jacobi else 0, ct.cast(it, ct.c_void_p), _stream())
    _zv_check(rc)
    return it[0] if single else list(it)


def _batch(x, shape2):
    if tuple(x.shape) == tuple(shape2):
        return 1, False
    if x.dim() == 3 and tuple(x.shape[1:]) == tuple(shape2):
        return x.shape[0], True
    raise ValueError(f"expected shape {tuple(shape2)} or (batch, {shape2[0]}, {shape2[1]}), got {tuple(x.shape)}")


def zvector_rhs(Cv, dE_dC):
    """b = Cv^T dE/dC, shape (n_virt, n_occ) (or a batch of them): the
    right-hand side of the Z-vector equations in the virtual-occupied block."""
    import torch
    M, nv = Cv.shape
    n = dE_dC.shape[-1]
    _check_dev(Cv, (M, nv))
    nb, bat = _batch(dE_dC, (M, n))
    _check_dev(dE_dC, tuple(dE_dC.shape))
    b = torch.empty(((nb,) if bat else ()) + (nv, n), dtype=torch.float64, device=Cv.device)
    _zv_check(lib().zvector_rhs(_ptr(Cv), M, nv, n, nb, _ptr(dE_dC), _ptr(b), _stream()))
    return b


def zvector_backmap(Cv, z):
    """Z = Cv z, shape (n_ao, n_occ) (or a batch): the response in the AO basis."""
    import torch
    M, nv = Cv.shape
    n = z.shape[-1]
    _check_dev(Cv, (M, nv))
    nb, bat = _batch(z, (nv, n))
    _check_dev(z, tuple(z.shape))
    Z = torch.empty(((nb,) if bat else ()) + (M, n), dtype=torch.float64, device=Cv.device)
    _zv_check(lib().zvector_backmap(_ptr(Cv), M, nv, n, nb, _ptr(z), _ptr(Z), _stream()))
    return Z


def jackknife_stats(x_jk):
    """Jackknife mean and standard error over the first dimension of the
    replicas x_jk (device, FP64): sqrt((nb - 1)/nb sum (x_b - mean)^2)."""
    import torch
    _check_dev(x_jk, tuple(x_jk.shape))
    nb = x_jk.shape[0]
    ln = x_jk[0].numel()
    mean = torch.empty(x_jk.shape[1:], dtype=torch.float64, device=x_jk.device)
    sigma = torch.empty_like(mean)
    _zv_check(lib().zvector_jackknife(_ptr(x_jk), nb, ln, _ptr(mean), _ptr(sigma), _stream()))
    return mean, sigma


def _make_energy_function():
    import torch

    class VMCEnergy(torch.autograd.Function):
        """Fixed-sample reweighted energy E_hat(C, R) on given walkers.

        forward : E_hat = sum_k w_k E_L,k / sum_k w_k with
                  w_k = exp(2 (ln|Psi_k(C,R)| - lnpsi0_k)) * Jac_k(R)
                  (electrons warped with the space-warp weights of R0);
        backward: exact derivative via the hand-written adjoint kernel;
                  nothing per walker is saved beyond E_L, the weights and E_hat.
        """

        @staticmethod
        def forward(fctx, C, R, context, walkers, R0, lnpsi0):
            C = C.detach().contiguous()
            R = R.detach().contiguous()
            out = context.eval(walkers, C, R, R0, lnpsi0)
            fctx.context = context
            fctx.save_for_backward(C, R, walkers, R0, out["EL"], out["wnorm"], out["Ehat"])
            return out["Ehat"][0].clone()

        @staticmethod
        def backward(fctx, gE):
            C, R, walkers, R0, EL, wnorm, Ehat = fctx.saved_tensors
            context = fctx.context
            g = context.energy_cotangents(float(gE), EL, wnorm, Ehat)
            dC, dR = context.adjoint(walkers, C, R, R0, g["gEL"], g["gPsi"], g["gJac"])
            return dC, dR, None, None, None, None

    return VMCEnergy


_VMCEnergy = None


def vmc_energy(C, R, context, walkers, R0, lnpsi0):
    """Differentiable fixed-sample energy (see VMCEnergy)."""
    global _VMCEnergy
    if _VMCEnergy is None:
        _VMCEnergy = _make_energy_function()
    return _VMCEnergy.apply(C, R, context, walkers, R0, lnpsi0)
