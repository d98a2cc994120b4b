"""Host-only checks of the C ABI: the library loads, exports every entry
point that include/vmc.h declares, and rejects bad inputs before any GPU
work (no GPU needed)."""
import copy
import os
import re

import numpy as np
import pytest

from paper_2511_05222_amd import inputs, vmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vmc_\w+|zvector_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = vmc.lib()
    names = declared_functions()
    assert "vmc_init" in names and "zvector_solve" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vmc.EXPORTED)


def test_strerror():
    L = vmc.lib()
    assert L.vmc_strerror(vmc.VMC_ENOTCONV) == b"VMC_ENOTCONV"
    assert L.vmc_strerror(-99) == b"VMC_UNKNOWN"


def _bad(mutate):
    mol = copy.deepcopy(inputs.make_config(1).molecule)
    mutate(mol)
    with pytest.raises(vmc.VmcError) as ei:
        vmc.Context(mol, 4)
    return ei.value


def test_rejects_f_shells():
    def m(mol):
        mol.basis.shell_l = mol.basis.shell_l.copy(); mol.basis.shell_l[3] = 3
    e = _bad(m)
    assert e.code == vmc.VMC_EINVAL and "l = 3" in str(e)


def test_rejects_nonpositive_exponent():
    def m(mol):
        mol.basis.prim_exp = mol.basis.prim_exp.copy(); mol.basis.prim_exp[5] = 0.0
    assert _bad(m).code == vmc.VMC_EINVAL


def test_rejects_nonfinite_coefficients():
    def m(mol):
        mol.C_full = mol.C_full.copy(); mol.C_full[2, 1] = np.inf
    assert _bad(m).code == vmc.VMC_EINVAL


def test_rejects_open_shell():
    def m(mol):
        mol.n_dn -= 1
    assert _bad(m).code == vmc.VMC_EINVAL


def test_rejects_bad_atom_index():
    def m(mol):
        mol.basis.shell_atom = mol.basis.shell_atom.copy(); mol.basis.shell_atom[0] = 99
    assert _bad(m).code == vmc.VMC_EINVAL


def test_rejects_too_many_orbitals():
    def m(mol):
        mol.n_up = mol.n_dn = 65   # C_full has 75 columns; 65 occupied > VMC_MAX_OCC
    e = _bad(m)
    assert e.code == vmc.VMC_EINVAL and "exceed" in str(e)


def test_rejects_bad_jastrow_form():
    def form(f, F):
        def m(mol):
            mol.jastrow = inputs.Jastrow(0.5, F, 0, 0.0, ee_form=f)
        return m
    assert _bad(form(2, 1.0)).code == vmc.VMC_EINVAL
    assert _bad(form(1, 0.0)).code == vmc.VMC_EINVAL   # the exponential form needs F > 0


def test_rejects_bad_options():
    mol = inputs.make_config(0).molecule
    with pytest.raises(vmc.VmcError) as ei:
        vmc.Context(mol, 4, refresh_period=0)
    assert ei.value.code == vmc.VMC_EINVAL
    with pytest.raises(vmc.VmcError):
        vmc.Context(mol, 0)


def test_zvector_rejects_bad_sizes():
    L = vmc.lib()
    import ctypes as ct
    it = ct.c_int32(0)
    assert L.zvector_solve(None, 0, 1, None, None, 1e-10, 10, 0, ct.byref(it), None) == vmc.VMC_EINVAL
    assert L.zvector_rhs(None, 5, 3, 2, 1, None, None, None) == vmc.VMC_EINVAL
    assert L.zvector_backmap(None, 5, 3, 2, 1, None, None, None) == vmc.VMC_EINVAL
    assert L.zvector_jackknife(None, 4, 3, None, None, None) == vmc.VMC_EINVAL
    assert L.vmc_jackknife(None, None, None, None, None, None) == vmc.VMC_EINVAL


def test_rejects_bad_body_jastrow():
    import dataclasses
    mol = inputs.with_body_jastrow(inputs.make_config(1).molecule, 7)
    xi3 = mol.jastrow.xi3.copy()
    xi3[0, 1] += 1e-3                       # not symmetric
    bad = dataclasses.replace(mol, jastrow=dataclasses.replace(mol.jastrow, xi3=xi3))
    with pytest.raises(vmc.VmcError) as ei:
        vmc.Context(bad, 4)
    assert ei.value.code == vmc.VMC_EINVAL and "symmetric" in str(ei.value)
    jb = mol.jastrow.jas_basis
    big = inputs.Basis(np.tile(jb.shell_atom, 4), np.tile(jb.shell_l, 4), np.tile(jb.shell_nprim, 4),
                       np.tile(jb.prim_exp, 4), np.tile(jb.prim_coef, 4))
    M4 = big.n_ao
    bad = dataclasses.replace(mol, jastrow=dataclasses.replace(mol.jastrow, jas_basis=big, xi1=np.zeros(M4),
                                                               xi3=np.zeros((M4, M4))))
    with pytest.raises(vmc.VmcError) as ei:
        vmc.Context(bad, 4)
    assert ei.value.code == vmc.VMC_EINVAL and "exceed" in str(ei.value)


def test_rejects_bad_pseudopotential():
    import dataclasses
    mol = inputs.with_ecp(inputs.make_config(1).molecule, 5)
    e = mol.ecp
    for field, value, word in (("term_l", np.where(e.term_l == 1, 4, e.term_l), "term"),
                               ("term_n", np.where(e.term_n == 2, 0, e.term_n), "term"),
                               ("term_exp", -e.term_exp, "term"),
                               ("rcut", np.full_like(e.rcut, np.nan), "cutoff"),
                              ("term_atom", np.where(e.term_atom == 0, 99, e.term_atom), "term")):
        bad = dataclasses.replace(mol, ecp=dataclasses.replace(e, **{field: value}))
        with pytest.raises(vmc.VmcError) as ei:
            vmc.Context(bad, 4)
        assert ei.value.code == vmc.VMC_EINVAL and word in str(ei.value), (field, str(ei.value))
