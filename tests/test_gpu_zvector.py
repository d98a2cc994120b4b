"""Z-vector step on the GPU (through the C ABI) against the oracle, at the
sizes of the 21-atom molecule: 47 occupied and 188 virtual orbitals (d = 8836,
right-hand side from a real dE/dC of the molecule) and the 47 x 203 rotation
space (d = 9541, seeded right-hand side).  Orbital Hessians are the seeded SPD
stand-ins diag(d) + G G^T / 64.

A batch of 12 seeded right-hand sides at 47 x 203 runs through the batched
solver (the reads of H shared by all of them) and is compared column by
column with the oracle's CG and with the one-at-a-time solver.

Checks: the projection b = C_virt^T dE/dC and the back-map Z = C_virt z
against the oracle to 1e-13 of their scale; CG (plain and Jacobi) against the
oracle's CG with the same stopping rule to 1e-9 (both stop at a relative
residual of 1e-12; the difference is the conditioning times that residual);
the residual ||H z + b|| <= rtol ||b|| recomputed on the host; and
Z^T S C_occ = 0 for the back-mapped response.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_05222_amd import inputs

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_05222_amd import vmc
    vmc.lib()
    return torch.device("cuda:0")


def close(gpu, ref, tol, what):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(gpu - ref).max()
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e} (rel {err / scale:.3e})"


def solve_both(dev, H, b, jacobi):
    from oracle import zvector
    from paper_2511_05222_amd import vmc
    tH = torch.tensor(H, device=dev)
    tb = torch.tensor(b, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z, it = vmc.zvector_solve(tH, tb, rtol=RTOL, maxit=2000, jacobi=jacobi)
    dt = time.perf_counter() - t0
    z = z.cpu().numpy()
    d = b.size
    print(f"\n[zvector] d={d} jacobi={jacobi}: {it} iterations, {dt * 1e3:.1f} ms "
          f"({8.0 * d * d * it / dt / 1e12:.2f} TB/s of H per iteration, host round trips included)")
    zr, itr, ok = zvector.cg_solve(H, b.ravel(), rtol=RTOL, maxit=2000, jacobi=jacobi)
    assert ok
    assert abs(it - itr) <= 2, (it, itr)
    bf = b.ravel()
    assert np.linalg.norm(H @ z.ravel() + bf) <= RTOL * np.linalg.norm(bf) * 1.0001
    close(z.ravel(), zr, 1e-9, f"z (jacobi={jacobi})")
    return z


def test_zvector_21atom_real_rhs(dev):
    """b from the oracle's dE/dC of the 21-atom molecule (64 walkers at their
    starting positions), projected on the GPU; CG; back-map; Z^T S C = 0."""
    from oracle import derivatives as dv, estimators, wavefunction as wf, zvector
    from paper_2511_05222_amd import vmc
    mol = inputs.make_config(2).molecule
    s = wf.System(mol)
    r = inputs.initial_walkers(mol, 64, 17)
    O, G, ev = dv.coefficient_derivatives(s, s.xyz, r)
    acc = estimators.Accumulator(s.A, s.M, s.C.shape[1])
    A = s.A
    zero = np.zeros((r.shape[0], A, 3))
    acc.add(dict(E_L=ev["E_L"], H=zero, P=zero, O=O, G=G))
    dEdC = acc.result()["dE_dC"]
    n = mol.n_occ
    Cv = np.ascontiguousarray(mol.C_full[:, n:])
    assert Cv.shape == (235, 188)
    tCv = torch.tensor(Cv, device=dev)
    b = vmc.zvector_rhs(tCv, torch.tensor(dEdC, device=dev)).cpu().numpy()
    b_ref = zvector.rhs(Cv, dEdC)
    close(b, b_ref, 1e-13, "b")
    H = inputs.seeded_spd(b.size, 21)
    for jacobi in (False, True):
        z = solve_both(dev, H, b_ref, jacobi)
    Z = vmc.zvector_backmap(tCv, torch.tensor(z, device=dev)).cpu().numpy()
    close(Z, zvector.backmap(Cv, z), 1e-13, "Z")
    S = inputs.overlap_matrix(mol.xyz, mol.basis)
    assert np.abs(Z.T @ S @ mol.C).max() < 1e-10 * np.abs(Z).max()


def test_zvector_47x203_seeded(dev):
    d = 47 * 203
    H = inputs.seeded_spd(d, 22)
    b = np.random.default_rng(23).standard_normal((203, 47))
    for jacobi in (False, True):
        solve_both(dev, H, b, jacobi)


def test_zvector_errors(dev):
    from paper_2511_05222_amd import vmc
    H = torch.tensor(inputs.seeded_spd(50, 2), device=dev)
    b = torch.tensor(np.random.default_rng(2).standard_normal(50), device=dev)
    with pytest.raises(vmc.VmcError) as ei:
        vmc.zvector_solve(H, b, rtol=1e-12, maxit=3)
    assert ei.value.code == vmc.VMC_ENOTCONV
    z, it = vmc.zvector_solve(H, torch.zeros_like(b), rtol=1e-12)
    assert it == 0 and float(z.abs().max()) == 0.0
    Hn = H.clone()
    Hn[3, 3] = float("nan")
    with pytest.raises(vmc.VmcError) as ei:
        vmc.zvector_solve(Hn, b, rtol=1e-12, jacobi=True)
    assert ei.value.code == vmc.VMC_ENONFINITE


def test_zvector_batched_47x203(dev):
    from oracle import zvector
    from paper_2511_05222_amd import vmc
    d, nr = 47 * 203, 12
    H = inputs.seeded_spd(d, 24)
    B = np.random.default_rng(25).standard_normal((nr, d))
    tH = torch.tensor(H, device=dev)
    tB = torch.tensor(B, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Z, its = vmc.zvector_solve(tH, tB, rtol=RTOL, maxit=2000, jacobi=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    z0, it0 = vmc.zvector_solve(tH, tB[0].contiguous(), rtol=RTOL, maxit=2000, jacobi=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    print(f"\n[zvector batched] {nr} right-hand sides at d={d}: {tb * 1e3:.1f} ms together, "
          f"{t1 * 1e3:.1f} ms for one alone; iterations {its}")
    Z = Z.cpu().numpy()
    for k in range(nr):
        zr, itr, ok = zvector.cg_solve(H, B[k], rtol=RTOL, maxit=2000, jacobi=True)
        assert ok and abs(its[k] - itr) <= 2
        assert np.linalg.norm(H @ Z[k] + B[k]) <= RTOL * np.linalg.norm(B[k]) * 1.0001
        close(Z[k], zr, 1e-9, f"z[{k}]")
    close(Z[0], z0.cpu().numpy(), 1e-10, "batched vs single")
