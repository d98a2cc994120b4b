"""The allocation-free Z-vector entry point (zvector_solve_noalloc) through
the C ABI against zvector_solve on the same inputs: two calls in a row, the
second smaller (its CG state reuses the fixed device array the first call
left dirty), bit for bit against the allocating entry point's one-at-a-time
solves, and the first against the oracle's CG (same stopping rule, 1e-9)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_05222_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_05222_amd import vmc
    vmc.lib()
    return torch.device("cuda:0")


def test_noalloc_matches_allocating_solver(dev):
    from oracle import zvector
    from paper_2511_05222_amd import vmc
    # call 1: d = 9541 (the 47 x 203 rotation space), Jacobi
    d1 = 9541
    H1 = inputs.seeded_spd(d1, 31)
    b1 = np.random.default_rng(32).standard_normal(d1)
    tH1, tb1 = torch.tensor(H1, device=dev), torch.tensor(b1, device=dev)
    z_ref, it_ref = vmc.zvector_solve(tH1, tb1, rtol=1e-12, maxit=2000, jacobi=True)
    z1 = torch.full_like(tb1, float("nan"))
    print(f"case: noalloc d={d1} jacobi", flush=True)
    it1 = vmc.zvector_solve_noalloc(tH1, tb1, z1, rtol=1e-12, maxit=2000, jacobi=True)
    assert it1 == it_ref
    assert torch.equal(z1, z_ref)
    zo, _, ok = zvector.cg_solve(H1, b1, rtol=1e-12, maxit=2000, jacobi=True)
    assert ok
    z1n = z1.cpu().numpy()
    assert np.abs(z1n - zo).max() <= 1e-9 * np.abs(zo).max()
    # call 2: smaller, two right-hand sides, no preconditioner
    d2 = 300
    H2 = inputs.seeded_spd(d2, 33)
    b2 = np.random.default_rng(34).standard_normal((2, d2))
    tH2, tb2 = torch.tensor(H2, device=dev), torch.tensor(b2, device=dev)
    z2 = torch.full_like(tb2, float("nan"))
    print(f"case: noalloc d={d2} x2", flush=True)
    it2 = vmc.zvector_solve_noalloc(tH2, tb2, z2, rtol=1e-12, maxit=2000)
    for k in range(2):
        zk, itk = vmc.zvector_solve(tH2, tb2[k].contiguous(), rtol=1e-12, maxit=2000)
        assert it2[k] == itk
        assert torch.equal(z2[k], zk)
    res = H2 @ z2.cpu().numpy().T + b2.T
    assert np.all(np.linalg.norm(res, axis=0) <= 1e-12 * np.linalg.norm(b2, axis=1) * 1.0001)


def test_noalloc_rejects_oversize(dev):
    from paper_2511_05222_amd import vmc
    d = vmc.ZVECTOR_NOALLOC_MAX_D + 1
    # a 1 x 1 view stands in: the size check happens before any device work
    H = torch.zeros((1,), dtype=torch.float64, device=dev)
    rc = vmc.lib().zvector_solve_noalloc(vmc._ptr(H), d, 1, vmc._ptr(H), vmc._ptr(H), 1e-12, 10, 0, None,
                                         vmc._stream())
    assert rc == vmc.VMC_EINVAL
