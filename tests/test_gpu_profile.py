"""Kernel timing through the C ABI (vmc_profile / vmc_profile_read): launch
counts and walker counts of every timed kernel over sweeps with measurement
split into several measurement launches, the totals cleared when timing is
enabled again, the one-/three-body Jastrow products timed with their own id,
and an unknown kernel id rejected."""
import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_05222_amd import inputs

pytestmark = pytest.mark.gpu

MAIN = ("adjoint", "dense", "mo_rows", "sweep", "proposals")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_05222_amd import vmc
    vmc.lib()
    return torch.device("cuda:0")


def _counts(ctx, names):
    return {k: ctx.profile_read(k) for k in names}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_launch_and_walker_counts(dev, precision):
    from paper_2511_05222_amd import vmc
    mol = inputs.make_config(1).molecule
    W, sweeps, chunk = 64, 2, 32
    ctx = vmc.Context(mol, max_walkers=W, staging_walkers=chunk, precision=precision)
    w = torch.tensor(inputs.initial_walkers(mol, W, 3), device=dev)
    print(f"case: 9-atom kernel timing, {precision}", flush=True)
    ctx.profile(True)
    ctx.sweep(w, sweeps, 17)
    torch.cuda.synchronize()
    got = _counts(ctx, MAIN + ("ecp_points", "ecp_energy", "ecp_adjoint", "jas_gemm"))
    ctx.profile(False)
    nm = sweeps * ((W + chunk - 1) // chunk)   # measurement launches
    want = {"sweep": sweeps, "proposals": sweeps, "mo_rows": nm, "dense": nm, "adjoint": nm}
    for k, n in want.items():
        ms, nl, nw = got[k]
        assert nl == n, (k, nl, n)
        assert nw == sweeps * W, (k, nw)
        assert ms > 0.0, (k, ms)
    for k in ("ecp_points", "ecp_energy", "ecp_adjoint", "jas_gemm"):
        assert got[k] == (0.0, 0, 0), (k, got[k])
    # enabling again clears the totals
    ctx.profile(True)
    assert all(v == (0.0, 0, 0) for v in _counts(ctx, MAIN).values())
    ctx.sweep(w, 1, 18, sweep_offset=sweeps, measure=False)
    torch.cuda.synchronize()
    got = _counts(ctx, MAIN)
    ctx.profile(False)
    assert got["sweep"][1] == 1 and got["proposals"][1] == 1 and got["adjoint"][1] == 0
    # an unknown kernel id
    ms, nl, nw = ct.c_double(0), ct.c_int64(0), ct.c_int64(0)
    rc = vmc.lib().vmc_profile_read(ctx._h, 99, ct.byref(ms), ct.byref(nl), ct.byref(nw))
    assert rc == vmc.VMC_EINVAL


def test_body_jastrow_products(dev):
    """The one-/three-body Jastrow products: one per sweep (the moves'
    differences) and two per measurement launch (values, xi3 h)."""
    from paper_2511_05222_amd import vmc
    mol = inputs.with_body_jastrow(inputs.make_config(1).molecule, 7)
    W, sweeps, chunk = 48, 2, 16
    ctx = vmc.Context(mol, max_walkers=W, staging_walkers=chunk, precision="mixed")
    w = torch.tensor(inputs.initial_walkers(mol, W, 5), device=dev)
    print("case: 9-atom J1/J3 kernel timing", flush=True)
    ctx.profile(True)
    ctx.sweep(w, sweeps, 23)
    torch.cuda.synchronize()
    ms, nl, nw = ctx.profile_read("jas_gemm")
    ctx.profile(False)
    nm = sweeps * ((W + chunk - 1) // chunk)
    assert nl == sweeps + 2 * nm, nl
    assert nw == sweeps * W + 2 * sweeps * W, nw
    assert ms > 0.0
