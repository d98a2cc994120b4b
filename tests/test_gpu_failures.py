"""Failure detection through the C ABI: a singular Slater block, a non-finite
walker, and the forced inverse refresh after an accepted move with a small
determinant ratio (its accept/reject sequence against the oracle's).

Every case is forced from the host with valid inputs of valid shapes; no
kernel is made to fault.  A walker with a coincident same-spin pair or a NaN
coordinate only turns its own arithmetic singular or non-finite: the other
walkers' chains are checked to be unaffected.
"""
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


@pytest.fixture(scope="module")
def mol9():
    return inputs.make_config(1).molecule


def _run(mol, w0, dev, precision="fp64", sweeps=2, seed=77):
    from paper_2511_05222_amd import vmc
    ctx = vmc.Context(mol, max_walkers=w0.shape[0], precision=precision)
    tw = torch.tensor(w0, device=dev)
    ctx.sweep(tw, sweeps, seed)
    torch.cuda.synchronize()
    err = None
    try:
        ctx.accumulate(reset=True)
    except vmc.VmcError as e:
        err = e.code
    # the error state is cleared by the reset: a clean batch then reads fine
    return err, tw.cpu().numpy(), ctx


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coincident_same_spin_pair_is_singular(dev, mol9, precision):
    from paper_2511_05222_amd import vmc
    W, bad = 8, 3
    w0 = inputs.initial_walkers(mol9, W, 5)
    ref_err, ref_pos, _ = _run(mol9, w0, dev, precision)
    assert ref_err is None
    w1 = w0.copy()
    w1[bad, 1] = w1[bad, 0]          # electrons 0 and 1 are both spin up
    print(f"case: coincident pair, walker {bad}, {precision}", flush=True)
    err, pos, ctx = _run(mol9, w1, dev, precision)
    assert err == vmc.VMC_ESINGULAR
    keep = np.arange(W) != bad
    assert np.array_equal(pos[keep], ref_pos[keep])
    # the reset cleared the error: the next batch of clean walkers is fine
    tw = torch.tensor(w0, device=dev)
    ctx.sweep(tw, 1, 78)
    ctx.accumulate(reset=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nan_walker_is_nonfinite(dev, mol9, precision):
    from paper_2511_05222_amd import vmc
    W, bad = 8, 5
    w0 = inputs.initial_walkers(mol9, W, 6)
    ref_err, ref_pos, _ = _run(mol9, w0, dev, precision)
    assert ref_err is None
    w1 = w0.copy()
    w1[bad, 2, 0] = np.nan
    print(f"case: NaN coordinate, walker {bad}, {precision}", flush=True)
    err, pos, _ = _run(mol9, w1, dev, precision)
    assert err == vmc.VMC_ENONFINITE
    keep = np.arange(W) != bad
    assert np.array_equal(pos[keep], ref_pos[keep])


def test_far_electron_is_singular(dev, mol9):
    """An electron so far out that every orbital underflows to zero: an
    all-zero row of its Slater block."""
    from paper_2511_05222_amd import vmc
    W, bad = 4, 1
    w1 = inputs.initial_walkers(mol9, W, 7)
    w1[bad, 20] = [4000.0, 0.0, 0.0]
    print("case: far electron", flush=True)
    err, _, _ = _run(mol9, w1, dev, "fp64", sweeps=1)
    assert err == vmc.VMC_ESINGULAR


@pytest.mark.parametrize("threshold", [0.3, 1.0])
def test_forced_refresh_matches_oracle(dev, mol9, threshold):
    """With the forced-refresh threshold raised, many accepted moves rebuild
    their block's inverse; the accept/reject sequence still matches the
    oracle's (which applies the same rule) bit for bit."""
    from oracle import sampler
    from oracle import wavefunction as wf
    from paper_2511_05222_amd import vmc
    W, sweeps, seed = 24, 3, 4242
    w0 = inputs.initial_walkers(mol9, W, 9)
    s = wf.System(mol9)
    ch, bits = sampler.run(s, w0, sweeps, seed, forced_ratio=threshold)
    assert ch.n_forced > 10, ch.n_forced      # the rule really fired
    print(f"case: forced refresh threshold {threshold}, {ch.n_forced} forced rebuilds in the oracle", flush=True)
    ctx = vmc.Context(mol9, max_walkers=W, forced_refresh_ratio=threshold)
    tw = torch.tensor(w0, device=dev)
    acc = torch.zeros((sweeps, mol9.n_elec, W), dtype=torch.uint8, device=dev)
    ctx.sweep(tw, sweeps, seed, measure=False, accept=acc)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy().astype(bool), bits)
    assert np.abs(tw.cpu().numpy() - ch.r).max() < 1e-12
