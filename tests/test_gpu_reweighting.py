"""Reweighted estimators (Appendix A, the reweighting equation: averages
<O W> / <W> with W = |Psi/Psi_G|^2 per walker) through the C ABI, against the
oracle's weighted accumulator.

9-atom molecule, FP64: three batches of configurations sampled by the oracle,
each added with vmc_accumulate_walkers and seeded weights in [0.2, 2), one
block per batch, measured in launches smaller than a batch (a ragged tail).
E, F_bare, dE/dC and <dE_L/dC> to 1e-10 of each array's scale, the blocked
error bar of weighted block means to 1e-8, the jackknife replicas to 1e-10.
Weights of one equal the sweeps' own unweighted accumulation bit for bit.
Mixed precision: the same weighted batches within the mixed-vs-FP64 bounds.
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


def close(gpu, ref, tol, what):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(gpu - ref).max()
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e} (rel {err / scale:.3e})"


@pytest.fixture(scope="module")
def batches():
    from oracle import sampler
    from oracle import wavefunction as wf
    mol = inputs.make_config(1).molecule
    s = wf.System(mol)
    W = 23
    out = []
    pos = inputs.initial_walkers(mol, W, 31)
    rng = np.random.default_rng(32)
    for b in range(3):
        ch, _ = sampler.run(s, pos, 2, 33, sweep_offset=2 * b)
        pos = ch.r
        out.append((pos.copy(), rng.uniform(0.2, 2.0, W)))
    return mol, out


def test_weighted_estimators_match_oracle(dev, batches):
    from oracle import derivatives as dv
    from oracle import estimators
    from oracle import wavefunction as wf
    from paper_2511_05222_amd import vmc
    mol, bs = batches
    s = wf.System(mol)
    acc = estimators.Accumulator(s.A, s.M, s.C.shape[1])
    ctx = vmc.Context(mol, max_walkers=23, staging_walkers=10, jackknife_blocks=4)
    for pos, wts in bs:
        acc.add(dv.measure(s, s.xyz, pos), wts)
        print(f"case: weighted batch of {pos.shape[0]} walkers", flush=True)
        ctx.accumulate_walkers(torch.tensor(pos, device=dev), torch.tensor(wts, device=dev))
    jk = ctx.jackknife()
    res = ctx.accumulate()
    ref = acc.result()
    close(res["E"], ref["E"], 1e-10, "E")
    close(res["F_bare"], ref["F_bare"], 1e-10, "F_bare")
    close(res["dE_dC"], ref["dE_dC"], 1e-10, "dE/dC")
    close(res["dEL_dC_mean"], ref["dEL_dC_mean"], 1e-10, "<dE_L/dC>")
    assert res["n_samples"] == 3 * 23
    assert abs(res["E_sigma"] - ref["E_sigma"]) <= 1e-8 * ref["E_sigma"]
    rjk = acc.jackknife()
    for k in ("E", "F_bare", "dE_dC"):
        close(jk[k].cpu().numpy(), rjk[k], 1e-10, f"replicas {k}")


def test_unit_weights_equal_unweighted(dev, batches):
    from paper_2511_05222_amd import vmc
    mol, bs = batches
    r = []
    for weights in (None, "ones"):
        ctx = vmc.Context(mol, max_walkers=23)
        for pos, _ in bs:
            tw = torch.tensor(pos, device=dev)
            wt = None if weights is None else torch.ones(pos.shape[0], dtype=torch.float64, device=dev)
            ctx.accumulate_walkers(tw, wt)
        r.append(ctx.accumulate())
    for k in ("E", "F_bare", "dE_dC", "dEL_dC_mean"):
        assert np.array_equal(np.asarray(r[0][k]), np.asarray(r[1][k])), k


def test_weighted_mixed_within_bounds(dev, batches):
    from paper_2511_05222_amd import vmc
    mol, bs = batches
    r = {}
    for prec in ("fp64", "mixed"):
        ctx = vmc.Context(mol, max_walkers=23, precision=prec)
        for pos, wts in bs:
            ctx.accumulate_walkers(torch.tensor(pos, device=dev), torch.tensor(wts, device=dev))
        r[prec] = ctx.accumulate()
    assert abs(r["mixed"]["E"] - r["fp64"]["E"]) < 1e-5
    assert np.abs(r["mixed"]["F_bare"] - r["fp64"]["F_bare"]).max() < 1e-4
