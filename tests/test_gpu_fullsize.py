"""Parity at the production size: the 21-atom molecule (94 electrons, 235
cartesian AOs, 47 occupied orbitals per spin) with all 65536 walkers, in the
launch configuration of the throughput run (inverse refresh every 32 moves,
the chunked measurement after every sweep, FP64 and mixed).

The oracle cannot run 65536 walkers, but every walker is an independent chain
whose random numbers are keyed on its own index, so the oracle runs a sample
of walker indices one by one (the first and last walker, the edges of a
four-walker sweep block and of a measurement chunk) and the GPU's rows for
those indices are compared with it:

  FP64   accept/reject bit-exact, positions to 1e-13 of their scale, and every
         per-walker measured quantity to 1e-10 of its array's scale;
  mixed  accept/reject agreement >= 99% on the sampled moves (an FP32 ratio
         can only differ from the FP64 one within its rounding of q), and
         walkers whose decisions all agree equal in position to 1e-13.

Whole-batch properties that hold at any size are checked on the full run:
the estimator invariants C^T dE/dC = 0 and sum_alpha F_alpha = 0 (both exact
per sample set), and mixed against FP64 on the same 65536 configurations
within the stated error bounds (|dE| < 5e-6 Ha, half the 1e-5 Ha target;
|dF| < 1e-4 Ha/bohr).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_05222_amd import inputs

pytestmark = pytest.mark.gpu

SWEEPS = 2
MEAS = ("EL", "lnpsi", "lnjac", "dEL_dR", "dlnpsi_dR", "dlnjac_dR", "O", "G")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_05222_amd import vmc
    vmc.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def full():
    spec = inputs.make_config(2)
    mol = spec.molecule
    W = spec.n_walkers
    return spec, mol, W, inputs.initial_walkers(mol, W, spec.seed)


def sample_ids(W, chunk):
    # measurement launches split W into equal chunks of at most `chunk`
    step = -(-W // -(-W // chunk))
    ids = {0, 3, 4, W // 2 + 1, step - 1, step, W - 1}
    return sorted(i for i in ids if 0 <= i < W)


def close(gpu, ref, tol, what):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(gpu - ref).max()
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e} (rel {err / scale:.3e})"


def run_gpu(dev, spec, mol, W, w0, precision):
    from paper_2511_05222_amd import vmc
    ctx = vmc.Context(mol, max_walkers=W, refresh_period=32, precision=precision)
    tw = torch.tensor(w0, device=dev)
    acc = torch.zeros((SWEEPS, mol.n_elec, W), dtype=torch.uint8, device=dev)
    ctx.sweep(tw, SWEEPS, spec.seed, sweep_offset=0, measure=True, accept=acc)
    res = ctx.accumulate()
    torch.cuda.synchronize()
    return ctx, tw, acc, res


def check_invariants(mol, res, W, tol):
    assert res["n_samples"] == W * SWEEPS
    C = np.asarray(mol.C)
    assert np.isfinite(res["E"]) and np.isfinite(res["F_bare"]).all() and np.isfinite(res["dE_dC"]).all()
    ctd = np.abs(C.T @ res["dE_dC"]).max() / (np.abs(C).max() * np.abs(res["dE_dC"]).max())
    fs = np.abs(res["F_bare"].sum(axis=0)).max() / np.abs(res["F_bare"]).max()
    print(f"\n[full size] E = {res['E']:.6f} +- {res['E_sigma']:.2e}, |C^T dE/dC| rel {ctd:.2e}, "
          f"|sum F| rel {fs:.2e}")
    assert ctd < tol
    assert fs < tol


def test_fullsize_fp64_sweep_and_measure(dev, full):
    from oracle import derivatives as dv, sampler, wavefunction as wf
    spec, mol, W, w0 = full
    ctx, tw, acc, res = run_gpu(dev, spec, mol, W, w0, "fp64")
    ids = sample_ids(W, ctx.chunk_walkers())
    s = wf.System(mol)
    ch, bits = sampler.run(s, w0[ids], SWEEPS, spec.seed, walker_ids=np.array(ids, np.uint64), refresh_period=32)
    assert np.array_equal(acc[:, :, ids].cpu().numpy().astype(bool), bits)
    close(tw[ids].cpu().numpy(), ch.r, 1e-13, "positions")
    check_invariants(mol, res, W, 1e-9)

    # the measurement of all 65536 walkers at their new positions, sampled
    out = ctx.measure(tw, outputs=MEAS)
    got = {k: v[ids].cpu().numpy() for k, v in out.items()}
    del out
    torch.cuda.synchronize()
    r = ch.r
    dE, dP, dJ = dv.nuclear_derivatives(s, s.xyz, s.xyz, r)
    O, G, ev = dv.coefficient_derivatives(s, s.xyz, r)
    ref = dict(EL=ev["E_L"], lnpsi=ev["lnpsi"], dEL_dR=dE, dlnpsi_dR=dP, dlnjac_dR=dJ, O=O, G=G)
    for k, v in ref.items():
        close(got[k], v, 1e-10, f"sampled {k}")
    assert np.abs(got["lnjac"]).max() == 0.0


def test_fullsize_mixed(dev, full):
    from oracle import sampler, wavefunction as wf
    from paper_2511_05222_amd import vmc
    spec, mol, W, w0 = full
    ctx, tw, acc, res = run_gpu(dev, spec, mol, W, w0, "mixed")
    ids = sample_ids(W, ctx.chunk_walkers())
    ch, bits = sampler.run(wf.System(mol), w0[ids], SWEEPS, spec.seed, walker_ids=np.array(ids, np.uint64),
                           refresh_period=32)
    gbits = acc[:, :, ids].cpu().numpy().astype(bool)
    agree = np.mean(gbits == bits)
    print(f"\n[full size mixed] sampled accept agreement {agree:.4f}")
    assert agree >= 0.99
    same = np.all(gbits == bits, axis=(0, 1))
    assert same.any()
    close(tw[ids].cpu().numpy()[same], ch.r[same], 1e-13, "positions of agreeing walkers")
    check_invariants(mol, res, W, 1e-5)

    # mixed against FP64 on the same 65536 configurations
    outs = ("EL", "lnjac", "dEL_dR", "dlnpsi_dR", "dlnjac_dR")
    c64 = vmc.Context(mol, max_walkers=W, refresh_period=32, precision="fp64")
    ef = {}
    for name, c in (("mixed", ctx), ("fp64", c64)):
        o = c.measure(tw, outputs=outs)
        E, H = o["EL"], o["dEL_dR"]
        P = o["dlnpsi_dR"] + 0.5 * o["dlnjac_dR"]
        assert torch.isfinite(E).all() and torch.isfinite(H).all()
        sft = E.mean()
        e = E - sft
        F = -H.mean(0) - 2.0 * ((e[:, None, None] * P).mean(0) - e.mean() * P.mean(0))
        ef[name] = ((sft + e.mean()).item(), F.cpu().numpy())
        del o
    dE = abs(ef["mixed"][0] - ef["fp64"][0])
    dF = np.abs(ef["mixed"][1] - ef["fp64"][1]).max()
    print(f"[full size mixed vs fp64] |dE| = {dE:.2e} Ha, max |dF| = {dF:.2e} Ha/bohr")
    assert dE < 5e-6
    assert dF < 1e-4


def test_fullsize_exponential_jastrow(dev, full):
    """The exponential two-body workload as the throughput run launches it:
    the 21-atom molecule with u = a(1 - e^{-F r})/F (eq. twobody_v_exp),
    16384 walkers.  FP64: accept bits, positions and every per-walker
    measured quantity of three sampled walkers against the oracle, the
    invariants on the whole batch; mixed against FP64 on the same
    configurations within the bounds."""
    import dataclasses
    from oracle import derivatives as dv, sampler, wavefunction as wf
    from paper_2511_05222_amd import vmc
    spec, mol, _, _ = full
    me = dataclasses.replace(mol, jastrow=dataclasses.replace(mol.jastrow, ee_form=1))
    W = 16384
    w0 = inputs.initial_walkers(me, W, spec.seed)
    print("case: 21-atom exponential two-body Jastrow, 16384 walkers, FP64", flush=True)
    ctx, tw, acc, res = run_gpu(dev, spec, me, W, w0, "fp64")
    step = -(-W // -(-W // ctx.chunk_walkers()))
    ids = sorted({0, step - 1, W - 1})
    s = wf.System(me)
    ch, bits = sampler.run(s, w0[ids], SWEEPS, spec.seed, walker_ids=np.array(ids, np.uint64), refresh_period=32)
    assert np.array_equal(acc[:, :, ids].cpu().numpy().astype(bool), bits)
    close(tw[ids].cpu().numpy(), ch.r, 1e-13, "positions")
    check_invariants(me, res, W, 1e-9)
    outs = ("EL", "lnpsi", "dEL_dR", "dlnpsi_dR", "O", "G")
    out = ctx.measure(tw, outputs=outs)
    got = {k: v[ids].cpu().numpy() for k, v in out.items()}
    dE, dP, _ = dv.nuclear_derivatives(s, s.xyz, s.xyz, ch.r)
    O, G, ev = dv.coefficient_derivatives(s, s.xyz, ch.r)
    ref = dict(EL=ev["E_L"], lnpsi=ev["lnpsi"], dEL_dR=dE, dlnpsi_dR=dP, O=O, G=G)
    for k, v in ref.items():
        close(got[k], v, 1e-10, f"sampled {k}")
    c32 = vmc.Context(me, max_walkers=W, refresh_period=32, precision="mixed")
    o32 = c32.measure(tw, outputs=("EL", "dEL_dR", "dlnpsi_dR"))
    torch.cuda.synchronize()

    def ef(o):
        E, H, Pp = o["EL"], o["dEL_dR"], o["dlnpsi_dR"]
        e = E - E.mean()
        return E.mean().item(), -H.mean(0) - 2.0 * ((e[:, None, None] * Pp).mean(0) - e.mean() * Pp.mean(0))

    E64, F64 = ef(out)
    E32, F32 = ef(o32)
    dEm, dFm = abs(E32 - E64), (F32 - F64).abs().max().item()
    print(f"[exponential Jastrow full size mixed vs fp64] |dE| = {dEm:.2e} Ha, max |dF| = {dFm:.2e} Ha/bohr")
    assert dEm <= 5e-6 and dFm < 1e-4
