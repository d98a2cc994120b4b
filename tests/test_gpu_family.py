"""The mixed-size family (64 seeded geometries of 9-21 atoms, 8192 walkers
each) as parity cases.  Five members are sampled so that every register
class of the sweep is covered, including the two occupied-orbital counts
that fill a class exactly (n = 16 and n = 32):

  g22  9 atoms, n = 13      g7  10 atoms, n = 16      g3  15 atoms, n = 32
  g0  18 atoms, n = 37      g1  21 atoms, n = 47

Beyond the family, a 23-atom member of the same composition rule (n = 53, the
largest register class) stands for the maximum size.

For each: FP64 accept/reject bit-exact and positions to 1e-13 against the
oracle (6 walkers, 2 sweeps, refresh every 32 moves); FP64 per-walker
measurement against the oracle to 1e-10 (2 walkers); mixed against FP64 on
the same 8192 configurations within |dE| < 5e-6 Ha (half the 1e-5 Ha target)
and |dF| < 1e-4 Ha/bohr.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_05222_amd import inputs

pytestmark = pytest.mark.gpu

# (family index, or 100 + atom count for the member beyond the family; n)
MEMBERS = [(22, 13), (7, 16), (3, 32), (0, 37), (1, 47), (123, 53)]


def member(g):
    if g < inputs.FAMILY_SIZE:
        return inputs.family_member(g)
    A = g - 100
    mol = inputs.make_molecule(inputs.composition(A), 1000 + g, 2000 + g, 3000 + g, f"{A}-atom (largest class)")
    return inputs.RunSpec(mol, 8192, 10, 4, precision="mixed")


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


def energy_force(o):
    E, H = o["EL"], o["dEL_dR"]
    P = o["dlnpsi_dR"] + 0.5 * o["dlnjac_dR"]
    s = E.mean()
    e = E - s
    F = -H.mean(0) - 2.0 * ((e[:, None, None] * P).mean(0) - e.mean() * P.mean(0))
    return (s + e.mean()).item(), F.cpu().numpy()


@pytest.mark.parametrize("g,n_occ", MEMBERS)
def test_family_member(dev, g, n_occ):
    from oracle import derivatives as dv, sampler, wavefunction as wf
    from paper_2511_05222_amd import vmc
    spec = member(g)
    mol = spec.molecule
    assert mol.n_occ == n_occ
    s = wf.System(mol)

    # sweeps: bit-exact decisions against the oracle
    W = 6
    w0 = inputs.initial_walkers(mol, W, 40 + g)
    ch, bits = sampler.run(s, w0, 2, 500 + g, refresh_period=32)
    ctx = vmc.Context(mol, max_walkers=W)
    tw = torch.tensor(w0, device=dev)
    acc = torch.zeros((2, mol.n_elec, W), dtype=torch.uint8, device=dev)
    ctx.sweep(tw, 2, 500 + g, measure=True, accept=acc)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy().astype(bool), bits)
    close(tw.cpu().numpy(), ch.r, 1e-13, f"g{g} positions")

    # measurement of two of them against the oracle
    r = ch.r[:2]
    out = ctx.measure(torch.tensor(r, device=dev))
    torch.cuda.synchronize()
    dE, dP, dJ = dv.nuclear_derivatives(s, s.xyz, s.xyz, r)
    O, G, ev = dv.coefficient_derivatives(s, s.xyz, r)
    ref = dict(EL=ev["E_L"], lnpsi=ev["lnpsi"], dEL_dR=dE, dlnpsi_dR=dP, dlnjac_dR=dJ, O=O, G=G)
    for k, v in ref.items():
        close(out[k].cpu().numpy(), v, 1e-10, f"g{g} {k}")

    # mixed against FP64 on the family's 8192 walkers
    Wf = spec.n_walkers
    tw = torch.tensor(inputs.initial_walkers(mol, Wf, spec.seed), device=dev)
    c64 = vmc.Context(mol, max_walkers=Wf, precision="fp64")
    c64.sweep(tw, 3, spec.seed, measure=False)
    c32 = vmc.Context(mol, max_walkers=Wf, precision="mixed")
    outs = ("EL", "lnjac", "dEL_dR", "dlnpsi_dR", "dlnjac_dR")
    E64, F64 = energy_force(c64.measure(tw, outputs=outs))
    E32, F32 = energy_force(c32.measure(tw, outputs=outs))
    dEm = abs(E32 - E64)
    dFm = np.abs(F32 - F64).max()
    print(f"\n[family g{g}] {mol.name}: N={mol.n_elec} M={mol.basis.n_ao} n={mol.n_occ}; mixed vs fp64 on {Wf} "
          f"walkers |dE|={dEm:.2e} Ha, max|dF|={dFm:.2e} Ha/bohr")
    assert dEm < 5e-6
    assert dFm < 1e-4
