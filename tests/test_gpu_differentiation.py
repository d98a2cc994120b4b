"""Differentiation at the 21-atom size (94 electrons, 235 AOs, 47 occupied
orbitals; 256 walkers on fixed samples), through the autograd function whose
backward is the hand-written adjoint:

* against the oracle: dE/dC of the fixed-sample energy on all 235 x 47
  coefficients equals the oracle's dE_dC + <dE_L/dC> (1e-10 of its scale), on
  walkers at their generated starting positions;
* against finite differences (the exactness pin of the estimators): after 50
  sweeps, central differences (h = 1e-4, Richardson-extrapolated with h/2,
  so the truncation error is O(h^4)) of the GPU forward agree with the
  backward on all 63 nuclear coordinates and on a seeded subset of 200
  coefficients, to 1e-6 of max(1, |derivative|).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_05222_amd import inputs

pytestmark = pytest.mark.gpu

W = 256


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_05222_amd import vmc
    vmc.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def mol():
    return inputs.make_config(2).molecule


def backward(ctx, tw, mol, dev):
    from paper_2511_05222_amd import vmc
    C = torch.tensor(mol.C, device=dev, requires_grad=True)
    R0 = torch.tensor(mol.xyz, device=dev)
    R = R0.clone().requires_grad_(True)
    lnpsi0 = ctx.measure(tw, outputs=("lnpsi",))["lnpsi"]
    E = vmc.vmc_energy(C, R, ctx, tw, R0, lnpsi0)
    E.backward()
    torch.cuda.synchronize()
    return E.item(), C.grad.cpu().numpy(), R.grad.cpu().numpy(), R0, lnpsi0


def test_dEdC_21atom_against_oracle(dev, mol):
    from oracle import derivatives as dv, estimators, wavefunction as wf
    from paper_2511_05222_amd import vmc
    r = inputs.initial_walkers(mol, W, 29)
    ctx = vmc.Context(mol, max_walkers=W)
    tw = torch.tensor(r, device=dev)
    E, gC, gR, _, _ = backward(ctx, tw, mol, dev)
    s = wf.System(mol)
    O, G, ev = dv.coefficient_derivatives(s, s.xyz, r)
    acc = estimators.Accumulator(s.A, s.M, s.C.shape[1])
    zero = np.zeros((W, s.A, 3))
    acc.add(dict(E_L=ev["E_L"], H=zero, P=zero, O=O, G=G))
    ref = acc.result()
    want = ref["dE_dC"] + ref["dEL_dC_mean"]
    assert gC.shape == want.shape == (235, 47)
    scale = np.abs(want).max()
    err = np.abs(gC - want).max()
    assert err <= 1e-10 * scale, (err, scale)
    assert abs(E - ref["E"]) <= 1e-10 * abs(ref["E"])


def test_fixed_sample_derivatives_21atom(dev, mol):
    from paper_2511_05222_amd import vmc
    spec = inputs.make_config(2)
    ctx = vmc.Context(mol, max_walkers=W)
    tw = torch.tensor(inputs.initial_walkers(mol, W, spec.seed), device=dev)
    ctx.sweep(tw, 50, spec.seed, measure=False)
    E, gC, gR, R0, lnpsi0 = backward(ctx, tw, mol, dev)
    C0 = torch.tensor(mol.C, device=dev)

    def ehat(Cv, Rv):
        return vmc.vmc_energy(Cv, Rv, ctx, tw, R0, lnpsi0).item()

    def fd(shift):
        h = 1e-4
        d1 = (ehat(*shift(h)) - ehat(*shift(-h))) / (2 * h)
        d2 = (ehat(*shift(h / 2)) - ehat(*shift(-h / 2))) / h
        return (4.0 * d2 - d1) / 3.0

    worst = 0.0
    for a in range(mol.n_atoms):
        for k in range(3):
            def shift(t, a=a, k=k):
                Rt = R0.clone()
                Rt[a, k] += t
                return C0, Rt
            f = fd(shift)
            rel = abs(f - gR[a, k]) / max(1.0, abs(f))
            worst = max(worst, rel)
            assert rel < 1e-6, ("R", a, k, f, gR[a, k])
    rng = np.random.default_rng(31)
    picks = rng.choice(mol.C.size, size=200, replace=False)
    for flat in picks:
        mu, i = divmod(int(flat), mol.C.shape[1])

        def shift(t, mu=mu, i=i):
            Ct = C0.clone()
            Ct[mu, i] += t
            return Ct, R0
        f = fd(shift)
        rel = abs(f - gC[mu, i]) / max(1.0, abs(f))
        worst = max(worst, rel)
        assert rel < 1e-6, ("C", mu, i, f, gC[mu, i])
    print(f"\n[differentiation 21 atoms] E_hat = {E:.6f}; worst relative FD mismatch {worst:.2e} "
          f"(63 R components, 200 C entries)")
