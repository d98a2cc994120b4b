"""Monte Carlo estimators of E, the bare force and dE/dC (oracle).

  E      = <E_L>                                     (eq. eval-observable)
  F_bare = -<H> - 2 (<E_L P> - <E_L><P>)             (Appendix A SWCT force;
           H = dE_L/dR_alpha + sum_i omega dE_L/dr_i,
           P = dlnPsi/dR_alpha + sum_i [omega dlnPsi/dr_i + 1/2 grad_i omega])
  dE/dC  = 2 (<E_L O> - <E_L><O>),  O = dln|Psi|/dC  (eq. fc-vmc-eval; the
           paper prints a leading minus, while defining B = dE/dC in the
           Z-vector equations; the sign is fixed here by B = dE/dC, which the
           finite-difference check confirms)
  <dE_L/dC> is reported separately; its expectation vanishes and the
  covariance form drops it, as the paper does.
  dE/dxi = 2 (<E_L O_xi> - <E_L><O_xi>), O_xi = dln|Psi|/dxi of the one- and
           three/four-body Jastrow parameters (xi1, and xi3 as a symmetric
           matrix), the same covariance form (the gradient the paper's
           stochastic reconfiguration of the Jastrow works with); present
           when the measurements carry Oxi1 and Oxi3.

All sums are FP64 with a shift s (the mean E_L of the first measured batch)
subtracted from E_L, so that the covariances do not cancel catastrophically
(E_L is hundreds of hartree).  Batches are summed by numpy (pairwise) and
accumulated across batches with Neumaier compensation.  Block sums of E_L - s
per `block_sweeps` sweeps give the blocked error bar.

Reweighting (Appendix A, the reweighting equation): when the configurations
x' come from a guiding distribution Psi_G^2 instead of Psi^2, every average
above becomes <O W>/<W> with W = |Psi/Psi_G|^2.  The paper names the
Attaccalite-Sorella guiding function but does not define it; the weights are
therefore an input here (one per walker, W = 1 for samples of Psi^2, which
reproduces the unweighted estimators exactly).  Every sum below carries the
walker's weight and K is the sum of the weights.

Jackknife (the resampling the paper uses for the error of B and of what the
Z-vector equations make of it, Sec. II): every complete block keeps its own
sums of all estimator terms; replica b is the estimate from all blocks but b,
and the jackknife error of any function of the replicas x_b is
sqrt((nb - 1)/nb * sum_b (x_b - mean)^2).
"""
import numpy as np


class _Neumaier:
    def __init__(self, shape):
        self.s = np.zeros(shape)
        self.c = np.zeros(shape)

    def add(self, x):
        t = self.s + x
        big = np.abs(self.s) >= np.abs(x)
        self.c += np.where(big, (self.s - t) + x, (x - t) + self.s)
        self.s = t

    @property
    def value(self):
        return self.s + self.c


class Accumulator:
    def __init__(self, n_atoms, n_ao, n_occ, block_sweeps=1):
        A, M, n = n_atoms, n_ao, n_occ
        self.shift = None
        self.K = 0.0
        self.sums = {k: _Neumaier(sh) for k, sh in dict(
            E=(), EE=(), H=(A, 3), P=(A, 3), EP=(A, 3), O=(M, n), EO=(M, n), G=(M, n)).items()}
        self.block_sweeps = block_sweeps
        self.block_sums = []
        self.block_counts = []
        self._cur_block = [0.0, 0.0]
        self._sweeps_in_block = 0
        self.block_F = []
        self._blk = None
        self.block_terms = []      # per complete block: dict of term sums and K
        self._terms = None
        self.xi = None             # Jastrow-parameter sums (Oxi1, EOxi1, Oxi3, EOxi3)

    def _block_force(self, e, wt, meas):
        """Per-block force estimate (for blocked error bars of F)."""
        if self._blk is None:
            self._blk = dict(K=0.0, E=0.0, H=0.0, P=0.0, EP=0.0)
        b = self._blk
        b["K"] += float(np.sum(wt))
        b["E"] += np.sum(wt * e)
        b["H"] = b["H"] + np.einsum("w,wak->ak", wt, meas["H"])
        b["P"] = b["P"] + np.einsum("w,wak->ak", wt, meas["P"])
        b["EP"] = b["EP"] + np.einsum("w,wak->ak", wt * e, meas["P"])

    def add(self, meas, weights=None):
        """Add a batch of measured walkers; weights[W] = |Psi/Psi_G|^2 of each
        (None: all 1, samples of Psi^2).  The shift is the mean E_L of the
        first batch (unweighted)."""
        E = np.asarray(meas["E_L"], dtype=np.float64)
        if self.shift is None:
            self.shift = float(np.mean(E))
        e = E - self.shift
        W = E.shape[0]
        wt = np.ones(W) if weights is None else np.asarray(weights, dtype=np.float64)
        Kb = float(np.sum(wt))
        self.K += Kb
        we = wt * e
        sm = self.sums
        sm["E"].add(np.sum(we))
        sm["EE"].add(np.sum(we * e))
        sm["H"].add(np.einsum("w,wak->ak", wt, meas["H"]))
        sm["P"].add(np.einsum("w,wak->ak", wt, meas["P"]))
        sm["EP"].add(np.einsum("w,wak->ak", we, meas["P"]))
        sm["O"].add(np.einsum("w,wmi->mi", wt, meas["O"]))
        sm["EO"].add(np.einsum("w,wmi->mi", we, meas["O"]))
        sm["G"].add(np.einsum("w,wmi->mi", wt, meas["G"]))
        if "Oxi1" in meas:
            if self.xi is None:
                self.xi = {k: _Neumaier(np.shape(meas[k.lstrip("E")])[1:]) for k in ("Oxi1", "EOxi1", "Oxi3", "EOxi3")}
            self.xi["Oxi1"].add(np.einsum("w,wm->m", wt, meas["Oxi1"]))
            self.xi["EOxi1"].add(np.einsum("w,wm->m", we, meas["Oxi1"]))
            self.xi["Oxi3"].add(np.einsum("w,wmn->mn", wt, meas["Oxi3"]))
            self.xi["EOxi3"].add(np.einsum("w,wmn->mn", we, meas["Oxi3"]))
        t = dict(K=Kb, E=np.sum(we), H=np.einsum("w,wak->ak", wt, meas["H"]),
                 P=np.einsum("w,wak->ak", wt, meas["P"]), EP=np.einsum("w,wak->ak", we, meas["P"]),
                 O=np.einsum("w,wmi->mi", wt, meas["O"]), EO=np.einsum("w,wmi->mi", we, meas["O"]))
        self._terms = t if self._terms is None else {k: self._terms[k] + t[k] for k in t}
        self._cur_block[0] += float(np.sum(we))
        self._cur_block[1] += Kb
        self._block_force(e, wt, meas)
        self._sweeps_in_block += 1
        if self._sweeps_in_block == self.block_sweeps:
            b = self._blk
            k = float(b["K"])
            self.block_F.append(-b["H"] / k - 2.0 * (b["EP"] / k - (b["E"] / k) * (b["P"] / k)))
            self._blk = None
            self.block_terms.append(self._terms)
            self._terms = None
            self.block_sums.append(self._cur_block[0])
            self.block_counts.append(self._cur_block[1])
            self._cur_block = [0.0, 0.0]
            self._sweeps_in_block = 0

    def result(self):
        K = float(self.K)
        v = {k: a.value / K for k, a in self.sums.items()}
        E = self.shift + v["E"]
        F = -v["H"] - 2.0 * (v["EP"] - v["E"] * v["P"])
        dEdC = 2.0 * (v["EO"] - v["E"] * v["O"])
        nb = len(self.block_sums)
        if nb >= 2:
            bm = np.array(self.block_sums) / np.array(self.block_counts)
            sigma = float(np.std(bm, ddof=1) / np.sqrt(nb))
            F_sigma = np.std(np.array(self.block_F), axis=0, ddof=1) / np.sqrt(nb)
        else:
            sigma = float("nan")
            F_sigma = np.full_like(F, np.nan)
        out = dict(E=E, E_sigma=sigma, F_sigma=F_sigma, F_bare=F, dE_dC=dEdC, dEL_dC_mean=v["G"],
                   var_E=v["EE"] - v["E"] ** 2, K=self.K, shift=self.shift)
        if self.xi is not None:
            x = {k: a.value / K for k, a in self.xi.items()}
            out["dE_dxi1"] = 2.0 * (x["EOxi1"] - v["E"] * x["Oxi1"])
            out["dE_dxi3"] = 2.0 * (x["EOxi3"] - v["E"] * x["Oxi3"])
        return out

    def jackknife(self):
        """Leave-one-block-out replicas of E, F_bare and dE/dC over the complete
        blocks: replica b sums the terms of every block except b."""
        nb = len(self.block_terms)
        out = dict(E=[], F_bare=[], dE_dC=[])
        for b in range(nb if nb >= 2 else 0):   # a replica needs another block
            rest = [self.block_terms[q] for q in range(nb) if q != b]
            K = float(sum(r["K"] for r in rest))
            v = {k: sum(r[k] for r in rest) / K for k in ("E", "H", "P", "EP", "O", "EO")}
            out["E"].append(self.shift + v["E"])
            out["F_bare"].append(-v["H"] - 2.0 * (v["EP"] - v["E"] * v["P"]))
            out["dE_dC"].append(2.0 * (v["EO"] - v["E"] * v["O"]))
        return {k: np.array(x) for k, x in out.items()}


def jackknife_stats(x):
    """Mean and jackknife standard error over the first axis of replicas x."""
    x = np.asarray(x, dtype=np.float64)
    nb = x.shape[0]
    m = x.mean(axis=0)
    return m, np.sqrt((nb - 1) / nb * ((x - m) ** 2).sum(axis=0))
