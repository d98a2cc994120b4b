"""Single-electron Metropolis sampling of |Psi|^2 (oracle).

The paper draws configurations from pi(x) = Psi^2 / int Psi^2 by Markov chain
Monte Carlo over independent chains (Appendix A, "Variational Monte Carlo
Methods"; chain counts in "Computational details").  It does not state the
move.  Reading (the move of the hot path being reproduced):
  * a sweep proposes, for e = 0 .. N-1 in order, r'_e = r_e + sigma z with
    z ~ N(0, I_3) (sigma = 0.5 bohr);
  * q = |Psi(x')/Psi(x)|^2 = (det ratio * exp(J(x') - J(x)))^2, accepted iff
    u < q with u uniform in [0, 1) (q >= 1 always accepts);
  * all draws come from Philox keyed by (seed; walker, sweep, electron), so any
    subset of walker ids reproduces the same chains.

Two ratio modes:
  exact  the determinant ratio from two fresh LU factorisations;
  sm     the ratio phi(r')^T K[:, e] from a Sherman-Morrison-updated inverse
         K = A^-1; after an accepted move
             K <- K - K[:, e] (phi(r')^T K - e_e^T) / ratio.
         The inverses of both spin blocks persist across sweeps.  A block's
         K is recomputed from scratch at the start of a run, after every
         `refresh_period`-th proposed move of that block (its own move index
         sweep * n_block + j, j the electron's index within the block), and
         after an accepted move of that block whose |ratio| is below
         forced_ratio (1e-8 unless given; the update divides by the ratio).
"""
import numpy as np

from . import gto
from . import philox
from . import wavefunction as wf

FORCED_REFRESH_RATIO = 1e-8


class Chains:
    """A batch of walkers and their sampler state."""

    def __init__(self, system, walkers, walker_ids=None, R=None):
        self.system = system
        self.r = np.array(walkers, dtype=np.float64, copy=True)      # [W,N,3]
        W = self.r.shape[0]
        self.ids = np.arange(W, dtype=np.uint64) if walker_ids is None else np.asarray(walker_ids, np.uint64)
        self.R = system.xyz if R is None else np.asarray(R, np.float64)
        self.K = None
        self.n_forced = 0          # forced refreshes so far (walker-moves)

    # ------------------------------------------------------------------
    def spin_of(self, e):
        s = self.system
        if e < s.n_up:
            return 0, e, slice(0, s.n_up), s.n_up
        return 1, e - s.n_up, slice(s.n_up, s.N), s.n_dn

    def orbitals_at(self, pts, n):
        val, _, _ = gto.eval_aos(self.system.table, self.R, pts)
        return val @ self.system.C[:, :n]

    def refresh(self, mask=None, blocks=(0, 1)):
        """Recompute K = A^-1 of the given spin blocks from the current
        positions (for the walkers in mask, default all)."""
        s = self.system
        phi = self.orbitals_at(self.r, s.C.shape[1])
        K = list(self.K) if self.K is not None else [None, None]
        for b, (sl, n) in enumerate(s.spin_blocks()):
            if b not in blocks and self.K is not None:
                continue
            Kn = np.linalg.inv(phi[:, sl, :n])
            if mask is not None and self.K is not None:
                Kn = np.where(mask[:, None, None], Kn, self.K[b])
            K[b] = Kn
        self.K = K

    def jastrow_delta(self, e, r_new):
        """J(x') - J(x) for moving electron e to r_new [W,3]."""
        s = self.system
        others = [j for j in range(s.N) if j != e]
        dJ = np.zeros(self.r.shape[0])
        if others:
            ro = self.r[:, others, :]
            dn = np.sqrt(np.sum((r_new[:, None, :] - ro) ** 2, axis=-1))
            do = np.sqrt(np.sum((self.r[:, e, None, :] - ro) ** 2, axis=-1))
            dJ += np.sum(wf.ee_pair(s, dn)[0] - wf.ee_pair(s, do)[0], axis=1)
        if s.jas_table is not None:
            # one- and three/four-body terms: only the pairs (e, j) change
            c_new, _, _ = gto.eval_aos(s.jas_table, self.R, r_new[:, None, :])
            c_old, _, _ = gto.eval_aos(s.jas_table, self.R, self.r[:, e, None, :])
            dchi = (c_new - c_old)[:, 0, :]                            # [W, MJ]
            dJ += dchi @ s.xi1
            if others:
                c_oth, _, _ = gto.eval_aos(s.jas_table, self.R, self.r[:, others, :])
                dJ += np.einsum("wm,mn,wjn->w", dchi, s.xi3, c_oth)
        if s.en_on:
            for al in range(s.A):
                dn = np.linalg.norm(r_new - self.R[al], axis=-1)
                do = np.linalg.norm(self.r[:, e] - self.R[al], axis=-1)
                dJ += wf.pade(dn, -s.Z[al], s.en_b)[0] - wf.pade(do, -s.Z[al], s.en_b)[0]
        return dJ

    # ------------------------------------------------------------------
    def sweep(self, seed, sweep_index, step_sigma=0.5, mode="sm", refresh_period=32,
              forced_ratio=FORCED_REFRESH_RATIO):
        """One sweep of N single-electron moves; returns accept bits [N, W]."""
        s = self.system
        W = self.r.shape[0]
        acc_bits = np.zeros((s.N, W), dtype=bool)
        if mode == "sm" and self.K is None:
            self.refresh()
        for e in range(s.N):
            b, j, sl, n = self.spin_of(e)
            z = philox.move_normals(seed, self.ids, sweep_index, e)
            u = philox.move_uniform(seed, self.ids, sweep_index, e)
            r_new = self.r[:, e, :] + step_sigma * z
            phi_new = self.orbitals_at(r_new, n)                      # [W, n]
            if mode == "exact":
                A_old = self.orbitals_at(self.r[:, sl, :], n)
                A_new = A_old.copy()
                A_new[:, j, :] = phi_new
                s0, l0 = wf.lu_logdet(A_old)
                s1, l1 = wf.lu_logdet(A_new)
                ratio = s0 * s1 * np.exp(l1 - l0)
            else:
                K = self.K[b]
                v = np.einsum("wi,wic->wc", phi_new, K)               # phi'^T K
                ratio = v[:, j]
            q = (ratio * np.exp(self.jastrow_delta(e, r_new))) ** 2
            acc = u < q
            acc_bits[e] = acc
            self.r[acc, e, :] = r_new[acc]
            if mode == "sm":
                colj = K[:, :, j].copy()                              # K[:, e]
                t = v.copy()
                t[:, j] -= 1.0
                upd = colj[:, :, None] * (t / ratio[:, None])[:, None, :]
                K[acc] -= upd[acc]
                forced = acc & (np.abs(ratio) < forced_ratio)
                self.n_forced += int(np.count_nonzero(forced))
                if np.any(forced):
                    self.refresh(mask=forced, blocks=(b,))
                m = sweep_index * n + j
                if (m + 1) % refresh_period == 0:
                    self.refresh(blocks=(b,))
        return acc_bits


def run(system, walkers, n_sweeps, seed, sweep_offset=0, walker_ids=None, step_sigma=0.5,
        mode="sm", refresh_period=32, measure=None, forced_ratio=FORCED_REFRESH_RATIO):
    """Sample n_sweeps sweeps; call measure(chains, sweep_index) after each.

    Returns (chains, accept bits [n_sweeps, N, W]).
    """
    ch = Chains(system, walkers, walker_ids)
    bits = []
    for t in range(n_sweeps):
        sidx = sweep_offset + t
        bits.append(ch.sweep(seed, sidx, step_sigma, mode, refresh_period, forced_ratio))
        if measure is not None:
            measure(ch, sidx)
    return ch, np.array(bits)
