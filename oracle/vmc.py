"""One VMC run: sample, measure after every sweep, accumulate (oracle).

A walker-step is one sweep of N single-electron moves followed by one
measurement of E_L, the SWCT force terms and the MO-coefficient derivatives
at the new configuration, accumulated into the estimators.
"""
import numpy as np

from . import derivatives
from . import estimators
from . import sampler
from . import wavefunction as wf


def run(mol, walkers, n_sweeps, seed, sweep_offset=0, walker_ids=None, step_sigma=0.5,
        mode="sm", refresh_period=32, block_sweeps=1, measure=True, C=None, keep_samples=False,
        n_burn=0):
    """n_burn unmeasured sweeps (indices sweep_offset ...) precede n_sweeps
    measured ones."""
    system = wf.System(mol, C)
    acc = estimators.Accumulator(system.A, system.M, system.C.shape[1], block_sweeps)
    samples = []

    def meas(ch, sidx):
        m = derivatives.measure(system, system.xyz, ch.r, C, frame=(ch.ids, sidx))
        acc.add(m)
        if keep_samples:
            samples.append(dict(m, r=ch.r.copy(), sweep=sidx))

    def maybe_meas(ch, sidx):
        if measure and sidx >= sweep_offset + n_burn:
            meas(ch, sidx)

    ch, bits = sampler.run(system, walkers, n_burn + n_sweeps, seed, sweep_offset, walker_ids, step_sigma,
                           mode, refresh_period, maybe_meas)
    out = dict(positions=ch.r, accept=bits, system=system)
    if measure:
        out.update(acc.result())
        out["jackknife"] = acc.jackknife()
    if keep_samples:
        out["samples"] = samples
    return out
