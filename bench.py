"""Throughput of the VMC force hot path on one MI355X.

A step is one sweep of N single-electron Metropolis moves for every walker
followed by one measurement (local energy, SWCT Hellmann-Feynman + Pulay force
terms, dE_L/dC and dln|Psi|/dC) accumulated into the estimators: one
walker-step per walker.  value = walkers x steps / seconds.

Prints ONE JSON line.  Besides the timed region it
  * times the dominant kernel (the measurement kernel) with HIP events on the
    stream it is launched on and reports its achieved FP64 rate against the
    FP64 vector peak (roofline);
  * times the FP64 oracle on a bounded sample of the same workload on the host
    (cpu_baseline), unless --no-cpu-baseline.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walker-steps/s (fwd+adjoint) mixed vs FP64 on 1 GPU; force err Ha/bohr"
FP64_VECTOR_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_measure_9atom_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2511_05222_amd", "csrc", "vmc_pipeline.hip")
COPY_BYTES = 1 << 30   # plain device copy used to calibrate the HBM byte counters
WORKLOADS = {"9atom": 1, "21atom": 2}


def measure_flops_per_walker(N, M, n):
    """Algorithmic FP64 flops of one walker's measurement (dense contractions):
    forward MO value/gradient/Laplacian 10 N M n, adjoint back-projections
    4 N M n, outer products dln|Psi|/dC and dE_L/dC 6 N M n, Slater inverses
    2 x 2 n^3, (K X K) 2 x 4 n^3.  AO, Jastrow and potential work is not
    counted (the figure is a lower bound on the work done)."""
    return 20.0 * N * M * n + 12.0 * n ** 3


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def cpu_baseline(spec, budget_s=15.0):
    """Time the oracle (sm mode + full measurement) on a bounded sample."""
    import resource
    from oracle import vmc as ovmc
    mol = spec.molecule
    w0 = __import__("paper_2511_05222_amd.inputs", fromlist=["x"]).initial_walkers(mol, 64, spec.seed)
    done = 0
    t0 = time.perf_counter()
    c0 = resource.getrusage(resource.RUSAGE_SELF)
    walkers = w0
    sweeps = 0
    while time.perf_counter() - t0 < budget_s:
        res = ovmc.run(mol, walkers, 1, spec.seed, sweep_offset=sweeps)
        walkers = res["positions"]
        sweeps += 1
        done += walkers.shape[0]
    dt = time.perf_counter() - t0
    c1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (c1.ru_utime - c0.ru_utime) + (c1.ru_stime - c0.ru_stime)
    return {"value": done / dt, "unit": "walker-steps/s", "cores": max(1, int(round(cpu / dt))),
            "kind": "oracle", "sample": f"{walkers.shape[0]} walkers x {sweeps} sweeps of the same molecule "
                                        f"({dt:.1f} s wall, {cpu:.1f} s CPU)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="9atom")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the measurement kernel and a plain copy of known size (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_05222_amd import inputs, vmc

    spec = inputs.make_config(WORKLOADS[args.workload])
    mol = spec.molecule
    W = args.walkers or spec.n_walkers
    dev = torch.device("cuda:0")
    ctx = vmc.Context(mol, max_walkers=W, refresh_period=32, precision=args.precision)
    walkers = torch.tensor(inputs.initial_walkers(mol, W, spec.seed), device=dev)
    if args.pmc_probe:
        ctx.sweep(walkers, 2, spec.seed, measure=False)
        outs = ctx.measure(walkers)
        for _ in range(args.kernel_reps):
            ctx.measure_into(walkers, outs)
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "walkers": W, "staging_walkers": ctx.chunk_walkers(),
                          "copy_bytes": COPY_BYTES, "kernel_source_sha": kernel_sha()}), flush=True)
        return
    sweep = 0
    for _ in range(args.warmup):
        ctx.sweep(walkers, 1, spec.seed, sweep_offset=sweep)
        sweep += 1
    torch.cuda.synchronize()
    ctx.accumulate(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.sweep(walkers, 1, spec.seed, sweep_offset=sweep)
        sweep += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = ctx.accumulate(reset=True)
    value = W * args.steps / dt

    # dominant kernel: the measurement kernel alone, HIP events on its stream
    stream = torch.cuda.current_stream()
    n_launch = (W + ctx.chunk_walkers() - 1) // ctx.chunk_walkers()
    outs = ctx.measure(walkers)   # warm
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.kernel_reps):
        ctx.measure_into(walkers, outs)
    ev1.record(stream)
    torch.cuda.synchronize()
    k_ms = ev0.elapsed_time(ev1) / (args.kernel_reps * n_launch)
    walkers_per_launch = W / n_launch
    flops = measure_flops_per_walker(mol.n_elec, mol.basis.n_ao, mol.n_occ) * walkers_per_launch
    achieved = flops / (k_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_source_sha") == kernel_sha() and t.get("walkers_per_launch") == walkers_per_launch:
            traffic = t["hbm_bytes_per_launch"]

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{mol.name}: {mol.n_atoms} atoms, {mol.n_elec} electrons, "
                               f"{mol.basis.n_ao} cartesian AOs, {W} walkers, FP64 path",
                   "walkers": W, "electrons": mol.n_elec, "n_ao": mol.basis.n_ao, "atoms": mol.n_atoms,
                   "precision": "fp64"},
        "roofline": {"bound": "alu", "kernel": "k_measure", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic, "avg_launch_ms": k_ms, "walkers_per_launch": walkers_per_launch},
        "estimates": {"E": res["E"], "E_sigma": res["E_sigma"], "n_samples": res["n_samples"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
