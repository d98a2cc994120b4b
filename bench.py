"""Throughput of the VMC force hot path on one MI355X.

A step is one sweep of N single-electron Metropolis moves for every walker
followed by one measurement (local energy, SWCT Hellmann-Feynman + Pulay
force terms, dE_L/dC and dln|Psi|/dC) accumulated into the estimators: one
walker-step per walker.  value = walkers x steps / seconds of the timed
vmc_sweep call (positions, MO matrices and accumulators resident in HBM).

Default workload: the 21-atom molecule (9 C, 4 O, 8 H; 94 electrons, 235
cartesian AOs, 47 occupied orbitals per spin), 65536 walkers, mixed
precision.  The same workload also runs through the FP64 path, and the line
reports both rates and their ratio, plus the mixed-vs-FP64 error table on
replayed configurations (the mixed run's final walkers measured in both
precisions): walker-averaged |dE|, max |dF| over the bare force components,
and the relative max error of dE/dC on a subset.

Also in the line:
  roofline     the dominant kernel (k_adjoint_mfma: back-projection and outer
               products on the matrix cores), timed with HIP events that the
               library records on its launch stream over the timed region;
               algorithmic flops per walker 10 N M n (kappa = K~ C^T and
               a = Abar C^T, 2 N M n each; O = psi^T K~, 2 N M n; G = psi^T
               Abar + q^T K~, 4 N M n) against the dense MFMA peak of the
               arithmetic type; traffic from the committed rocprofv3 counter
               summary when it matches this kernel source and launch size;
  cpu_baseline the FP64 oracle on a bounded sample of the same molecule on
               the host cores (unless --no-cpu-baseline).
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
MFMA_PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}   # dense FP32 / FP64 matrix-core peaks
KERNEL = "k_adjoint_mfma"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2511_05222_amd", "csrc", f)
               for f in ("vmc_adjoint.hip", "vmc_mfma.hpp", "vmc_device.hpp", "vmc_pipeline.hpp")]
COPY_BYTES = 1 << 30   # plain device copy used to calibrate the HBM byte counters
WORKLOADS = {"9atom": 1, "21atom": 2}


def adjoint_flops_per_walker(N, M, n):
    return 10.0 * N * M * n


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_file(workload, precision):
    return os.path.join(ROOT, "profiles", f"{KERNEL}_{workload}_{precision}_traffic.json")


def cpu_baseline(spec, budget_s=12.0):
    """Time the oracle (sm sweep + full measurement) on a bounded sample."""
    import resource
    from oracle import vmc as ovmc
    from paper_2511_05222_amd import inputs
    mol = spec.molecule
    walkers = inputs.initial_walkers(mol, 8, spec.seed)
    done = sweeps = 0
    t0 = time.perf_counter()
    c0 = resource.getrusage(resource.RUSAGE_SELF)
    while time.perf_counter() - t0 < budget_s:
        res = ovmc.run(mol, walkers, 1, spec.seed, sweep_offset=sweeps)
        walkers = res["positions"]
        sweeps += 1
        done += walkers.shape[0]
    dt = time.perf_counter() - t0
    c1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (c1.ru_utime - c0.ru_utime) + (c1.ru_stime - c0.ru_stime)
    return {"value": done / dt, "unit": "walker-steps/s", "cores": max(1, int(round(cpu / dt))),
            "kind": "oracle", "sample": f"{walkers.shape[0]} walkers x {sweeps} sweeps (sweep + measurement) of the "
                                        f"same molecule, {dt:.1f} s wall, {cpu:.1f} s CPU"}


def run_steps(ctx, walkers, seed, warmup, steps):
    """One vmc_sweep call of `warmup` sweeps, then the timed call of `steps`."""
    import torch
    ctx.sweep(walkers, warmup, seed, sweep_offset=0)
    torch.cuda.synchronize()
    ctx.accumulate(reset=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sweep(walkers, steps, seed, sweep_offset=warmup)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = {k: ctx.profile_read(k) for k in ("adjoint", "dense", "mo_rows", "sweep")}
    ctx.profile(False)
    return dt, ctx.accumulate(reset=True), prof


def error_table(mol, W_sub, walkers, ctx32, ctx64):
    """Mixed vs FP64 on the same configurations."""
    import torch
    outs = ("EL", "lnpsi", "lnjac", "dEL_dR", "dlnpsi_dR", "dlnjac_dR")
    o = {}
    for name, ctx in (("mixed", ctx32), ("fp64", ctx64)):
        r = ctx.measure(walkers, outputs=outs)
        E, H = r["EL"], r["dEL_dR"]
        P = r["dlnpsi_dR"] + 0.5 * r["dlnjac_dR"]
        s = E.mean()
        e = E - s
        F = -H.mean(0) - 2.0 * ((e[:, None, None] * P).mean(0) - e.mean() * P.mean(0))
        o[name] = (s + e.mean(), F)
        del r
    sub = walkers[:W_sub].contiguous()
    dC = {}
    for name, ctx in (("mixed", ctx32), ("fp64", ctx64)):
        r = ctx.measure(sub, outputs=("EL", "O"))
        e = r["EL"] - r["EL"].mean()
        dC[name] = 2.0 * (e[:, None, None] * r["O"]).mean(0)
        del r
    torch.cuda.synchronize()
    dE = abs((o["mixed"][0] - o["fp64"][0]).item())
    dF = (o["mixed"][1] - o["fp64"][1]).abs().max().item()
    rC = ((dC["mixed"] - dC["fp64"]).abs().max() / dC["fp64"].abs().max()).item()
    return {"walkers": int(walkers.shape[0]), "dE_Ha": dE, "dF_max_Ha_per_bohr": dF,
            "dEdC_rel_max": rC, "dEdC_walkers": W_sub,
            "bounds": {"dE_Ha": 1e-5, "dF_max_Ha_per_bohr": 1e-4}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed sweeps (with measurement) before the timed call: the chains leave their "
                         "starting positions, so the timed sweeps see equilibrated walkers")
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="21atom")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference run and the error table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the measurement and a plain copy of known size (for counter runs)")
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
    w0 = torch.tensor(inputs.initial_walkers(mol, W, spec.seed), device=dev)
    ctx = vmc.Context(mol, max_walkers=W, refresh_period=32, precision=args.precision)
    if args.pmc_probe:
        # the measurement as the timed run launches it: one sweep with
        # measurement after two without
        walkers = w0.clone()
        ctx.sweep(walkers, 2, spec.seed, measure=False)
        ctx.sweep(walkers, 1, spec.seed, sweep_offset=2)
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "walkers": W, "staging_walkers": ctx.chunk_walkers(),
                          "copy_bytes": COPY_BYTES, "kernel_source_sha": kernel_sha()}), flush=True)
        return

    walkers = w0.clone()
    dt, res, prof = run_steps(ctx, walkers, spec.seed, args.warmup, args.steps)
    value = W * args.steps / dt
    print(f"# {args.precision}: {value:.4g} walker-steps/s, {dt / args.steps * 1e3:.2f} ms/step", file=sys.stderr,
          flush=True)

    # the dominant kernel
    k_ms, k_launches, k_walkers = prof["adjoint"]
    avg_ms = k_ms / max(k_launches, 1)
    wpl = k_walkers / max(k_launches, 1)
    flops = adjoint_flops_per_walker(mol.n_elec, mol.basis.n_ao, mol.n_occ) * wpl
    achieved = flops / (avg_ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[args.precision]
    traffic = None
    tf = traffic_file(args.workload, args.precision)
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("kernel_source_sha") == kernel_sha() and abs(t.get("walkers_per_launch", -1) - wpl) < 0.5:
            traffic = t["hbm_bytes_per_launch"]
    step_ms = dt / args.steps * 1e3
    shares = {k: v[0] / args.steps / step_ms for k, v in prof.items()}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{mol.name}: {mol.n_atoms} atoms, {mol.n_elec} electrons, {mol.basis.n_ao} "
                               f"cartesian AOs, {mol.n_occ} occupied orbitals per spin, {W} walkers",
                   "walkers": W, "electrons": mol.n_elec, "n_ao": mol.basis.n_ao, "atoms": mol.n_atoms,
                   "precision": args.precision, "refresh_period": 32},
        "roofline": {"bound": "mfma", "kernel": KERNEL, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic, "avg_launch_ms": avg_ms,
                     "walkers_per_launch": wpl, "flops_per_walker": adjoint_flops_per_walker(
                         mol.n_elec, mol.basis.n_ao, mol.n_occ)},
        "kernel_share_of_step": shares,
        "estimates": {"E": res["E"], "E_sigma": res["E_sigma"], "n_samples": res["n_samples"]},
    }
    if args.precision == "mixed" and not args.no_fp64:
        ctx64 = vmc.Context(mol, max_walkers=W, refresh_period=32, precision="fp64")
        w64 = w0.clone()
        dt64, _, _ = run_steps(ctx64, w64, spec.seed, args.warmup, args.steps)
        v64 = W * args.steps / dt64
        print(f"# fp64: {v64:.4g} walker-steps/s, {dt64 / args.steps * 1e3:.2f} ms/step", file=sys.stderr,
              flush=True)
        line["fp64_value"] = v64
        line["fp64_ms_per_step"] = dt64 / args.steps * 1e3
        line["mixed_over_fp64"] = value / v64
        del w64
        line["errors"] = error_table(mol, min(W, 1024), walkers, ctx, ctx64)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
