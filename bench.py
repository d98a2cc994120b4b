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
and the relative max error of dE/dC on a subset.  The 9-atom molecule with
16384 walkers through the FP64 path is timed as well (`fp64_9atom`).

Also in the line:
  roofline       the kernel with the largest share of the step, timed with
                 HIP events that the library records on its launch stream
                 over the timed region, against the roof of its algorithmic
                 work (work_model: matrix-core flops, vector-ALU flops and
                 HBM bytes per unit; the bound is the resource whose work
                 takes longest at its peak); traffic from the committed
                 rocprofv3 counter summary when it matches the kernel source
                 and launch size;
  kernels        the same for every timed kernel;
  step_roofline  the whole walker-step: the summed work of the step against
                 the same peaks, T_roof / T_measured;
  ecp_9atom      the pseudopotential workload (the 9-atom molecule made
                 valence-only with a seeded semilocal pseudopotential, 16384
                 walkers, both precisions) with its kernels' rooflines;
  next_rows      on the 21-atom molecule with 16384 walkers: the one- and
                 three/four-body Jastrow (mixed, FP64, and mixed with the
                 Jastrow-parameter gradient sums), the exponential two-body
                 Jastrow (mixed), reweighted accumulation of given walkers,
                 and the jackknife error pipeline through the Z-vector solve;
  family_64      the 64-geometry mixed-size family (9-21 atoms, 8192 walkers
                 each, mixed precision), one context per geometry, their
                 sweeps on four streams (and on one, for comparison);
  cpu_baseline   the FP64 oracle on a bounded sample of the same molecule on
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
# MI355X peaks.  Matrix cores: dense FP32 157.3, FP64 78.6 TFLOP/s.  Vector
# ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (one FMA) x 2.4 GHz = 78.6
# TFLOP/s for FP32 and FP64 alike (the 157.3 TFLOP/s FP32 vector figure needs
# packed FP32 instructions, which this library does not emit).  HBM 8 TB/s.
PEAK_MFMA = {"mixed": 157.3, "fp64": 78.6}
PEAK_ALU = 78.6
PEAK_HBM = 8000.0
KERNELS = {"sweep": "k_sweep_r", "proposals": "k_mo_rows_mfma_proposals", "mo_rows": "k_mo_rows_mfma",
           "dense": "k_dense", "adjoint": "k_adjoint_mfma"}
KERNEL_SRCS = {
    "sweep": ("vmc_sweep.hip", "vmc_regs.hpp", "vmc_device.hpp", "vmc_pipeline.hpp"),
    "proposals": ("vmc_sweep.hip", "vmc_mo.hip", "vmc_mfma.hpp", "vmc_device.hpp", "vmc_pipeline.hpp"),
    "mo_rows": ("vmc_mo.hip", "vmc_mfma.hpp", "vmc_device.hpp", "vmc_pipeline.hpp"),
    "dense": ("vmc_dense.hip", "vmc_mfma.hpp", "vmc_regs.hpp", "vmc_device.hpp", "vmc_pipeline.hpp"),
    "adjoint": ("vmc_adjoint.hip", "vmc_mfma.hpp", "vmc_device.hpp", "vmc_pipeline.hpp"),
}
COPY_BYTES = 1 << 30   # plain device copy used to calibrate the HBM byte counters
WORKLOADS = {"9atom": 1, "21atom": 2}


def work_model(mol, precision, p_acc):
    """Algorithmic work per unit of each kernel: {"mfma": flops, "alu": flops,
    "hbm": bytes}; the unit is a walker-sweep for the sweep, a walker for the
    measurement kernels.  Counts are what the method computes (no padding,
    no recomputation beyond the design's recompute-not-store rule), with
    N electrons, n orbitals per spin, M AOs, P primitives, S shells, A
    atoms, p the measured acceptance:
      proposals  per walker-sweep, the N proposals' AO values (per
               primitive alpha*rho and c*e, per shell rho, per AO monomial
               x radial: 3P + 6S + 3M each) and MO rows psi^T C (2NMn on the
               matrix cores); bytes: positions read, proposals written and
               read, the N n orbital values written.
      sweep    per move: the ratio (2n), the Jastrow difference (N - 1
               pairs, old and new distance, 24 flops), on accept the
               Sherman-Morrison update (2n^2); per block every 32 moves an
               inverse (2n^3, FP64).  Bytes: positions and proposals in,
               positions out, the proposals' orbital rows in, both blocks'
               inverses in and out (in the arithmetic type), MO rows
               written on accept, read back at each rebuild.
      mo_rows  AO value, gradient, Laplacian (10 flops per primitive, 15 per
               AO) and the five products psi C (10 NMn on the matrix cores);
               bytes: the 5Nn orbital values written.
      dense    per block a Newton step of the inverse (4n^3), T = X K and
               Abar = T^T K^T (4n^3) on the matrix cores; Jastrow pairs
               (40 flops each), determinant gradients (8Nn).
      adjoint  AO derivatives through third order (60 flops per AO, 12 per
               primitive, per electron); kappa = K~ C^T, a = Abar C^T,
               O = psi^T K~, G = psi^T Abar + q^T K~ (10 NMn).
    """
    b = mol.basis
    N, n, M, P, S, A = mol.n_elec, mol.n_occ, b.n_ao, b.n_prim, b.n_shells, mol.n_atoms
    ts = 4 if precision == "mixed" else 8
    ao_val = 3 * P + 6 * S + 3 * M
    sweep_alu = N * (2 * n + 24 * (N - 1) + p_acc * 2 * n * n) + (N / 32.0) * 2 * n ** 3
    sweep_hbm = 3 * 24 * N + N * n * ts + 2 * 2 * (n * n * ts) + p_acc * N * n * ts + (N / 32.0) * n * n * ts
    return {
        "proposals": {"mfma": 2.0 * N * M * n, "alu": float(N * ao_val), "hbm": float(3 * 24 * N + N * n * ts)},
        "sweep": {"mfma": 0.0, "alu": float(sweep_alu), "hbm": float(sweep_hbm)},
        "mo_rows": {"mfma": 10.0 * N * M * n, "alu": float(N * (10 * P + 6 * S + 15 * M)),
                    "hbm": float(24 * N + 5 * N * n * ts)},
        "dense": {"mfma": 16.0 * n ** 3, "alu": float(40 * N * (N - 1) / 2 + 8 * N * n),
                  "hbm": float(5 * N * n * ts + 2 * N * n * ts)},
        "adjoint": {"mfma": 10.0 * N * M * n, "alu": float(N * (60 * M + 12 * P)),
                    "hbm": float(24 * N + 2 * N * n * ts + 2 * M * n * ts)},
    }


def roof(work, precision, t_s):
    """Roofline of `work` done in t_s seconds: bound, achieved, peak, frac."""
    times = {"mfma": work["mfma"] / (PEAK_MFMA[precision] * 1e12), "alu": work["alu"] / (PEAK_ALU * 1e12),
             "hbm": work["hbm"] / (PEAK_HBM * 1e9)}
    bound = max(times, key=times.get)
    if bound == "hbm":
        ach, peak, unit = work["hbm"] / t_s / 1e9, PEAK_HBM, "GB/s"
    else:
        ach, peak = work[bound] / t_s / 1e12, (PEAK_MFMA[precision] if bound == "mfma" else PEAK_ALU)
        unit = "TFLOP/s"
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "t_roof_ns": times[bound] * 1e9, "t_measured_ns": t_s * 1e9}


def kernel_sha(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SRCS[kernel]:
        with open(os.path.join(ROOT, "paper_2511_05222_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(kernel, workload, precision):
    return os.path.join(ROOT, "profiles", f"{KERNELS[kernel]}_{workload}_{precision}_traffic.json")


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
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done / dt, "unit": "walker-steps/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "cpu_model": model, "threads_busy": round(cpu / dt, 2),
            "sample": f"{walkers.shape[0]} walkers x {sweeps} sweeps (sweep + measurement) of the same molecule, "
                      f"{dt:.1f} s wall, {cpu:.1f} s CPU; numpy with its BLAS threads over the host cores"}


def run_steps(ctx, walkers, seed, warmup, steps, kernels=("adjoint", "dense", "mo_rows", "sweep", "proposals")):
    """One vmc_sweep call of `warmup` sweeps, then the timed call of `steps`
    (the kernels' HIP-event times over it)."""
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
    prof = {k: ctx.profile_read(k) for k in kernels}
    ctx.profile(False)
    res = ctx.accumulate(reset=True)
    # acceptance of one more sweep on a copy (untimed, not accumulated)
    wc = walkers.clone()
    acc = torch.zeros((1, wc.shape[1], wc.shape[0]), dtype=torch.uint8, device=wc.device)
    ctx.sweep(wc, 1, seed, sweep_offset=warmup + steps, measure=False, accept=acc)
    p_acc = acc.float().mean().item()
    del wc, acc
    return dt, res, prof, p_acc


ECP_KERNELS = {"ecp_points": "k_ecp_count/scan/place + k_mo_rows_mfma (points)", "ecp_energy": "k_ecp_energy",
               "ecp_adjoint": "k_ecp_adjoint"}


def ecp_work(mol, precision, pairs):
    """Algorithmic work per walker of the pseudopotential kernels, with
    `pairs` (electron, nucleus) pairs inside the cutoffs per walker, Q = 12
    pairs quadrature points:
      ecp_points   the AOs and their gradients at the points (10 flops per
                   primitive, 6 per shell, 15 per AO) and psi C for the five
                   components (10 Q M n on the matrix cores); bytes: the
                   points and their MO rows written;
      ecp_energy   per point the ratio (2n), the Jastrow difference (N pairs,
                   about 30 flops each) and Z (2n); per spin block
                   K~ Z K~ (4 n^3); bytes: the points' values, K~ and Abar;
      ecp_adjoint  per point and AO the value and gradient (~30 flops),
                   kappa = C y and G += psi y (4n), the chain (6n + 60 N);
                   bytes: the points' gradients, K~, G read and written."""
    b = mol.basis
    N, n, M, P, S = mol.n_elec, mol.n_occ, b.n_ao, b.n_prim, b.n_shells
    ts = 4 if precision == "mixed" else 8
    Q = 12.0 * pairs
    return {
        "ecp_points": {"mfma": 10.0 * Q * M * n, "alu": Q * (10 * P + 6 * S + 15 * M),
                       "hbm": Q * (24 + 5 * n * ts)},
        "ecp_energy": {"mfma": 0.0, "alu": Q * (4 * n + 30 * N) + 2 * 4.0 * n ** 3,
                       "hbm": Q * n * ts + 3.0 * N * n * ts},
        "ecp_adjoint": {"mfma": 0.0, "alu": Q * (M * (30 + 4 * n) + 6 * n + 60 * N),
                        "hbm": Q * (3 * n * ts + 24) + N * n * ts + 2.0 * M * n * 8},
    }


def ecp_entry(args, dev):
    """The pseudopotential workload: the 9-atom molecule made valence-only
    with the seeded semilocal pseudopotential (20 electrons), 16384 walkers,
    both precisions; walker-steps/s and the pseudopotential kernels'
    rooflines."""
    import torch
    from paper_2511_05222_amd import inputs, vmc
    spec9 = inputs.make_config(1)
    m = inputs.with_ecp(spec9.molecule, 5)
    W = spec9.n_walkers
    out = {"workload": f"{m.name}: {m.n_atoms} atoms, {m.n_elec} valence electrons, {m.basis.n_ao} cartesian AOs, "
                       f"s and p projectors on C and O, 12-point quadrature, {W} walkers"}
    for prec in ("mixed", "fp64"):
        ctx = vmc.Context(m, max_walkers=W, refresh_period=32, precision=prec)
        w = torch.tensor(inputs.initial_walkers(m, W, spec9.seed), device=dev)
        ctx.sweep(w, args.warmup, spec9.seed, sweep_offset=0)
        torch.cuda.synchronize()
        ctx.accumulate(reset=True)
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.sweep(w, args.steps, spec9.seed, sweep_offset=args.warmup)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = {k: ctx.profile_read(k) for k in ECP_KERNELS}
        ctx.profile(False)
        ctx.accumulate(reset=True)
        # pairs inside the cutoffs per walker, from the final positions
        r = w.cpu().numpy()
        e = m.ecp
        nl = [a for a in range(m.n_atoms) if e.rcut[a] > 0]
        d = np.linalg.norm(r[:, :, None, :] - np.asarray(m.xyz)[None, None, nl, :], axis=-1)
        pairs = float((d < np.asarray(e.rcut)[nl][None, None, :]).sum(axis=(1, 2)).mean())
        work = ecp_work(m, prec, pairs)
        kern = {}
        step_ms = dt / args.steps * 1e3
        for k, (ms, nl_, nw) in prof.items():
            if nl_ < 1:
                continue
            rf = roof(work[k], prec, ms * 1e-3 / max(nw, 1))
            rf.update({"kernel": ECP_KERNELS[k], "share_of_step": ms / args.steps / step_ms,
                       "avg_launch_ms": ms / nl_, "units_per_launch": nw / nl_, "work_per_unit": work[k]})
            kern[k] = rf
        out[prec] = {"value": W * args.steps / dt, "ms_per_step": step_ms, "pairs_per_walker": pairs,
                     "kernels": kern}
        print(f"# ecp 9-atom {prec}: {W * args.steps / dt:.4g} walker-steps/s, {step_ms:.2f} ms/step",
              file=sys.stderr, flush=True)
        del ctx, w
    out["mixed_over_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    return out


def next_rows_entry(args, dev, W=16384, warmup=5, steps=3):
    """The rows beyond the headline path, each on the 21-atom molecule:
    the one- and three/four-body Jastrow (mixed and FP64, and mixed with the
    Jastrow-parameter gradient sums), the exponential two-body form (mixed),
    reweighted accumulation of given walkers with weights, and the jackknife
    error pipeline through the Z-vector solve (4 replicas)."""
    import dataclasses
    import torch
    from paper_2511_05222_amd import inputs, vmc
    spec = inputs.make_config(2)
    mol = spec.molecule
    out = {}

    def rate(m, prec, **kw):
        ctx = vmc.Context(m, max_walkers=W, refresh_period=32, precision=prec, **kw)
        w = torch.tensor(inputs.initial_walkers(m, W, spec.seed), device=dev)
        jas = m.jastrow.jas_basis is not None
        dt, _, prof, _ = run_steps(ctx, w, spec.seed, warmup, steps, kernels=("jas_gemm",) if jas else ())
        del ctx, w
        r = {"value": W * steps / dt, "ms_per_step": dt / steps * 1e3}
        ms, nl, nw = prof.get("jas_gemm", (0.0, 0, 0))
        if nl > 0:
            # k_jas_gemm: per walker and launch 2 N MJ^2 matrix-core flops
            # (the xi1 column is a dot product); A rows of MJ entries (V,
            # Q: 1 and 4 components, the sweep's differences 2) and MJ + 1
            # output columns in the arithmetic type
            MJ, ts = m.jastrow.jas_basis.n_ao, 4 if prec == "mixed" else 8
            work = {"mfma": 2.0 * m.n_elec * MJ * MJ, "alu": 0.0,
                    "hbm": float(m.n_elec * ts * (2 * MJ + MJ + 1))}
            rf = roof(work, prec, ms * 1e-3 / max(nw, 1))
            rf.update({"kernel": "k_jas_gemm", "share_of_step": ms / steps / r["ms_per_step"],
                       "avg_launch_ms": ms / nl, "launches": nl, "units_per_launch": nw / nl,
                       "work_per_unit": work})
            r["kernels"] = {"jas_gemm": rf}
        return r

    mj = inputs.with_body_jastrow(mol, 7)
    out["body_jastrow"] = {
        "workload": f"{mol.name} + one-/three-body Jastrow on {mj.jastrow.jas_basis.n_ao} Jastrow basis functions, "
                    f"{W} walkers",
        "mixed": rate(mj, "mixed"), "fp64": rate(mj, "fp64"),
        "mixed_with_xi_gradient": rate(mj, "mixed", jastrow_gradient=True)}
    out["body_jastrow"]["mixed_over_fp64"] = out["body_jastrow"]["mixed"]["value"] / out["body_jastrow"]["fp64"][
        "value"]
    me = dataclasses.replace(mol, jastrow=dataclasses.replace(mol.jastrow, ee_form=1))
    out["exp_jastrow"] = {"workload": f"{mol.name}, exponential two-body Jastrow, {W} walkers",
                          "mixed": rate(me, "mixed")}
    # reweighted accumulation: measurement + weighted estimator sums of W
    # given walkers (the weights from the caller)
    ctx = vmc.Context(mol, max_walkers=W, refresh_period=32, precision="mixed")
    w = torch.tensor(inputs.initial_walkers(mol, W, spec.seed), device=dev)
    ctx.sweep(w, warmup, spec.seed, measure=False)
    wt = torch.exp(torch.randn(W, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev)
                               .manual_seed(5)) * 0.5)
    ctx.accumulate_walkers(w, wt)
    torch.cuda.synchronize()
    ctx.accumulate(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.accumulate_walkers(w, wt)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.accumulate(reset=True)
    out["reweighted"] = {"workload": f"{mol.name}, {W} given walkers with weights, mixed",
                         "walkers_per_s": W * steps / dt, "ms_per_call": dt / steps * 1e3}
    del ctx, w, wt
    # jackknife error pipeline: replicas of dE/dC, their right-hand sides,
    # one batched Jacobi-CG solve at d = 188 n, jackknife statistics
    ctx = vmc.Context(mol, max_walkers=W, precision="mixed", block_sweeps=1, jackknife_blocks=4)
    w = torch.tensor(inputs.initial_walkers(mol, W, spec.seed), device=dev)
    ctx.sweep(w, 4, spec.seed)
    n = mol.n_occ
    Cv = torch.tensor(np.ascontiguousarray(mol.C_full[:, n:]), device=dev)
    H = torch.tensor(inputs.seeded_spd(188 * n, 13), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    jk = ctx.jackknife()
    b = vmc.zvector_rhs(Cv, jk["dE_dC"])
    z, its = vmc.zvector_solve(H, b.reshape(b.shape[0], -1), rtol=1e-12, maxit=2000, jacobi=True)
    vmc.jackknife_stats(z)
    vmc.jackknife_stats(jk["F_bare"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["jackknife"] = {"workload": f"{mol.name}, {W} walkers x 4 sweeps in 4 blocks; Z-vector d = {188 * n}",
                        "replicas": int(b.shape[0]), "ms": dt * 1e3, "cg_iterations": its}
    del ctx, w, H
    for k, v in out.items():
        print(f"# next row {k}: {json.dumps(v)}", file=sys.stderr, flush=True)
    return out


def family_entry(args, dev, n_streams=4):
    """The mixed-size family: 64 seeded geometries of 9-21 atoms, 8192
    walkers each, mixed precision, one context per geometry.  Every context
    runs its sweeps (with measurement) on one of n_streams streams in turn,
    so that the small members' launches overlap; the same with one stream
    for comparison.  value = 64 x 8192 x steps / seconds."""
    import torch
    from paper_2511_05222_amd import inputs, vmc
    G = inputs.FAMILY_SIZE
    specs = [inputs.family_member(g) for g in range(G)]
    ctxs, ws = [], []
    for sp in specs:
        ctxs.append(vmc.Context(sp.molecule, max_walkers=sp.n_walkers, refresh_period=32, precision="mixed",
                                staging_walkers=4096))
        ws.append(torch.tensor(inputs.initial_walkers(sp.molecule, sp.n_walkers, sp.seed), device=dev))
    walkers = sum(sp.n_walkers for sp in specs)
    out = {"workload": f"{G} seeded geometries of {min(inputs.family_sizes())}-{max(inputs.family_sizes())} atoms, "
                       f"8192 walkers each ({walkers} in all), mixed precision, one context per geometry"}
    off = 0
    for ns in (n_streams, 1):
        streams = [torch.cuda.Stream() for _ in range(ns)]

        def run(nsteps, offset):
            for g, (c, w) in enumerate(zip(ctxs, ws)):
                with torch.cuda.stream(streams[g % ns]):
                    c.sweep(w, nsteps, specs[g].seed + g, sweep_offset=offset)

        run(2, off)
        torch.cuda.synchronize()
        for c in ctxs:
            c.accumulate(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(args.steps, off + 2)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        off += 2 + args.steps
        for c in ctxs:
            c.accumulate(reset=True)
        out[f"streams_{ns}"] = {"value": walkers * args.steps / dt, "ms_per_step": dt / args.steps * 1e3}
        print(f"# family, {ns} streams: {walkers * args.steps / dt:.4g} walker-steps/s, "
              f"{dt / args.steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    out["value"] = out[f"streams_{n_streams}"]["value"]
    out["unit"] = "walker-steps/s"
    del ctxs, ws
    return out


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
    ap.add_argument("--no-ecp", action="store_true", help="skip the pseudopotential workload")
    ap.add_argument("--no-family", action="store_true", help="skip the 64-geometry mixed-size family")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the Jastrow, reweighting and jackknife entries")
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
                          "copy_bytes": COPY_BYTES,
                          "kernel_source_sha": {k: kernel_sha(k) for k in KERNEL_SRCS}}), flush=True)
        return

    walkers = w0.clone()
    dt, res, prof, p_acc = run_steps(ctx, walkers, spec.seed, args.warmup, args.steps)
    value = W * args.steps / dt
    step_ms = dt / args.steps * 1e3
    print(f"# {args.precision}: {value:.4g} walker-steps/s, {step_ms:.2f} ms/step", file=sys.stderr, flush=True)

    work = work_model(mol, args.precision, p_acc)
    kern = {}
    for k, (ms, nl, nw) in prof.items():
        if nl < 1:
            continue
        # per unit: walker-sweeps for the sweep (one launch per sweep), walkers otherwise
        t_unit = ms * 1e-3 / max(nw, 1)
        r = roof(work[k], args.precision, t_unit)
        r.update({"kernel": KERNELS[k], "share_of_step": ms / args.steps / step_ms, "avg_launch_ms": ms / nl,
                  "units_per_launch": nw / nl, "work_per_unit": work[k]})
        kern[k] = r
    dom = max(kern, key=lambda k: kern[k]["share_of_step"])
    d = kern[dom]
    traffic = None
    tf = traffic_file(dom, args.workload, args.precision)
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("kernel_source_sha") == kernel_sha(dom) and abs(t.get("walkers_per_launch", -1) -
                                                                 d["units_per_launch"]) < 0.5:
            traffic = t["hbm_bytes_per_launch"]
    # the whole walker-step: work of all kernels (finalize and the estimator
    # reductions are small beside them and are timed only as part of the step)
    tot = {r: sum(work[k][r] for k in work) for r in ("mfma", "alu", "hbm")}
    step_roof = roof(tot, args.precision, step_ms * 1e-3 / W)

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
        "roofline": {"bound": d["bound"], "kernel": d["kernel"], "achieved": d["achieved"], "peak": d["peak"],
                     "unit": d["unit"], "frac": d["frac"], "traffic": traffic, "avg_launch_ms": d["avg_launch_ms"],
                     "units_per_launch": d["units_per_launch"], "work_per_unit": d["work_per_unit"]},
        "kernels": kern,
        "step_roofline": step_roof,
        "acceptance": p_acc,
        "estimates": {"E": res["E"], "E_sigma": res["E_sigma"], "n_samples": res["n_samples"]},
    }
    if args.precision == "mixed" and not args.no_fp64:
        ctx64 = vmc.Context(mol, max_walkers=W, refresh_period=32, precision="fp64")
        w64 = w0.clone()
        dt64, _, _, _ = run_steps(ctx64, w64, spec.seed, args.warmup, args.steps)
        v64 = W * args.steps / dt64
        print(f"# fp64: {v64:.4g} walker-steps/s, {dt64 / args.steps * 1e3:.2f} ms/step", file=sys.stderr,
              flush=True)
        line["fp64_value"] = v64
        line["fp64_ms_per_step"] = dt64 / args.steps * 1e3
        line["mixed_over_fp64"] = value / v64
        del w64
        line["errors"] = error_table(mol, min(W, 1024), walkers, ctx, ctx64)
        del ctx64
    if args.workload == "21atom" and not args.no_fp64:
        # the 9-atom molecule, 16384 walkers, FP64 path
        spec9 = inputs.make_config(1)
        m9 = spec9.molecule
        c9 = vmc.Context(m9, max_walkers=spec9.n_walkers, refresh_period=32, precision="fp64")
        w9 = torch.tensor(inputs.initial_walkers(m9, spec9.n_walkers, spec9.seed), device=dev)
        dt9, _, _, _ = run_steps(c9, w9, spec9.seed, args.warmup, args.steps)
        v9 = spec9.n_walkers * args.steps / dt9
        print(f"# 9-atom fp64: {v9:.4g} walker-steps/s, {dt9 / args.steps * 1e3:.2f} ms/step", file=sys.stderr,
              flush=True)
        line["fp64_9atom"] = {"workload": f"{m9.name}: {m9.n_atoms} atoms, {m9.n_elec} electrons, "
                                          f"{m9.basis.n_ao} cartesian AOs, {spec9.n_walkers} walkers, FP64",
                              "value": v9, "ms_per_step": dt9 / args.steps * 1e3}
        del c9, w9
    if args.workload == "21atom" and not args.no_ecp:
        line["ecp_9atom"] = ecp_entry(args, dev)
    if args.workload == "21atom" and not args.no_next:
        line["next_rows"] = next_rows_entry(args, dev)
    if args.workload == "21atom" and not args.no_family:
        del ctx
        line["family_64"] = family_entry(args, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
