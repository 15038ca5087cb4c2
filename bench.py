"""Benchmark: short-range non-bonded MD on one MI355X.

Default workload (one JSON line): the 24,000-atom Ewald dynamics system (cubic
6.2 nm box, LJ sigma 0.30 nm / epsilon 0.5 kJ/mol, charges +/-0.4 e, Ewald
real-space beta 3.12 nm^-1, r_cut 1.0, r_list 1.1, 16 amu, 300 K Maxwell
velocities), relaxed by steepest descent, then velocity-Verlet steps at dt 2 fs
with the pair list rebuilt every 10 steps.  A "step" is one MD step: position
update, list rebuild when due, staging, force kernel, force gather, velocity
update -- the whole hot path, inputs resident in HBM.

    python bench.py [--steps K] [--warmup W] [--workload dynamics|ensemble|serve|large]

value = useful pair interactions/s (pairs with r < r_cut per step x steps / s).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s + ns/day (24k atoms); ensemble p50/p99 latency vs plain"
FP32_PEAK_TFLOPS = 157.3        # MI355X published FP32 vector peak (packed FP32)
FP32_PEAK_UNPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0

# Algorithmic flops per useful pair (plain formula: add/sub/mul = 1, FMA = 2,
# each rsqrt/exp/erfc = 1), force-only pass.
FLOPS_PER_PAIR = {"ewald": 36, "rf": 30, "none": 26}


# HBM bytes per launch of the force kernel on the default workload, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes over the MD steps, scaled by
# what the same counters read for a 512 MiB device copy (FETCH_SIZE reads half
# the copied bytes: x2.0; WRITE_SIZE reads them exactly: x1.0).  Valid only for
# the sources they were taken on (keyed by the SHA-256 of the force kernel's
# source followed by the list builder's, which sets the work items and so the
# partials written) and the default cluster size / j-tile; otherwise the
# traffic is reported as null.
TIMING_STRIDE = 7

FORCE_TRAFFIC = {
    "83f88b2a0f01864a5d161cd42cfc64c9f1b5b91c73ea47d0f3d3c91213695a81":
        {"fetch_bytes": 2.7970 * 2 ** 20, "write_bytes": 8.2260 * 2 ** 20},
}


def force_kernel_traffic(cluster: int, jtile: int):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1506_00716_amd", "csrc")
    h = hashlib.sha256()
    for name in ("nb_force.hip", "nb_build.hip"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    t = FORCE_TRAFFIC.get(h.hexdigest())
    if t is None or cluster not in (0, 8) or jtile != 0:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def ns_per_day(steps_per_s: float, dt_ps: float) -> float:
    return steps_per_s * dt_ps * 1e-3 * 86400.0


def cpu_baseline(sysm, budget_s: float = 12.0):
    """Time the FP64 O(N^2) oracle on the host: whole force evaluations of the
    same workload (its generator positions), repeated until the budget is spent,
    reported as useful pair interactions/s."""
    import oracle
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    # useful pairs (r < r_cut, min image) at these positions, counted outside the timing
    useful = int(oracle.pairs(sysm.x, sysm.box, sysm.model.r_cut, nthreads=nthreads).shape[0])
    evals, elapsed = 0, 0.0
    while elapsed < budget_s:
        t0 = time.perf_counter()
        oracle.forces(sysm, nthreads=nthreads)
        elapsed += time.perf_counter() - t0
        evals += 1
    return {"value": useful * evals / elapsed, "unit": "pair interactions/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{evals} full force evaluations of the {sysm.n}-atom system at its generator "
                      f"positions ({useful} pairs within r_cut each), {elapsed:.1f} s"}


def calibration_copy(mb: int):
    """A plain device copy of a known size: its FETCH_SIZE / WRITE_SIZE counters
    calibrate the per-dispatch HBM byte counts of the profiled kernels."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def run_dynamics(args):
    import torch

    from paper_1506_00716_amd import inputs, nb

    ctx = nb.Context(0)
    if args.calib_copy_mb > 0:
        calibration_copy(args.calib_copy_mb)
    sysm = inputs.dynamics_ewald(velocities=True)
    dt = 0.002
    s = nb.System(ctx, sysm, cluster=args.cluster, jtile=args.jtile)
    x, v, f = nb.device_state(sysm)
    # pre-relaxation of the literal lattice (steepest descent on the same force path)
    fmax, iters = s.minimize(x, f, n_iter=500, f_tol=1000.0, max_disp=0.002)
    v.copy_(torch.tensor(sysm.v, dtype=torch.float64, device="cuda:0"))
    s.step = 0
    s.build_pairlist(x)
    st = s.stats()
    s.set_build_checks(False)
    # warm-up steps (untimed)
    if args.warmup > 0:
        s.md_step(x, v, f, dt, args.warmup, nstlist=10, nstenergy=0)
    torch.cuda.synchronize()
    # HIP events bracket one of every TIMING_STRIDE force launches and rebuilds
    # of the timed run (stride coprime with nstlist: every step of the list
    # period is sampled); each event record costs the stream a few microseconds
    s.set_timing(True, every=TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.md_step(x, v, f, dt, args.steps, nstlist=10, nstenergy=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = s.timings()
    s.set_timing(False)
    wall = t1 - t0
    # useful pairs (r < r_cut) at the end of the run: one more build for the count
    s.build_pairlist(x)
    st_end = s.stats()
    useful = 0.5 * (st["pairs_rcut"] + st_end["pairs_rcut"])
    steps_per_s = args.steps / wall
    value = useful * args.steps / wall
    force_us = 1000.0 * tm["force_ms"] / max(1, tm["force_launches"])
    flops = FLOPS_PER_PAIR[sysm.model.coulomb] * useful
    achieved = flops / (force_us * 1e-6) / 1e12
    # energy drift over a separate short NVE leg (energies every 10 steps, not timed)
    tr = s.md_step(x, v, f, dt, 200, nstlist=10, nstenergy=10)
    t_ps = tr[:, 0] * dt
    drift = float(np.polyfit(t_ps, tr[:, 4] / sysm.n, 1)[0]) if len(tr) > 2 else float("nan")
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "24000-atom Ewald dynamics (6.2 nm box, rc 1.0, rlist 1.1, beta 3.12, "
                               "dt 2 fs, nstlist 10, FP32 forces, FP64 update)",
                   "n_atoms": sysm.n, "cluster": st["clusters"] and s.params.cluster or 8,
                   "jtile": s.params.jtile},
        "ns_per_day": ns_per_day(steps_per_s, dt),
        "useful_pairs_per_step": useful,
        "evaluated_pairs_per_step": st["evaluated_pairs"],
        "list": {"entries": st["entries"], "cluster_pairs": st["cluster_pairs"], "items": st["items"],
                 "groups": st["groups"], "clusters": st["clusters"]},
        "list_pairs_rlist": st["atom_pairs_rlist"],
        "force_kernel_us": force_us,
        "rebuild_us": 1000.0 * tm["build_ms"] / max(1, tm["builds"]),
        "timed_launches": {"stride": TIMING_STRIDE, "force": tm["force_launches"], "rebuilds": tm["builds"]},
        "nve_drift_kj_mol_ps_atom": drift,
        "relax": {"fmax": fmax, "iterations": iters},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": force_kernel_traffic(args.cluster, args.jtile), "traffic_unit": "HBM bytes per launch",
                     "peak_unpacked": FP32_PEAK_UNPACKED_TFLOPS,
                     "frac_unpacked": achieved / FP32_PEAK_UNPACKED_TFLOPS,
                     "flops_per_pair": FLOPS_PER_PAIR[sysm.model.coulomb]},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inputs.dynamics_ewald(velocities=False), budget_s=args.cpu_budget)
    return res


def relax_inplace(ctx, nb, sysm, n_iter=300, f_tol=1000.0):
    """Steepest-descent relaxation on the GPU force path; returns relaxed x (host)."""
    import torch
    g = nb.System(ctx, sysm)
    x = torch.tensor(sysm.x, dtype=torch.float64, device="cuda:0")
    f = torch.zeros((sysm.n, 3), dtype=torch.float32, device="cuda:0")
    g.minimize(x, f, n_iter=n_iter, f_tol=f_tol, max_disp=0.002)
    g.build_pairlist(x)
    useful = g.stats()["pairs_rcut"]
    out = x.cpu().numpy()
    g.close()
    return out, useful


def autotune_table(ctx, nb, inputs, sizes, dt=0.002):
    """(cluster, jtile) per size class, tuned once on a representative member of
    each class; a system's choice is then a function of its size only."""
    import torch
    edges = [1000, 2000, 4000, 8000, 16000, 32000]
    table = []
    for lo, hi in zip(edges, edges[1:]):
        n = int(round(math.sqrt(lo * hi) / 2)) * 2
        s = inputs.ensemble_member(10_000 + lo, n)
        x, _ = relax_inplace(ctx, nb, s, n_iter=100)
        s.x = x
        g = nb.System(ctx, s)
        xx = torch.tensor(x, dtype=torch.float64, device="cuda:0")
        f = torch.zeros((s.n, 3), dtype=torch.float32, device="cuda:0")
        c, j, us = g.autotune(xx, f, clusters=(4, 8), jtiles=(8, 16, 32, 64))
        table.append({"lo": lo, "hi": hi, "cluster": c, "jtile": j, "force_us": us})
        g.close()
    return table


def pick(table, n):
    for row in table:
        if row["lo"] <= n < row["hi"]:
            return row["cluster"], row["jtile"]
    return table[-1]["cluster"], table[-1]["jtile"]


def run_ensemble(args):
    """512 independent systems, batched (one launch per kernel per step, graph
    replay) vs 512 plain per-system md_step calls on the same GPU."""
    import torch

    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    dt = 0.002
    sizes = inputs.ensemble_sizes(args.n_systems)
    t_setup = time.perf_counter()
    tune = autotune_table(ctx, nb, inputs, sizes) if args.autotune else None
    members = []
    for k, n in enumerate(sizes):
        s = inputs.ensemble_member(k, n)
        s.x, useful = relax_inplace(ctx, nb, s, n_iter=args.relax_iter)
        c, j = pick(tune, n) if tune else (args.cluster, args.jtile)
        members.append((s, useful, c, j))
    setup_s = time.perf_counter() - t_setup
    useful_total = sum(m[1] for m in members)

    def fresh_state():
        out = []
        for s, useful, c, j in members:
            g = nb.System(ctx, s, cluster=c, jtile=j)
            x, v, f = nb.device_state(s)
            out.append((g, x, v, f))
        return out

    # plain: one system at a time, each with its own launches
    plain = fresh_state()
    for g, x, v, f in plain:
        g.md_step(x, v, f, dt, args.warmup, nstlist=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, x, v, f in plain:
        g.md_step(x, v, f, dt, args.steps, nstlist=10)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    xs_plain = [x.cpu().numpy() for _, x, _, _ in plain[:4]]
    for g, *_ in plain:
        g.close()
    del plain
    # batched
    batch = fresh_state()
    ens = nb.Ensemble(ctx, len(batch))
    for g, x, v, f in batch:
        ens.add(g, x, v, f)
    ens.step(args.warmup, dt, nstlist=10, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(args.steps, dt, nstlist=10, use_graph=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(a, x.cpu().numpy()) for a, (_, x, _, _) in zip(xs_plain, batch[:4]))
    ens.close()
    v_batch = useful_total * args.steps / t_batch
    v_plain = useful_total * args.steps / t_plain
    return {
        "metric": METRIC, "value": v_batch, "unit": "pair interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * t_batch / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched ensemble of {len(sizes)} systems, N log-uniform 1000-30000, RF rc 0.9, "
                               f"rlist 1.0, dt 2 fs, nstlist 10, {args.steps} steps", "total_atoms": int(sum(sizes))},
        "plain_value": v_plain, "batched_over_plain": v_batch / v_plain,
        "plain_ms_per_step": 1000.0 * t_plain / args.steps,
        "useful_pairs_per_step": useful_total, "alone_equals_batched_bitwise": bool(same),
        "autotune": tune, "setup_s": setup_s,
    }


def run_serve(args):
    """Poisson stream of MD jobs through the continuous-batching server vs the same
    trace served one job at a time (FIFO)."""
    import torch

    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    dt = 0.002
    # capacity calibration: a batch of typical jobs, atom-steps/s
    cal = inputs.job_trace(24, rate=1.0, seed=505)
    srv = nb.Server(ctx, pool_bytes=int(args.pool_gib * (1 << 30)), max_slots=64, dt=dt)
    cal_sys = []
    for j in cal:
        s = inputs.job_system(j, seed=505)
        s.x, _ = relax_inplace(ctx, nb, s, n_iter=args.relax_iter)
        cal_sys.append(s)
    t0 = time.perf_counter()
    for s in cal_sys:
        srv.submit(s, 100)
    srv.wait_idle(600)
    cap = srv.stats()["atom_steps"] / (time.perf_counter() - t0)
    srv.close()
    mean_work = np.mean([j.n_atoms * j.n_steps for j in inputs.job_trace(args.n_jobs, rate=1.0)])
    results = {}
    for load in args.loads:
        rate = load * cap / mean_work
        jobs = inputs.job_trace(args.n_jobs, rate=rate)
        systems = []
        for j in jobs:
            s = inputs.job_system(j)
            s.x, _ = relax_inplace(ctx, nb, s, n_iter=args.relax_iter)
            systems.append(s)
        for mode, slots in (("batched", 64), ("serial", 1)):
            srv = nb.Server(ctx, pool_bytes=int(args.pool_gib * (1 << 30)), max_slots=slots, dt=dt)
            t0 = time.perf_counter()
            ids = []
            for j, s in zip(jobs, systems):
                delay = j.arrival - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                ids.append(srv.submit(s, j.n_steps))
            srv.wait_idle(3600)
            wall = time.perf_counter() - t0
            polls = [srv.poll(i) for i in ids]
            lat = np.array([q["t_done"] - q["t_submit"] for q in polls])
            errors = [{"n_atoms": int(j.n_atoms), "error": int(q["error"])}
                      for j, q in zip(jobs, polls) if q["state"] == "failed"]
            st = srv.stats()
            results.setdefault(str(load), {})[mode] = {
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "atom_steps_per_s": st["atom_steps"] / wall,
                "ns_per_day_aggregate": ns_per_day(st["atom_steps"] / wall / np.mean([j.n_atoms for j in jobs]), dt),
                "done": st["done"], "failed": st["failed"], "failed_jobs": errors, "wall_s": wall}
            srv.close()
    key = str(args.loads[0])
    b, s_ = results[key]["batched"], results[key]["serial"]
    return {
        "metric": METRIC, "value": b["p99_s"], "unit": "s (p99 job latency)", "n_gpus": 1,
        "steps": args.n_jobs, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served Poisson stream of {args.n_jobs} MD jobs, N log-uniform 2000-200000, "
                               f"steps U(100,5000), RF, load {args.loads} of batched capacity",
                   "capacity_atom_steps_per_s": cap},
        "p50_s": b["p50_s"], "serial_p50_s": s_["p50_s"], "serial_p99_s": s_["p99_s"],
        "by_load": results,
    }


def run_large(args):
    """1M-atom slab (dense central slab, LB mixing, Ewald): list build and force
    kernel timings, and the precision study V64r vs V32 against the FP64 oracle
    on a sampled subset of atoms (forces) and on a 1/8-volume system (energies)."""
    import torch

    import oracle
    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    out = {}
    sysm = inputs.slab_system()
    x = torch.tensor(sysm.x, dtype=torch.float64, device="cuda:0")
    f = torch.zeros((sysm.n, 3), dtype=torch.float32, device="cuda:0")
    rng = np.random.default_rng((3, 99))
    idx = np.sort(rng.choice(sysm.n, size=args.sample, replace=False))
    t0 = time.perf_counter()
    fr, _ = oracle.forces_subset(sysm, idx)
    t_oracle = time.perf_counter() - t0
    for name, fp32 in (("V64r", False), ("V32", True)):
        g = nb.System(ctx, sysm, fp32_reduce=fp32, force_fixed_bits=16)
        g.build_pairlist(x)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(5):
            g.build_pairlist(x)
        torch.cuda.synchronize()
        build_ms = 1000.0 * (time.perf_counter() - tb) / 5
        st = g.stats()
        g.compute_forces(x, f, energies=False)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        for _ in range(args.steps):
            g.compute_forces(x, f, energies=False)
        torch.cuda.synchronize()
        force_ms = 1000.0 * (time.perf_counter() - tf) / args.steps
        fg = f.cpu().numpy().astype(np.float64)
        err = float(np.sqrt(((fg[idx] - fr) ** 2).sum() / (fr ** 2).sum()))
        out[name] = {"force_rel_rms": err, "build_ms": build_ms, "force_call_ms": force_ms,
                     "useful_pairs": st["pairs_rcut"], "evaluated_pairs": st["evaluated_pairs"],
                     "pairs_per_s": st["pairs_rcut"] / (force_ms * 1e-3)}
        g.close()
    # energies on a 1/8-volume slab system (same densities), full oracle sum
    small = inputs.slab_system(n_atoms=125_000, box=21.5 / 2)
    t0 = time.perf_counter()
    _, er, _ = oracle.forces(small)
    t_small = time.perf_counter() - t0
    xs = torch.tensor(small.x, dtype=torch.float64, device="cuda:0")
    fs = torch.zeros((small.n, 3), dtype=torch.float32, device="cuda:0")
    for name, fp32 in (("V64r", False), ("V32", True)):
        g = nb.System(ctx, small, fp32_reduce=fp32, force_fixed_bits=16)
        g.build_pairlist(xs)
        e, _ = g.compute_forces(xs, fs)
        out[name]["energy_rel_err_125k"] = [float(abs(e[k] - er[k]) / abs(er[k])) for k in range(2)]
        g.close()
    v = out["V64r"]["pairs_per_s"]
    return {
        "metric": METRIC, "value": v, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": out["V64r"]["force_call_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1,000,000-atom slab (21.5 nm box, 1.5x density slab, LB mixing, Ewald beta 3.12, "
                               "rc 1.0, rlist 1.1), one force evaluation per step"},
        "precision": out, "oracle_sample_atoms": int(args.sample), "oracle_sample_s": t_oracle,
        "oracle_125k_s": t_small,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="dynamics", choices=["dynamics", "ensemble", "serve", "large"])
    ap.add_argument("--sample", type=int, default=50000)
    ap.add_argument("--calib-copy-mb", type=int, default=0)
    ap.add_argument("--n-systems", type=int, default=512)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--relax-iter", type=int, default=500)
    ap.add_argument("--n-jobs", type=int, default=400)
    ap.add_argument("--pool-gib", type=float, default=64.0)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.7])
    ap.add_argument("--cluster", type=int, default=0)
    ap.add_argument("--jtile", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ensemble":
        res = run_ensemble(args)
    elif args.workload == "serve":
        res = run_serve(args)
    elif args.workload == "large":
        res = run_large(args)
    else:
        res = run_dynamics(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
