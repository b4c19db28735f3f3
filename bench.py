#!/usr/bin/env python3
"""Time-to-solve benchmark of the VBARMS hot path on one MI355X.

Default workload: 74^3 mesh nodes (405,224) on the 14-neighbour random stencil, a block of
1 to 7 unknowns per node drawn uniformly (n = 1,619,907, nnz = 96.6M), upwind convection
values with cell Peclet numbers LogUniform(0.1, 100); tau = 1 (exact node blocks), 4
levels whose independent sets are groups of supernodes of up to 32 rows, drop tolerance
1e-4, FGMRES(60) to a true relative residual of 1e-8, b = A 1.
`--workload grid40` runs the 40^3 five-unknown workload instead (n = 320,000, 10% block
perturbation, tau = 0.8, 3 levels with groups of up to 16 rows, FGMRES(50)); `--batch`
runs 256 systems of that recipe (one supernode per group there: the host greedy over all
systems of a chunk costs more than the groups save).

One step = the whole hot path from the device-resident CSR: compress (Sec. 2.1), factor
(Sec. 3, all levels and the last-level block ILUT), solve (FGMRES with the
preconditioner applied every iteration, Alg. 2).  Both precisions run the same steps:
plain FP64, and FP32 factors with FP64 FGMRES (mixed).  For each: W untimed steps, then
K timed steps between device synchronizations, with no instrumentation inside the timed
region.  One further untimed step per precision records HIP events around every launch
class for the per-kernel figures and the roofline.  The oracle (CPU, FP64) solves a
smaller grid of the same recipe on the host for the CPU-baseline figure.

Prints one JSON line; `value` is the mixed-precision time-to-solve.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solve @1e-8 rel residual + SpMV/solve GB/s, mixed/learned vs FP64 plain"
HBM_PEAK_GBPS = 8000.0
TOL, MAXIT = 1e-8, 1000

WORKLOADS = {
    "upwind74": dict(desc="74^3 nodes, 14-neighbour random stencil, 1..7 unknowns per node, upwind "
                          "convection (cell Peclet LogUniform(0.1, 100))",
                     make=lambda side: __import__("paper_1508_02219_amd.synth", fromlist=["x"]).upwind_system(
                         side, side, side, seed=3),
                     side=74, sample_side=48, tau=1.0, levels=4, droptol=1e-4, restart=60, group_rows=32),
    "grid40": dict(desc="40^3 nodes, 14-neighbour random stencil, 5 unknowns per node, 10% block perturbation",
                   make=lambda side: __import__("paper_1508_02219_amd.synth", fromlist=["x"]).grid_system(
                       side, side, side, 5, "14rand", 0.10, seed=2),
                   side=40, sample_side=40, tau=0.8, levels=3, droptol=1e-4, restart=50, group_rows=16),
}


def _sources_sha256():
    """Hash of the library's kernel and header sources (a traffic record applies only to the
    sources it was measured on)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1508_02219_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h")))
    for f in files + [os.path.join(ROOT, "include", "vbarms.h")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic(kernel, workload, group_rows, weighted):
    """HBM bytes per dispatch of `kernel` from the committed counter record (FETCH_SIZE and
    WRITE_SIZE scaled by the copy calibration), or None when no record matches this kernel,
    this workload and the current sources."""
    path = os.path.join(ROOT, "profiles", "k_ilut_wave_upwind74_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("kernel") != kernel or workload != "upwind74" or group_rows != 32 or weighted
            or rec.get("sources_sha256") != _sources_sha256()):
        return None
    return rec["bytes_per_dispatch"]


def _host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 0


def _cpu_baseline(wl, n_full):
    """The oracle, single-threaded, on a smaller grid of the same recipe: compress +
    factor + FGMRES; the time is scaled to the full workload by the ratio of unknowns."""
    from oracle import oracle as O

    system = wl["make"](wl["sample_side"])
    t0 = time.perf_counter()
    po, bo = O.compress(system.n, system.rowptr, system.col, wl["tau"])
    orc = O.Oracle(system.n, system.rowptr, system.col, system.val, po, bo, wl["levels"], wl["droptol"], 1, 0,
                   wl["group_rows"])
    x, st, its, rel, _ = O.fgmres(system.n, system.rowptr, system.col, system.val, system.b, orc, TOL,
                                  wl["restart"], MAXIT)
    dt = time.perf_counter() - t0
    model, ncpu = _host_cpu()
    side = wl["sample_side"]
    return {"value": round(dt * n_full / system.n, 3), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"the same recipe on a {side}^3 grid (n={system.n}): one compress + factor + FGMRES solve "
                      f"took {dt:.2f} s (status {st}, {its} iterations, true rel. residual {rel:.2e}); value "
                      f"scales it by n_full/n_sample = {n_full / system.n:.3f}",
            "host_cpu": model, "host_logical_cpus": ncpu}


def _comparators(wl, side, V, torch):
    """Sec. 4 comparison (Table 5's claim): the same system solved with VBARMS, with block
    ILUT alone on the compressed blocks (VBILUT) and with pointwise ILUT; median of three
    timed runs each after one warm-up, FP64."""
    system = wl["make"](side)
    dev = V.csr_to_device(system)
    b = torch.as_tensor(system.b, device="cuda")
    n = system.n
    single_perm = torch.arange(n, dtype=torch.int32, device="cuda")
    single_bptr = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    methods = {"VBARMS": (wl["levels"], False), "VBILUT": (0, False), "ILUT (pointwise)": (0, True)}
    if wl["group_rows"]:
        methods = {"VBARMS (groups)": (wl["levels"], False), "VBARMS (one supernode per group)": (wl["levels"], False),
                   "VBILUT": (0, False), "ILUT (pointwise)": (0, True)}
    out = {"comparators": {}, "workload": wl["desc"].replace("74^3", f"{side}^3").replace("40^3", f"{side}^3"),
           "n": n, "nnz": system.nnz, "tau": wl["tau"], "droptol": wl["droptol"], "krylov": f"FGMRES({wl['restart']})"}
    for name, (lev, pointwise) in methods.items():
        sv = V.Solver()
        runs = []
        for k in range(4):
            t0 = time.perf_counter()
            if pointwise:
                st = sv.set_partition(*dev, single_perm, single_bptr)
            else:
                _, _, st = sv.compress(*dev, wl["tau"])
            try:
                sv.factor(lev, wl["droptol"], group_rows=wl["group_rows"] if "(groups)" in name else 0)
            except V.VbarmsError as e:  # e.g. a pointwise row longer than the block ILUT holds
                print(f"[comparators] {name}: factorization failed: {e}", file=sys.stderr, flush=True)
                out["comparators"][name] = {"failed": str(e)}
                break
            x, info = sv.solve(b, tol=TOL, restart=wl["restart"], maxit=MAXIT)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            fs = sv.stats()
            if k > 0:
                runs.append((dt, fs, info, st))
            print(f"[comparators] {name} run {k}: {dt * 1e3:.1f} ms its {info.iters} status {info.status}",
                  file=sys.stderr, flush=True)
        if not runs:
            sv.close()
            continue
        runs.sort(key=lambda r: r[0])
        dt, fs, info, st = runs[1]
        out["comparators"][name] = {
            "s_per_solve": round(dt, 4), "iters": info.iters, "converged": info.status == 0,
            "true_relres": info.true_relres, "blocks": st.nblocks, "av_bd": round(st.av_bd, 4),
            "compress_ms": round(fs.compress_ms, 2), "factor_ms": round(fs.factor_ms, 2),
            "solve_ms": round(fs.solve_ms, 2), "levels": fs.levels, "last_level_blocks": fs.last_p,
            "ilut_waves": fs.ilut_waves, "mem_ratio": round(fs.factor_values / max(fs.nnz, 1), 3)}
        sv.close()
    print(json.dumps(out), flush=True)
    return 0


def _batch_systems(count, seed=4):
    """The batched workload: `count` systems of the 40^3 recipe (14-neighbour stencil, 10%
    block perturbation) with n log-uniform in [5k, 200k] and ell in {3, 5, 6}; each grid is
    as close to a cube as the node count allows."""
    import numpy as np
    from paper_1508_02219_amd import synth

    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        n = float(np.exp(rng.uniform(np.log(5e3), np.log(2e5))))
        ell = int(rng.choice([3, 5, 6]))
        nodes = max(8, int(round(n / ell)))
        nx = max(2, int(round(nodes ** (1.0 / 3.0))))
        ny = max(2, int(round((nodes / nx) ** 0.5)))
        nz = max(2, int(round(nodes / (nx * ny))))
        out.append(synth.grid_system(nx, ny, nz, ell, "14rand", 0.10, seed=1000 + q))
    return out


def _batch_bench(args, V, torch):
    """Batched uneven systems: all systems compressed, factored and solved for every
    right-hand side through shared launches, against one-at-a-time solves on a sample."""
    import numpy as np

    count, nrhs, tau, levels, droptol, restart = args.batch, 16, 0.8, 3, 1e-4, 50
    group_rows = 0 if args.group_rows < 0 else args.group_rows  # groups did not pay off on the batch
    t0 = time.perf_counter()
    systems = _batch_systems(count)
    print(f"[bench] generated {count} systems (n = {sum(s.n for s in systems)}) in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    devs = [V.csr_to_device(s) for s in systems]
    N = sum(s.n for s in systems)
    rng = np.random.default_rng(16)
    B = torch.as_tensor(rng.standard_normal((nrhs, N)), device="cuda")
    off = np.concatenate([[0], np.cumsum([s.n for s in systems])])
    # the systems go through the batched path `chunk` at a time (each chunk one combined
    # factorization and one lockstep solve of all right-hand sides)
    chunk = max(1, min(args.batch_chunk, count))
    chunks = [(q, min(q + chunk, count)) for q in range(0, count, chunk)]
    Bc = [B[:, off[a]:off[b]].contiguous() for a, b in chunks]
    bs = V.BatchSolver()

    def batched():
        info = []
        for (a, b), Bq in zip(chunks, Bc):
            bs.factor(devs[a:b], tau, levels, droptol, group_rows=group_rows)
            X, inf = bs.solve(Bq, tol=TOL, restart=restart, maxit=MAXIT)
            info += [list(r) for r in zip(*inf)]  # per system: its right-hand sides
        return info

    for w in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = batched()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    ok = all(i.status == 0 and i.true_relres <= TOL for row in info for i in row)
    its = [i.iters for row in info for i in row]
    fs = bs.handle().stats()  # of the last chunk
    bs.close()
    # one at a time: every 16th system, each compressed, factored and solved for its 16
    # right-hand sides on its own handle; scaled to the whole batch by the unknowns
    sample = list(range(0, count, max(1, count // 16)))
    sv = V.Solver()
    for q in sample[:1]:  # warm-up
        sv.compress(*devs[q], tau)
        sv.factor(levels, droptol, group_rows=group_rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_sample = 0
    for q in sample:
        sv.compress(*devs[q], tau)
        sv.factor(levels, droptol, group_rows=group_rows)
        for r in range(nrhs):
            x, inf = sv.solve(B[r, off[q]:off[q + 1]].contiguous(), tol=TOL, restart=restart, maxit=MAXIT)
            ok = ok and inf.status == 0
        n_sample += systems[q].n
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) * N / n_sample
    sv.close()
    solves = count * nrhs
    out = {"metric": "aggregate solves/s, batched vs one-at-a-time", "value": round(solves / tb, 3),
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1000.0 * tb, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{count} systems of the 40^3 recipe, n log-uniform in [5k, 200k], ell in "
                                  f"{{3, 5, 6}}, {nrhs} N(0,1) right-hand sides each", "systems": count,
                      "n_total": N, "nnz_total": int(sum(s.nnz for s in systems)), "tau": tau, "levels": levels,
                      "droptol": droptol, "krylov": f"FGMRES({restart})", "tol": TOL,
                      "systems_per_batched_factorization": chunk, "batched_factorizations": len(chunks),
                      "group_rows": group_rows,
                      "right_hand_sides": "all 16 of a chunk in one lockstep FGMRES (multi-vector SpMV and "
                                          "preconditioner launches)"},
           "all_converged": bool(ok), "iters_min_median_max": [int(min(its)), int(np.median(its)), int(max(its))],
           "batched_s": round(tb, 4), "last_chunk_phases_ms": {"compress": round(fs.compress_ms, 2),
                                                            "factor": round(fs.factor_ms, 2),
                                                            "solve_all_rhs": round(fs.solve_ms, 2)},
           "one_at_a_time_s": round(ts, 3), "one_at_a_time_solves_per_s": round(solves / ts, 3),
           "one_at_a_time_sample": f"{len(sample)} of {count} systems ({n_sample} unknowns), each compressed, "
                                   f"factored and solved for its {nrhs} right-hand sides on its own handle; time "
                                   f"scaled by total/sample unknowns",
           "batched_speedup": round(ts / tb, 3)}
    print(json.dumps(out), flush=True)
    return 0


def _learned_bench(args, V, torch):
    """Learned parameter selection on held-out matrices of the training recipe at 74^3
    nodes (n = 1.2M to 2.4M): the network is trained on the stored sweeps of the 20^3-34^3
    training matrices with the library's kernels, then each held-out matrix is solved with
    the predicted (tau, per-level t) in FP64 and with FP32 factors, with the defaults in
    FP64 (the plain method) and with the best constant setting of the sweeps in FP64.  A
    setting that does not converge within the sweeps' iteration limit is charged its run
    plus the defaults' run, as the method falls back to the defaults."""
    import math

    import numpy as np
    from paper_1508_02219_amd import learned as Lr

    meta, recs = Lr.load_dataset(os.path.join(ROOT, "paper_1508_02219_amd", "data", "x4_training_sweeps.json"))
    X = np.array([r["features"] for r in recs], np.float32)
    Y = np.array([Lr.target(r["label"]) for r in recs], np.float32)
    pred = Lr.Predictor(seed=0)
    pred.fit(X, Y, epochs=200, lr=2e-3, batch=32)
    (ctau, ctol), _ = Lr.best_constant(recs)
    rows = []
    for k in range(args.learned):
        r = Lr.recipe(9000 + k, side_range=(74, 74))
        t0 = time.perf_counter()
        s = Lr.make_system(r)
        print(f"[learned] {s.name} n={s.n} ell={r['ell']} pe={r['pe']:.2f} aniso={r['aniso']:.1f} "
              f"(generated in {time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
        dev = V.csr_to_device(s)
        b = torch.as_tensor(s.b, device="cuda")
        sv = V.Solver()
        (tau, tols), = pred.predict(sv.features(*dev))

        def measure(tau_, tols_, prec):
            Lr.run_once(sv, dev, b, tau_, tols_, precision=prec)  # warm-up of this setting
            return Lr.run_once(sv, dev, b, tau_, tols_, precision=prec)

        dflt = measure(Lr.DEFAULT_TAU, Lr.DEFAULT_TOL, V.F64)
        res = {"defaults_f64": dflt, "learned_f64": measure(tau, tols, V.F64),
               "learned_f32": measure(tau, tols, V.F32), "constant_f64": measure(ctau, ctol, V.F64)}
        sv.close()
        row = {"n": s.n, "pe": round(r["pe"], 2), "ell": r["ell"], "predicted_tau": round(tau, 3),
               "predicted_t": [float(f"{t:.2e}") for t in tols]}
        for key, rr in res.items():
            ms = rr.ms if rr.ok else (rr.ms + dflt.ms if dflt.ok else math.inf)
            row[key] = {"ms": round(ms, 1), "iters": rr.iters, "converged": bool(rr.ok)}
        rows.append(row)
        print(f"[learned] {json.dumps(row)}", file=sys.stderr, flush=True)
    solved = [r for r in rows if r["defaults_f64"]["converged"]]

    def gm(a, b):
        v = [r[a]["ms"] / r[b]["ms"] for r in solved if math.isfinite(r[a]["ms"]) and math.isfinite(r[b]["ms"])]
        return round(float(np.exp(np.mean(np.log(v)))), 3) if v else None

    out = {"metric": "time-to-solve, learned (tau, per-level t) vs the defaults (FP64 plain) and vs the best "
                     "constant setting", "unit": "x (geometric mean of time ratios)", "n_gpus": 1,
           "data": "synthetic", "config": {"workload": "held-out matrices of the learned-selection recipe at 74^3 "
                                                       "nodes", "levels": Lr.LEVELS, "restart": Lr.RESTART,
                                           "maxit": Lr.MAXIT, "tol": Lr.RTOL, "defaults": [Lr.DEFAULT_TAU, Lr.DEFAULT_TOL],
                                           "best_constant": [ctau, ctol], "training_matrices": len(recs)},
           "matrices": rows, "solved_by_defaults": len(solved),
           "speedup_learned_f64_vs_defaults_f64": gm("defaults_f64", "learned_f64"),
           "speedup_learned_f32_vs_defaults_f64": gm("defaults_f64", "learned_f32"),
           "speedup_learned_f64_vs_constant_f64": gm("constant_f64", "learned_f64")}
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="upwind74")
    ap.add_argument("--precisions", default="f64,f32", help="comma list of f64 / f32 (the last one is `value`)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three 1 GiB device-to-device copies (the reference for counter scaling)")
    ap.add_argument("--batch", type=int, default=0, metavar="COUNT",
                    help="instead of the benchmark, time COUNT uneven systems with 16 right-hand sides each, "
                         "batched and one at a time")
    ap.add_argument("--batch-chunk", type=int, default=64, metavar="K",
                    help="systems per batched factorization (the batch is processed K systems at a time)")
    ap.add_argument("--group-rows", type=int, default=-1, metavar="K",
                    help="groups of supernodes in the independent sets, at most K rows each (0: one supernode; "
                         "default: the workload's setting)")
    ap.add_argument("--learned", type=int, default=0, metavar="K",
                    help="instead of the benchmark, evaluate the learned parameter selection on K held-out "
                         "matrices of its recipe at 74^3 nodes")
    ap.add_argument("--weighted-is", action="store_true",
                    help="visit supernodes by the weighted order in the independent sets (default: natural order)")
    ap.add_argument("--comparators", type=int, default=0, metavar="SIDE",
                    help="instead of the benchmark, compare VBARMS with block ILUT alone (VBILUT, levels = 0) and "
                         "with pointwise ILUT (1x1 blocks, levels = 0) on a SIDE^3 grid of the workload's recipe")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the whole problem fits on one MI355X and this build has no "
              "multi-GPU path (--gpus must be 1)", file=sys.stderr)
        return 2

    import torch

    from paper_1508_02219_amd import vbarms as V

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: each copy reads and writes exactly 1 GiB
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 3}), flush=True)
        return 0
    if args.batch:
        return _batch_bench(args, V, torch)
    if args.learned:
        return _learned_bench(args, V, torch)
    wl = WORKLOADS[args.workload]
    tau, levels, droptol, restart = wl["tau"], wl["levels"], wl["droptol"], wl["restart"]
    group_rows = wl["group_rows"] if args.group_rows < 0 else args.group_rows
    is_order = V.IS_WEIGHTED if args.weighted_is else V.IS_NATURAL
    if args.comparators:
        return _comparators(wl, args.comparators, V, torch)
    system = wl["make"](wl["side"])
    print(f"[bench] workload {system.name} n={system.n} nnz={system.nnz}", file=sys.stderr, flush=True)
    rp, ci, va = V.csr_to_device(system)
    b = torch.as_tensor(system.b, device="cuda")
    sv = V.Solver()
    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]

    def step(prec):
        _, _, st = sv.compress(rp, ci, va, tau)
        sv.factor(levels, droptol, 1, V.F32 if prec == "f32" else V.F64, is_order, group_rows)
        x, info = sv.solve(b, tol=TOL, restart=restart, maxit=MAXIT)
        return st, info

    runs = {}
    for prec in precs:
        for w in range(args.warmup):
            print(f"[bench] {prec} warmup {w + 1}/{args.warmup}", file=sys.stderr, flush=True)
            step(prec)
        phases = {"compress_ms": [], "factor_ms": [], "solve_ms": [], "ilut_ms": []}
        iters, relres = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            st, info = step(prec)
            if info.status != 0 or info.true_relres > TOL:
                print(f"[bench] {prec} step {k + 1} did not converge: status {info.status} "
                      f"relres {info.true_relres:.3e}", file=sys.stderr, flush=True)
                return 1
            fs = sv.stats()
            for key in phases:
                phases[key].append(getattr(fs, key))
            iters.append(info.iters)
            relres.append(info.true_relres)
            print(f"[bench] {prec} step {k + 1}/{args.steps}: its {info.iters} relres {info.true_relres:.2e} "
                  f"compress {fs.compress_ms:.1f} factor {fs.factor_ms:.1f} (ilut {fs.ilut_ms:.1f}, "
                  f"{fs.ilut_waves} waves) solve {fs.solve_ms:.1f} ms", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        fs = sv.stats()
        # measurement pass (untimed): HIP events around every launch class
        sv.set_timing(True)
        step(prec)
        kst = sv.kernel_stats()
        sv.set_timing(False)
        fsm = sv.stats()
        runs[prec] = dict(s=elapsed / args.steps, phases=phases, iters=iters, relres=relres, st=st, fs=fs, kst=kst,
                          fsm=fsm)

    mem = V.device_memory()
    sv.close()
    head = precs[-1]
    R = runs[head]
    ms_per_step = 1000.0 * R["s"]

    def per_class(kst):
        return {k: {"calls": v[0], "ms": round(v[1], 3), "avg_us": round(1000.0 * v[1] / v[0], 3) if v[0] else None,
                    "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 2) if v[1] > 0 and v[2] > 0 else None}
                for k, v in kst.items()}

    # Roofline of the dominant launch class (by event time in the measurement pass).  For
    # the block ILUT, the algorithmic bytes are those of its result: read the matrix handed
    # to it, write L, U and the pivot-block LU factors (exported sizes), divided over its
    # launches; the other classes count the bytes their launches must move (see the
    # library's kernel table).
    kst, fsm = R["kst"], R["fsm"]
    timed = {k: v for k, v in kst.items() if v[0] > 0}
    dom = max(timed, key=lambda k: timed[k][1])
    calls, ms, nbytes = timed[dom]
    if dom == "ilut_wave":
        nbytes = calls * (fsm.ilut_result_bytes / max(calls, 1))
    achieved = (nbytes / calls) / (ms / calls * 1e-3) / 1e9 if nbytes > 0 else None
    roofline = {"bound": "hbm", "kernel": dom, "calls": calls, "avg_us": round(1000.0 * ms / calls, 3),
                "bytes_per_launch": round(nbytes / calls), "achieved": None if achieved is None else round(achieved, 3),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": None if achieved is None else round(achieved / HBM_PEAK_GBPS, 6), "traffic": None}
    if dom == "ilut_wave":
        roofline["traffic"] = _traffic("k_ilut_wave<float>" if head == "f32" else "k_ilut_wave<double>",
                                       args.workload, group_rows, args.weighted_is)

    def summary(prec):
        r = runs[prec]
        pc = per_class(r["kst"])
        f = r["fs"]
        mean = {k: round(sum(v) / len(v), 2) for k, v in r["phases"].items()}
        return {"s_per_solve": round(r["s"], 4), "phases_ms_mean": mean,
                "phases_ms_spread": {k: round(max(v) - min(v), 2) for k, v in r["phases"].items()},
                "iters": r["iters"], "max_true_relres": max(r["relres"]),
                "levels_factored": f.levels, "last_level_supernodes": f.last_p, "ilut_waves": f.ilut_waves,
                "ilut_attempts": f.ilut_attempts, "mem_ratio": round(f.factor_values / max(f.nnz, 1), 3),
                "factor_breakdown_ms": {"levels": [round(f.factor_level_ms[l], 2) for l in range(f.levels)],
                                        "last_level_ilut": round(f.ilut_ms, 2)},
                "spmv_GBps": pc["spmv"]["GBps"], "apply_GBps": pc["apply"]["GBps"],
                "trsv_GBps": pc["trsv_sweeps"]["GBps"], "kernels": pc}

    out = {
        "metric": METRIC,
        "value": round(R["s"], 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factors + f64 fgmres" if head == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": system.n, "nnz": system.nnz, "blocks": R["st"].nblocks,
                   "tau": tau, "levels": levels, "droptol": droptol, "group_rows": group_rows,
                   "independent_set_order": "weighted" if args.weighted_is else "natural",
                   "krylov": f"FGMRES({restart})", "tol": TOL, "rhs": "A*1"},
        "runs": {p: summary(p) for p in precs},
        "device_memory_GiB": {"peak_live": round(mem["peak"] / 2**30, 2), "cached": round(mem["cached"] / 2**30, 2),
                              "runtime_allocs": mem["runtime_allocs"]},
        "roofline": roofline,
    }
    if "f64" in runs and "f32" in runs:
        out["mixed_speedup_vs_fp64"] = round(runs["f64"]["s"] / runs["f32"]["s"], 4)
    if not args.no_cpu_baseline:
        print("[bench] oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(wl, system.n)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
