"""Benchmark of the LBRS hot path on one MI355X.

Workload: the four-quadrant 2D Riemann problem, 4096 x 4096 cells on [0,1]^2,
D2Q4, FP64, gamma = 1.4, omega = 1, CFL 0.5, transmissive sides, t_end = 0.3.
One "step" is one fused collide-and-stream LBRS step over the whole grid
(moments, flux, equilibria, relaxation, streaming, sides, next-step lambda*).

Prints one JSON line: MLUPS (value), the HBM roofline of the step kernel
(algorithmic 256 B per lattice update: 16 FP64 populations read + 16 written),
and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline: plain vs batched vs adjoint step, 1 MI355X"

# HBM bytes per launch of the step kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# (calibrated against a plain copy), valid for the kernel source they were taken
# on (profiles/step2d_d2q4_riemann4096.md); null once the source changes.
TRAFFIC_BYTES = 4.432e9
TRAFFIC_SOURCE_HASH = "79bd4658efd82c8a"
TRAFFIC_SHAPE = {"rows": 0, "wpb": 16, "layout": 1}


def kernel_source_hash() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_1504_07034_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("lbrs_step2d.hip", "lbrs_device.hpp"))
    return hashlib.sha256(src).hexdigest()[:16]
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = 256  # 16 FP64 populations in + 16 out per lattice update


def cpu_baseline(nsteps: int = 2):
    """The oracle on the same 4096^2 workload for a bounded number of steps
    (single thread), init time excluded by differencing two runs."""
    import oracle
    from paper_1504_07034_amd import workloads as wl

    w = wl.riemann2d(4096)
    P = oracle.Problem(model=w.model, nx=w.nx, ny=w.ny, domain=w.domain, gamma=w.gamma,
                       omega=w.omega, cfl=w.cfl, sides=w.sides)
    U0 = oracle.prim_to_cons(P, w.W)
    del w
    t0 = time.perf_counter()
    oracle.run(P, U0, t_end=0.3, max_steps=0, record=False)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oracle.run(P, U0, t_end=0.3, max_steps=nsteps, record=False)
    t_run = time.perf_counter() - t0
    secs = max(t_run - t_init, 1e-9)
    lups = 4096 * 4096 * r.nsteps
    return {"value": lups / secs / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"4096x4096 four-quadrant problem, {r.nsteps} steps from t=0 "
                      f"({secs:.1f} s of stepping; init excluded)"}


def batched_1d(chunks=(510, 1022, 2046), subset=32):
    """Ragged 1D batch: 1024 seeded shock tubes (200..20000 cells, own t_end) in
    one persistent launch (chunk autotuned), against sequential single-domain
    runs of a seeded subset of the same tubes (the plain library path: one
    persistent launch per tube of <= 2048 cells, one launch per step above)."""
    import numpy as np
    import torch

    from paper_1504_07034_amd import lbrs
    from paper_1504_07034_amd import workloads as wl

    tubes = wl.tube_batch(1024, seed=0)

    def make(sel, chunk):
        units = [lbrs.make_params(t.model, t.nx, 1, t.domain, t.gamma, t.omega, t.cfl)
                 for t in sel]
        B = lbrs.Batch1D(units, [t.t_end for t in sel], chunk=chunk)
        W = torch.from_numpy(np.concatenate([t.W[:, 0, :] for t in sel], axis=1)).cuda()
        U0 = torch.empty_like(W)
        lbrs.lbrs_prim_to_cons(lbrs.make_params(units[0].model, B.total, 1), W, U0)
        return B, U0

    def timed_batch(sel, chunk):
        B, U0 = make(sel, chunk)
        B.init(U0)
        B.run(10**6)  # capture the graph and warm up
        B.init(U0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B.run(10**6)
        e1.record()
        st = B.state()
        ms = e0.elapsed_time(e1)
        lups = sum(n * t.nx for n, t in zip(st["nsteps"], sel))
        assert st["rc"] == 0 and all(x == t.t_end for x, t in zip(st["t"], sel))
        B.close()
        return ms, lups

    tuned = {}
    for c in chunks:
        try:
            tuned[c] = timed_batch(tubes, c)
        except lbrs.LBRSError:  # chunk too large for this device's LDS
            pass
    best = min(tuned, key=lambda c: tuned[c][0])
    ms, lups = tuned[best]
    rng = np.random.default_rng(1)
    sub = [tubes[i] for i in sorted(rng.choice(len(tubes), size=subset, replace=False))]
    ms_b, lups_b = timed_batch(sub, best)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in sub:
        sim = lbrs.Sim(t.model, t.nx, 1, domain=t.domain, gamma=t.gamma, omega=t.omega, cfl=t.cfl)
        sim.init_primitive(t.W)
        sim.run(t.t_end, chunk=100000)
        sim.close()
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3
    return {"units": len(tubes), "cells": int(sum(t.nx for t in tubes)), "chunk": best,
            "ms": round(ms, 2), "MLUPS": round(lups / ms / 1e3, 1),
            "chunk_ms": {str(c): round(v[0], 2) for c, v in tuned.items()},
            "subset": {"units": subset, "batched_ms": round(ms_b, 2),
                       "sequential_ms": round(ms_s, 2), "speedup": round(ms_s / ms_b, 2)}}


def _time_ms(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def adjoint_2d(n=2048, steps=2000, k=50):
    """Adjoint configuration (2048^2 periodic acoustic pulse, frozen lattice
    speed, 2000 steps, J over [0.7,0.8]^2): time of a plain step, of a step
    writing the U^n tape, of an adjoint step, and of the whole sqrt(T)
    checkpointed gradient (forward with checkpoints + recompute + reverse)."""
    import torch

    from paper_1504_07034_amd import adjoint, lbrs
    from paper_1504_07034_amd import workloads as wl

    w = wl.acoustic_pulse(n, steps=steps)
    rho0 = torch.from_numpy(w.W[0].copy()).cuda()
    run = adjoint.GradientRunner(adjoint.GradientSpec(n=n, steps=steps), rho0)
    sim = run.sim
    run.forward(rho0, keep=False)
    fwd = _time_ms(lambda: sim.step(k)) / k
    tape = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    tap = _time_ms(lambda: [lbrs.lbrs_step_tape(sim.ctx, tape) for _ in range(k)]) / k
    g = torch.empty_like(run.fbar)
    adj = _time_ms(lambda: [lbrs.lbrs_adjoint_step(sim.ctx, tape, run.fbar, g) for _ in range(k)]) / k
    r = rho0.clone().requires_grad_(True)

    def grad():
        J = adjoint.LBRSFunction.apply(r, run)
        J.backward()

    grad()
    t_grad = _time_ms(grad)
    t_fwd = _time_ms(lambda: run.forward(rho0, keep=False))
    run.close()
    cells = n * n
    return {"n": n, "steps": steps, "segment": run.spec.seg,
            "forward_step_ms": round(fwd, 4), "tape_step_ms": round(tap, 4),
            "adjoint_step_ms": round(adj, 4),
            "adjoint_over_forward": round((tap + adj) / fwd, 3),
            "adjoint_step_GBs": round(288 * cells / (adj * 1e-3) / 1e9, 1),
            "gradient_ms": round(t_grad, 1), "forward_run_ms": round(t_fwd, 1),
            "gradient_over_forward_run": round(t_grad / t_fwd, 3)}


def batched_2d(k=10):
    """128 seeded periodic domains (sides 256..2048): one launch per step for all
    domains, against the same domains stepped one at a time."""
    import torch

    from paper_1504_07034_amd import lbrs
    from paper_1504_07034_amd import workloads as wl

    ws = wl.domain_batch(128, seed=0)
    doms = [lbrs.make_params(lbrs.LBRS_D2Q4, w.nx, w.ny, w.domain, w.gamma, w.omega, w.cfl,
                             w.sides, lbrs.LBRS_LAMBDA_FROZEN_INIT, 0.0, lbrs.LBRS_LAYOUT_ROWS)
            for w in ws]
    Us = []
    for w, p in zip(ws, doms):
        Wt = torch.from_numpy(w.W).cuda()
        U = torch.empty_like(Wt)
        lbrs.lbrs_prim_to_cons(p, Wt, U)
        Us.append(U)
    B = lbrs.Batch2D(doms)
    B.init(torch.cat([U.reshape(4, -1) for U in Us], dim=1))
    B.step(2)
    ms_b = _time_ms(lambda: B.step(k)) / k
    total = B.total
    B.close()
    del B
    torch.cuda.empty_cache()
    ms_s = 0.0
    for w, U in zip(ws, Us):
        sim = lbrs.Sim(lbrs.LBRS_D2Q4, w.nx, w.ny, domain=w.domain, gamma=w.gamma, cfl=w.cfl,
                       bc=w.sides, lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT,
                       layout=lbrs.LBRS_LAYOUT_ROWS)
        sim.init(U)
        sim.step(2)
        ms_s += _time_ms(lambda: sim.step(k)) / k
        sim.close()
    return {"domains": len(ws), "cells": int(total), "batched_ms_per_step": round(ms_b, 3),
            "MLUPS": round(total / ms_b / 1e3, 1),
            "sequential_ms_per_step": round(ms_s, 3), "speedup": round(ms_s / ms_b, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--rows", type=int, default=-1,
                    help="rows per tile (0 = automatic); default: autotune")
    ap.add_argument("--wpb", type=int, default=4)
    ap.add_argument("--layout", type=int, default=1, help="0 planar, 1 row-interleaved")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and adjoint figures reported beside the main value")
    ap.add_argument("--only", choices=["adjoint", "batch1d", "batch2d"], default=None,
                    help="run only one of the secondary measurements and print it (profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, run one plain copy of the populations (lbrs_get_f: "
                         "16 planes read and written) as a known-size reference for counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1504_07034_amd import autotune, lbrs
    from paper_1504_07034_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.only:
        fn = {"adjoint": adjoint_2d, "batch1d": batched_1d, "batch2d": batched_2d}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    n = 4096
    t_end = 0.3
    w = wl.riemann2d(n, t_end=t_end)
    sim = lbrs.Sim(w.model, n, n, domain=w.domain, gamma=w.gamma, omega=w.omega, cfl=w.cfl,
                   bc=w.sides, layout=args.layout)
    W = torch.from_numpy(w.W).cuda()
    U0 = sim.prim_to_cons(W)
    del W, w

    shape = {"rows": args.rows, "wpb": args.wpb}

    def fresh():
        sim.init(U0)
        if shape["rows"] >= 0:
            sim.set_tile(shape["rows"], shape["wpb"])

    if args.rows < 0:  # autotune the launch shape (untimed), then start over
        sim.init(U0)
        sim.step(20, t_end)
        best = autotune.tune(sim, t_end, use_cache=False)
        shape = {"rows": best["rows"], "wpb": best["wpb"]}
        print("autotune: " + ", ".join(f"({c['rows']},{c['wpb']}) {c['ms']:.3f} ms"
                                       for c in best["candidates"]), file=sys.stderr, flush=True)

    # The run reaches t_end after ~7.8k steps; time in segments that stay
    # inside [0, t_end) so that every timed step does real work.
    seg_cap = 6000
    fresh()
    sim.step(args.warmup, t_end)
    done_in_seg = args.warmup
    stream = torch.cuda.current_stream()
    total_ms = 0.0
    left = args.steps
    while left > 0:
        if done_in_seg >= seg_cap:
            fresh()
            done_in_seg = 0
        k = min(left, seg_cap - done_in_seg)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(k, t_end)
        e1.record(stream)
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        st = sim.state()
        if st["rc"] != 0 or st["nsteps"] != done_in_seg + k:
            raise RuntimeError(f"timed steps did not all run: {st}")
        done_in_seg += k
        left -= k

    if args.calibrate_copy:
        f_copy = sim.get_f()
        torch.cuda.synchronize()
        del f_copy

    ms_per_step = total_ms / args.steps
    cells = n * n
    mlups = cells / (ms_per_step * 1e-3) / 1e6
    achieved = BYTES_PER_LUP * cells / (ms_per_step * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D four-quadrant Riemann problem, plain LBRS D2Q4",
                   "nx": n, "ny": n, "domain": "[0,1]^2", "gamma": 1.4, "omega": 1.0,
                   "cfl": 0.5, "sides": "transmissive", "t_end": t_end,
                   "tile_rows": shape["rows"], "waves_per_block": shape["wpb"],
                   "layout": "row-interleaved" if args.layout == 1 else "planar"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (TRAFFIC_BYTES if kernel_source_hash() == TRAFFIC_SOURCE_HASH
                                 and shape["wpb"] == TRAFFIC_SHAPE["wpb"]
                                 and args.layout == TRAFFIC_SHAPE["layout"] else None)},
    }
    sim.close()
    del U0
    torch.cuda.empty_cache()
    if not args.no_extras:
        rec["adjoint_2d"] = adjoint_2d()
        torch.cuda.empty_cache()
        rec["batched_1d"] = batched_1d()
        torch.cuda.empty_cache()
        rec["batched_2d"] = batched_2d()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
