"""Benchmark of the LBRS hot path on one MI355X.

Workload: the four-quadrant 2D Riemann problem, 4096 x 4096 cells on [0,1]^2,
D2Q4, FP64, gamma = 1.4, omega = 1, CFL 0.5, transmissive sides, t_end = 0.3,
per-step lattice speed.  One "step" is one collide-and-stream LBRS step over
the whole grid (moments, flux, equilibria, relaxation, streaming, sides,
next-step lambda*).  The K timed steps (after W untimed ones) are taken from
the middle of the run to t_end, in the autotuned launch form (single steps,
or two fused steps per launch).

Prints one JSON line: MLUPS (value), the HBM roofline of the timed kernel on
its own algorithmic bytes (256 B per lattice update for a single step, 128 B
for two fused steps: f^{n+1} stays in registers), whole runs to t_end, and the
CPU oracle timed on a bounded sample of the same workload (one thread and all
host cores).
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
# (calibrated against a plain copy), by launch shape "waves_per_block,alternate"
# (automatic row segments, row-interleaved layout), valid for the kernel code
# they were taken on (profiles/step2d_d2q4_riemann4096.md); null once the code
# changes or for a shape not profiled.
TRAFFIC_BYTES = {"16,0": 4.430e9}
TRAFFIC_SOURCE_HASH = "c1666d2a85a1b74c"
SINGLE_SOURCES = ("lbrs_step2d.hip", "lbrs_device.hpp", "lbrs_rowops.hpp")
# The same for the fused multi-step kernel, by "steps_per_launch,waves_per_block":
# HBM bytes per launch that does work (profiles/step2d_pair_riemann4096.md);
# the window's figure is that times the share of the enqueued launches that
# did work (per-step lattice speeds: one launch per step, of which those past
# the steps done exit at once, moving nothing).
PAIR_TRAFFIC_BYTES = {"4,8": 4.498e9, "2,8": 4.428e9}
PAIR_TRAFFIC_SOURCE_HASH = "317c0476b9c364cb"
PAIR_SOURCES = ("lbrs_pair2d.hip", "lbrs_device.hpp", "lbrs_rowops.hpp")


def traffic_bytes(shape, layout, active_share=1.0):
    """HBM bytes per enqueued launch of the timed form (fused: per launch that
    did work, times the share of such launches), or None."""
    if shape["rows"] != 0 or layout != 1:
        return None
    if shape.get("fuse", 1) >= 2:
        if kernel_source_hash(PAIR_SOURCES) != PAIR_TRAFFIC_SOURCE_HASH:
            return None
        b = PAIR_TRAFFIC_BYTES.get(f"{shape['fuse']},{shape['wpb']}")
        return None if b is None else round(b * active_share)
    if kernel_source_hash(SINGLE_SOURCES) != TRAFFIC_SOURCE_HASH:
        return None
    return TRAFFIC_BYTES.get(f"{shape['wpb']},{shape['alt']}")


def _code_only(text: str) -> str:
    """Source text without comments and blank lines (what the compiler sees)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.split("\n") if line.strip())


def kernel_source_hash(files=SINGLE_SOURCES) -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_1504_07034_amd", "csrc")
    src = "".join(_code_only(open(os.path.join(csrc, f)).read()) for f in files)
    return hashlib.sha256(src.encode()).hexdigest()[:16]


HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = 256  # single step: 16 FP64 populations in + 16 out per lattice update
# k fused steps: f^n in, f^{n+k} out per k updates, 256/k B per update


def form_bytes(fuse: int) -> float:
    return BYTES_PER_LUP / fuse


def cpu_baseline(nsteps_one: int = 8, nsteps_all: int = 48):
    """The oracle on the same 4096^2 workload for a bounded number of steps from
    t = 0, init time excluded by differencing two runs: its timing build (the
    same source, -O3 -march=native, OpenMP over cells, no contraction of
    multiply-adds) on one thread (8 steps, ~12 s), then on every host core the
    process may use (48 steps, ~10 s on 16 cores)."""
    import oracle
    from paper_1504_07034_amd import workloads as wl

    w = wl.riemann2d(4096)
    P = oracle.Problem(model=w.model, nx=w.nx, ny=w.ny, domain=w.domain, gamma=w.gamma,
                       omega=w.omega, cfl=w.cfl, sides=w.sides)
    U0 = oracle.prim_to_cons(P, w.W)
    del w
    host = _host_cpu()

    def timed(threads, nsteps):
        used = oracle.use("omp", threads)
        t0 = time.perf_counter()
        oracle.run(P, U0, t_end=0.3, max_steps=0, record=False)
        t_init = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = oracle.run(P, U0, t_end=0.3, max_steps=nsteps, record=False)
        t_run = time.perf_counter() - t0
        secs = max(t_run - t_init, 1e-9)
        return used, 4096 * 4096 * r.nsteps / secs / 1e6, secs, r.nsteps

    try:
        one = timed(1, nsteps_one)
        allc = timed(host["affinity"], nsteps_all)
    finally:
        oracle.use("serial")
    return {"value": round(allc[1], 2), "unit": "MLUPS", "cores": allc[0], "kind": "oracle",
            "sample": f"4096x4096 four-quadrant problem, {allc[3]} steps from t=0 on {allc[0]} "
                      f"threads ({allc[2]:.1f} s of stepping; init excluded)",
            "build": "g++ -O3 -march=native -fopenmp -ffp-contract=off",
            "single_thread": {"value": round(one[1], 2), "cores": 1,
                              "sample": f"{one[3]} steps ({one[2]:.1f} s)"},
            "host": host}


def _host_cpu() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def batched_1d(chunks=(1022, 2046, 3070), sequential=True):
    """Ragged 1D batch: 1024 seeded shock tubes (200..20000 cells, own t_end) in
    one persistent launch (chunk autotuned).  Beside it: the critical path --
    the largest unit alone in the same batched kernel (its team's serial chain
    of steps bounds the batch's time from below) -- and the same 1024 tubes run
    one after another through the plain single-domain path (one persistent
    launch per tube of <= 2048 cells, one launch per step above), timed on
    the GPU only: every tube is set up and initialised before the timed region,
    whose launches are enqueued back to back.  sequential=False runs the batch
    alone (for HBM counters of the batched launch)."""
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
        return ms, lups, st["nsteps"]

    tuned = {}
    for c in chunks:
        try:
            tuned[c] = timed_batch(tubes, c)
        except lbrs.LBRSError:  # chunk too large for this device's LDS
            pass
    best = min(tuned, key=lambda c: tuned[c][0])
    ms, lups, nsteps = tuned[best]
    out = {"units": len(tubes), "cells": int(sum(t.nx for t in tubes)), "chunk": best,
           "ms": round(ms, 2), "MLUPS": round(lups / ms / 1e3, 1),
           # a single 1D D1Q3 step's 144 B per update at this rate (the batch
           # keeps its populations on chip: not HBM traffic)
           "single_step_equivalent_GBs": round(144 * lups / ms / 1e6, 1),
           "chunk_ms": {str(c): round(v[0], 2) for c, v in tuned.items()}}
    # critical path: the unit with the longest serial chain (cells per member
    # times steps) alone in the batched kernel
    def chain(b):
        t = tubes[b]
        return nsteps[b] * min(t.nx, best)
    crit = max(range(len(tubes)), key=chain)
    ms_c, _, st_c = timed_batch([tubes[crit]], best)
    out["critical_path"] = {
        "unit": crit, "cells": tubes[crit].nx, "steps": int(st_c[0]),
        "members": -(-tubes[crit].nx // best), "alone_ms": round(ms_c, 2),
        "per_step_us": round(1e3 * ms_c / st_c[0], 3),
        "batch_over_critical_path": round(ms / ms_c, 3)}
    if not sequential:
        return out
    sims = []
    for t in tubes:
        sim = lbrs.Sim(t.model, t.nx, 1, domain=t.domain, gamma=t.gamma, omega=t.omega, cfl=t.cfl)
        sim.init_primitive(t.W)
        sims.append(sim)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for sim, t, k in zip(sims, tubes, nsteps):
        sim.step(int(k), t.t_end)
    e1.record()
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    done = [sim.state() for sim in sims]
    assert all(d["rc"] == 0 and d["t"] == t.t_end and d["nsteps"] == k
               for d, t, k in zip(done, tubes, nsteps))
    for sim in sims:
        sim.close()
    out["sequential"] = {"units": len(tubes), "kind": "single-domain launches, GPU time only",
                         "ms": round(ms_s, 2), "speedup": round(ms_s / ms, 2)}
    return out


def sod_400():
    """The 400-cell Sod tube (D1Q3, omega = 1, cfl 0.5, transmissive) run to
    t = 0.2: the whole run is one persistent launch (one workgroup, the tube in
    LDS); latency-bound, so MLUPS here is not a roofline figure."""
    import torch

    from paper_1504_07034_amd import lbrs
    from paper_1504_07034_amd import workloads as wl

    w = wl.sod(400)
    sim = lbrs.Sim(w.model, w.nx, 1, domain=w.domain, gamma=w.gamma, omega=w.omega, cfl=w.cfl)
    U0 = sim.prim_to_cons(torch.from_numpy(w.W).cuda())
    sim.init(U0)
    sim.step(10**6, 0.2)  # warm up
    times = []
    for _ in range(5):
        sim.init(U0)
        times.append(_time_ms(lambda: sim.step(10**6, 0.2)))
    st = sim.state()
    assert st["rc"] == 0 and st["t"] == 0.2
    sim.close()
    ms = sorted(times)[len(times) // 2]
    return {"workload": "Sod shock tube, D1Q3, 400 cells, t = 0.2", "steps": st["nsteps"],
            "launches": 1, "ms": round(ms, 3), "us_per_step": round(1e3 * ms / st["nsteps"], 3),
            "MLUPS": round(400 * st["nsteps"] / ms / 1e3, 2)}


def _time_ms(fn, reps=1, warm=False):
    """Milliseconds of fn (mean of reps), after one untimed call with warm
    (first launches of a kernel load its code)."""
    import torch
    if warm:
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def adjoint_2d(n=2048, steps=2000, k=50, steps_only=False):
    """Adjoint configuration (2048^2 periodic acoustic pulse, frozen lattice
    speed, 2000 steps, J over [0.7,0.8]^2): time of a plain step, of a step
    writing the U^n tape, of an adjoint step, of the whole sqrt(T)
    checkpointed gradient (forward with checkpoints + recompute + reverse),
    and of the gradient with every step's moments kept when they fit."""
    import torch

    from paper_1504_07034_amd import adjoint, lbrs
    from paper_1504_07034_amd import workloads as wl

    w = wl.acoustic_pulse(n, steps=steps)
    rho0 = torch.from_numpy(w.W[0].copy()).cuda()
    run = adjoint.GradientRunner(adjoint.GradientSpec(n=n, steps=steps), rho0)
    best = run.tune(rho0)
    sim = run.sim
    run.forward(rho0, keep=False)
    fwd = _time_ms(lambda: sim.step(k), warm=True) / k
    sim.set_fusion(1)
    fwd1 = _time_ms(lambda: sim.step(k), warm=True) / k
    sim.set_fusion(best["fuse"])
    # the taped and adjoint steps in the tuned number per launch (what the
    # gradient's recompute and reverse sweep use), in pairs and single
    kf = best["fuse"]
    tapes = torch.empty((kf, 4, n, n), dtype=torch.float64, device="cuda")
    tape = tapes[0]
    tap = _time_ms(lambda: [lbrs.lbrs_step_tape(sim.ctx, tape) for _ in range(k)], warm=True) / k
    kk = max(1, k // kf)
    tapk = _time_ms(lambda: [lbrs.lbrs_step_tapes(sim.ctx, kf, tapes)
                             for _ in range(kk)], warm=True) / (kf * kk)
    g = torch.empty_like(run.fbar)
    adj = _time_ms(lambda: [lbrs.lbrs_adjoint_step(sim.ctx, tape, run.fbar, g) for _ in range(k)],
                   warm=True) / k
    adjk = _time_ms(lambda: [lbrs.lbrs_adjoint_steps(sim.ctx, kf, tapes, run.fbar, g)
                             for _ in range(kk)], warm=True) / (kf * kk)
    pair = None
    if kf > 2:
        k2 = max(1, k // 2)
        pair = {"tape_step_ms": round(_time_ms(lambda: [lbrs.lbrs_step_tapes(sim.ctx, 2, tapes)
                                                        for _ in range(k2)], warm=True)
                                      / (2 * k2), 4),
                "adjoint_step_ms": round(_time_ms(lambda: [
                    lbrs.lbrs_adjoint_steps(sim.ctx, 2, tapes, run.fbar, g)
                    for _ in range(k2)], warm=True) / (2 * k2), 4)}
    if steps_only:  # the per-step figures alone (profiling)
        run.close()
        return {"n": n, "forward_step_ms": round(fwd, 4), "tape_step_ms": round(tapk, 4),
                "adjoint_step_ms": round(adjk, 4), "single_forward_step_ms": round(fwd1, 4),
                "steps_per_launch": kf, "waves_per_block": best["wpb"]}
    r = rho0.clone().requires_grad_(True)

    def grad():
        J = adjoint.LBRSFunction.apply(r, run)
        J.backward()

    grad()
    t_grad = _time_ms(grad)
    t_fwd = _time_ms(lambda: run.forward(rho0, keep=False))
    tile, fuse, seg = run.spec.tile, run.spec.fuse, run.spec.seg
    run.close()
    del run, r, sim, tape, tapes, g
    torch.cuda.empty_cache()
    # the same gradient with every step's moments kept (no checkpoints, no
    # recompute) when the tape fits in device memory
    run2 = adjoint.GradientRunner(adjoint.GradientSpec(n=n, steps=steps, tile=tile, fuse=fuse,
                                                       store_all=None), rho0)
    store_all = {"used": run2.store_all, "tape_GiB": round(steps * 32 * n * n / 2**30, 1)}
    if run2.store_all:
        r2 = rho0.clone().requires_grad_(True)

        def grad2():
            J = adjoint.LBRSFunction.apply(r2, run2)
            J.backward()

        grad2()
        t_sa = _time_ms(grad2)
        store_all.update(gradient_ms=round(t_sa, 1),
                         gradient_over_forward_run=round(t_sa / t_fwd, 3),
                         speedup_over_checkpointed=round(t_grad / t_sa, 3))
        del r2
    run2.close()
    del run2
    torch.cuda.empty_cache()
    cells = n * n
    return {"n": n, "steps": steps, "segment": seg,
            "tile_rows": best["rows"], "waves_per_block": best["wpb"], "alternate": best["alt"],
            "steps_per_launch": kf,
            # per step: forward, taped recompute and adjoint, in the tuned
            # (fused) form and as single steps
            "forward_step_ms": round(fwd, 4), "tape_step_ms": round(tapk, 4),
            "adjoint_step_ms": round(adjk, 4),
            "adjoint_over_forward": round((tapk + adjk) / fwd, 3),
            # the timed forms' own bytes per lattice update: k fused adjoint
            # steps (256 + 32 k) / k (fbar^{n+k} 128 + k tapes 32 + fbar^n
            # 128 per k updates), the single adjoint 288 (128 + 32 + 128)
            "adjoint_step_bytes_per_lup": round((256 + 32 * kf) / kf, 2),
            "adjoint_step_GBs": round((256 + 32 * kf) / kf * cells / (adjk * 1e-3) / 1e9, 1),
            "adjoint_step_single_equivalent_GBs": round(288 * cells / (adjk * 1e-3) / 1e9, 1),
            "two_per_launch": pair,
            "single": {"forward_step_ms": round(fwd1, 4), "tape_step_ms": round(tap, 4),
                       "adjoint_step_ms": round(adj, 4),
                       "adjoint_over_forward": round((tap + adj) / fwd1, 3),
                       "adjoint_step_GBs": round(288 * cells / (adj * 1e-3) / 1e9, 1)},
            "gradient_ms": round(t_grad, 1), "forward_run_ms": round(t_fwd, 1),
            "gradient_over_forward_run": round(t_grad / t_fwd, 3),
            "gradient_store_all": store_all}


def batched_2d(k=12, ws=None):
    """128 seeded periodic domains (sides 256..2048): one launch per step (or
    per 2, 3, 4 fused steps) for all domains, against the same domains
    stepped one at a time in the same forms; the fastest fused form is the
    main figure."""
    import torch

    from paper_1504_07034_amd import lbrs
    from paper_1504_07034_amd import workloads as wl

    ws = ws or wl.domain_batch(128, seed=0)
    doms = [lbrs.make_params(lbrs.LBRS_D2Q4, w.nx, w.ny, w.domain, w.gamma, w.omega, w.cfl,
                             w.sides, lbrs.LBRS_LAMBDA_FROZEN_INIT, 0.0, lbrs.LBRS_LAYOUT_ROWS)
            for w in ws]
    Us = []
    for w, p in zip(ws, doms):
        Wt = torch.from_numpy(w.W).cuda()
        U = torch.empty_like(Wt)
        lbrs.lbrs_prim_to_cons(p, Wt, U)
        Us.append(U)
    forms = (1, 2, 3, 4)
    B = lbrs.Batch2D(doms)
    B.init(torch.cat([U.reshape(4, -1) for U in Us], dim=1))
    ms_b = {}
    for fuse in forms:
        B.set_fusion(fuse)
        B.step(fuse)
        ms_b[fuse] = _time_ms(lambda: B.step(k)) / k
    total = B.total
    B.close()
    del B
    torch.cuda.empty_cache()
    # the same domains one at a time, in the same forms
    ms_s = {f: 0.0 for f in forms}
    for w, U in zip(ws, Us):
        sim = lbrs.Sim(lbrs.LBRS_D2Q4, w.nx, w.ny, domain=w.domain, gamma=w.gamma, cfl=w.cfl,
                       bc=w.sides, lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT,
                       layout=lbrs.LBRS_LAYOUT_ROWS)
        sim.init(U)
        for fuse in forms:
            sim.set_fusion(fuse)
            sim.step(fuse)
            ms_s[fuse] += _time_ms(lambda: sim.step(k)) / k
        sim.close()
    best = min(forms[1:], key=lambda f: ms_b[f])

    def form(f):
        return {"batched_ms_per_step": round(ms_b[f], 3), "MLUPS": round(total / ms_b[f] / 1e3, 1),
                "sequential_ms_per_step": round(ms_s[f], 3), "speedup": round(ms_s[f] / ms_b[f], 3),
                "GBs": round(256.0 / f * total / (ms_b[f] * 1e-3) / 1e9, 1)}

    return dict({"domains": len(ws), "cells": int(total), "steps_per_launch": best}, **form(best),
                forms={str(f): form(f) for f in forms})


def batched_grad_2d(steps=1000, subset=16, mem_frac=0.6, ws=None, fuse=4):
    """Batched forward+adjoint: dJ_d/dU0 of the 128 seeded periodic domains after
    1000 steps (frozen lattice speeds, J over [0.7,0.8]^2), sqrt(T) checkpointed.
    The pools run in memory waves, each wave one captured hipGraph (capture
    included in the time: every wave runs once); against the single-domain
    checkpointed path run domain by domain on a seeded subset."""
    import math

    import numpy as np
    import torch

    from paper_1504_07034_amd import adjoint, lbrs
    from paper_1504_07034_amd import workloads as wl

    ws = ws or wl.domain_batch(128, seed=0, steps=steps)
    # near the minimum of 128*ceil(T/s) + 32*s bytes per cell (s = 2 sqrt(T)),
    # a multiple of the steps per launch
    seg = max(fuse, round(2 * math.sqrt(steps) / fuse) * fuse)
    nck = math.ceil(steps / seg)
    per_cell = 8 * (16 * (nck + 4) + 4 * (seg + 2))  # ckpt, f0 f1 fbar work, tape, U0 Ubar0

    def doms_of(sel):
        return [lbrs.make_params(lbrs.LBRS_D2Q4, w.nx, w.ny, w.domain, w.gamma, w.omega, w.cfl,
                                 w.sides, lbrs.LBRS_LAMBDA_FROZEN_INIT, 0.0,
                                 lbrs.LBRS_LAYOUT_ROWS) for w in sel]

    def U0_of(sel, doms):
        out = []
        for w, p in zip(sel, doms):
            Wt = torch.from_numpy(w.W).cuda()
            U = torch.empty_like(Wt)
            lbrs.lbrs_prim_to_cons(p, Wt, U)
            out.append(U.reshape(4, -1))
        return torch.cat(out, dim=1).contiguous()

    def run_wave(sel, replays=0, seg=seg, nck=nck, bufs=None):
        # nck = 0: one segment, every step's moments taped (no checkpoints);
        # bufs: flat buffers reused across waves (else allocated here)
        doms = doms_of(sel)
        B = lbrs.Batch2D(doms)
        U0 = U0_of(sel, doms)
        B.init(U0)
        B.set_fusion(fuse)
        B.set_window(0.7, 0.8)
        T = B.total
        if bufs is None:
            bufs = alloc(T, seg, nck)
        ck = bufs["ck"][:max(1, nck * 16 * T)]
        tp = bufs["tp"][:seg * 4 * T]
        fb = bufs["fb"][:16 * T]
        wk = bufs["wk"][:16 * T]
        Ub = bufs["Ub"][:4 * T].view(4, T)
        J = torch.zeros(len(sel), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        t0 = time.perf_counter()
        B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=True)  # capture + launch
        host_ms = (time.perf_counter() - t0) * 1e3
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = B.state()
        assert st["rc"] == 0 and bool(torch.isfinite(J).all()) and bool(torch.isfinite(Ub).all())
        Jh = J.cpu().numpy()
        replay_ms = None
        if replays:
            replay_ms = _time_ms(lambda: B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub,
                                                    use_graph=True), replays)
        B.close()
        del B, ck, tp, fb, wk, Ub, U0, bufs
        return ms, T, Jh, host_ms, replay_ms

    def alloc(cells, seg, nck):
        def z(k):
            return torch.empty(max(1, k), dtype=torch.float64, device="cuda")
        return {"ck": z(nck * 16 * cells), "tp": z(seg * 4 * cells), "fb": z(16 * cells),
                "wk": z(16 * cells), "Ub": z(4 * cells)}

    def run_all(per_cell, name, seg=seg, nck=nck):
        torch.cuda.empty_cache()
        free = torch.cuda.mem_get_info()[0]
        cap = int(mem_frac * free / per_cell)
        order = sorted(range(len(ws)), key=lambda b: -ws[b].nx * ws[b].ny)
        waves, cur, cells = [], [], 0
        for b in order:  # first fit into the current wave, largest domains first
            c = ws[b].nx * ws[b].ny
            if cur and cells + c > cap:
                waves.append(cur)
                cur, cells = [], 0
            cur.append(b)
            cells += c
        waves.append(cur)
        # one set of buffers for the largest wave, reused by every wave
        bufs = alloc(max(sum(ws[b].nx * ws[b].ny for b in wv) for wv in waves), seg, nck)
        total_ms, total_cells, wave_info = 0.0, 0, []
        for i, wv in enumerate(waves):
            ms, T, _, host_ms, _ = run_wave([ws[b] for b in wv], seg=seg, nck=nck, bufs=bufs)
            total_ms += ms
            total_cells += T
            wave_info.append({"domains": len(wv), "cells": int(T), "ms": round(ms, 1),
                              "capture_ms": round(host_ms, 1)})
            print(f"bench: batched_grad_2d {name} wave {i + 1}/{len(waves)}: {ms:.0f} ms",
                  file=sys.stderr, flush=True)
        del bufs
        torch.cuda.empty_cache()
        return total_ms, total_cells, wave_info

    total_ms, total_cells, wave_info = run_all(per_cell, "checkpointed")
    # the same gradients with one segment: every step's moments taped in the
    # forward sweep, no checkpoints, no recompute (more, smaller waves)
    per_cell_w = 8 * (16 * 4 + 4 * (steps + 2))
    ms_w, _, info_w = run_all(per_cell_w, "whole tape", seg=steps, nck=0)

    rng = np.random.default_rng(2)
    sub = [ws[b] for b in sorted(rng.choice(len(ws), size=subset, replace=False))]
    ms_first, T_b, J_b, _, ms_b = run_wave(sub, replays=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J_s = []
    for w, p in zip(sub, doms_of(sub)):
        sim = lbrs.Sim(lbrs.LBRS_D2Q4, w.nx, w.ny, domain=w.domain, gamma=w.gamma, omega=w.omega,
                       cfl=w.cfl, bc=w.sides, lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT,
                       layout=lbrs.LBRS_LAYOUT_ROWS)
        Wt = torch.from_numpy(w.W).cuda()
        U0 = torch.empty_like(Wt)
        lbrs.lbrs_prim_to_cons(p, Wt, U0)
        sim.init(U0)
        sim.set_fusion(fuse)
        cells = w.nx * w.ny
        ck = torch.empty(nck * 16 * cells, dtype=torch.float64, device="cuda")
        tp = torch.empty(seg * 4 * cells, dtype=torch.float64, device="cuda")
        fb = torch.empty(16 * cells, dtype=torch.float64, device="cuda")
        wk = torch.empty_like(fb)
        J = torch.zeros(1, dtype=torch.float64, device="cuda")
        Ub = torch.empty_like(U0)
        lbrs.lbrs_forward_checkpointed(sim.ctx, steps, seg, ck)
        i0, i1 = adjoint.window_range(w.nx, 0.7, 0.8)
        lbrs.lbrs_window_objective(sim.ctx, i0, i1, i0, i1, J, fb)
        lbrs.lbrs_backward_checkpointed(sim.ctx, steps, seg, ck, tp, fb, wk)
        lbrs.lbrs_adjoint_init(sim.ctx, fb, U0, Ub)
        J_s.append(J.item())
        sim.close()
        del ck, tp, fb, wk
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3
    rel = float(np.max(np.abs(np.asarray(J_s) - J_b) / np.abs(np.asarray(J_s))))
    lups = total_cells * steps
    return {"domains": len(ws), "cells": int(total_cells), "steps": steps, "segment": seg,
            "steps_per_launch": fuse, "waves": wave_info, "ms": round(total_ms, 1),
            "forward_equiv_MLUPS": round(lups / total_ms / 1e3, 1),
            "whole_tape": {"ms": round(ms_w, 1), "waves": len(info_w),
                           "bytes_per_cell": per_cell_w,
                           "speedup_over_checkpointed": round(total_ms / ms_w, 3)},
            "subset": {"domains": subset, "cells": int(T_b),
                       "batched_first_call_ms": round(ms_first, 1),
                       "batched_replay_ms": round(ms_b, 1),
                       "sequential_ms": round(ms_s, 1), "speedup": round(ms_s / ms_b, 3),
                       "speedup_incl_capture": round(ms_s / ms_first, 3),
                       "J_max_rel_diff": rel}}


def dirichlet_2d(nx=12288, ny=4096, steps=200, warmup=20):
    """The oblique-shock reflection (prescribed inflow and post-shock sides,
    free-slip wall; omega = 1.8) at nx x ny: the step kernel with Dirichlet
    ghosts, autotuned launch shape, HIP events."""
    import torch

    from paper_1504_07034_amd import autotune, lbrs
    from paper_1504_07034_amd import workloads as wl

    w = wl.oblique_shock(nx, ny, omega=1.8)
    sim = lbrs.Sim(w.model, nx, ny, domain=w.domain, gamma=w.gamma, omega=w.omega, cfl=w.cfl,
                   bc=w.sides, layout=lbrs.LBRS_LAYOUT_ROWS, dirichlet_W=w.dirichlet_W)
    U0 = sim.prim_to_cons(torch.from_numpy(w.W))
    del w
    sim.init(U0)
    sim.step(5)
    best = autotune.tune(sim, use_cache=False)
    sim.init(U0)
    sim.set_tile(best["rows"], best["wpb"], best["alt"])
    sim.step(warmup)
    ms = _time_ms(lambda: sim.step(steps)) / steps
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == warmup + steps
    sim.close()
    cells = nx * ny
    gbs = BYTES_PER_LUP * cells / (ms * 1e-3) / 1e9
    return {"workload": "oblique shock reflection, Dirichlet inflow/top, wall below",
            "nx": nx, "ny": ny, "omega": 1.8, "tile_rows": best["rows"],
            "waves_per_block": best["wpb"], "alternate": best["alt"],
            "ms_per_step": round(ms, 4), "MLUPS": round(cells / ms / 1e3, 1),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def bodies_2d(nx=7680, ny=2560, steps=200, warmup=20):
    """Solid bodies: the forward-facing step case (Mach 3 channel, inflow
    side, walls, the step as a mask of solid cells) at nx x ny with the body
    kernel (2-byte node code per cell on top of the 256 B of populations;
    solid cells are streamed like the others), autotuned launch shape, HIP
    events.  Beside it, the wall-clock time of whole runs of the three Sec. III
    body cases at the paper's grids (launch-bound: a few ten thousand cells)."""
    import torch

    from paper_1504_07034_amd import autotune, lbrs
    from paper_1504_07034_amd import workloads as wl

    def make(w):
        return lbrs.Sim(w.model, w.nx, w.ny, domain=w.domain, gamma=w.gamma, omega=w.omega,
                        cfl=w.cfl, bc=w.sides, layout=lbrs.LBRS_LAYOUT_ROWS,
                        dirichlet_W=w.dirichlet_W, solid=w.solid)

    w = wl.forward_step(nx, ny, omega=1.6)
    solid_frac = float(w.solid.mean())
    sim = make(w)
    U0 = sim.prim_to_cons(torch.from_numpy(w.W))
    del w
    sim.init(U0)
    sim.step(5)
    best = autotune.tune(sim, use_cache=False)
    sim.init(U0)
    sim.set_tile(best["rows"], best["wpb"], 0)
    sim.step(warmup)
    ms = _time_ms(lambda: sim.step(steps)) / steps
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == warmup + steps
    sim.close()
    del U0
    cells = nx * ny
    bytes_per_lup = BYTES_PER_LUP + 2
    gbs = bytes_per_lup * cells / (ms * 1e-3) / 1e9
    out = {"workload": "forward-facing step, Mach 3, step as solid cells",
           "nx": nx, "ny": ny, "omega": 1.6, "solid_fraction": round(solid_frac, 4),
           "tile_rows": best["rows"], "waves_per_block": best["wpb"],
           "ms_per_step": round(ms, 4), "MLUPS": round(cells / ms / 1e3, 1),
           "fluid_MLUPS": round(cells * (1.0 - solid_frac) / ms / 1e3, 1),
           "bytes_per_lup": bytes_per_lup, "GBs": round(gbs, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    runs = {}
    for w in (wl.forward_step(), wl.ramp(), wl.shock_diffraction()):
        sim = make(w)
        rec = {"grid": f"{w.nx}x{w.ny}", "t_end": w.t_end}
        for label in ("default", "tuned"):
            sim.init_primitive(w.W)
            if label == "tuned":
                sim.step(20)
                best = autotune.tune(sim, w.t_end, use_cache=False)
                rec["tile_rows"], rec["waves_per_block"] = best["rows"], best["wpb"]
            else:
                sim.step(10)  # first launches
            sim.init_primitive(w.W)
            if label == "tuned":
                sim.set_tile(best["rows"], best["wpb"], 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.run(w.t_end, chunk=4000)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            assert st["rc"] == 0 and st["t"] == w.t_end
            rec["steps"] = st["nsteps"]
            rec[f"run_ms_{label}"] = round(sec * 1e3, 1)
        runs[w.name] = rec
        sim.close()
    out["paper_grids"] = runs
    return out


def scalar_laws(n2=8192, n1=1 << 26, steps=200, warmup=20):
    """Scalar LBRS: the 2D Burgers case 1 (prescribed sides) at n2 x n2 on
    D2Q4 (64 B per lattice update: 4 populations in and out) with an autotuned
    launch shape, and the 1D Burgers shock tube on n1 cells (the 2D case's
    cell count), D1Q2 (32 B per update), planar 1D layout (and the blocked one
    for comparison).  HIP events."""
    import torch

    from paper_1504_07034_amd import autotune, lbrs
    from paper_1504_07034_amd import workloads as wl

    out = {}
    w = wl.spekreijse(1, n2)
    sim = lbrs.Sim(w.model, n2, n2, domain=w.domain, omega=w.omega, cfl=w.cfl, bc=w.sides,
                   layout=lbrs.LBRS_LAYOUT_ROWS, dirichlet_W=w.dirichlet_W,
                   law=lbrs.LBRS_LAW_SCALAR, scalar_flux=w.quad)
    U0 = sim.prim_to_cons(torch.from_numpy(w.W))
    sim.init(U0)
    sim.step(5)
    best = autotune.tune(sim, use_cache=False, alts=(1,))
    sim.init(U0)
    sim.set_tile(best["rows"], best["wpb"])
    sim.step(warmup)
    ms = _time_ms(lambda: sim.step(steps)) / steps
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == warmup + steps
    sim.close()
    del U0
    gbs = 64 * n2 * n2 / (ms * 1e-3) / 1e9
    out["burgers_2d"] = {"workload": "2D Burgers case 1 (Dirichlet sides), D2Q4", "n": n2,
                         "tile_rows": best["rows"], "waves_per_block": best["wpb"],
                         "ms_per_step": round(ms, 4), "MLUPS": round(n2 * n2 / ms / 1e3, 1),
                         "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    torch.cuda.empty_cache()
    w = wl.burgers_riemann(n1, 1.0, 0.0, t_end=10.0)
    blocked_ms = None
    for layout in (lbrs.LBRS_LAYOUT_ROWS, lbrs.LBRS_LAYOUT_PLANAR):
        sim = lbrs.Sim(w.model, n1, 1, domain=w.domain, omega=w.omega, cfl=w.cfl, bc=w.sides,
                       law=lbrs.LBRS_LAW_SCALAR, scalar_flux=w.quad, layout=layout)
        sim.init_primitive(w.W)
        sim.step(warmup, w.t_end)
        ms = _time_ms(lambda: sim.step(steps, w.t_end)) / steps
        st = sim.state()
        assert st["rc"] == 0 and st["nsteps"] == warmup + steps
        if layout == lbrs.LBRS_LAYOUT_ROWS:
            blocked_ms = ms
            sim.close()
    sim.close()
    gbs = 32 * n1 / (ms * 1e-3) / 1e9
    gbs_b = 32 * n1 / (blocked_ms * 1e-3) / 1e9
    out["burgers_1d"] = {"workload": "1D Burgers shock tube, D1Q2", "n": n1, "layout": "planar",
                         "ms_per_step": round(ms, 4), "MLUPS": round(n1 / ms / 1e3, 1),
                         "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "blocked": {"ms_per_step": round(blocked_ms, 4),
                                     "frac": round(gbs_b / HBM_PEAK_GBS, 4)}}
    return out


def euler_1d_long(n=1 << 24, steps=200, warmup=20):
    """The Euler shock tube (Sod) on n cells with D1Q3: the one-launch-per-step
    1D kernel (512-cell LDS tiles), 144 B per lattice update, in the blocked
    population layout (the planes of each 64-cell block contiguous) and, for
    comparison, the planar one."""
    import torch

    from paper_1504_07034_amd import lbrs
    from paper_1504_07034_amd import workloads as wl

    w = wl.sod(n, t_end=0.2)
    out = {"workload": "Sod shock tube, D1Q3", "n": n}
    for layout in (lbrs.LBRS_LAYOUT_PLANAR, lbrs.LBRS_LAYOUT_ROWS):
        sim = lbrs.Sim(w.model, n, 1, domain=w.domain, gamma=w.gamma, omega=w.omega, cfl=w.cfl,
                       layout=layout)
        sim.init_primitive(w.W)
        sim.step(warmup, 0.2)
        ms = _time_ms(lambda: sim.step(steps, 0.2)) / steps
        st = sim.state()
        assert st["rc"] == 0 and st["nsteps"] == warmup + steps
        sim.close()
        torch.cuda.empty_cache()
        gbs = 144 * n / (ms * 1e-3) / 1e9
        if layout == lbrs.LBRS_LAYOUT_PLANAR:
            out["planar"] = {"ms_per_step": round(ms, 4), "frac": round(gbs / HBM_PEAK_GBS, 4)}
        else:
            out.update({"layout": "blocked", "ms_per_step": round(ms, 4),
                        "MLUPS": round(n / ms / 1e3, 1), "GBs": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4)})
    return out


def copy_bandwidth(src, dst, reps=20):
    """Measured copy reference on this GPU: torch's device-to-device copy of
    one population buffer (read + write counted), HIP events."""
    dst.copy_(src)
    ms = _time_ms(lambda: dst.copy_(src), reps)
    nbytes = 2 * src.numel() * src.element_size()
    return {"kind": "torch copy_ of one population buffer", "bytes": nbytes,
            "ms": round(ms, 4), "GBs": round(nbytes / (ms * 1e-3) / 1e9, 1)}


def slab_step(steps=200, warmup=20):
    """One GPU's share of an eight-way slab decomposition of the 4096^2
    four-quadrant problem: the step on a 4096 x 512 slab through the middle of
    the domain (own transmissive sides; no halo exchange), launch shape
    autotuned for the slab."""
    import torch

    from paper_1504_07034_amd import autotune, lbrs
    from paper_1504_07034_amd import workloads as wl

    n, h, y0 = 4096, 512, 1792
    w = wl.riemann2d(n)
    W = torch.from_numpy(w.W[:, y0:y0 + h, :].copy()).cuda()
    sim = lbrs.Sim(w.model, n, h, domain=(0.0, 1.0, y0 / n, (y0 + h) / n), gamma=w.gamma,
                   omega=w.omega, cfl=w.cfl, bc=w.sides, layout=lbrs.LBRS_LAYOUT_ROWS)
    U0 = sim.prim_to_cons(W)
    del w, W
    sim.init(U0)
    sim.step(5, 0.3)
    best = autotune.tune(sim, 0.3, use_cache=False, rows=(0, 16, 32, 64, 128))
    sim.init(U0)
    sim.set_tile(best["rows"], best["wpb"], best["alt"])
    sim.set_fusion(best["fuse"])
    sim.step(warmup, 0.3)
    ms = _time_ms(lambda: sim.step(steps, 0.3)) / steps
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == warmup + steps
    sim.close()
    cells = n * h
    bpl = form_bytes(best["fuse"])
    gbs = bpl * cells / (ms * 1e-3) / 1e9
    return {"nx": n, "ny": h, "tile_rows": best["rows"], "waves_per_block": best["wpb"],
            "alternate": best["alt"], "steps_per_launch": best["fuse"], "ms_per_step": round(ms, 4),
            "MLUPS": round(cells / ms / 1e3, 1), "bytes_per_lup": round(bpl, 2),
            "GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "single_step_equivalent_GBs": round(BYTES_PER_LUP * cells / (ms * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--rows", type=int, default=-1,
                    help="rows per tile (0 = automatic); default: autotune")
    ap.add_argument("--wpb", type=int, default=4)
    ap.add_argument("--alt", type=int, default=1, choices=[0, 1],
                    help="march odd row segments upwards (with --rows >= 0)")
    ap.add_argument("--layout", type=int, default=1, help="0 planar, 1 row-interleaved")
    ap.add_argument("--fuse", type=int, default=1, choices=[1, 2, 3, 4],
                    help="time steps per launch (with --rows >= 0; autotuned otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and adjoint figures reported beside the main value")
    ap.add_argument("--only", choices=["adjoint", "adjoint_steps", "batch1d", "batch1d_run",
                                       "batch2d", "batchgrad", "dirichlet", "scalar", "euler1d",
                                       "slab", "bodies", "sod"],
                    default=None,
                    help="run only one of the secondary measurements and print it (profiling)")
    ap.add_argument("--mid", type=int, default=-1,
                    help="first step of the timed window (default: the middle of a whole run, "
                         "which is then run first); with --rows >= 0 nothing else runs before "
                         "the window (profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, run one plain copy of the populations (lbrs_get_f: "
                         "16 planes read and written) as a known-size reference for counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1504_07034_amd import autotune, lbrs
    from paper_1504_07034_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.only:
        fn = {"adjoint": adjoint_2d, "adjoint_steps": lambda: adjoint_2d(steps_only=True),
              "batch1d": batched_1d, "batch2d": batched_2d,
              "batchgrad": batched_grad_2d, "dirichlet": dirichlet_2d,
              "scalar": scalar_laws, "euler1d": euler_1d_long, "slab": slab_step,
              "bodies": bodies_2d,
              "batch1d_run": lambda: batched_1d(chunks=(3070,), sequential=False),
              "sod": sod_400}[args.only]
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

    shape = {"rows": args.rows, "wpb": args.wpb, "alt": args.alt, "fuse": args.fuse}
    single = None  # the best single-step shape, when the fused one wins
    stream = torch.cuda.current_stream()

    def use(sh):
        sim.set_tile(sh["rows"], sh["wpb"], sh["alt"])
        sim.set_fusion(sh["fuse"])

    def whole_run(sh):
        """The whole run from t = 0 to t_end, timed in calls of 1000 steps."""
        sim.init(U0)
        use(sh)
        total_ms, steps = 0.0, 0
        while True:
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sim.step(1000, t_end)
            e1.record(stream)
            torch.cuda.synchronize()
            total_ms += e0.elapsed_time(e1)
            st = sim.state()
            if st["rc"] != 0:
                raise RuntimeError(f"whole run failed: {st}")
            if st["t"] >= t_end:
                steps = st["nsteps"]
                break
        out = {"steps": steps, "ms": round(total_ms, 1), "ms_per_step": round(total_ms / steps, 4),
               "MLUPS": round(n * n * steps / (total_ms * 1e-3) / 1e6, 1)}
        if sh["fuse"] >= 2:
            out["launches"] = sim.pair_stats()
        return out

    # The timed window sits in the middle of the run to t_end: the whole run
    # in a default shape gives its step count, then the state at the window's
    # start is kept, and the tuner and every timed form start from it.
    default = dict(shape) if args.rows >= 0 else {"rows": 0, "wpb": 6, "alt": 0, "fuse": 2}
    if args.mid >= 0:
        first, n_total, mid = None, None, args.mid
    else:
        first = whole_run(default)
        n_total = first["steps"]
        mid = max(0, (n_total - args.warmup - args.steps) // 2)
    sim.init(U0)
    use(default)
    if mid:
        sim.step(mid, t_end)
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == mid, st
    f_mid, t_mid = sim.get_f(), st["t"]
    whole = f" ({first['ms_per_step']} ms/step, {first['MLUPS']} MLUPS)" if first else ""
    print(f"bench: whole run {n_total} steps{whole}; window from step {mid} (t = {t_mid:.5f})",
          file=sys.stderr, flush=True)

    if args.rows < 0:  # autotune the launch shape from the window's start (untimed)
        # automatic row segments (one balanced round of the resident waves);
        # single and fused launches, every (waves per workgroup, march order)
        # candidate
        best = autotune.tune(sim, t_end, steps=20, use_cache=False, rows=(0,))
        shape = {k: best[k] for k in ("rows", "wpb", "alt", "fuse")}
        print("autotune: " + ", ".join(f"({c['rows']},{c['wpb']},{c['alt']},{c['fuse']}) "
                                       f"{c['ms']:.3f} ms" for c in best["candidates"]),
              file=sys.stderr, flush=True)
        if shape["fuse"] >= 2:
            s1 = min((c for c in best["candidates"] if c["fuse"] == 1), key=lambda c: c["ms"])
            single = {k: s1[k] for k in ("rows", "wpb", "alt", "fuse")}

    def timed_window(sh, steps, warmup):
        """ms per step over `steps` steps after `warmup` untimed ones, from the
        state at step `mid` of the run; the steps taken (fewer only where the
        run reaches t_end first)."""
        sim.set_f(f_mid, t_mid, mid)
        use(sh)
        if warmup:
            sim.step(warmup, t_end)
        st0 = sim.state()
        c0 = sim.pair_stats() if sh["fuse"] >= 2 else None
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps, t_end)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st1 = sim.state()
        done = st1["nsteps"] - st0["nsteps"]
        if st1["rc"] != 0 or (done != steps and st1["t"] < t_end) or done < 1:
            raise RuntimeError(f"timed steps did not all run: {st0} -> {st1}")
        if c0 is not None:
            c1 = sim.pair_stats()
            window_launches[sh["fuse"], sh["wpb"], sh["alt"]] = {k: c1[k] - c0[k] for k in c1}
        return ms, done

    window_launches = {}

    def roofline(sh, ms, done):
        """The kernel's own algorithmic bytes: 256 B per lattice update for a
        single step (16 FP64 populations in, 16 out), 256/k B for k fused
        steps (f^n in and f^{n+k} out per k updates: the states between never
        leave the registers); per launch: the step-kernel launches the window
        enqueued (a call of K single steps enqueues K; a fused call counts its
        own, those that found the work done included)."""
        bpl = BYTES_PER_LUP / sh["fuse"]
        cells = n * n
        alg = bpl * cells * done
        launches = args.steps
        achieved = alg / (ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
             "traffic": traffic_bytes(sh, args.layout),
             "kernel": "step2d_pair" if sh["fuse"] >= 2 else "step2d_d2q4",
             "bytes_per_lup": round(bpl, 2), "launches": launches,
             "avg_launch_ms": round(ms / launches, 5),
             "alg_bytes_per_launch": round(alg / launches),
             # the single step's 256 B per update over the same time
             "single_step_equivalent_GBs": round(256 * cells * done / (ms * 1e-3) / 1e9, 1)}
        if sh["fuse"] >= 2:
            # what the window's launches did: pairs that stood, pairs rolled
            # back, bound-only passes, single steps, predictions of the next
            # bound made / standing / rolled back, cells evaluated for them;
            # the launches that did work (the others exit at once) and their
            # mean time, prediction kernels and gaps included
            lc = window_launches.get((sh["fuse"], sh["wpb"], sh["alt"]))
            r["launch_counts"] = lc
            if lc:
                active = lc["pairs"] + lc["rejected"] + lc["bound_only"] + lc["single"]
                r["active_launches"] = active
                r["avg_active_launch_ms"] = round(ms / max(active, 1), 5)
                launches = max(lc["enqueued"], 1)
                r["launches"] = launches
                r["avg_launch_ms"] = round(ms / launches, 5)
                r["alg_bytes_per_launch"] = round(alg / launches)
                r["traffic"] = traffic_bytes(sh, args.layout, active / launches)
            else:
                r["traffic"] = None
        return r

    ms_win, done = timed_window(shape, args.steps, args.warmup)
    ms_per_step = ms_win / done

    if args.calibrate_copy:
        f_copy = sim.get_f()
        torch.cuda.synchronize()
        del f_copy
    copy_ref = None if args.no_extras else copy_bandwidth(sim.f0, sim.f1)

    cells = n * n
    mlups = cells / (ms_per_step * 1e-3) / 1e6
    rf = roofline(shape, ms_win, done)
    rec = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": done,
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
                   "lambda": "per step", "window_first_step": mid, "run_steps": n_total,
                   "tile_rows": shape["rows"], "waves_per_block": shape["wpb"],
                   "alternate_march": shape["alt"], "steps_per_launch": shape["fuse"],
                   "layout": "row-interleaved" if args.layout == 1 else "planar"},
        "roofline": rf,
    }
    if not args.no_extras:
        full = {"default_shape": dict(default, **first)} if first else {}
        if single is not None:
            ms1, done1 = timed_window(single, args.steps, args.warmup)
            rec["single_step"] = {
                "tile_rows": single["rows"], "waves_per_block": single["wpb"],
                "alternate_march": single["alt"], "ms_per_step": round(ms1 / done1, 4),
                "MLUPS": round(cells * done1 / (ms1 * 1e-3) / 1e6, 1),
                "roofline": roofline(single, ms1, done1)}
            full["fused"] = whole_run(shape)
            full["single"] = whole_run(single)
        else:
            full["tuned"] = whole_run(shape)
        rec["full_run"] = full
    if copy_ref is not None:
        copy_ref["frac_of_copy"] = round(rf["achieved"] / copy_ref["GBs"], 4)
        rec["copy_reference"] = copy_ref
    del f_mid
    sim.close()
    del U0, sim
    torch.cuda.empty_cache()

    def stage(name, fn):
        rec[name] = fn()
        torch.cuda.empty_cache()
        print(f"bench: {name} done", file=sys.stderr, flush=True)

    if not args.no_extras:
        stage("sod_400", sod_400)
        stage("slab_4096x512", slab_step)
        stage("dirichlet_2d", dirichlet_2d)
        stage("bodies_2d", bodies_2d)
        stage("scalar_laws", scalar_laws)
        stage("euler_1d_long", euler_1d_long)
        stage("adjoint_2d", adjoint_2d)
        stage("batched_1d", batched_1d)
        ws = wl.domain_batch(128, seed=0, steps=1000)
        stage("batched_2d", lambda: batched_2d(ws=ws))
        stage("batched_grad_2d", lambda: batched_grad_2d(ws=ws))
        del ws
    if not args.no_cpu_baseline:
        stage("cpu_baseline", cpu_baseline)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
