"""Autotuner for the launch shape of the 2D step kernel.

Candidates are (rows_per_tile, waves_per_block, alternate, fuse) tuples;
rows_per_tile = 0 is the library's automatic choice (one balanced round of the
resident waves), alternate = 1 marches odd row segments upwards (same results,
different memory order; a domain with a solid body marches one way only),
fuse = 2, 3 or 4 takes that many fused steps per launch (2D Euler without body or
Dirichlet side; such launches march one way).  Candidates are compared in time per step.
Each candidate is timed with HIP events over a few steps that start from the
same checkpoint of the populations (lbrs_get_f / lbrs_set_f), so tuning does
not advance the caller's solution; the fastest few are timed again over four
times as many steps before one is chosen.  The best shape is applied to the context
and cached per (device, model, nx, ny, side conditions, body or not) in a
JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import lbrs

CACHE = os.environ.get("LBRS_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "lbrs_tune.json"))

DEFAULT_ROWS = (0, 32, 64, 96, 128)
DEFAULT_WPB = (4, 6, 8, 12, 16)
DEFAULT_ALT = (0, 1)
# Grids up to SMALL_CELLS cells are latency-bound (a step is a chain of a few
# row latencies): short row segments and small workgroups are candidates.
SMALL_CELLS = 1 << 20
SMALL_ROWS = (0, 1, 2, 3, 4, 6, 8)
SMALL_WPB = (1, 2, 4, 8)


def _key(sim: "lbrs.Sim") -> str:
    p = sim.p
    name = torch.cuda.get_device_name(sim.device)
    body = "|body" if getattr(sim, "body", False) else ""
    return f"{name}|m{p.model}|{p.nx}x{p.ny}|bc{tuple(p.bc)}{body}|lm{p.lambda_mode}|v4"


def _load_cache() -> dict:
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as fh:
            json.dump(c, fh, indent=1, sort_keys=True)
    except OSError:
        pass


def time_shape(sim: "lbrs.Sim", rows: int, wpb: int, steps: int, f0: torch.Tensor,
               t0: float, n0: int, t_end: float, alternate: int = 1, fuse: int = 1) -> float:
    """Milliseconds per step of one launch shape, from the checkpoint (f0, t0, n0)."""
    sim.set_tile(rows, wpb, alternate)
    sim.set_fusion(fuse)
    sim.set_f(f0, t0, n0)
    sim.step(2, t_end)  # warm the shape
    sim.set_f(f0, t0, n0)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps, t_end)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(sim: "lbrs.Sim", t_end: float = float("inf"), steps: int = 10, rows=None,
         wpbs=None, alts=DEFAULT_ALT, use_cache: bool = True,
         verbose: bool = False, confirm: int = 4, fuses=None) -> dict:
    """Pick and apply the fastest 2D launch shape for `sim` (already initialised).
    rows / wpbs default to the candidate sets for the grid's size; fuses to
    (1, 2, 3, 4) where fused launches are available."""
    small = sim.nx * sim.ny <= SMALL_CELLS
    if rows is None:
        rows = SMALL_ROWS if small else DEFAULT_ROWS
    if wpbs is None:
        wpbs = SMALL_WPB if small else DEFAULT_WPB
    key = _key(sim)
    if getattr(sim, "body", False):
        alts = (0,)
    if fuses is None:
        fuses = (1, 2, 3, 4) if getattr(sim, "fusable", False) else (1,)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]
        sim.set_tile(best["rows"], best["wpb"], best.get("alt"))
        sim.set_fusion(best.get("fuse", 1))
        return best
    st = sim.state()
    f0 = sim.get_f()
    results = []
    for fu in fuses:
        for a in (alts if fu == 1 else (0,)):
            # fused launches run at most 12 waves per group, those of three or
            # more steps 8
            for w in (wpbs if fu == 1 else [v for v in wpbs if v <= (12 if fu == 2 else 8)]):
                for r in rows:
                    ms = time_shape(sim, r, w, steps, f0, st["t"], st["nsteps"], t_end, a, fu)
                    results.append({"rows": r, "wpb": w, "alt": a, "fuse": fu, "ms": ms})
                    if verbose:
                        print(f"autotune rows={r} wpb={w} alt={a} fuse={fu}: {ms:.4f} ms/step",
                              flush=True)
    # the short timings are noisy: re-time the best few over longer runs
    finalists = sorted(results, key=lambda d: d["ms"])[:confirm]
    for d in finalists:
        d["ms_confirm"] = time_shape(sim, d["rows"], d["wpb"], 4 * steps, f0, st["t"],
                                     st["nsteps"], t_end, d["alt"], d["fuse"])
    best = min(finalists, key=lambda d: d["ms_confirm"])
    sim.set_f(f0, st["t"], st["nsteps"])
    sim.set_tile(best["rows"], best["wpb"], best["alt"])
    sim.set_fusion(best["fuse"])
    best = dict(best, candidates=results)
    if use_cache:
        cache[key] = best
        _save_cache(cache)
    return best
