"""GPU parity of the fused launches of 2, 3 and 4 steps (lbrs_set_fusion).

The fused kernel streams every row of f^{n+1} straight into the next step,
k times; with the per-step lattice speed it guesses the later steps' bounds
(predictions, else the current bound) and the next launch checks every
guess (falling back to f^n on a mismatch).  The bar is the oracle's:
max-abs <= 1e-10 on U, identical step counts, times, lattice speeds and
non-physical reports, on the shapes, sides, speed modes and omegas of the
single-step tests, plus agreement with single steps and exact step-count
semantics of every call.  The oracle's runs are kept for the session and
shared by the step counts per launch that compare against them.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import TOL, gpu_sim, max_abs, oracle_problem, report

pytestmark = pytest.mark.gpu


_ORACLE_RUNS = {}


def _oracle_run(P, w, serial=True, **kw):
    """oracle.run on the workload's initial state, kept per problem, initial
    state and stopping rule for the session (the oracle is deterministic)."""
    key = (repr(P), w.name, w.nx, w.ny, float(np.sum(w.W)), float(np.sum(w.W * w.W)),
           tuple(sorted(kw.items())), serial)
    if key not in _ORACLE_RUNS:
        U0 = oracle.prim_to_cons(P, w.W)
        _ORACLE_RUNS[key] = oracle.run(P, U0, **kw) if serial else _oracle_omp_run(P, U0, **kw)
    return _ORACLE_RUNS[key]


def _riemann_rect(nx=301, ny=201):
    """Four-quadrant states on a rectangle (dx = dy), split at its centre."""
    w = wl.riemann2d(nx)
    x = wl.centres(nx, 0.0, nx / ny)
    y = wl.centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y, indexing="xy")
    st = w.meta["states"]
    east, north = X > 0.5 * nx / ny, Y > 0.5
    W = np.empty((4, ny, nx))
    for k in range(4):
        W[k] = np.where(north, np.where(east, st["NE"][k], st["NW"][k]),
                        np.where(east, st["SE"][k], st["SW"][k]))
    return wl.Workload("riemann_rect", wl.D2Q4, nx, ny, (0.0, nx / ny, 0.0, 1.0), W, t_end=0.03)


def _fused(w, tile=None, layout=0, fuse=2, **kw):
    sim = gpu_sim(w, layout=layout, **kw)
    sim.init_primitive(w.W)
    if tile:
        sim.set_tile(*tile)
    sim.set_fusion(fuse)
    return sim


# steps per fused launch
FUSE = pytest.mark.parametrize("fuse", [2, 3, 4])


def _compare(w, t_end=math.inf, max_steps=10**9, omega=None, sides=None, lam_mode=0,
             lam_user=0.0, tile=None, layout=0, name="", chunks=None, fuse=2):
    """Run the oracle and the fused GPU path; chunks: the GPU's lbrs_step calls
    (default one call, as many steps as the oracle took, +5 when t_end stops it)."""
    P = oracle_problem(w, omega=omega, sides=sides, lam_mode=lam_mode, lam_user=lam_user)
    ref = _oracle_run(P, w, t_end=t_end, max_steps=max_steps)
    sim = _fused(w, tile=tile, layout=layout, omega=omega, sides=sides, lam_mode=lam_mode,
                 lam_user=lam_user, fuse=fuse)
    total = ref.nsteps + (5 if ref.status == 0 and ref.t >= t_end else 0)
    for k in (chunks or [total]):
        sim.step(k, t_end)
    st = sim.state()
    U = sim.moments().cpu().numpy()
    sim.close()
    err = max_abs(U, ref.U)
    report(name or w.name, steps=st["nsteps"], oracle_steps=ref.nsteps, t=st["t"], err=err,
           status=(st["rc"], ref.status), fail=(st["fail_step"], ref.fail_step))
    if ref.status == oracle.NONPHYSICAL:
        assert st["rc"] == lbrs.LBRS_E_NONPHYSICAL and st["fail_step"] == ref.fail_step
        assert st["nsteps"] == ref.nsteps
        return U, ref, st
    assert st["rc"] == 0 and ref.status == 0
    assert st["nsteps"] == ref.nsteps
    assert st["t"] == pytest.approx(ref.t, rel=1e-12, abs=0)
    if ref.nsteps:
        assert st["lambda"] == pytest.approx(ref.lam[-1], rel=1e-12)
    assert err <= TOL, err
    return U, ref, st


@pytest.mark.parametrize("tile", [(0, 4), (0, 8), (0, 1), (0, 2), (0, 6), (0, 12), (0, 16),
                                  (1, 4), (2, 2), (3, 8), (4, 1), (7, 4), (50, 2), (200, 8)])
@FUSE
def test_tile_shapes_full_run(tile, fuse):
    """Ragged strips (<= 60 columns) and row segments shorter than the two halo
    rows, every workgroup shape, the per-step speed to t_end (clipped last
    step) on a transmissive rectangle."""
    w = _riemann_rect()
    _compare(w, t_end=0.03, omega=1.4, tile=tile, name=f"fused{fuse} tile {tile}", fuse=fuse)


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.4])
@FUSE
def test_riemann_256_to_end(omega, fuse):
    """The benchmark's problem at 256^2 to t = 0.3: the bound changes at
    dozens of steps, so guesses are rejected and repeated along the way."""
    w = wl.riemann2d(256)
    _compare(w, t_end=0.3, omega=omega, name=f"fused{fuse} riemann 256 w{omega}", fuse=fuse)


def _oracle_omp_run(P, U0, **kw):
    """The oracle's OpenMP build (cells in parallel; bitwise the serial
    build's results) for the large whole runs."""
    oracle.use("omp")
    try:
        return oracle.run(P, U0, **kw)
    finally:
        oracle.use("serial")


@pytest.mark.parametrize("n", [512, 1024])
@FUSE
def test_riemann_to_end_large(n, fuse):
    """The benchmark's problem to t = 0.3 at 512^2 and 1024^2, fused launches
    with per-step speeds in the benchmark's row-interleaved layout.  The bound
    changes at nearly every step after the first few hundred, so guesses are
    rejected, bounds reduced alone and predictions taken along the way.  Two
    GPU runs: one call for the whole run (every cell at the end), and calls of
    37 steps (t and lambda after every call against the oracle's sequence, so
    a wrong dt anywhere shows in t)."""
    w = wl.riemann2d(n)
    P = oracle_problem(w)
    ref = _oracle_run(P, w, serial=False, t_end=0.3)
    assert ref.status == 0 and ref.t == 0.3
    cum = np.cumsum(ref.dt)
    for chunk in (None, 37):
        sim = _fused(w, layout=1, fuse=fuse)
        done = 0
        while done < ref.nsteps:
            k = ref.nsteps + 5 if chunk is None else min(chunk, ref.nsteps - done)
            sim.step(k, 0.3)
            done = min(done + k, ref.nsteps)
            st = sim.state()
            assert st["rc"] == 0 and st["nsteps"] == done
            assert st["t"] == pytest.approx(cum[done - 1], rel=1e-12, abs=0), done
            assert st["lambda"] == pytest.approx(ref.lam[done - 1], rel=1e-12), done
        stats = sim.pair_stats()
        U = sim.moments().cpu().numpy()
        sim.close()
        err = max_abs(U, ref.U)
        report(f"fused{fuse} riemann {n} to end, calls of {chunk or 'all'}", steps=st["nsteps"],
               oracle_steps=ref.nsteps, t=st["t"], err=err, **stats)
        assert st["t"] == ref.t
        assert err <= TOL, err
        # the path of the whole run went through checked guesses
        assert stats["rejected"] + stats["bound_only"] + stats["pred_hit"] > 0
        # every step accounted for: accepted multi-step launches count two,
        # three-step ones one more, four-step ones two more, single steps one
        steps = 2 * stats["pairs"] + stats["steps3"] + 2 * stats["steps4"] + stats["single"]
        assert steps == ref.nsteps
        assert stats["steps3"] == 0 or fuse >= 3
        assert stats["steps4"] == 0 or fuse >= 4
        # launches that did work are among those enqueued
        active = stats["pairs"] + stats["rejected"] + stats["bound_only"] + stats["single"]
        assert active <= stats["enqueued"]


@pytest.mark.parametrize("sides", [(1, 1, 1, 1), (1, 1, 0, 0), (0, 0, 1, 1)])
@FUSE
def test_periodic(sides, fuse):
    w = wl.fourier_modes(130, seed=3)
    w.sides = sides
    _compare(w, max_steps=61, omega=1.2, sides=sides, name=f"fused{fuse} periodic {sides}",
             fuse=fuse)


@pytest.mark.parametrize("sides", [(1, 1, 2, 2), (0, 0, 0, 2), (2, 0, 1, 1), (0, 2, 0, 0),
                                   (0, 0, 2, 0), (2, 2, 0, 0)])
@pytest.mark.parametrize("omega", [0.7, 1.6])
@FUSE
def test_walls(sides, omega, fuse):
    """Free-slip walls on every side, with per-step speeds."""
    w = wl.explosion(96)
    _compare(w, max_steps=81, omega=omega, sides=sides, name=f"fused{fuse} wall {sides} w{omega}",
             fuse=fuse)


@pytest.mark.parametrize("tile", [(0, 4), (3, 2), (0, 16), (1, 8), (2, 4)])
@pytest.mark.parametrize("layout", [0, 1])
@FUSE
def test_walls_and_layouts_small_segments(tile, layout, fuse):
    """Row segments of 1 to 4 rows: a segment that begins 1 or 2 rows above a
    clamped or wall side still computes the rows below it for the later
    steps, by the side rules (the blast reaches the sides, so a wrong ghost
    row would show)."""
    w = wl.explosion(70)
    _compare(w, max_steps=45, omega=1.3, sides=(2, 2, 0, 0), tile=tile, layout=layout,
             name=f"fused{fuse} walls x l{layout} {tile}", fuse=fuse)
    _compare(w, max_steps=45, omega=1.3, sides=(0, 0, 2, 2), tile=tile, layout=layout,
             name=f"fused{fuse} walls y l{layout} {tile}", fuse=fuse)


@pytest.mark.parametrize("sides", [(2, 2, 0, 0), (0, 0, 2, 2), (0, 0, 0, 0), (0, 2, 1, 1)])
@pytest.mark.parametrize("tile", [(1, 8), (2, 8), (1, 2)])
@FUSE
def test_narrow_strips_and_segments(sides, tile, fuse):
    """A 16 x 16 domain in 8-wave workgroups: strips of 2 columns begin 2 to 4
    columns from a side, so their halo lanes hold the wall or ghost column."""
    w = wl.explosion(16)
    _compare(w, max_steps=30, omega=1.3, sides=sides, tile=tile,
             name=f"fused{fuse} narrow {sides} {tile}", fuse=fuse)


@FUSE
def test_fixed_speeds(fuse):
    w = wl.acoustic_pulse(128, steps=50)
    _compare(w, max_steps=51, lam_mode=2, lam_user=3.0, name="pair user lambda", fuse=fuse)
    _compare(w, max_steps=50, lam_mode=1, name="pair frozen lambda", fuse=fuse)


@pytest.mark.parametrize("chunks", [[1, 2, 3, 5, 8, 13], [7, 7, 7], [2] * 11, [1] * 9, [40]])
@pytest.mark.parametrize("lam_mode", [0, 1])
@FUSE
def test_step_counts_per_call(chunks, lam_mode, fuse):
    """Every call takes exactly its max_steps (odd and even counts, one-step
    calls), whatever the guesses do."""
    w = _riemann_rect(130, 90)
    P = oracle_problem(w, omega=1.2, lam_mode=lam_mode)
    sim = _fused(w, omega=1.2, lam_mode=lam_mode, fuse=fuse)
    done = 0
    for k in chunks:
        sim.step(k)
        done += k
        st = sim.state()
        assert st["rc"] == 0 and st["nsteps"] == done
    ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=done)
    U = sim.moments().cpu().numpy()
    sim.close()
    assert ref.nsteps == done
    assert st["t"] == pytest.approx(ref.t, rel=1e-12, abs=0)
    assert max_abs(U, ref.U) <= TOL


@FUSE
def test_call_far_past_t_end(fuse):
    """A call of far more steps than the run to t_end takes (100000 against a
    few dozen) stops at t_end with the oracle's state, and enqueues at most
    one round of 512 launches beyond those that did work."""
    w = _riemann_rect(130, 90)
    P = oracle_problem(w)
    ref = _oracle_run(P, w, t_end=w.t_end)
    assert ref.status == 0 and ref.t == w.t_end
    sim = _fused(w, fuse=fuse)
    sim.step(100000, w.t_end)
    st = sim.state()
    stats = sim.pair_stats()
    U = sim.moments().cpu().numpy()
    sim.close()
    assert st["rc"] == 0 and st["nsteps"] == ref.nsteps and st["t"] == ref.t
    assert max_abs(U, ref.U) <= TOL
    active = stats["pairs"] + stats["rejected"] + stats["bound_only"] + stats["single"]
    assert active <= stats["enqueued"] <= active + 512, stats


@pytest.mark.parametrize("lam_mode", [0, 1])
@pytest.mark.parametrize("fuse", [1, 2, 3, 4])
def test_fused_calls_replayed_from_a_graph(lam_mode, fuse):
    """A fused lbrs_step call captured in a HIP graph (torch.cuda.graph on the
    context's own stream) enqueues its launches without waiting, rounded up
    to a multiple of six, so each replay continues the run by the call's
    steps from where the last one left it (single steps: a call of six, one
    launch each).  One eager call first, then the capture (which runs
    nothing: the state stays at the eager call's), then three replays with
    eager work and synchronisation between them, each against the same calls
    made eagerly on another context: step count, time, lattice speed and U
    bit for bit, and the last one against the oracle."""
    w = _riemann_rect(130, 90)
    first, k = 3, (6 if fuse == 1 else 7)
    ref = _fused(w, omega=1.2, lam_mode=lam_mode, fuse=fuse)
    ref.step(first)
    want = []
    for _ in range(3):
        ref.step(k)
        want.append((ref.state(), ref.moments().cpu().numpy()))
    ref.close()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sim = _fused(w, omega=1.2, lam_mode=lam_mode, fuse=fuse)
        sim.step(first)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            sim.step(k)
        torch.cuda.synchronize()
        st = sim.state()
        assert st["rc"] == 0 and st["nsteps"] == first
        for i in range(3):
            g.replay()
            torch.cuda.synchronize()
            st = sim.state()
            U = sim.moments().cpu().numpy()
            torch.cuda.synchronize()
            ws, wU = want[i]
            assert st["rc"] == 0 and st["nsteps"] == ws["nsteps"] == first + (i + 1) * k
            assert st["t"] == ws["t"] and st["lambda"] == ws["lambda"]
            assert max_abs(U, wU) == 0.0, i
        sim.close()
    P = oracle_problem(w, omega=1.2, lam_mode=lam_mode)
    o = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=first + 3 * k)
    assert o.nsteps == first + 3 * k
    assert st["t"] == pytest.approx(o.t, rel=1e-12, abs=0)
    assert max_abs(U, o.U) <= TOL


@FUSE
def test_lattice_speed_sequence(fuse):
    """After every call (of 3 to 14 steps) the reported lattice speed and time
    are the oracle's after that many steps."""
    w = wl.riemann2d(128)
    P = oracle_problem(w)
    ref = oracle.run(P, oracle.prim_to_cons(P, w.W), t_end=0.3)
    sim = _fused(w, fuse=fuse)
    done = 0
    for k in [3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14] * 4:
        if done + k > ref.nsteps:
            break
        sim.step(k, 0.3)
        done += k
        st = sim.state()
        assert st["nsteps"] == done
        assert st["lambda"] == pytest.approx(ref.lam[done - 1], rel=1e-12), done
        assert st["t"] == pytest.approx(float(np.sum(ref.dt[:done])), rel=1e-12)
    sim.close()


@pytest.mark.parametrize("lam_user,fail", [(1.0, 3), (1.2, 4), (1.8, 9), (2.2, 24)])
@FUSE
def test_nonphysical_fixed_speed(lam_user, fail, fuse):
    """Lattice speeds below the bound lose positivity at odd and even steps: a
    non-physical f^{n+1} inside a fused launch sends the next launch back to
    f^n for one step, a non-physical f^{n+2} is reported when accepted."""
    w = wl.explosion(64)
    _, ref, st = _compare(w, max_steps=400, omega=1.6, lam_mode=2, lam_user=lam_user,
                          name=f"fused{fuse} nonphysical user {lam_user}", fuse=fuse)
    assert ref.fail_step == fail and st["fail_step"] == fail


@FUSE
def test_nonphysical_per_step(fuse):
    w = _riemann_rect(300, 200)
    _, ref, st = _compare(w, t_end=0.04, omega=1.8, name=f"fused{fuse} nonphysical rect",
                          fuse=fuse)
    assert ref.fail_step == 2
    w = wl.explosion(96)
    w.cfl = 1.0
    _, ref, st = _compare(w, max_steps=300, omega=1.95,
                          name=f"fused{fuse} nonphysical explosion", fuse=fuse)
    assert ref.fail_step == 210


@FUSE
def test_nonphysical_initial_state(fuse):
    w = wl.riemann2d(64)
    w.W[3, 10, 10] = -1.0
    sim = _fused(w, fuse=fuse)
    sim.step(5)
    st = sim.state()
    assert st["rc"] == lbrs.LBRS_E_NONPHYSICAL and st["fail_step"] == 0 and st["nsteps"] == 0
    sim.close()


@pytest.mark.parametrize("sides", [(0, 0, 0, 0), (1, 1, 1, 1), (2, 2, 0, 0), (0, 0, 2, 2)])
@FUSE
def test_matches_single_steps(sides, fuse):
    """Fused and single-step runs: identical step counts, status, times,
    speeds and populations, bit for bit (the per-cell arithmetic is written
    with its multiply-adds spelled out and contraction off, so both kernels
    round alike, and every guess of the next bound is checked exactly)."""
    w = wl.explosion(150)
    outs = []
    for k in (1, fuse):
        sim = gpu_sim(w, sides=sides, omega=1.3, layout=1)
        sim.init_primitive(w.W)
        sim.set_fusion(k)
        sim.step(57, 0.25)
        outs.append((sim.state(), sim.get_f()))
        sim.close()
    (s1, f1), (s2, f2) = outs
    diff = float((f1 - f2).abs().max())
    report(f"fused{fuse} vs single {sides}", max_abs_f=diff, bitwise=bool(torch.equal(f1, f2)),
           t=(s1["t"], s2["t"]), lam=(s1["lambda"], s2["lambda"]))
    assert (s1["nsteps"], s1["rc"]) == (s2["nsteps"], s2["rc"])
    assert s2["t"] == s1["t"] and s2["lambda"] == s1["lambda"]
    assert torch.equal(f1, f2), diff


@FUSE
def test_uniform_flow_bitwise(fuse):
    n = 70
    W = np.zeros((4, n, n))
    W[0], W[1], W[2], W[3] = 0.8, 0.3, -0.2, 0.7
    w = wl.Workload("uniform", wl.D2Q4, n, n, (0, 1, 0, 1), W, omega=1.7)
    sim = _fused(w, fuse=fuse)
    sim.step(31)
    f = sim.get_f().reshape(16, -1)
    assert torch.all(f == f[:, :1])
    sim.close()


@FUSE
def test_mixed_with_single_steps_tape_and_checkpoints(fuse):
    """Fused calls interleaved with single-step calls, taped steps and
    get_f / set_f continue the same run."""
    w = wl.acoustic_pulse(96, steps=40)
    P = oracle_problem(w, lam_mode=oracle.LAM_FROZEN)
    ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=40)
    sim = gpu_sim(w, lam_mode=1)
    sim.init_primitive(w.W)
    sim.set_fusion(fuse)
    sim.step(9)
    sim.set_fusion(1)
    sim.step(4)
    tape = torch.empty((4, 96, 96), dtype=torch.float64, device="cuda")
    lbrs.lbrs_step_tape(sim.ctx, tape)
    sim.set_fusion(fuse)
    sim.step(6)
    s20 = sim.state()
    f20 = sim.get_f()
    sim.step(20)
    U40 = sim.moments().clone()
    sim.set_f(f20, s20["t"], s20["nsteps"])
    sim.step(20)
    st = sim.state()
    assert s20["nsteps"] == 20 and st["nsteps"] == 40
    assert torch.equal(sim.moments(), U40)
    assert max_abs(U40.cpu().numpy(), ref.U) <= TOL
    sim.close()


def test_checkpointed_gradient_with_fused_forward():
    """The gradient's forward sweeps run through lbrs_step, so fused launches
    take them (segments of odd length included); the gradient equals the
    single-step one to rounding."""
    from paper_1504_07034_amd import adjoint
    w = wl.acoustic_pulse(64, steps=30)
    rho0 = torch.from_numpy(w.W[0].copy()).cuda()
    out = []
    for fuse in (1, 2, 3, 4):
        run = adjoint.GradientRunner(adjoint.GradientSpec(n=64, steps=30, segment=7, fuse=fuse),
                                     rho0)
        J = run.forward(rho0)
        g = run.backward(rho0)
        out.append((float(J), g.clone()))
        run.close()
    J1, g1 = out[0]
    scale = float(g1.abs().max())
    for fuse, (J2, g2) in zip((2, 3, 4), out[1:]):
        assert J2 == pytest.approx(J1, rel=1e-13)
        diff = float((g1 - g2).abs().max())
        report(f"fused{fuse} gradient", J=J1, rel_diff=diff / scale)
        assert diff <= 1e-11 * scale


def test_mode_restrictions():
    w = wl.explosion(32)
    sim = gpu_sim(w)
    sim.init_primitive(w.W)
    for bad in (0, 5):
        with pytest.raises(lbrs.LBRSError) as e:
            sim.set_fusion(bad)
        assert e.value.code == lbrs.LBRS_E_INVAL
    sim.close()
    w1 = wl.sod(100)
    sim = gpu_sim(w1)
    sim.init_primitive(w1.W)
    with pytest.raises(lbrs.LBRSError) as e:
        sim.set_fusion(2)
    assert e.value.code == lbrs.LBRS_E_STATE
    sim.set_fusion(1)
    sim.close()
    wf = wl.forward_step()
    sim = lbrs.Sim(wf.model, wf.nx, wf.ny, domain=wf.domain, gamma=wf.gamma, omega=wf.omega,
                   cfl=wf.cfl, bc=tuple(wf.sides), solid=wf.solid, dirichlet_W=wf.dirichlet_W)
    sim.init_primitive(wf.W)
    with pytest.raises(lbrs.LBRSError) as e:
        sim.set_fusion(2)
    assert e.value.code == lbrs.LBRS_E_STATE
    sim.close()


@pytest.mark.parametrize("tile", [(0, 8), (0, 4), (0, 12)])
@FUSE
def test_full_size_4096_first_steps(tile, fuse):
    """Full size (4096^2, transmissive, omega = 1, row-interleaved) in fused
    launch shapes: five steps (two fused launches and a single one) against
    the oracle on every cell."""
    w = wl.riemann2d(4096)
    _compare(w, max_steps=5, tile=tile, layout=1, name=f"fused{fuse} riemann 4096 x5 {tile}",
             fuse=fuse)


@FUSE
def test_full_size_4096_cone_samples(fuse):
    """Full size, 100 fused steps at the oracle's fixed lattice speed, checked
    on sampled cells against the oracle on the (2k+3)^2 patch around each
    (a cell after k steps depends only on the (2k+1)^2 patch around it)."""
    n, k = 4096, 100
    w = wl.riemann2d(n)
    Pfull = oracle_problem(w)
    lam = oracle.initial_lattice_speed(Pfull, oracle.prim_to_cons(Pfull, w.W))
    sim = _fused(w, tile=(0, 8), layout=1, lam_mode=lbrs.LBRS_LAMBDA_USER, lam_user=lam,
                 fuse=fuse)
    sim.step(k)
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == k
    U = sim.moments().cpu().numpy()
    sim.close()
    rng = np.random.default_rng(13)
    samples = [(0, 0), (n - 1, n - 1), (0, n - 1), (n // 2, n // 2), (n // 2 - 1, n // 2),
               (1, n // 2 + 5)] + [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(4)]
    R = k + 1
    worst = 0.0
    for (j, i) in samples:
        y0, y1 = max(0, j - R), min(n, j + R + 1)
        x0, x1 = max(0, i - R), min(n, i + R + 1)
        P = oracle.Problem(model=oracle.D2Q4, nx=x1 - x0, ny=y1 - y0,
                           domain=(0.0, (x1 - x0) / n, 0.0, (y1 - y0) / n), gamma=w.gamma,
                           omega=w.omega, cfl=w.cfl, sides=(0, 0, 0, 0),
                           lam_mode=oracle.LAM_USER, lam_user=lam)
        ref = oracle.run(P, oracle.prim_to_cons(P, w.W[:, y0:y1, x0:x1]), max_steps=k,
                         record=False)
        err = float(np.max(np.abs(U[:, j, i] - ref.U[:, j - y0, i - x0])))
        worst = max(worst, err)
        assert err <= TOL, ((j, i), err)
    report("pair riemann 4096 cone", steps=k, samples=len(samples), err=worst)
