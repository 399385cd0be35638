"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Element-by-element comparison of U = (rho, rho u, [rho v,] rho E) at max-abs
<= 1e-10, identical step counts and final times, on seeded workloads that span
several tiles and ragged tails, for every model, omega in {0.6, 1.0, 1.4, 1.8}
and every side condition; plus the full-size 4096^2 configuration for a few
steps in the launch shape the benchmark times.
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

OMEGAS = [0.6, 1.0, 1.4, 1.8]


def _compare(w, t_end=math.inf, max_steps=10**9, omega=None, sides=None, model=None,
             lam_mode=0, lam_user=0.0, tile=None, name="", relative=False, layout=0):
    P = oracle_problem(w, omega=omega, sides=sides, model=model, lam_mode=lam_mode,
                       lam_user=lam_user)
    U0 = oracle.prim_to_cons(P, w.W)
    ref = oracle.run(P, U0, t_end=t_end, max_steps=max_steps)
    sim = gpu_sim(w, omega=omega, sides=sides, model=model, lam_mode=lam_mode, lam_user=lam_user,
                  layout=layout)
    sim.init_primitive(w.W)
    if tile:
        sim.set_tile(*tile)
    steps = ref.nsteps if math.isinf(t_end) else max(ref.nsteps + 5, 1)
    sim.step(steps, t_end)
    st = sim.state()
    U = sim.moments().cpu().numpy()
    if relative:  # per component, in units of the component's largest magnitude
        err = max(max_abs(U[k], ref.U[k]) / max(1.0, np.abs(ref.U[k]).max())
                  for k in range(U.shape[0]))
    else:
        err = max_abs(U, ref.U)
    report(name or w.name, steps=st["nsteps"], oracle_steps=ref.nsteps, t=st["t"], err=err,
           status=(st["rc"], ref.status), fail=(st["fail_step"], ref.fail_step))
    if ref.status == oracle.NONPHYSICAL:
        # over-relaxation is not positivity preserving: both sides must stop at
        # the same step with the same report
        assert st["rc"] == -4 and st["fail_step"] == ref.fail_step
        assert st["nsteps"] == ref.nsteps
        sim.close()
        return U, ref
    assert st["rc"] == 0 and ref.status == 0
    assert st["nsteps"] == ref.nsteps
    assert st["t"] == pytest.approx(ref.t, rel=1e-12, abs=0)
    assert err <= TOL, err
    sim.close()
    return U, ref


@pytest.mark.parametrize("omega", OMEGAS)
@pytest.mark.parametrize("model", [wl.D1Q2, wl.D1Q3])
def test_sod_full_run(model, omega):
    """Shock tube, 400 cells, to t = 0.2 (the persistent one-workgroup form)."""
    w = wl.sod(400, model=model, omega=omega)
    _compare(w, t_end=0.2, name=f"sod m{model} w{omega}")


def test_sod_paper_dimensional():
    """The paper's dimensional shock tube (p ~ 1e5 Pa, rho E ~ 2.5e5): the bar is
    1e-10 relative to each component's magnitude (round-off scales with it)."""
    w = wl.sod_dimensional()
    _compare(w, t_end=0.01, name="sod dimensional", relative=True)


@pytest.mark.parametrize("omega", [0.6, 1.8])
def test_1d_periodic(omega):
    w = wl.sod(300, omega=omega)
    _compare(w, max_steps=200, sides=(1, 1, 0, 0), name=f"1d periodic w{omega}")


@pytest.mark.parametrize("model", [wl.D1Q2, wl.D1Q3])
@pytest.mark.parametrize("periodic", [False, True])
def test_1d_long_tiled(model, periodic):
    """5003 cells (beyond the one-workgroup form, ragged against 512-cell tiles)."""
    w = wl.sod(5003, model=model, omega=1.3, t_end=0.02)
    sides = (1, 1, 0, 0) if periodic else (0, 0, 0, 0)
    _compare(w, t_end=0.02, sides=sides, name=f"1d long m{model} p{periodic}")


@pytest.mark.parametrize("n,model,periodic", [(62000, wl.D1Q3, False), (62001, wl.D1Q2, True),
                                               (400063, wl.D1Q3, True), (1 << 20, wl.D1Q2, False)])
def test_1d_long_tubes(n, model, periodic):
    """Long tubes in many 512-cell tiles: a ragged last tile, one cell past a
    multiple of the tile, a power of two, periodic wrap across the ends."""
    w = wl.sod(n, model=model, omega=1.2, t_end=0.02)
    sides = (1, 1, 0, 0) if periodic else (0, 0, 0, 0)
    _compare(w, max_steps=25, sides=sides, name=f"1d long n{n} m{model} p{periodic}")


@pytest.mark.parametrize("n,model,periodic", [(400, wl.D1Q3, False), (400, wl.D1Q2, True),
                                               (5003, wl.D1Q3, False), (62001, wl.D1Q2, True),
                                               (400063, wl.D1Q3, True)])
def test_1d_blocked_layout(n, model, periodic):
    """The blocked 1D layout (LAYOUT_ROWS: the planes of each 64-cell block
    contiguous, last block padded) in the one-workgroup form and the tiled
    form, ragged against the block, periodic wrap across the ends."""
    w = wl.sod(n, model=model, omega=1.3, t_end=0.02)
    sides = (1, 1, 0, 0) if periodic else (0, 0, 0, 0)
    _compare(w, max_steps=40, sides=sides, layout=1, name=f"1d blocked n{n} m{model} p{periodic}")


@pytest.mark.parametrize("n", [300, 5003])
def test_1d_layouts_bitwise_and_f_round_trip(n):
    """Planar and blocked 1D layouts give the same bits (moments, populations,
    state); populations read with get_f and written back with set_f in the
    blocked layout continue the run exactly."""
    w = wl.sod(n, omega=1.4, t_end=0.05)
    outs = []
    for layout in (0, 1):
        sim = gpu_sim(w, layout=layout)
        sim.init_primitive(w.W)
        sim.step(30, w.t_end)
        outs.append((sim.moments(), sim.to_planar(sim.get_f()), sim.state()))
        sim.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]
    sim = gpu_sim(w, layout=1)
    sim.init_primitive(w.W)
    sim.step(10, w.t_end)
    st = sim.state()
    f = sim.from_planar(sim.to_planar(sim.get_f()))
    sim.step(20, w.t_end)
    ref = sim.moments().clone()
    sim.set_f(f, st["t"], st["nsteps"])
    sim.step(20, w.t_end)
    assert torch.equal(sim.moments(), ref)
    assert sim.state()["nsteps"] == 30
    sim.close()


@pytest.mark.parametrize("model,omega", [(wl.D1Q3, 1.0), (wl.D1Q2, 1.6)])
def test_steady_shock(model, omega):
    """The paper's steady shock (M = 2, 400 points on [-1, 1]) to t = 2."""
    w = wl.steady_shock(400, model=model, omega=omega, t_end=2.0)
    _compare(w, t_end=w.t_end, name=f"steady shock m{model} w{omega}")


@pytest.mark.parametrize("omega", [1.0, 1.7])
def test_steady_contact(omega):
    """The paper's steady contact (100 points, t = 2)."""
    w = wl.steady_contact(100, omega=omega)
    _compare(w, t_end=2.0, name=f"steady contact w{omega}")


def test_paper_riemann2d_400():
    """The paper's own four-quadrant case at its resolution (400^2), 300 steps
    (its end time is not given)."""
    w = wl.riemann2d_paper(400)
    _compare(w, max_steps=300, name="paper riemann 400")


def test_steady_shock_long_tiled():
    """The steady shock on 20011 cells (512-cell tiles, ragged), 600 steps."""
    w = wl.steady_shock(20011, omega=1.2)
    _compare(w, max_steps=600, name="steady shock 20011")


def _riemann_rect(nx=300, ny=200):
    """Four-quadrant states on a rectangle [0, 1.5] x [0, 1] (dx = dy)."""
    w = wl.riemann2d(nx)
    x = wl.centres(nx, 0.0, 1.5)
    y = wl.centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y, indexing="xy")
    st = w.meta["states"]
    east, north = X > 0.75, Y > 0.5
    W = np.empty((4, ny, nx))
    for k in range(4):
        W[k] = np.where(north, np.where(east, st["NE"][k], st["NW"][k]),
                        np.where(east, st["SE"][k], st["SW"][k]))
    return wl.Workload("riemann_rect", wl.D2Q4, nx, ny, (0.0, 1.5, 0.0, 1.0), W, t_end=0.04)


@pytest.mark.parametrize("omega", OMEGAS)
def test_2d_transmissive(omega):
    """Four-quadrant states on a 300 x 200 rectangle (at omega = 1.8 the oracle and
    the GPU both lose positivity at step 2 and must agree on it)."""
    w = _riemann_rect()
    _compare(w, t_end=0.04, omega=omega, name=f"2d transmissive w{omega}")


@pytest.mark.parametrize("omega", OMEGAS)
def test_2d_explosion(omega):
    """Explosion (Sec. III) at 200^2 on [-1,1]^2, 120 steps, every omega."""
    w = wl.explosion(200)
    _compare(w, max_steps=120, omega=omega, name=f"2d explosion w{omega}")


@pytest.mark.parametrize("tile", [(64, 4), (7, 1), (50, 2), (200, 4), (0, 6), (0, 8), (33, 12),
                                  (0, 16), (64, 4, 0), (7, 2, 0), (0, 16, 0), (1, 1), (1, 4, 0),
                                  (2, 8), (3, 2, 0), (3, 16)])
def test_2d_tile_shapes(tile):
    """Ragged row segments and every workgroup shape (lockstep groups of 1 to 16
    waves, strip widths below 62) give the same answer."""
    w = _riemann_rect(301, 201)
    w.domain = (0.0, 301 / 201, 0.0, 1.0)
    _compare(w, t_end=0.03, omega=1.4, tile=tile, name=f"2d tile {tile}")


@pytest.mark.parametrize("sides", [(1, 1, 1, 1), (1, 1, 0, 0), (0, 0, 1, 1)])
def test_2d_periodic(sides):
    w = wl.fourier_modes(130, seed=3)
    w.sides = sides
    _compare(w, max_steps=60, omega=1.2, name=f"2d periodic {sides}")


@pytest.mark.parametrize("sides", [(1, 1, 2, 2), (0, 0, 0, 2), (2, 0, 1, 1), (0, 2, 0, 0)])
@pytest.mark.parametrize("omega", [0.7, 1.6])
def test_2d_walls(sides, omega):
    """Specular free-slip walls (Sec. II.E) on each side."""
    w = wl.explosion(96)
    _compare(w, max_steps=80, omega=omega, sides=sides, name=f"2d wall {sides} w{omega}")


def test_2d_full_run_riemann_256():
    """The benchmark's four-quadrant problem at 256^2, run to t = 0.3."""
    w = wl.riemann2d(256)
    _compare(w, t_end=0.3, name="riemann 256 full")


def test_2d_user_lambda_and_frozen():
    w = wl.acoustic_pulse(128, steps=50)
    _compare(w, max_steps=50, lam_mode=2, lam_user=3.0, name="user lambda")
    _compare(w, max_steps=50, lam_mode=1, name="frozen lambda")


@pytest.mark.parametrize("layout,tile", [(0, (0, 4)), (1, (0, 4)), (1, (0, 16, 0)),
                                         (1, (0, 8, 1))])
def test_full_size_4096_first_steps(layout, tile):
    """Full size (4096^2, transmissive, omega = 1) in the benchmark's launch shapes
    (automatic row segments, 4-, 16- and 8-wave groups, both march orders, both
    population layouts): three steps against the oracle on every cell."""
    w = wl.riemann2d(4096)
    _compare(w, max_steps=3, tile=tile, layout=layout, name=f"riemann 4096 x3 l{layout} {tile}")


@pytest.mark.parametrize("tile", [(0, 16, 0), (0, 8, 1)])
def test_full_size_4096_cone_samples(tile):
    """Full size, 100 steps, in the benchmark's launch shapes, checked on
    sampled cells.  With a fixed lattice speed a cell after k steps depends
    only on the (2k+1)^2 patch around it, so the oracle computes each sample on
    a patch of radius k+1 (the real sides where the patch reaches them, any
    side elsewhere: errors from an artificial patch edge travel one cell per
    step and do not reach the centre).  The fixed speed is the oracle's own
    lambda*(U0)/cfl of the whole grid."""
    n, k = 4096, 100
    w = wl.riemann2d(n)
    Pfull = oracle_problem(w)
    lam = oracle.initial_lattice_speed(Pfull, oracle.prim_to_cons(Pfull, w.W))
    assert lam > 0
    sim = gpu_sim(w, lam_mode=lbrs.LBRS_LAMBDA_USER, lam_user=lam, layout=1)
    sim.init_primitive(w.W)
    sim.set_tile(*tile)
    sim.step(k)
    st = sim.state()
    assert st["rc"] == 0 and st["nsteps"] == k
    U = sim.moments().cpu().numpy()
    sim.close()
    rng = np.random.default_rng(12)
    samples = [(0, 0), (n - 1, n - 1), (0, n - 1), (n // 2, n // 2), (n // 2 - 1, n // 2),
               (3, n // 2 + 7)] + [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(4)]
    R = k + 1
    worst = 0.0
    for (j, i) in samples:  # (row, column)
        y0, y1 = max(0, j - R), min(n, j + R + 1)
        x0, x1 = max(0, i - R), min(n, i + R + 1)
        P = oracle.Problem(model=oracle.D2Q4, nx=x1 - x0, ny=y1 - y0,
                           domain=(0.0, (x1 - x0) / n, 0.0, (y1 - y0) / n), gamma=w.gamma,
                           omega=w.omega, cfl=w.cfl, sides=(0, 0, 0, 0),
                           lam_mode=oracle.LAM_USER, lam_user=lam)
        ref = oracle.run(P, oracle.prim_to_cons(P, w.W[:, y0:y1, x0:x1]), max_steps=k,
                         record=False)
        assert ref.status == 0 and ref.nsteps == k
        err = float(np.max(np.abs(U[:, j, i] - ref.U[:, j - y0, i - x0])))
        worst = max(worst, err)
        assert err <= TOL, ((j, i), err)
    report(f"riemann 4096 cone {tile}", steps=k, samples=len(samples), err=worst)


@pytest.mark.parametrize("sides", [(0, 0, 0, 0), (1, 1, 2, 2), (2, 0, 1, 1)])
def test_rows_layout_matches_planar_bitwise(sides):
    """The row-interleaved population layout runs the same arithmetic: moments and
    populations equal the planar layout's bit for bit."""
    w = wl.explosion(150)
    outs = []
    for layout in (0, 1):
        sim = gpu_sim(w, sides=sides, omega=1.3, layout=layout)
        sim.init_primitive(w.W)
        sim.step(70)
        outs.append((sim.moments(), sim.to_planar(sim.get_f()), sim.state()))
        sim.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


@pytest.mark.parametrize("sides", [(0, 0, 0, 0), (1, 1, 2, 2), (2, 0, 1, 1), (0, 0, 2, 0),
                                   (1, 1, 1, 1)])
@pytest.mark.parametrize("layout", [0, 1])
def test_alternate_march_bitwise(sides, layout):
    """Odd row segments marched upwards through the y-mirrored view give the
    same bits as marching every segment downwards: populations, moments,
    state, and the moment tape of a fixed-speed step."""
    w = wl.explosion(150)
    outs = []
    for alt in (0, 1):
        sim = gpu_sim(w, sides=sides, omega=1.3, layout=layout, lam_mode=1)
        sim.init_primitive(w.W)
        sim.set_tile(7, 4, alt)  # 22 segments, half of them mirrored
        sim.step(60)
        tape = torch.empty((4, w.ny, w.nx), dtype=torch.float64, device="cuda")
        lbrs.lbrs_step_tape(sim.ctx, tape)
        outs.append((sim.moments(), sim.to_planar(sim.get_f()), sim.state(), tape))
        sim.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]
    assert torch.equal(outs[0][3], outs[1][3])


def test_rows_layout_parity():
    w = _riemann_rect(301, 201)
    w.domain = (0.0, 301 / 201, 0.0, 1.0)
    _compare(w, t_end=0.03, omega=0.6, layout=1, name="2d rows layout")


def test_symmetry_4096_long():
    """After 400 steps at 4096^2 the solution keeps the x <-> y symmetry of the
    initial data (a property that holds at any size; Sec. III notes it)."""
    w = wl.riemann2d(4096)
    sim = gpu_sim(w)
    sim.init_primitive(w.W)
    sim.set_tile(64, 4)
    sim.step(400, 0.3)
    st = sim.state()
    U = sim.moments()
    rho, m, n = U[0], U[1], U[2]
    e1 = (rho - rho.T).abs().max().item()
    e2 = (m - n.T).abs().max().item()
    report("symmetry 4096", steps=st["nsteps"], rho=e1, mom=e2)
    assert st["rc"] == 0 and st["nsteps"] == 400
    assert e1 <= 1e-13 and e2 <= 1e-13
    sim.close()


@pytest.mark.parametrize("sides", [(0, 0, 0, 0), (1, 1, 1, 1), (1, 1, 2, 2)])
def test_uniform_flow_bitwise(sides):
    n = 70
    W = np.zeros((4, n, n))
    W[0], W[1], W[2], W[3] = 0.8, 0.3, (0.0 if 2 in sides else -0.2), 0.7
    w = wl.Workload("uniform", wl.D2Q4, n, n, (0, 1, 0, 1), W, omega=1.7, sides=sides)
    sim = gpu_sim(w)
    sim.init_primitive(w.W)
    sim.step(30)
    f = sim.get_f().reshape(16, -1)
    assert torch.all(f == f[:, :1])
    sim.close()


def test_nonphysical_reported_at_same_step():
    """A lattice speed far below the bound loses positivity; the GPU stops at the
    same step as the oracle and reports LBRS_E_NONPHYSICAL."""
    w = wl.sod(40, model=wl.D1Q2, omega=1.9)
    P = oracle_problem(w, lam_mode=oracle.LAM_USER, lam_user=0.2)
    ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=500)
    assert ref.status == oracle.NONPHYSICAL
    sim = gpu_sim(w, lam_mode=2, lam_user=0.2)
    sim.init_primitive(w.W)
    sim.step(500)
    st = sim.state()
    report("nonphysical", gpu=st["fail_step"], oracle=ref.fail_step)
    assert st["rc"] == -4 and st["fail_step"] == ref.fail_step and st["nsteps"] == ref.fail_step


def test_nonphysical_initial_state():
    w = wl.riemann2d(64)
    w.W[3, 10, 10] = -1.0
    sim = gpu_sim(w)
    sim.init_primitive(w.W)
    sim.step(5)
    st = sim.state()
    assert st["rc"] == -4 and st["fail_step"] == 0 and st["nsteps"] == 0


def test_get_set_f_roundtrip():
    w = wl.riemann2d(128)
    sim = gpu_sim(w)
    sim.init_primitive(w.W)
    sim.step(20, 0.3)
    s20 = sim.state()
    f20 = sim.get_f()
    sim.step(15, 0.3)
    U35 = sim.moments().clone()
    sim.set_f(f20, s20["t"], s20["nsteps"])
    sim.step(15, 0.3)
    st = sim.state()
    assert st["nsteps"] == 35
    assert torch.equal(sim.moments(), U35)


def test_deterministic():
    w = wl.riemann2d(512)
    outs = []
    for _ in range(2):
        sim = gpu_sim(w)
        sim.init_primitive(w.W)
        sim.step(50, 0.3)
        outs.append(sim.get_f())
        sim.close()
    assert torch.equal(outs[0], outs[1])
