"""DIRICHLET sides on the GPU (the prescribed inflow and top boundaries of the
oblique-shock reflection case, Sec. III) against the oracle, cell by cell."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import TOL, max_abs, report
from test_oracle_dirichlet import oracle_problem

pytestmark = pytest.mark.gpu


def gpu_sim(w, omega=None, lam_mode=0, lam_user=0.0, layout=1, sides=None):
    return lbrs.Sim(w.model, w.nx, w.ny, domain=w.domain, gamma=w.gamma,
                    omega=w.omega if omega is None else omega, cfl=w.cfl,
                    bc=tuple(w.sides if sides is None else sides), lambda_mode=lam_mode,
                    lambda_user=lam_user, layout=layout, dirichlet_W=w.dirichlet_W)


def compare(w, max_steps=10**9, t_end=math.inf, omega=None, tile=None, lam_mode=0, lam_user=0.0,
            layout=1, name=""):
    P = oracle_problem(w, omega=omega, lam_mode=lam_mode, lam_user=lam_user)
    U0 = oracle.prim_to_cons(P, w.W)
    ref = oracle.run(P, U0, t_end=t_end, max_steps=max_steps, record=False)
    sim = gpu_sim(w, omega=omega, lam_mode=lam_mode, lam_user=lam_user, layout=layout)
    sim.init_primitive(w.W)
    if tile:
        sim.set_tile(*tile)
    sim.step(ref.nsteps if math.isinf(t_end) else ref.nsteps + 5, t_end)
    st = sim.state()
    U = sim.moments().cpu().numpy()
    err = max_abs(U, ref.U)
    report(name or w.name, steps=st["nsteps"], oracle_steps=ref.nsteps, err=err,
           status=(st["rc"], ref.status), tile=tile)
    sim.close()
    return st, ref, err


@pytest.mark.parametrize("omega", [1.0, 1.8])
@pytest.mark.parametrize("tile", [None, (0, 16, 0), (0, 8, 1), (7, 4, 1), (13, 2, 0)])
def test_oblique_shock_parity(omega, tile):
    """The paper's oblique-shock reflection (inflow and post-shock states
    prescribed, free-slip wall below), 240 x 80, to t = 0.6, in several launch
    shapes, both march orders."""
    w = wl.oblique_shock(240, 80, t_end=0.6, omega=omega)
    st, ref, err = compare(w, t_end=w.t_end, tile=tile, name=f"oblique w{omega} {tile}")
    assert st["rc"] == 0 and ref.status == oracle.OK
    assert st["nsteps"] == ref.nsteps and st["t"] == pytest.approx(ref.t, rel=1e-12, abs=0)
    assert err <= TOL


def _smooth_side(n, seed, base):
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, 1.0, n)
    out = np.empty((4, n))
    for k in range(4):
        a, f, ph = rng.uniform(0.05, 0.2), rng.integers(1, 4), rng.uniform(0, 2 * np.pi)
        out[k] = base[k] + a * np.sin(2 * np.pi * f * s + ph)
    return out


@pytest.mark.parametrize("sides", [(3, 3, 3, 3), (1, 1, 3, 3), (3, 3, 1, 1), (3, 0, 2, 3),
                                   (2, 3, 3, 0), (3, 3, 2, 2)])
@pytest.mark.parametrize("alt", [0, 1])
def test_varying_dirichlet_data_vs_oracle(sides, alt):
    """Different, smoothly varying prescribed states along every Dirichlet side
    (corners take the y-side's state), random smooth interior, odd sizes, with
    periodic, wall and transmissive neighbours."""
    nx, ny = 131, 97
    w = wl.fourier_modes(nx, seed=11)
    w.ny, w.W = ny, w.W[:, :ny, :].copy()
    w.domain = (0.0, 1.0, 0.0, ny / nx)
    w.sides = sides
    base = np.array([1.0, 0.2, -0.1, 1.0])
    w.dirichlet_W = tuple(_smooth_side(ny if s < 2 else nx, 30 + s, base) if sides[s] == 3 else None
                          for s in range(4))
    st, ref, err = compare(w, max_steps=60, omega=1.3, tile=(9, 4, alt),
                           name=f"dirichlet sides {sides} alt{alt}")
    assert st["rc"] == 0 and ref.status == oracle.OK and st["nsteps"] == ref.nsteps
    assert err <= TOL


@pytest.mark.parametrize("lam_mode", [1, 2])
def test_dirichlet_fixed_lattice_speeds(lam_mode):
    w = wl.oblique_shock(120, 40, omega=1.5)
    st, ref, err = compare(w, max_steps=150, lam_mode=lam_mode, lam_user=6.0,
                           name=f"oblique lam_mode {lam_mode}")
    assert st["rc"] == 0 and ref.status == oracle.OK and err <= TOL


def test_dirichlet_planar_layout():
    w = wl.oblique_shock(240, 80, t_end=0.3, omega=1.8)
    st, ref, err = compare(w, t_end=w.t_end, layout=0, name="oblique planar")
    assert st["rc"] == 0 and err <= TOL


def test_oblique_shock_large_first_steps():
    """The case at 16x the paper's resolution (3840 x 1280) in the automatic
    launch shape: three steps against the oracle on every cell."""
    w = wl.oblique_shock(3840, 1280, omega=1.8)
    st, ref, err = compare(w, max_steps=3, name="oblique 3840x1280 x3")
    assert st["rc"] == 0 and st["nsteps"] == 3 and err <= TOL


def test_dirichlet_nonadmissible_state_reported_at_step_0():
    w = wl.oblique_shock(60, 20)
    top = w.dirichlet_W[3].copy()
    top[3, 7] = -1.0
    w.dirichlet_W = (w.dirichlet_W[0], None, None, top)
    sim = gpu_sim(w)
    sim.init_primitive(w.W)
    sim.step(5)
    st = sim.state()
    assert st["rc"] == lbrs.LBRS_E_NONPHYSICAL and st["fail_step"] == 0 and st["nsteps"] == 0
    sim.close()


def test_dirichlet_rejections():
    """No tape step on a Dirichlet context (the tape serves the periodic
    adjoint); no Dirichlet data for a side -> invalid."""
    w = wl.oblique_shock(60, 20)
    sim = gpu_sim(w, lam_mode=1)
    sim.init_primitive(w.W)
    tape = torch.empty((4, 20, 60), dtype=torch.float64, device="cuda")
    with pytest.raises(lbrs.LBRSError) as e:
        lbrs.lbrs_step_tape(sim.ctx, tape)
    assert e.value.code == lbrs.LBRS_E_STATE
    sim.close()
    with pytest.raises(lbrs.LBRSError) as e:
        lbrs.Sim(2, 60, 20, domain=(0, 3, 0, 1), bc=(3, 0, 2, 3), layout=1)
    assert e.value.code == lbrs.LBRS_E_INVAL
