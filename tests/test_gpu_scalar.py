"""Scalar laws on the GPU (Burgers D1Q2/D1Q3, Sec. II.A; the 2D Burgers cases
of Sec. III on D2Q4; a general quadratic flux) against the oracle, cell by
cell."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import TOL, max_abs, report
from test_oracle_scalar import problem

pytestmark = pytest.mark.gpu


def gpu_sim(w, omega=None, lam_mode=0, lam_user=0.0, layout=1, sides=None):
    return lbrs.Sim(w.model, w.nx, w.ny, domain=w.domain, omega=w.omega if omega is None else omega,
                    cfl=w.cfl, bc=tuple(w.sides if sides is None else sides), lambda_mode=lam_mode,
                    lambda_user=lam_user, layout=layout, dirichlet_W=w.dirichlet_W,
                    law=lbrs.LBRS_LAW_SCALAR, scalar_flux=w.quad)


def compare(w, t_end=math.inf, max_steps=10**9, omega=None, tile=None, lam_mode=0, layout=1,
            name=""):
    P = problem(w, omega=omega, lam_mode=lam_mode)
    ref = oracle.run(P, w.W.copy(), t_end=t_end, max_steps=max_steps, record=False)
    sim = gpu_sim(w, omega=omega, lam_mode=lam_mode, layout=layout)
    sim.init_primitive(w.W)
    if tile:
        sim.set_tile(*tile)
    sim.step(ref.nsteps if math.isinf(t_end) else ref.nsteps + 5, t_end)
    st = sim.state()
    U = sim.moments().cpu().numpy()
    err = max_abs(U, ref.U)
    report(name or w.name, steps=st["nsteps"], oracle_steps=ref.nsteps, err=err,
           status=(st["rc"], ref.status))
    sim.close()
    assert st["rc"] == 0 and ref.status == oracle.OK
    assert st["nsteps"] == ref.nsteps
    if not math.isinf(t_end):
        assert st["t"] == pytest.approx(ref.t, rel=1e-12, abs=0)
    assert err <= TOL, err
    return U, ref


@pytest.mark.parametrize("model", [wl.D1Q2, wl.D1Q3])
@pytest.mark.parametrize("uL,uR", [(1.0, 0.0), (-0.5, 1.0), (1.2, -0.8)])
@pytest.mark.parametrize("n", [400, 1000, 2500])
def test_burgers_1d(model, uL, uR, n):
    """Shock, rarefaction and a stationary-ish shock, to t = 0.5, on one
    1024-cell tile (400, 1000 cells) and on three with a ragged last one
    (2500 cells)."""
    w = wl.burgers_riemann(n, uL, uR, t_end=0.5, model=model)
    compare(w, t_end=w.t_end, name=f"burgers m{model} ({uL},{uR}) n{n}")


@pytest.mark.parametrize("model", [wl.D1Q2, wl.D1Q3])
def test_burgers_1d_layouts(model):
    """Planar and blocked (64-cell blocks) 1D layouts, a tube ragged against
    both the block and the tile: same result as the oracle, same bits."""
    w = wl.burgers_riemann(5003, 1.0, -0.5, t_end=0.3, model=model)
    U0, _ = compare(w, t_end=w.t_end, layout=0, name=f"burgers planar m{model}")
    U1, _ = compare(w, t_end=w.t_end, layout=1, name=f"burgers blocked m{model}")
    assert np.array_equal(U0, U1)


@pytest.mark.parametrize("omega", [0.7, 1.6])
def test_burgers_1d_omega_and_dirichlet(omega):
    """Prescribed u on both sides (Dirichlet), over-/under-relaxed."""
    w = wl.burgers_riemann(700, 0.9, -0.3, t_end=0.8)
    w.sides = (wl.DIRICHLET, wl.DIRICHLET, 0, 0)
    w.dirichlet_W = (np.array([[0.9]]), np.array([[-0.3]]), None, None)
    compare(w, t_end=w.t_end, omega=omega, name=f"burgers dirichlet w{omega}")


def test_linear_advection_periodic_1d():
    n = 300
    x = wl.centres(n, 0.0, 1.0)
    W = (1.0 + 0.5 * np.sin(2 * np.pi * x))[None, None, :]
    w = wl.Workload("advect", wl.D1Q2, n, 1, (0.0, 1.0, 0.0, 1.0), W, sides=(1, 1, 0, 0),
                    flux=wl.FLUX_QUADRATIC, quad=(0.7, 0.0, 0.0, 0.0))
    compare(w, max_steps=400, omega=1.3, name="advection 1d")


@pytest.mark.parametrize("case", [1, 2])
@pytest.mark.parametrize("tile", [None, (0, 16), (5, 4), (13, 1)])
def test_spekreijse_cases(case, tile):
    """The paper's 2D Burgers cases, 64 x 64, to the steady state (t = 3)."""
    w = wl.spekreijse(case, 64, t_end=3.0)
    compare(w, t_end=w.t_end, tile=tile, name=f"spekreijse {case} {tile}")


@pytest.mark.parametrize("sides", [(1, 1, 1, 1), (0, 0, 1, 1), (3, 3, 3, 3), (1, 1, 3, 0)])
@pytest.mark.parametrize("layout", [0, 1])
def test_general_quadratic_2d(sides, layout):
    """A general quadratic flux pair on odd sizes, random smooth data, every
    side condition the scalar laws take, both layouts."""
    nx, ny = 131, 97
    rng = np.random.default_rng(5)
    c = wl.centres(nx, 0.0, 1.0)
    X, Y = np.meshgrid(c, c[:ny], indexing="xy")
    W = (0.4 + 0.3 * np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y)
         + 0.05 * rng.standard_normal((ny, nx)))[None]
    dirichlet = tuple((0.3 + 0.2 * np.sin(np.linspace(0, 3, ny if s < 2 else nx)))[None, :]
                      if sides[s] == wl.DIRICHLET else None for s in range(4))
    w = wl.Workload("quad2d", wl.D2Q4, nx, ny, (0.0, 1.0, 0.0, ny / nx), W, sides=sides,
                    dirichlet_W=dirichlet, flux=wl.FLUX_QUADRATIC, quad=(0.3, 1.0, -0.7, 0.5))
    compare(w, max_steps=80, omega=1.4, layout=layout, name=f"quad2d {sides} L{layout}")


def test_scalar_frozen_lambda():
    w = wl.spekreijse(2, 64)
    compare(w, max_steps=100, lam_mode=1, name="spekreijse frozen")


def test_spekreijse_large_first_steps():
    """The 2D Burgers case at 2048^2 in the automatic launch shape: ten steps
    against the oracle on every cell."""
    w = wl.spekreijse(1, 2048)
    compare(w, max_steps=10, name="spekreijse 2048 x10")


def test_scalar_rejects_euler_only_calls():
    w = wl.spekreijse(1, 64)
    sim = gpu_sim(w, lam_mode=1)
    sim.init_primitive(w.W)
    tape = torch.empty((1, 64, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(lbrs.LBRSError) as e:
        lbrs.lbrs_step_tape(sim.ctx, tape)
    assert e.value.code == lbrs.LBRS_E_STATE
    f = sim.get_f()
    sim.set_f(f, 0.0, 0)  # round trip keeps the state
    sim.step(3)
    assert sim.state()["rc"] == 0
    sim.close()
