"""Seeded synthetic inputs for the LBRS hot path.

This module holds input *data* only: grids, piecewise-constant states, smooth
pulses and seeded random draws, as primitive variables W = (rho, u, [v,] p) in
SoA planes ``[K][ny][nx]`` (float64, numpy).  It contains none of the scheme's
arithmetic (no conversion to conserved variables, no fluxes, no equilibria), so
both the GPU library's tests and the CPU oracle can start from the same arrays.

Grids are cell-centred: x_j = x0 + (j + 1/2) dx with dx = (x1 - x0)/nx.  With
an even cell count no centre lies on a mid-domain interface, so no tie-break
is needed at the discontinuities below.

Model ids: 0 = D1Q2, 1 = D1Q3, 2 = D2Q4.  Side ids: 0 transmissive,
1 periodic, 2 wall, 3 Dirichlet; side order (x-low, x-high, y-low, y-high).
Bodies (the Sec. III step, backward step and ramp cases) are masks of solid
cells, a cell being solid when its centre lies inside the body.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

D1Q2, D1Q3, D2Q4 = 0, 1, 2
TRANSMISSIVE, PERIODIC, WALL, DIRICHLET = 0, 1, 2, 3


FLUX_EULER, FLUX_LINEAR, FLUX_QUADRATIC = 0, 1, 2


@dataclass
class Workload:
    name: str
    model: int
    nx: int
    ny: int
    domain: tuple            # (x0, x1, y0, y1)
    W: np.ndarray            # primitive SoA [K][ny][nx]
    gamma: float = 1.4
    omega: float = 1.0
    cfl: float = 0.5
    sides: tuple = (TRANSMISSIVE,) * 4
    t_end: float = math.inf
    steps: int | None = None  # fixed step count (frozen lattice speed runs)
    meta: dict = field(default_factory=dict)
    # prescribed primitive states of Dirichlet sides (xlo, xhi, ylo, yhi):
    # [K][n] along the side (n = ny for the x-sides, nx for the y-sides)
    dirichlet_W: tuple = (None, None, None, None)
    # conservation law: the Euler equations, or a scalar law with
    # g1(u) = quad[0] u + quad[1] u^2/2, g2(u) = quad[2] u + quad[3] u^2/2
    flux: int = FLUX_EULER
    quad: tuple = (0.0, 0.0, 0.0, 0.0)
    # solid cells of a body [ny][nx] (uint8, nonzero = solid), or None
    solid: np.ndarray | None = None


def centres(n: int, a: float, b: float) -> np.ndarray:
    dx = (b - a) / n
    return a + (np.arange(n) + 0.5) * dx


def _tube(n, domain, xi, left, right, model=D1Q3):
    x = centres(n, domain[0], domain[1])
    W = np.empty((3, 1, n))
    for k in range(3):
        W[k, 0, :] = np.where(x < xi, left[k], right[k])
    return W


def sod(n: int = 400, model: int = D1Q3, omega: float = 1.0, cfl: float = 0.5,
        t_end: float = 0.2) -> Workload:
    """Sod shock tube on [0,1], interface 0.5: (rho,u,p) = (1,0,1) | (0.125,0,0.1)."""
    W = _tube(n, (0.0, 1.0), 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    return Workload("sod", model, n, 1, (0.0, 1.0, 0.0, 1.0), W, omega=omega, cfl=cfl,
                    t_end=t_end, meta={"left": (1.0, 0.0, 1.0), "right": (0.125, 0.0, 0.1),
                                       "x_interface": 0.5})


def sod_dimensional(model: int = D1Q3, omega: float = 1.0, cfl: float = 0.5) -> Workload:
    """The paper's dimensional shock tube (Sec. III): [-10, 10], 50 cells,
    (1 kg/m^3, 0, 1e5 Pa) | (0.125, 0, 1e4), t = 0.01 s."""
    W = _tube(50, (-10.0, 10.0), 0.0, (1.0, 0.0, 1.0e5), (0.125, 0.0, 1.0e4))
    return Workload("sod_dimensional", model, 50, 1, (-10.0, 10.0, 0.0, 1.0), W, omega=omega,
                    cfl=cfl, t_end=0.01, meta={"left": (1.0, 0.0, 1.0e5),
                                               "right": (0.125, 0.0, 1.0e4), "x_interface": 0.0})


def steady_shock(n: int = 400, model: int = D1Q3, omega: float = 1.0, t_end: float = 1.0,
                 mach: float = 2.0, gamma: float = 1.4) -> Workload:
    """Steady shock (Sec. III, after Zhang and Shu) on [-1, 1], shock at x = 0:
    pre-shock rho = 1, p = 1, u = M a with M = 2 (the paper gives only the Mach
    number); post-shock state by the normal-shock relations; transmissive
    sides."""
    rhoL, pL = 1.0, 1.0
    uL = mach * math.sqrt(gamma * pL / rhoL)
    m2 = mach * mach
    rhoR = rhoL * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    pR = pL * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    uR = uL * rhoL / rhoR
    W = _tube(n, (-1.0, 1.0), 0.0, (rhoL, uL, pL), (rhoR, uR, pR), model=model)
    return Workload("steady_shock", model, n, 1, (-1.0, 1.0, 0.0, 1.0), W, gamma=gamma,
                    omega=omega, t_end=t_end,
                    meta={"left": (rhoL, uL, pL), "right": (rhoR, uR, pR)})


def steady_contact(n: int = 100, model: int = D1Q3, omega: float = 1.0,
                   t_end: float = 2.0) -> Workload:
    """Stationary contact (Sec. III): rho 1.4 | 1.0, u = 0, p = 1 on [0,1], split at 0.5."""
    W = _tube(n, (0.0, 1.0), 0.5, (1.4, 0.0, 1.0), (1.0, 0.0, 1.0))
    return Workload("steady_contact", model, n, 1, (0.0, 1.0, 0.0, 1.0), W, omega=omega,
                    t_end=t_end)


def riemann2d(n: int = 4096, states=None, t_end: float = 0.3, omega: float = 1.0,
              cfl: float = 0.5) -> Workload:
    """Four-quadrant 2D Riemann problem on [0,1]^2 split at x = y = 0.5.

    Default quadrant states (rho, u, v, p):
      NE (1.5, 0, 0, 1.5), NW (0.5323, 1.206, 0, 0.3),
      SW (0.138, 1.206, 1.206, 0.029), SE (0.5323, 0, 1.206, 0.3)."""
    if states is None:
        states = {"NE": (1.5, 0.0, 0.0, 1.5), "NW": (0.5323, 1.206, 0.0, 0.3),
                  "SW": (0.138, 1.206, 1.206, 0.029), "SE": (0.5323, 0.0, 1.206, 0.3)}
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")  # [y][x]
    east, north = X > 0.5, Y > 0.5
    W = np.empty((4, n, n))
    for k in range(4):
        W[k] = np.where(north, np.where(east, states["NE"][k], states["NW"][k]),
                        np.where(east, states["SE"][k], states["SW"][k]))
    return Workload("riemann2d", D2Q4, n, n, (0.0, 1.0, 0.0, 1.0), W, omega=omega, cfl=cfl,
                    t_end=t_end, meta={"states": states})


def riemann2d_paper(n: int = 400, t_end: float = 0.25) -> Workload:
    """The paper's 2D Riemann case (Sec. III): quadrants split at the domain
    centre (its garbled "x >= 0, y >= 0" read as x, y >= 0.5 on [0,1]^2)."""
    states = {"NE": (1.1, 0.0, 0.0, 1.1), "NW": (0.5065, 0.8939, 0.0, 0.35),
              "SW": (1.1, 0.8939, 0.8939, 1.1), "SE": (0.5065, 0.0, 0.8939, 0.35)}
    w = riemann2d(n, states=states, t_end=t_end)
    w.name = "riemann2d_paper"
    return w


# Oblique shock reflection (Sec. III): the inflow state and the post-shock state
# the paper prints for the top boundary.
OBLIQUE_INFLOW = (1.0, 2.9, 0.0, 1.0 / 1.4)
OBLIQUE_POST_SHOCK = (1.69997, 2.61934, -0.50633, 1.52819)


def oblique_shock(nx: int = 240, ny: int = 80, t_end: float = 4.0, omega: float = 1.0) -> Workload:
    """Oblique shock reflection (Sec. III) on an nx x ny grid: the inflow state
    prescribed on the left side, the post-shock state on the top side, a
    free-slip wall at the bottom, a transmissive (supersonic outflow) right
    side; the interior starts at the inflow state.  The domain extent is not
    given: [0, nx/ny] x [0, 1], i.e. [0, 3] x [0, 1] with square cells at
    240 x 80, so that the shock enters at the top-left corner."""
    W = np.empty((4, ny, nx))
    for k in range(4):
        W[k] = OBLIQUE_INFLOW[k]
    inflow = np.repeat(np.asarray(OBLIQUE_INFLOW, dtype=np.float64)[:, None], ny, axis=1)
    top = np.repeat(np.asarray(OBLIQUE_POST_SHOCK, dtype=np.float64)[:, None], nx, axis=1)
    return Workload("oblique_shock", D2Q4, nx, ny, (0.0, nx / ny, 0.0, 1.0), W, omega=omega,
                    t_end=t_end, sides=(DIRICHLET, TRANSMISSIVE, WALL, DIRICHLET),
                    dirichlet_W=(inflow, None, None, top))


def _uniform(nx: int, ny: int, state) -> np.ndarray:
    W = np.empty((4, ny, nx))
    for k in range(4):
        W[k] = state[k]
    return W


def _along(state, n: int) -> np.ndarray:
    return np.repeat(np.asarray(state, dtype=np.float64)[:, None], n, axis=1)


def _cell_mask(nx: int, ny: int, domain, inside) -> np.ndarray:
    """uint8 [ny][nx]: 1 where inside(x, y) holds at the cell centre."""
    X, Y = np.meshgrid(centres(nx, domain[0], domain[1]), centres(ny, domain[2], domain[3]))
    return inside(X, Y).astype(np.uint8)


def forward_step(nx: int = 240, ny: int = 80, t_end: float = 4.0, omega: float = 1.0,
                 mach: float = 3.0, step_x: float = 0.6, step_h: float = 0.2) -> Workload:
    """Mach 3 flow over a forward-facing step in the channel [0, 3] x [0, 1]
    (Sec. III; 240 x 80 cells, t = 4, the interior starts at the inflow
    state, free-slip walls).  The step itself is not given: a step of height
    0.2 from x = 0.6 to the outflow.  Inflow (rho, u, v, p) = (1.4, M, 0, 1),
    so that the sound speed is 1; prescribed on the left side, transmissive
    (supersonic outflow) right side, walls at the bottom and the top."""
    domain = (0.0, 3.0, 0.0, 1.0)
    inflow = (1.4, mach, 0.0, 1.0)
    solid = _cell_mask(nx, ny, domain, lambda x, y: (x > step_x) & (y < step_h))
    return Workload("forward_step", D2Q4, nx, ny, domain, _uniform(nx, ny, inflow), omega=omega,
                    t_end=t_end, sides=(DIRICHLET, TRANSMISSIVE, WALL, WALL),
                    dirichlet_W=(_along(inflow, ny), None, None, None), solid=solid,
                    meta={"mach": mach, "step_x": step_x, "step_h": step_h})


def moving_shock_state(mach: float, rho1: float = 1.4, p1: float = 1.0,
                       gamma: float = 1.4) -> tuple:
    """(rho, u, v, p) behind a normal shock of Mach number `mach` running
    into gas at rest (rho1, p1): the normal-shock relations in the shock's
    frame, shifted by the shock speed mach * a1."""
    a1 = math.sqrt(gamma * p1 / rho1)
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    u2 = mach * a1 * (1.0 - rho1 / rho2)
    return (rho2, u2, 0.0, p2)


def shock_diffraction(n: int = 400, t_end: float = 0.1561, omega: float = 1.0,
                      mach: float = 5.09, corner=(0.2, 0.5)) -> Workload:
    """A Mach 5.09 shock diffracting over a backward-facing step in [0, 1]^2
    (Sec. III; 400 x 400 cells, t = 0.1561), the shock starting at the
    step's tip.  The step is not given: the body is [0, 0.2] x [0, 0.5] (a
    shock starting at x = 0.2 runs 0.795 in that time, reaching the right
    side).  Gas at rest (1.4, 0, 0, 1) ahead of the shock, the post-shock
    state behind it and prescribed on the left side; the other sides are
    transmissive."""
    domain = (0.0, 1.0, 0.0, 1.0)
    xc, yc = corner
    post = moving_shock_state(mach)
    rest = (1.4, 0.0, 0.0, 1.0)
    X, _ = np.meshgrid(centres(n, 0.0, 1.0), centres(n, 0.0, 1.0))
    W = np.empty((4, n, n))
    for k in range(4):
        W[k] = np.where(X < xc, post[k], rest[k])
    solid = _cell_mask(n, n, domain, lambda x, y: (x < xc) & (y < yc))
    return Workload("shock_diffraction", D2Q4, n, n, domain, W, omega=omega, t_end=t_end,
                    sides=(DIRICHLET, TRANSMISSIVE, TRANSMISSIVE, TRANSMISSIVE),
                    dirichlet_W=(_along(post, n), None, None, None), solid=solid,
                    meta={"mach": mach, "corner": corner, "post": post})


def ramp(nx: int = 240, ny: int = 80, t_end: float = 4.0, omega: float = 1.0, mach: float = 2.0,
         angle_deg: float = 15.0, x_start: float = 0.5, x_end: float = 1.5) -> Workload:
    """Mach 2 flow over a compression ramp in a channel (Sec. III; 240 x 80
    cells).  Channel, ramp and end time are not given: the channel
    [0, 3] x [0, 1] of the step case, a 15-degree ramp from x = 0.5 to 1.5
    followed by a flat top (a compression corner and an expansion corner),
    t = 4, the interior starting at the inflow state (1.4, M, 0, 1); inflow
    prescribed on the left, transmissive right side, walls at the bottom and
    the top.  Cells whose centres lie below the ramp's surface are solid."""
    domain = (0.0, 3.0, 0.0, 1.0)
    inflow = (1.4, mach, 0.0, 1.0)
    slope = math.tan(math.radians(angle_deg))

    def below(x, y):
        h = slope * (np.clip(x, x_start, x_end) - x_start)
        return y < h

    solid = _cell_mask(nx, ny, domain, below)
    return Workload("ramp", D2Q4, nx, ny, domain, _uniform(nx, ny, inflow), omega=omega,
                    t_end=t_end, sides=(DIRICHLET, TRANSMISSIVE, WALL, WALL),
                    dirichlet_W=(_along(inflow, ny), None, None, None), solid=solid,
                    meta={"mach": mach, "angle_deg": angle_deg, "x_start": x_start,
                          "x_end": x_end})


def burgers_riemann(n: int = 400, uL: float = 1.0, uR: float = 0.0, t_end: float = 0.5,
                    model: int = D1Q2, omega: float = 1.0) -> Workload:
    """Inviscid Burgers equation u_t + (u^2/2)_x = 0 (Sec. II.A) on [-1, 1]
    with a jump at x = 0, transmissive sides."""
    x = centres(n, -1.0, 1.0)
    W = np.where(x < 0.0, uL, uR)[None, None, :].astype(np.float64)
    return Workload("burgers_riemann", model, n, 1, (-1.0, 1.0, 0.0, 1.0), W, omega=omega,
                    t_end=t_end, flux=FLUX_QUADRATIC, quad=(0.0, 1.0, 0.0, 0.0),
                    meta={"uL": uL, "uR": uR})


def spekreijse(case: int = 1, n: int = 64, t_end: float = 3.0, omega: float = 1.0) -> Workload:
    """2D inviscid Burgers u_t + (u^2/2)_x + u_y = 0 on [0,1]^2 (Sec. III,
    after Spekreijse), n x n, D2Q4, prescribed u on the left, right and bottom
    sides (case 1: 1, -1, 1 - 2x; case 2: 1.5, -0.5, 1.5 - 2x), outflow
    (transmissive) on top.  The initial state is not given: u = 0 inside,
    run to a steady state."""
    left, right, c0 = (1.0, -1.0, 1.0) if case == 1 else (1.5, -0.5, 1.5)
    x = centres(n, 0.0, 1.0)
    W = np.zeros((1, n, n))
    dirichlet = (np.full((1, n), left), np.full((1, n), right), (c0 - 2.0 * x)[None, :].copy(),
                 None)
    return Workload(f"spekreijse{case}", D2Q4, n, n, (0.0, 1.0, 0.0, 1.0), W, omega=omega,
                    t_end=t_end, sides=(DIRICHLET, DIRICHLET, DIRICHLET, TRANSMISSIVE),
                    dirichlet_W=dirichlet, flux=FLUX_QUADRATIC, quad=(0.0, 1.0, 1.0, 0.0),
                    meta={"case": case})


def explosion(n: int = 400, t_end: float = 0.25, omega: float = 1.0) -> Workload:
    """Explosion (Sec. III): [-1,1]^2, (1,0,0,1) for r < 0.4, (0.125,0,0,0.1) outside."""
    x = centres(n, -1.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    inside = X * X + Y * Y < 0.4 * 0.4
    W = np.empty((4, n, n))
    W[0] = np.where(inside, 1.0, 0.125)
    W[1] = 0.0
    W[2] = 0.0
    W[3] = np.where(inside, 1.0, 0.1)
    return Workload("explosion", D2Q4, n, n, (-1.0, 1.0, -1.0, 1.0), W, omega=omega, t_end=t_end)


def acoustic_pulse(n: int = 2048, steps: int = 2000, gamma: float = 1.4) -> Workload:
    """Periodic [0,1]^2, rho = 1 + 0.01 exp(-r^2/0.05^2) about (0.5, 0.5), u = v = 0,
    p = rho^gamma/gamma (isentropic), run for a fixed number of steps at a frozen
    lattice speed; objective J = sum of rho^2 over cells centred in [0.7,0.8]^2."""
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    W = np.empty((4, n, n))
    W[0] = 1.0 + 0.01 * np.exp(-r2 / 0.05 ** 2)
    W[1] = 0.0
    W[2] = 0.0
    W[3] = W[0] ** gamma / gamma
    return Workload("acoustic_pulse", D2Q4, n, n, (0.0, 1.0, 0.0, 1.0), W, gamma=gamma,
                    sides=(PERIODIC,) * 4, steps=steps,
                    meta={"window": (0.7, 0.8), "isentropic": True})


def window_mask(n: int, lo: float = 0.7, hi: float = 0.8) -> np.ndarray:
    """Boolean [n][n] mask of cells whose centres lie in the closed square [lo,hi]^2."""
    x = centres(n, 0.0, 1.0)
    inx = (x >= lo) & (x <= hi)
    return inx[:, None] & inx[None, :]


def fourier_modes(n: int, seed: int, nmodes: int = 8, gamma: float = 1.4,
                  steps: int = 1000) -> Workload:
    """Random smooth periodic state: rho = 1 + 0.05 * sum of nmodes seeded modes,
    u, v = 0.1 * seeded modes, p = rho^gamma/gamma.  Each mode is
    cos(2 pi (kx x + ky y) + theta) with integer (kx, ky) in [-4,4]^2 \\ {0},
    theta ~ U[0, 2 pi) and a random sign, normalised by nmodes."""
    rng = np.random.default_rng(seed)
    x = centres(n, 0.0, 1.0)

    def field():
        # cos(a + b) = cos a cos b - sin a sin b with a = 2 pi kx x + theta and
        # b = 2 pi ky y: each mode is a sum of two outer products ([y][x])
        acc = np.zeros((n, n))
        for _ in range(nmodes):
            while True:
                kx, ky = rng.integers(-4, 5, size=2)
                if kx != 0 or ky != 0:
                    break
            th = rng.uniform(0.0, 2.0 * math.pi)
            sg = rng.choice([-1.0, 1.0])
            a = 2.0 * math.pi * kx * x + th
            b = 2.0 * math.pi * ky * x
            acc += sg * (np.outer(np.cos(b), np.cos(a)) - np.outer(np.sin(b), np.sin(a)))
        return acc / nmodes

    W = np.empty((4, n, n))
    W[0] = 1.0 + 0.05 * field()
    W[1] = 0.1 * field()
    W[2] = 0.1 * field()
    W[3] = W[0] ** gamma / gamma
    return Workload(f"fourier{seed}", D2Q4, n, n, (0.0, 1.0, 0.0, 1.0), W, gamma=gamma,
                    sides=(PERIODIC,) * 4, steps=steps, meta={"seed": seed})


def tube_batch(count: int = 1024, seed: int = 0, nmin: int = 200, nmax: int = 20000):
    """Ragged batch of shock tubes: cell counts log-uniform in [nmin, nmax], left and
    right states rho ~ U[0.1,1], u ~ U[-0.5,0.5], p ~ U[0.1,1], t_end ~ U[0.1,0.25];
    domain [0,1], interface 0.5, D1Q3, omega = 1, cfl = 0.5, transmissive."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count)).astype(np.int64)
    ns += ns % 2  # even counts: no cell centre on the interface
    tubes = []
    for b in range(count):
        left = (rng.uniform(0.1, 1.0), rng.uniform(-0.5, 0.5), rng.uniform(0.1, 1.0))
        right = (rng.uniform(0.1, 1.0), rng.uniform(-0.5, 0.5), rng.uniform(0.1, 1.0))
        t_end = rng.uniform(0.1, 0.25)
        W = _tube(int(ns[b]), (0.0, 1.0), 0.5, left, right)
        tubes.append(Workload(f"tube{b}", D1Q3, int(ns[b]), 1, (0.0, 1.0, 0.0, 1.0), W,
                              t_end=t_end, meta={"left": left, "right": right,
                                                 "x_interface": 0.5}))
    return tubes


def domain_batch(count: int = 128, seed: int = 0, sides=(256, 512, 1024, 2048),
                 steps: int = 1000):
    """Ragged batch of periodic 2D domains with side lengths drawn uniformly from
    `sides`; domain b gets the random smooth state fourier_modes(n_b, seed*100000 + b)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sides), size=count)
    return [fourier_modes(int(ns[b]), seed * 100000 + b, steps=steps) for b in range(count)]


def random_states(count: int, seed: int, dim: int = 2):
    """Random admissible primitive states (rho, u, [v,] p), one per row."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 2.0, size=count)
    p = rng.uniform(0.05, 3.0, size=count)
    vel = rng.uniform(-2.0, 2.0, size=(count, dim))
    return np.column_stack([rho, vel, p])


def bump_direction(n: int, seed: int, nbumps: int = 4, width: float = 0.05) -> np.ndarray:
    """Smooth perturbation direction on the periodic [0,1]^2 grid: a sum of nbumps
    Gaussian bumps of the given width with random centres and signs (periodic
    distance), scaled so that max |d| = 1.  Shape [n][n]."""
    rng = np.random.default_rng(seed)
    x = centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x, indexing="xy")
    d = np.zeros((n, n))
    for _ in range(nbumps):
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        sg = rng.choice([-1.0, 1.0])
        dx = np.abs(X - cx)
        dy = np.abs(Y - cy)
        dx = np.minimum(dx, 1.0 - dx)
        dy = np.minimum(dy, 1.0 - dy)
        d += sg * np.exp(-(dx * dx + dy * dy) / width ** 2)
    return d / np.max(np.abs(d))
