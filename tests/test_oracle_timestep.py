"""Pins of the oracle's time-step rule (no GPU).

The rule under test (readings of Sec. II.A, II.C and II.D): every step n takes
lambda*_n = the largest local wave-speed bound over the cells of U^n (the
moments before collision), dt_n = min(cfl dx / lambda*_n, t_end - t_n) and the
lattice speed dx/dt_n (exact hopping, lambda dt = dx); the clipped last step
lands on t_end.  With a frozen speed, lambda = lambda*(U0)/cfl for every step.

Nothing here reuses the oracle's bound formula: lambda* is recomputed from
each U^n as the largest |eigenvalue| of the flux Jacobian (1D) or of
s_x A_1 + s_y A_2 over s in {+-1}^2 (2D), the Jacobians by complex-step
differentiation of the Euler fluxes and the eigenvalues by numpy; and the
first steps of the paper's cases are checked against hand values.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1504_07034_amd import workloads as wl


def problem(w, **kw):
    args = dict(model=w.model, nx=w.nx, ny=w.ny, domain=w.domain, gamma=w.gamma, omega=w.omega,
                cfl=w.cfl, sides=w.sides)
    args.update(kw)
    return oracle.Problem(**args)


# ------------------------------------------------------------ independent bound
def _euler_flux(U, gamma, axis):
    """Euler flux along x (axis 0) or y (axis 1) of conserved states U [K, n]
    (K = 3: (rho, rho u, rho E); K = 4: (rho, rho u, rho v, rho E)); complex-safe."""
    K = U.shape[0]
    rho = U[0]
    if K == 3:
        u = U[1] / rho
        p = (gamma - 1.0) * (U[2] - 0.5 * rho * u * u)
        return np.stack([U[1], U[1] * u + p, u * (U[2] + p)])
    u, v = U[1] / rho, U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    if axis == 0:
        return np.stack([U[1], U[1] * u + p, U[2] * u, u * (U[3] + p)])
    return np.stack([U[2], U[1] * v, U[2] * v + p, v * (U[3] + p)])


def _jacobians(U, gamma, axis):
    """dG/dU per cell [n, K, K] by complex steps (exact to rounding)."""
    K, n = U.shape
    J = np.empty((n, K, K))
    h = 1e-30
    for j in range(K):
        Uc = U.astype(complex)
        Uc[j] += 1j * h
        J[:, :, j] = (_euler_flux(Uc, gamma, axis).imag / h).T
    return J


def spectral_bound(U, gamma):
    """Largest |eigenvalue| over cells of A (1D) or of s_x A1 + s_y A2 (2D)."""
    K = U.shape[0]
    U = U.reshape(K, -1)
    if K == 3:
        return float(np.max(np.abs(np.linalg.eigvals(_jacobians(U, gamma, 0)))))
    A1, A2 = _jacobians(U, gamma, 0), _jacobians(U, gamma, 1)
    return float(max(np.max(np.abs(np.linalg.eigvals(A1 + s * A2))) for s in (1.0, -1.0)))


def _states(P, U0, t_end, nsteps):
    """U^n for n = 0 .. nsteps-1 (each by a fresh run of n steps)."""
    out = [oracle.run(P, U0, t_end=t_end, max_steps=0).U]
    for n in range(1, nsteps):
        r = oracle.run(P, U0, t_end=t_end, max_steps=n)
        assert r.nsteps == n
        out.append(r.U)
    return out


def _check_sequence(P, U0, t_end, ref, states, complete=True):
    """dt_n = min(cfl dx / lambda*(U^n), t_end - t_n), lambda_n = dx/dt_n,
    t_{n+1} = t_n + dt_n; a complete run ends on the first step that reaches
    t_end."""
    dx = P.dx
    t = 0.0
    lam_star = []
    for n, Un in enumerate(states):
        ls = spectral_bound(Un, P.gamma)
        lam_star.append(ls)
        want = P.cfl * dx / ls
        rem = t_end - t
        last = complete and n == ref.nsteps - 1
        if last:
            assert want >= rem * (1 - 1e-12), "the run stopped before t_end"
            assert ref.dt[n] == rem           # clipped onto t_end exactly
        else:
            assert want < rem
            assert ref.dt[n] == pytest.approx(want, rel=1e-12), n
        assert ref.lam[n] == pytest.approx(dx / ref.dt[n], rel=1e-15)
        t = t_end if last else t + ref.dt[n]
    assert ref.t == t
    if complete:
        assert ref.t == t_end and len(states) == ref.nsteps
    return np.array(lam_star)


def test_dt_rule_four_quadrant_riemann():
    """The 2D Riemann problem of the benchmark (D2Q4, cfl 0.5) at 32^2 to a
    t_end that clips the last step: every dt and lattice speed from lambda* of
    U^n, recomputed by eigenvalues.  lambda* moves by more than 1e-5 relative
    between steps here, so taking it from U^{n+1} (after collision and
    streaming) instead of U^n, or a missing cfl factor, fails."""
    w = wl.riemann2d(32)
    P = problem(w)
    U0 = oracle.prim_to_cons(P, w.W)
    t_end = 0.1531
    ref = oracle.run(P, U0, t_end=t_end)
    assert ref.status == 0 and 20 < ref.nsteps < 40
    lam_star = _check_sequence(P, U0, t_end, ref, _states(P, U0, t_end, ref.nsteps))
    steps = np.abs(np.diff(lam_star)) / lam_star[1:]
    assert np.max(steps) > 1e-5


def test_dt_rule_sod_d1q3():
    """Sod's tube (D1Q3, cfl 0.5, 400 cells): the same rule over the first 60
    steps, checked step by step, and the clip at t = 0.2 on a run of 100 cells."""
    w = wl.sod(400)
    P = problem(w)
    U0 = oracle.prim_to_cons(P, w.W)
    ref = oracle.run(P, U0, t_end=0.2)
    assert ref.status == 0 and ref.t == 0.2
    head = oracle.run(P, U0, t_end=0.2, max_steps=60)
    _check_sequence(P, U0, 0.2, head, _states(P, U0, 0.2, 60), complete=False)
    np.testing.assert_array_equal(head.dt, ref.dt[:60])
    w = wl.sod(100)
    P = problem(w)
    U0 = oracle.prim_to_cons(P, w.W)
    ref = oracle.run(P, U0, t_end=0.2)
    _check_sequence(P, U0, 0.2, ref, _states(P, U0, 0.2, ref.nsteps))


def test_first_steps_hand_values():
    """Hand values of the first step.  Sod: the left state (1, 0, 1) bounds
    the speeds, lambda*_0 = |u| + a = sqrt(1.4), dt_0 = 0.5 (1/400)/sqrt(1.4), lattice
    speed 2 sqrt(1.4).  The four-quadrant problem: the SW quadrant (0.138, 1.206,
    1.206, 0.029) bounds them, lambda*_0 = |u + v| + sqrt(2) a = 2.412 +
    sqrt(2 * 1.4 * 0.029 / 0.138) = 3.17909..."""
    w = wl.sod(400)
    P = problem(w)
    r = oracle.run(P, oracle.prim_to_cons(P, w.W), t_end=0.2, max_steps=1)
    assert r.dt[0] == pytest.approx(0.5 * (1.0 / 400) / math.sqrt(1.4), rel=1e-14)
    assert r.lam[0] == pytest.approx(2.0 * math.sqrt(1.4), rel=1e-14)
    assert oracle.initial_lattice_speed(P, oracle.prim_to_cons(P, w.W)) == \
        pytest.approx(2.0 * math.sqrt(1.4), rel=1e-14)
    n = 64
    w = wl.riemann2d(n)
    P = problem(w)
    r = oracle.run(P, oracle.prim_to_cons(P, w.W), t_end=0.3, max_steps=1)
    lam0 = 2.412 + math.sqrt(2.0 * 1.4 * 0.029 / 0.138)
    assert lam0 == pytest.approx(3.179, abs=5e-4)
    assert r.dt[0] == pytest.approx(0.5 * (1.0 / n) / lam0, rel=1e-13)
    assert r.lam[0] == pytest.approx(lam0 / 0.5, rel=1e-13)


def test_frozen_acoustic_pulse_speed():
    """Frozen mode on the acoustic pulse: u = v = 0 and p = rho^gamma/gamma give
    a = rho^0.2 and the bound sqrt(2) a, largest at the densest cell centre, so
    the lattice speed is 2 sqrt(2) rho_max^0.2 (-> 2 sqrt(2) 1.01^0.2 = 2.834
    as the grid refines); dt = dx/lambda on every step, no clip at t_end."""
    for n in (32, 2048):
        w = wl.acoustic_pulse(n, steps=4)
        rho_max = float(w.W[0].max())
        lam = 2.0 * math.sqrt(2.0) * rho_max ** 0.2
        if n == 2048:
            # the densest centre sits sqrt(2) half a cell from the pulse centre
            assert lam == pytest.approx(2.0 * math.sqrt(2.0) * 1.01 ** 0.2, rel=2e-7)
            assert lam == pytest.approx(2.834, abs=5e-4)
            continue
        P = problem(w, lam_mode=oracle.LAM_FROZEN)
        U0 = oracle.prim_to_cons(P, w.W)
        r = oracle.run(P, U0, max_steps=4)
        assert r.nsteps == 4
        np.testing.assert_allclose(r.lam, lam, rtol=1e-14)
        np.testing.assert_allclose(r.dt, P.dx / lam, rtol=1e-14)
        # t_end stops a frozen run after the step that reaches it, unclipped
        r = oracle.run(P, U0, t_end=1.5 * P.dx / lam)
        assert r.nsteps == 2 and r.t == 2 * (P.dx / lam)


# ------------------------------------------------------------ Dirichlet corner (D2)
def _feq_d2q4(U, lam, gamma):
    """D2Q4 equilibria U/4 + (s_x G1 + s_y G2)/(4 lambda), velocities in the
    paper's order (-,-), (+,-), (+,+), (-,+) (Sec. II.D)."""
    U = np.asarray(U, float).reshape(4, 1)
    G1, G2 = _euler_flux(U, gamma, 0)[:, 0], _euler_flux(U, gamma, 1)[:, 0]
    s = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    return np.array([U[:, 0] / 4 + (sx * G1 + sy * G2) / (4 * lam) for sx, sy in s])


@pytest.mark.parametrize("periodic_x", [False, True])
def test_dirichlet_corner_ghost_takes_the_y_side(periodic_x):
    """Reading D2: a ghost cell beyond two sides (a corner) holds the y-side's
    prescribed state at the x index brought onto the grid (clamped, or wrapped
    on a periodic x axis); ghosts beyond one side hold that side's state.
    After one step at a fixed lattice speed the populations pulled from ghosts
    are exactly those equilibria (hand-built here), e.g. f_(+,+) of cell (0, 0)
    comes from the corner ghost (-1, -1)."""
    nx = ny = 6
    D = oracle.DIRICHLET
    sides = (oracle.PERIODIC, oracle.PERIODIC, D, oracle.TRANSMISSIVE) if periodic_x else \
        (D, oracle.TRANSMISSIVE, D, oracle.TRANSMISSIVE)
    rng = np.random.default_rng(5)

    def states(n):
        W = np.stack([rng.uniform(0.8, 1.2, n), rng.uniform(-0.3, 0.3, n),
                      rng.uniform(-0.3, 0.3, n), rng.uniform(0.8, 1.2, n)])
        rho, u, v, p = W
        return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])

    Ux, Uy = states(ny), states(nx)
    lam = 9.0
    P = oracle.Problem(model=oracle.D2Q4, nx=nx, ny=ny, domain=(0.0, 1.0, 0.0, 1.0), sides=sides,
                       lam_mode=oracle.LAM_USER, lam_user=lam,
                       dirichlet=(None if periodic_x else Ux, None, Uy, None))
    W0 = np.stack([np.full((ny, nx), 1.0), np.full((ny, nx), 0.1), np.full((ny, nx), -0.1),
                   np.full((ny, nx), 1.0)])
    r = oracle.run(P, oracle.prim_to_cons(P, W0), max_steps=1, want_f=True)
    assert r.status == 0
    f = r.f  # [Q][K][ny][nx]
    corner = Uy[:, nx - 1] if periodic_x else Uy[:, 0]
    np.testing.assert_allclose(f[2, :, 0, 0], _feq_d2q4(corner, lam, 1.4)[2], rtol=0, atol=1e-15)
    # (+,+) of cell (3, 0): from (2, -1), beyond the y-side only
    np.testing.assert_allclose(f[2, :, 0, 3], _feq_d2q4(Uy[:, 2], lam, 1.4)[2], rtol=0, atol=1e-15)
    # (-,+) of cell (1, 0): from (2, -1)
    np.testing.assert_allclose(f[3, :, 0, 1], _feq_d2q4(Uy[:, 2], lam, 1.4)[3], rtol=0, atol=1e-15)
    if not periodic_x:
        # (+,+) and (+,-) of cell (0, 2): from (-1, 1) and (-1, 3), beyond the x-side only
        np.testing.assert_allclose(f[2, :, 2, 0], _feq_d2q4(Ux[:, 1], lam, 1.4)[2], rtol=0,
                                   atol=1e-15)
        np.testing.assert_allclose(f[1, :, 2, 0], _feq_d2q4(Ux[:, 3], lam, 1.4)[1], rtol=0,
                                   atol=1e-15)
        # the x-side's state is not the corner's (the test can tell the two apart)
        assert np.max(np.abs(_feq_d2q4(Ux[:, 0], lam, 1.4)[2] - f[2, :, 0, 0])) > 1e-3


def test_cfl_max_per_model():
    """Bouchut's condition (Sec. II.D) on the Sec. II.C D1Q3 equilibria
    U/3 -+ G/(2 lambda) needs lambda >= 1.5 max|u -+ a|, i.e. cfl <= 2/3;
    D1Q2 and D2Q4 take cfl <= 1.  A larger cfl is rejected."""
    w = wl.sod(50)
    for model, ok, bad in [(oracle.D1Q2, 1.0, 1.0 + 1e-12), (oracle.D1Q3, 2.0 / 3.0, 0.6667)]:
        P = problem(w, model=model, cfl=ok)
        assert oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=1).status == oracle.OK
        P = problem(w, model=model, cfl=bad)
        assert oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=1).status == oracle.INVAL
    w = wl.riemann2d(16)
    P = problem(w, cfl=1.0)
    assert oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=1).status == oracle.OK
    P = problem(w, cfl=1.0 + 1e-12)
    assert oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=1).status == oracle.INVAL
