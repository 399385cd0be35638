"""GPU adjoint (hand-written VJP of the fixed-speed D2Q4 step) against the
oracle's forward-mode dual numbers, and the checkpointed gradient against
central finite differences at the full 2048^2 / 2000-step size."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import adjoint, lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import report

pytestmark = pytest.mark.gpu

LAYOUTS = [0, 1]


def _sim(n, lam, layout, omega=1.0):
    return lbrs.Sim(lbrs.LBRS_D2Q4, n, n, omega=omega, bc=(1, 1, 1, 1),
                    lambda_mode=lbrs.LBRS_LAMBDA_USER, lambda_user=lam, layout=layout)


def _oracle_problem(n, lam, omega=1.0):
    return oracle.Problem(model=oracle.D2Q4, nx=n, ny=n, omega=omega, sides=(1, 1, 1, 1),
                          lam_mode=oracle.LAM_USER, lam_user=lam)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("omega", [0.7, 1.0, 1.6])
def test_adjoint_step_equals_bruteforce_transpose(omega, layout):
    """Every entry of L^T fbar, L = d(step)/df at f^3, against the transpose built
    column by column from the oracle's tangent (dual numbers) on a 6 x 6 grid."""
    n, lam, steps = 6, 3.0, 3
    w = wl.fourier_modes(n, seed=11)
    P = _oracle_problem(n, lam, omega)
    ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=steps, want_f=True)
    fbar = np.random.default_rng(5).standard_normal((4, 4, n, n))
    expect = np.zeros(16 * n * n)
    for j in range(16 * n * n):
        e = np.zeros(16 * n * n)
        e[j] = 1.0
        _, col = oracle.step_fixed(P, ref.f, lam, df=e)
        expect[j] = np.sum(col * fbar)
    sim = _sim(n, lam, layout, omega)
    sim.init_primitive(w.W)
    sim.step(steps)
    tape = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    lbrs.lbrs_step_tape(sim.ctx, tape)
    gn = sim.from_planar(torch.from_numpy(fbar).cuda())
    g = torch.empty_like(gn)
    lbrs.lbrs_adjoint_step(sim.ctx, tape, gn, g)
    got = sim.to_planar(g).cpu().numpy().ravel()
    err = np.max(np.abs(got - expect)) / np.max(np.abs(expect))
    report("adjoint bruteforce", omega=omega, layout=layout, rel=err)
    assert err <= 1e-12


@pytest.mark.parametrize("layout", LAYOUTS)
def test_tape_equals_moments_and_dot_product(layout):
    """130^2 periodic (three strips, ragged): the tape written by lbrs_step_tape is
    U^n bit for bit, and <L df, fbar> (oracle tangent) = <df, L^T fbar> (GPU)."""
    n, lam = 130, 2.9
    w = wl.fourier_modes(n, seed=4)
    sim = _sim(n, lam, layout, omega=1.3)
    sim.init_primitive(w.W)
    sim.step(7)
    U7 = sim.moments().clone()
    tape = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    lbrs.lbrs_step_tape(sim.ctx, tape)
    assert torch.equal(tape, U7)
    P = _oracle_problem(n, lam, omega=1.3)
    ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=7, want_f=True)
    rng = np.random.default_rng(9)
    df = rng.standard_normal((4, 4, n, n))
    fbar = rng.standard_normal((4, 4, n, n))
    _, Ldf = oracle.step_fixed(P, ref.f, lam, df=df)
    lhs = float(np.sum(Ldf * fbar))
    g = torch.empty(sim.f_shape, dtype=torch.float64, device="cuda")
    lbrs.lbrs_adjoint_step(sim.ctx, tape, sim.from_planar(torch.from_numpy(fbar).cuda()), g)
    rhs = float(np.sum(df * sim.to_planar(g).cpu().numpy()))
    report("dot product", layout=layout, lhs=lhs, rhs=rhs)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_adjoint_init_dot_product():
    """<d f^0, fbar0> with d f^0 = (df^eq/dU0) dU0 from the oracle's dual numbers
    equals <dU0, Ubar0> from lbrs_adjoint_init."""
    n, lam = 40, 3.1
    w = wl.fourier_modes(n, seed=2)
    P = _oracle_problem(n, lam)
    U0 = oracle.prim_to_cons(P, w.W)
    rng = np.random.default_rng(3)
    dU0 = rng.standard_normal(U0.shape)
    fbar0 = rng.standard_normal((4, 4, n, n))
    _, df0 = oracle.init_tangent(P, U0, dU0, lam)
    lhs = float(np.sum(df0 * fbar0))
    sim = _sim(n, lam, 1)
    Ug = torch.from_numpy(U0).cuda()
    sim.init(Ug)
    Ub = torch.empty_like(Ug)
    lbrs.lbrs_adjoint_init(sim.ctx, sim.from_planar(torch.from_numpy(fbar0).cuda()), Ug, Ub)
    rhs = float(np.sum(dU0 * Ub.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _oracle_dJ(n, steps, rho0, d, window):
    """Directional derivative of J along d by the oracle's dual numbers (its own
    frozen lattice speed of the unperturbed state)."""
    W0 = np.zeros((4, n, n))
    W0[0] = rho0
    W0[3] = rho0 ** 1.4 / 1.4
    Pf = oracle.Problem(model=oracle.D2Q4, nx=n, ny=n, sides=(1, 1, 1, 1),
                        lam_mode=oracle.LAM_FROZEN)
    lam = oracle.initial_lattice_speed(Pf, oracle.prim_to_cons(Pf, W0))
    P = _oracle_problem(n, lam)
    dW = np.zeros_like(W0)
    dW[0] = d
    U, dU = oracle.run_tangent(P, W0, dW, lam, steps, isentropic=True)
    m = wl.window_mask(n, *window)
    return float(np.sum(U[0][m] ** 2)), float(np.sum(2.0 * U[0][m] * dU[0][m]))


@pytest.mark.parametrize("fuse,segment,store_all", [(1, 8, False), (2, 8, False), (2, 7, False),
                                                    (3, 7, False), (4, 7, False),
                                                    (1, None, True), (2, None, True),
                                                    (3, None, True), (4, None, True)])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_gradient_matches_oracle_dual_numbers(layout, fuse, segment, store_all):
    """Gradient (48^2, 60 steps) against the oracle's exact directional
    derivatives along three smooth directions: checkpointed, in single launches
    or with fused forward, recompute and adjoint steps (forward sweeps in two
    to four steps per launch, recompute and adjoint in two; an odd segment
    leaves one single step of each), and with every step's moments
    kept (no checkpoints, no recompute)."""
    n, steps = 48, 60
    w = wl.acoustic_pulse(n, steps=steps)
    rho0 = torch.from_numpy(w.W[0].copy()).cuda()
    spec = adjoint.GradientSpec(n=n, steps=steps, layout=layout, segment=segment, fuse=fuse,
                                store_all=store_all)
    run = adjoint.GradientRunner(spec, rho0)
    r = rho0.clone().requires_grad_(True)
    J = adjoint.LBRSFunction.apply(r, run)
    J.backward()
    grad = r.grad.cpu().numpy()
    for k in range(3):
        d = wl.bump_direction(n, seed=200 + k)
        J_o, dJ_o = _oracle_dJ(n, steps, w.W[0], d, (0.7, 0.8))
        dJ_g = float(np.sum(grad * d))
        report("grad vs dual", k=k, layout=layout, fuse=fuse, store_all=store_all, J=J.item(),
               J_oracle=J_o, gpu=dJ_g, oracle=dJ_o)
        assert abs(J.item() - J_o) <= 1e-12 * abs(J_o)
        assert abs(dJ_g - dJ_o) <= 1e-9 * abs(dJ_o)
    run.close()


@pytest.mark.parametrize("fuse", [1, 2])
def test_gradient_finite_differences_full_size(fuse):
    """Full size: 2048^2 periodic acoustic pulse, 2000 steps, sqrt(T) checkpoints
    (segments of 45), single or fused launches; the gradient dJ/drho0 against
    central differences (h = 1e-4) along 16 seeded smooth directions, relative
    error <= 1e-5."""
    n, steps = 2048, 2000
    w = wl.acoustic_pulse(n, steps=steps)
    rho0 = torch.from_numpy(w.W[0].copy()).cuda()
    spec = adjoint.GradientSpec(n=n, steps=steps, fuse=fuse)
    run = adjoint.GradientRunner(spec, rho0)
    report("fd setup", lam=spec.lam, segment=spec.seg, window=run.win)
    r = rho0.clone().requires_grad_(True)
    J = adjoint.LBRSFunction.apply(r, run)
    J.backward()
    grad = r.grad
    h = 1e-4
    worst = 0.0
    for k in range(16):
        d = torch.from_numpy(wl.bump_direction(n, seed=100 + k)).cuda()
        Jp = run.forward(rho0 + h * d, keep=False).item()
        Jm = run.forward(rho0 - h * d, keep=False).item()
        fd = (Jp - Jm) / (2 * h)
        ad = float(torch.sum(grad * d))
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
        report("fd", k=k, J=J.item(), fd=fd, adjoint=ad, rel=rel)
        assert rel <= 1e-5
    report("fd worst", rel=worst)
    run.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", [48, 130])
def test_adjoint_step2_equals_two_steps(layout, n):
    """lbrs_adjoint_step2 (two reverse steps per launch) against two calls of
    lbrs_adjoint_step on the same tapes and random fbar, ragged strips and
    segments included."""
    w = wl.fourier_modes(n, seed=5)
    sim = lbrs.Sim(lbrs.LBRS_D2Q4, n, n, gamma=w.gamma, omega=1.3, cfl=w.cfl, bc=(1, 1, 1, 1),
                   lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT, layout=layout)
    sim.init_primitive(w.W)
    t0 = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    t1 = torch.empty_like(t0)
    lbrs.lbrs_step_tape(sim.ctx, t0)
    lbrs.lbrs_step_tape(sim.ctx, t1)
    rng = np.random.default_rng(4)
    g2 = torch.from_numpy(rng.standard_normal(16 * n * n)).cuda()
    g1 = torch.empty_like(g2)
    g0 = torch.empty_like(g2)
    lbrs.lbrs_adjoint_step(sim.ctx, t1, g2, g1)
    lbrs.lbrs_adjoint_step(sim.ctx, t0, g1, g0)
    h0 = torch.empty_like(g2)
    for tile in [(0, 4), (0, 8), (3, 2), (0, 1)]:
        sim.set_tile(*tile)
        h0.fill_(float("nan"))
        lbrs.lbrs_adjoint_step2(sim.ctx, t1, t0, g2, h0)
        diff = float((h0 - g0).abs().max())
        report("adjoint step2", n=n, layout=layout, tile=tile, max_abs=diff,
               bitwise=bool(torch.equal(h0, g0)))
        assert diff <= 1e-12 * float(g0.abs().max())
    with pytest.raises(lbrs.LBRSError):
        lbrs.lbrs_adjoint_step2(sim.ctx, t1, t0, g2, g2)
    sim.close()


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", [48, 130])
def test_adjoint_steps_equals_single_steps(layout, n, k):
    """lbrs_adjoint_steps (k reverse steps per launch) against k calls of
    lbrs_adjoint_step on the same tapes and random fbar, ragged strips and
    segments included; tapes from lbrs_step_tapes against k taped single
    steps."""
    w = wl.fourier_modes(n, seed=5)
    sim = lbrs.Sim(lbrs.LBRS_D2Q4, n, n, gamma=w.gamma, omega=1.3, cfl=w.cfl, bc=(1, 1, 1, 1),
                   lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT, layout=layout)
    sim.init_primitive(w.W)
    f0 = sim.get_f()
    st0 = sim.state()
    tapes = torch.empty((k, 4, n, n), dtype=torch.float64, device="cuda")
    for s in range(k):
        lbrs.lbrs_step_tape(sim.ctx, tapes[s])
    f_single = sim.get_f()
    # the same k taped steps in one fused launch
    sim.set_f(f0, st0["t"], st0["nsteps"])
    tk = torch.full_like(tapes, float("nan"))
    lbrs.lbrs_step_tapes(sim.ctx, k, tk)
    dt = float((tk - tapes).abs().max())
    df = float((sim.get_f() - f_single).abs().max())
    report("step tapes", k=k, n=n, layout=layout, tape_diff=dt, f_diff=df)
    assert sim.state()["nsteps"] == k
    assert dt <= 1e-12 * float(tapes.abs().max()) and df <= 1e-12 * float(f_single.abs().max())
    rng = np.random.default_rng(4 + k)
    g = torch.from_numpy(rng.standard_normal(16 * n * n)).cuda()
    ref = g.clone()
    nxt = torch.empty_like(g)
    for s in reversed(range(k)):
        lbrs.lbrs_adjoint_step(sim.ctx, tapes[s], ref, nxt)
        ref, nxt = nxt, ref
    h0 = torch.empty_like(g)
    for tile in [(0, 4), (0, 8), (3, 2), (0, 1)]:
        sim.set_tile(*tile)
        h0.fill_(float("nan"))
        lbrs.lbrs_adjoint_steps(sim.ctx, k, tapes, g, h0)
        diff = float((h0 - ref).abs().max())
        report("adjoint steps", k=k, n=n, layout=layout, tile=tile, max_abs=diff,
               bitwise=bool(torch.equal(h0, ref)))
        assert diff <= 1e-12 * float(ref.abs().max())
    with pytest.raises(lbrs.LBRSError):
        lbrs.lbrs_adjoint_steps(sim.ctx, k, tapes, g, g)
    with pytest.raises(lbrs.LBRSError):
        lbrs.lbrs_adjoint_steps(sim.ctx, 5, tapes, g, h0)
    sim.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", [70, 130])
def test_step_tape2_equals_two_taped_steps(layout, n):
    """lbrs_step_tape2 (two taped steps in fused launches) against two calls of
    lbrs_step_tape from the same state: tapes, populations, time and count."""
    w = wl.fourier_modes(n, seed=6)
    outs = []
    for fused in (False, True):
        sim = lbrs.Sim(lbrs.LBRS_D2Q4, n, n, gamma=w.gamma, omega=1.3, cfl=w.cfl,
                       bc=(1, 1, 1, 1), lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT, layout=layout)
        sim.init_primitive(w.W)
        sim.step(3)
        t0 = torch.full((4, n, n), float("nan"), dtype=torch.float64, device="cuda")
        t1 = torch.full_like(t0, float("nan"))
        if fused:
            lbrs.lbrs_step_tape2(sim.ctx, t0, t1)
            with pytest.raises(lbrs.LBRSError):
                lbrs.lbrs_step_tape2(sim.ctx, t0, t0)
        else:
            lbrs.lbrs_step_tape(sim.ctx, t0)
            lbrs.lbrs_step_tape(sim.ctx, t1)
        outs.append((t0, t1, sim.get_f(), sim.state()))
        sim.close()
    (a0, a1, fa, sa), (b0, b1, fb, sb) = outs
    assert sa["nsteps"] == sb["nsteps"] == 5 and sa["t"] == sb["t"]
    d = max(float((a0 - b0).abs().max()), float((a1 - b1).abs().max()),
            float((fa - fb).abs().max()))
    report("step_tape2", n=n, layout=layout, max_abs=d,
           bitwise=bool(torch.equal(a0, b0) and torch.equal(a1, b1) and torch.equal(fa, fb)))
    assert d <= 1e-12


def _gradient(spec, rho0):
    run = adjoint.GradientRunner(spec, rho0)
    r = rho0.clone().requires_grad_(True)
    J = adjoint.LBRSFunction.apply(r, run)
    J.backward()
    used = run.store_all
    run.close()
    del run
    torch.cuda.empty_cache()
    return J.item(), r.grad.cpu(), used


@pytest.mark.parametrize("n,steps", [(70, 37), (2048, 2000)])
def test_store_all_equals_checkpointed(n, steps):
    """Every step's moments kept (lbrs_forward_taped / lbrs_backward_taped)
    against sqrt(T) checkpoints, fused launches, at a ragged size with an odd
    step count and at full size (2048^2, 2000 steps: a 250 GiB tape): the
    same J and the same gradient (fixed speed: the taped steps are the same
    bits either way)."""
    w = wl.acoustic_pulse(n, steps=steps)
    rho0 = torch.from_numpy(w.W[0].copy()).cuda()
    Jc, gc, used_c = _gradient(adjoint.GradientSpec(n=n, steps=steps, fuse=2), rho0)
    # the full-size tape is taken only if the device holds it (automatic choice)
    store_all = True if n < 1024 else None
    Js, gs, used_s = _gradient(adjoint.GradientSpec(n=n, steps=steps, fuse=2, store_all=store_all),
                               rho0)
    assert not used_c
    if not used_s:
        free, total = torch.cuda.mem_get_info()
        pytest.skip(f"a {steps * 32 * n * n / 2**30:.0f} GiB tape does not fit "
                    f"({free / 2**30:.0f} of {total / 2**30:.0f} GiB free)")
    diff = float((gs - gc).abs().max() / gc.abs().max())
    report("store all vs checkpointed", n=n, steps=steps, J=Js, J_ckpt=Jc, rel=diff,
           bitwise=bool(torch.equal(gs, gc)))
    assert abs(Js - Jc) <= 1e-13 * abs(Jc)
    assert diff <= 1e-12
