"""Batch of independent 2D domains (one launch per step for all domains) against
the single-domain library (bitwise), the oracle, and, for the gradient, the
oracle's dual numbers; graph replays against eager runs."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import TOL, report

pytestmark = pytest.mark.gpu

SIDES_P = (1, 1, 1, 1)


def _doms(ws, mode=lbrs.LBRS_LAMBDA_FROZEN_INIT, lam=None, sides=None, omega=1.0):
    out = []
    for i, w in enumerate(ws):
        lu = 0.0 if lam is None else lam[i]
        m = mode if lam is None else lbrs.LBRS_LAMBDA_USER
        out.append(lbrs.make_params(lbrs.LBRS_D2Q4, w.nx, w.ny, w.domain, w.gamma, omega, w.cfl,
                                    sides[i] if sides else w.sides, m, lu, lbrs.LBRS_LAYOUT_ROWS))
    return out


def _pool_U0(ws, doms):
    U = []
    for w, p in zip(ws, doms):
        Wt = torch.from_numpy(w.W).cuda()
        Uw = torch.empty_like(Wt)
        lbrs.lbrs_prim_to_cons(p, Wt, Uw)
        U.append(Uw.reshape(4, -1))
    return torch.cat(U, dim=1).contiguous()


def _ragged_domains():
    sizes = [32, 130, 64, 200, 45, 96]
    return [wl.fourier_modes(n, seed=20 + i) for i, n in enumerate(sizes)]


def test_batch2d_forward_bitwise_vs_single_domains():
    ws = _ragged_domains()
    doms = _doms(ws)
    B = lbrs.Batch2D(doms)
    B.init(_pool_U0(ws, doms))
    B.step(40)
    U = B.moments()
    st = B.state()
    assert st["rc"] == 0 and st["nsteps"] == 40
    for d, (w, p) in enumerate(zip(ws, doms)):
        sim = lbrs.Sim(lbrs.LBRS_D2Q4, w.nx, w.ny, domain=w.domain, gamma=w.gamma, omega=1.0,
                       cfl=w.cfl, bc=w.sides, lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT,
                       layout=lbrs.LBRS_LAYOUT_ROWS)
        sim.init_primitive(w.W)
        sim.step(40)
        same = torch.equal(sim.moments().reshape(4, -1), U[:, B.unit_slice(d)])
        assert sim.state()["lambda"] == st["lambda"][d]
        report("batch2d vs single", dom=d, n=w.nx, bitwise=same)
        assert same
        sim.close()
    B.close()


@pytest.mark.parametrize("omega", [0.7, 1.5])
def test_batch2d_mixed_sides_vs_oracle(omega):
    """Transmissive, periodic and wall sides in one batch, against the oracle."""
    ws = [wl.explosion(60), wl.riemann2d(80), wl.explosion(50), wl.fourier_modes(40, seed=3)]
    sides = [(0, 0, 0, 0), (1, 1, 0, 0), (1, 1, 2, 2), (2, 0, 1, 1)]
    doms = _doms(ws, sides=sides, omega=omega)
    B = lbrs.Batch2D(doms)
    B.init(_pool_U0(ws, doms))
    B.step(30)
    U = B.moments().cpu().numpy()
    st = B.state()
    for d, w in enumerate(ws):
        P = oracle.Problem(model=oracle.D2Q4, nx=w.nx, ny=w.ny, domain=w.domain, omega=omega,
                           sides=sides[d], lam_mode=oracle.LAM_FROZEN)
        ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=30)
        err = float(np.max(np.abs(U[:, B.unit_slice(d)] - ref.U.reshape(4, -1))))
        report("batch2d vs oracle", dom=d, sides=sides[d], err=err, status=st["status"][d])
        assert ref.status == 0 and st["status"][d] == 0 and err <= TOL
    B.close()


def test_batch2d_adjoint_step_matches_single():
    ws = _ragged_domains()
    doms = _doms(ws)
    B = lbrs.Batch2D(doms)
    B.init(_pool_U0(ws, doms))
    B.step(5)
    tape = torch.empty((4, B.total), dtype=torch.float64, device="cuda")
    B.step_tape(tape)
    rng = np.random.default_rng(1)
    gn = torch.from_numpy(rng.standard_normal(16 * B.total)).cuda()
    g = torch.empty_like(gn)
    B.adjoint_step(tape, gn, g)
    for d, w in enumerate(ws):
        sim = lbrs.Sim(lbrs.LBRS_D2Q4, w.nx, w.ny, domain=w.domain, gamma=w.gamma, cfl=w.cfl,
                       bc=w.sides, lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT,
                       layout=lbrs.LBRS_LAYOUT_ROWS)
        sim.init_primitive(w.W)
        sim.step(5)
        t1 = torch.empty((4, w.ny, w.nx), dtype=torch.float64, device="cuda")
        lbrs.lbrs_step_tape(sim.ctx, t1)
        assert torch.equal(t1.reshape(4, -1), tape[:, B.unit_slice(d)])
        sl = slice(16 * B.offsets[d], 16 * B.offsets[d + 1])
        g1 = torch.empty(16 * w.nx * w.ny, dtype=torch.float64, device="cuda")
        lbrs.lbrs_adjoint_step(sim.ctx, t1, gn[sl].contiguous(), g1)
        assert torch.equal(g1, g[sl])
        sim.close()
    B.close()


def _oracle_dJ_dU(w, steps, dU, window=(0.7, 0.8)):
    """Directional derivative of J along a conserved-state direction dU by dual
    numbers: U0 + eps dU has primitive tangent obtained through the oracle's own
    conversion (run from conserved variables)."""
    P = oracle.Problem(model=oracle.D2Q4, nx=w.nx, ny=w.ny, domain=w.domain, sides=w.sides,
                       lam_mode=oracle.LAM_FROZEN)
    U0 = oracle.prim_to_cons(P, w.W)
    lam = oracle.initial_lattice_speed(P, U0)
    Pu = oracle.Problem(model=oracle.D2Q4, nx=w.nx, ny=w.ny, domain=w.domain, sides=w.sides,
                        lam_mode=oracle.LAM_USER, lam_user=lam)
    f0, df0 = oracle.init_tangent(Pu, U0, dU, lam)
    f, df = f0, df0
    for _ in range(steps):
        f, df = oracle.step_fixed(Pu, f, lam, df=df)
    rho, drho = f[:, 0].sum(0), df[:, 0].sum(0)
    m = wl.window_mask(w.nx, *window)
    return float(np.sum(rho[m] ** 2)), float(np.sum(2 * rho[m] * drho[m]))


def test_batch2d_gradient_graph_vs_oracle_and_replays():
    """Checkpointed gradient of every domain's J through the captured graph:
    J_d and <dJ_d/dU0, dU> against the oracle's dual numbers; three replays with
    eager work in between give the eager result bit for bit."""
    ws = [wl.fourier_modes(n, seed=40 + i) for i, n in enumerate([24, 40, 32])]
    steps, seg = 30, 6
    doms = _doms(ws)
    B = lbrs.Batch2D(doms)
    U0 = _pool_U0(ws, doms)
    B.init(U0)
    B.set_window(0.7, 0.8)
    nck = math.ceil(steps / seg)
    T = B.total
    ck = torch.empty(nck * 16 * T, dtype=torch.float64, device="cuda")
    tp = torch.empty(seg * 4 * T, dtype=torch.float64, device="cuda")
    fb = torch.empty(16 * T, dtype=torch.float64, device="cuda")
    wk = torch.empty_like(fb)
    J = torch.zeros(len(ws), dtype=torch.float64, device="cuda")
    Ub = torch.empty((4, T), dtype=torch.float64, device="cuda")
    B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=False)
    J_e, Ub_e = J.clone(), Ub.clone()
    # the state the sequence leaves (the gradient's recompute ends at the first segment)
    M_e, n_e = B.moments().clone(), B.state()["nsteps"]
    for rep in range(3):
        J.zero_()
        Ub.zero_()
        B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(J, J_e) and torch.equal(Ub, Ub_e), rep
        # after a replay the host reads the state the graph left, although
        # eager steps moved it in between (the buffer of f^n and the count)
        assert B.state()["nsteps"] == n_e, rep
        assert torch.equal(B.moments(), M_e), rep
        B.step(3)  # eager work between replays
        torch.cuda.synchronize()
        assert B.state()["nsteps"] == n_e + 3
    # other arguments recapture the graph instead of replaying the old one
    steps2, seg2 = 17, 4
    B.gradient(U0, steps2, seg2, ck, tp, fb, wk, J, Ub, use_graph=False)
    J_e2, Ub_e2 = J.clone(), Ub.clone()
    J.zero_()
    Ub.zero_()
    B.gradient(U0, steps2, seg2, ck, tp, fb, wk, J, Ub, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(J, J_e2) and torch.equal(Ub, Ub_e2)
    assert not torch.equal(J_e2, J_e)
    rng = np.random.default_rng(8)
    for d, w in enumerate(ws):
        dU = rng.standard_normal((4, w.ny, w.nx)) * np.array([1.0, 0.1, 0.1, 1.0])[:, None, None]
        Jo, dJo = _oracle_dJ_dU(w, steps, dU)
        dJg = float(np.sum(Ub_e[:, B.unit_slice(d)].cpu().numpy().reshape(dU.shape) * dU))
        report("batch2d grad", dom=d, J=J_e[d].item(), J_oracle=Jo, gpu=dJg, oracle=dJo)
        assert abs(J_e[d].item() - Jo) <= 1e-12 * abs(Jo)
        assert abs(dJg - dJo) <= 1e-9 * abs(dJo)
    B.close()


def test_batch2d_full_configuration_wave():
    """128 seeded periodic domains with sides from {256, 512, 1024, 2048}: one
    launch steps them all, 20 steps against the oracle -- the two smallest
    domains on every cell, the largest on sampled cells (a cell after k steps
    depends only on the (2k+1)^2 patch around it, which the oracle runs at the
    domain's frozen lattice speed); a memory wave of about 16M cells runs the
    1000-step checkpointed gradient in a captured graph, every J finite and
    every domain admissible."""
    ws = wl.domain_batch(128, seed=0)
    doms = _doms(ws)
    B = lbrs.Batch2D(doms)
    B.init(_pool_U0(ws, doms))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k = 20
    e0.record()
    B.step(k)
    e1.record()
    st = B.state()
    ms = e0.elapsed_time(e1) / k
    report("batch2d 128 forward", cells=B.total, ms_per_step=ms, mlups=B.total / ms / 1e3)
    assert st["rc"] == 0
    U = B.moments().cpu().numpy()
    B.close()

    def problem(w, nx, ny, domain, **kw):
        return oracle.Problem(model=oracle.D2Q4, nx=nx, ny=ny, domain=domain, gamma=w.gamma,
                              omega=1.0, cfl=w.cfl, **kw)

    order = sorted(range(len(ws)), key=lambda d: ws[d].nx * ws[d].ny)
    for d in order[:2]:
        w = ws[d]
        P = problem(w, w.nx, w.ny, w.domain, sides=w.sides, lam_mode=oracle.LAM_FROZEN)
        ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=k, record=False)
        err = float(np.max(np.abs(U[:, B.unit_slice(d)] - ref.U.reshape(4, -1))))
        report("batch2d 128 vs oracle", dom=d, n=w.nx, err=err)
        assert ref.status == 0 and err <= TOL
    d = order[-1]
    w = ws[d]
    Pf = problem(w, w.nx, w.ny, w.domain, sides=w.sides, lam_mode=oracle.LAM_FROZEN)
    lam = oracle.initial_lattice_speed(Pf, oracle.prim_to_cons(Pf, w.W))
    Ud = U[:, B.unit_slice(d)].reshape(4, w.ny, w.nx)
    dx = (w.domain[1] - w.domain[0]) / w.nx
    dy = (w.domain[3] - w.domain[2]) / w.ny
    R = k + 1
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(4):
        j = int(rng.integers(R, w.ny - R))
        i = int(rng.integers(R, w.nx - R))
        m = 2 * R + 1
        P = problem(w, m, m, (0.0, m * dx, 0.0, m * dy), sides=(0, 0, 0, 0),
                    lam_mode=oracle.LAM_USER, lam_user=lam)
        ref = oracle.run(P, oracle.prim_to_cons(P, w.W[:, j - R:j + R + 1, i - R:i + R + 1]),
                         max_steps=k, record=False)
        err = float(np.max(np.abs(Ud[:, j, i] - ref.U[:, R, R])))
        worst = max(worst, err)
        assert ref.status == 0 and err <= TOL, ((j, i), err)
    report("batch2d 128 cone samples", dom=d, n=w.nx, err=worst)
    del B
    torch.cuda.empty_cache()
    sub, cells = [], 0
    for w in ws:  # one memory wave of about 16M cells
        if cells + w.nx * w.ny > 16_000_000:
            continue
        sub.append(w)
        cells += w.nx * w.ny
    doms = _doms(sub)
    B = lbrs.Batch2D(doms)
    U0 = _pool_U0(sub, doms)
    B.init(U0)
    B.set_window(0.7, 0.8)
    steps, seg = 1000, 32
    T = B.total
    ck = torch.empty(math.ceil(steps / seg) * 16 * T, dtype=torch.float64, device="cuda")
    tp = torch.empty(seg * 4 * T, dtype=torch.float64, device="cuda")
    fb = torch.empty(16 * T, dtype=torch.float64, device="cuda")
    wk = torch.empty_like(fb)
    J = torch.zeros(len(sub), dtype=torch.float64, device="cuda")
    Ub = torch.empty((4, T), dtype=torch.float64, device="cuda")
    B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=True)  # capture + run
    torch.cuda.synchronize()
    e0.record()
    B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=True)
    e1.record()
    st = B.state()
    ms = e0.elapsed_time(e1)
    report("batch2d gradient wave", domains=len(sub), cells=T, ms=ms,
           ms_per_fwd_step_equiv=ms / steps)
    assert st["rc"] == 0 and torch.isfinite(J).all() and torch.isfinite(Ub).all()
    B.close()


@pytest.mark.parametrize("nsteps", [1, 2, 7, 40])
def test_batch2d_fused_vs_single_launches(nsteps):
    """Fused batch launches (k = 2, 3, 4 steps each, one more launch for the
    remainder) give the fused single-domain path's results bit for bit, and
    the single-step batch's to rounding."""
    ws = _ragged_domains()
    doms = _doms(ws)
    U0 = _pool_U0(ws, doms)
    outs = {}
    for fuse in (1, 2, 3, 4):
        B = lbrs.Batch2D(doms)
        B.init(U0)
        B.set_fusion(fuse)
        B.step(nsteps)
        st = B.state()
        assert st["rc"] == 0 and st["nsteps"] == nsteps
        outs[fuse] = B.moments()
        B.close()
    for fuse in (2, 3, 4):
        diff = float((outs[1] - outs[fuse]).abs().max())
        report("batch2d fused vs single", fuse=fuse, nsteps=nsteps, max_abs=diff,
               bitwise=bool(torch.equal(outs[1], outs[fuse])))
        assert diff <= 1e-12
        for d, w in enumerate(ws):
            sim = lbrs.Sim(lbrs.LBRS_D2Q4, w.nx, w.ny, domain=w.domain, gamma=w.gamma,
                           omega=1.0, cfl=w.cfl, bc=w.sides,
                           lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT, layout=lbrs.LBRS_LAYOUT_ROWS)
            sim.init_primitive(w.W)
            sim.set_fusion(fuse)
            sim.step(nsteps)
            assert torch.equal(sim.moments().reshape(4, -1), outs[fuse][:, lbrs_slice(d, ws)])
            sim.close()


def lbrs_slice(d, ws):
    off = [0]
    for w in ws:
        off.append(off[-1] + w.nx * w.ny)
    return slice(off[d], off[d + 1])


@pytest.mark.parametrize("fuse", [2, 3, 4])
@pytest.mark.parametrize("omega", [0.7, 1.5])
def test_batch2d_fused_mixed_sides_vs_oracle(omega, fuse):
    """Transmissive, periodic and wall sides in one fused batch, 31 steps,
    against the oracle."""
    ws = [wl.explosion(60), wl.riemann2d(80), wl.explosion(50), wl.fourier_modes(40, seed=3)]
    sides = [(0, 0, 0, 0), (1, 1, 0, 0), (1, 1, 2, 2), (2, 0, 1, 1)]
    doms = _doms(ws, sides=sides, omega=omega)
    B = lbrs.Batch2D(doms)
    B.init(_pool_U0(ws, doms))
    B.set_fusion(fuse)
    B.step(31)
    U = B.moments().cpu().numpy()
    st = B.state()
    for d, w in enumerate(ws):
        P = oracle.Problem(model=oracle.D2Q4, nx=w.nx, ny=w.ny, domain=w.domain, omega=omega,
                           sides=sides[d], lam_mode=oracle.LAM_FROZEN)
        ref = oracle.run(P, oracle.prim_to_cons(P, w.W), max_steps=31)
        err = float(np.max(np.abs(U[:, B.unit_slice(d)] - ref.U.reshape(4, -1))))
        report("batch2d fused vs oracle", fuse=fuse, dom=d, sides=sides[d], err=err,
               status=st["status"][d])
        assert ref.status == 0 and st["status"][d] == 0 and err <= TOL
    B.close()


def test_batch2d_gradient_fused_forward():
    """The gradient with fused forward sweeps (graph captured anew when the
    fusion changes): J and dJ/dU0 equal the single-launch gradient's to
    rounding; replays repeat the eager result bit for bit."""
    ws = [wl.fourier_modes(n, seed=40 + i) for i, n in enumerate([24, 40, 32])]
    steps, seg = 30, 7
    doms = _doms(ws)
    B = lbrs.Batch2D(doms)
    U0 = _pool_U0(ws, doms)
    B.init(U0)
    B.set_window(0.7, 0.8)
    nck = math.ceil(steps / seg)
    T = B.total
    ck = torch.empty(nck * 16 * T, dtype=torch.float64, device="cuda")
    tp = torch.empty(seg * 4 * T, dtype=torch.float64, device="cuda")
    fb = torch.empty(16 * T, dtype=torch.float64, device="cuda")
    wk = torch.empty_like(fb)
    J = torch.zeros(len(ws), dtype=torch.float64, device="cuda")
    Ub = torch.empty((4, T), dtype=torch.float64, device="cuda")
    res = {}
    for fuse in (1, 2, 4):
        B.set_fusion(fuse)
        B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=False)
        res[fuse] = (J.clone(), Ub.clone())
        J.zero_()
        Ub.zero_()
        B.gradient(U0, steps, seg, ck, tp, fb, wk, J, Ub, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(J, res[fuse][0]) and torch.equal(Ub, res[fuse][1]), fuse
    J1, U1 = res[1]
    scale = float(U1.abs().max())
    for fuse in (2, 4):
        J2, U2 = res[fuse]
        report("batch2d gradient fused", fuse=fuse, J=J1.tolist(),
               rel=float((U1 - U2).abs().max()) / scale)
        assert torch.allclose(J1, J2, rtol=1e-13, atol=0)
        assert float((U1 - U2).abs().max()) <= 1e-11 * scale
    B.close()


@pytest.mark.parametrize("fuse", [1, 2, 4])
def test_batch2d_gradient_whole_tape(fuse):
    """segment >= nsteps: one forward sweep writes every step's moments and the
    adjoint runs straight back (no checkpoint, no recompute).  J and dJ/dU0
    equal the checkpointed gradient's (segments of 7, odd step count), eager
    and graph-replayed."""
    ws = [wl.fourier_modes(n, seed=50 + i) for i, n in enumerate([24, 40, 32])]
    steps = 31
    doms = _doms(ws)
    B = lbrs.Batch2D(doms)
    U0 = _pool_U0(ws, doms)
    B.init(U0)
    B.set_window(0.7, 0.8)
    B.set_fusion(fuse)
    T = B.total
    ck = torch.empty(math.ceil(steps / 7) * 16 * T, dtype=torch.float64, device="cuda")
    tp = torch.empty(steps * 4 * T, dtype=torch.float64, device="cuda")
    fb = torch.empty(16 * T, dtype=torch.float64, device="cuda")
    wk = torch.empty_like(fb)
    J = torch.zeros(len(ws), dtype=torch.float64, device="cuda")
    Ub = torch.empty((4, T), dtype=torch.float64, device="cuda")
    B.gradient(U0, steps, 7, ck, tp, fb, wk, J, Ub, use_graph=False)
    Jc, Uc = J.clone(), Ub.clone()
    ck.fill_(float("nan"))  # not read by the whole-tape sweep
    for use_graph in (False, True, True):
        J.zero_()
        Ub.zero_()
        B.gradient(U0, steps, steps, ck, tp, fb, wk, J, Ub, use_graph=use_graph)
        torch.cuda.synchronize()
        scale = float(Uc.abs().max())
        rel = float((Ub - Uc).abs().max()) / scale
        report("batch2d gradient whole tape", fuse=fuse, graph=use_graph, rel=rel,
               bitwise=bool(torch.equal(Ub, Uc)))
        assert torch.allclose(J, Jc, rtol=1e-13, atol=0)
        assert rel <= 1e-12
    assert B.state()["rc"] == 0
    B.close()
