"""Ragged 1D batch (one persistent, graph-captured launch) against the oracle
per unit, and bitwise against the single-domain library path."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import TOL, report

pytestmark = pytest.mark.gpu


def _units(tubes, model=wl.D1Q3, omega=None, periodic=False, lam_user=None):
    bc = (1, 1, 0, 0) if periodic else (0, 0, 0, 0)
    out = []
    for i, t in enumerate(tubes):
        om = t.omega if omega is None else (omega[i] if isinstance(omega, (list, tuple)) else omega)
        mode = lbrs.LBRS_LAMBDA_PER_STEP
        lu = 0.0
        if lam_user is not None and lam_user.get(i) is not None:
            mode, lu = lbrs.LBRS_LAMBDA_USER, lam_user[i]
        out.append(lbrs.make_params(model, t.nx, 1, t.domain, t.gamma, om, t.cfl, bc, mode, lu))
    return out


def _batch(tubes, chunk, **kw):
    units = _units(tubes, **kw)
    B = lbrs.Batch1D(units, [t.t_end for t in tubes], chunk=chunk)
    W = torch.from_numpy(np.concatenate([t.W[:, 0, :] for t in tubes], axis=1)).cuda()
    U0 = torch.empty_like(W)
    lbrs.lbrs_prim_to_cons(lbrs.make_params(units[0].model, B.total, 1), W, U0)
    B.init(U0)
    return B, units


def _oracle_tube(t, model=wl.D1Q3, omega=None, periodic=False, lam_user=None):
    P = oracle.Problem(model=model, nx=t.nx, domain=t.domain, gamma=t.gamma,
                       omega=t.omega if omega is None else omega, cfl=t.cfl,
                       sides=(1, 1, 0, 0) if periodic else (0, 0, 0, 0),
                       lam_mode=oracle.LAM_USER if lam_user else oracle.LAM_PER_STEP,
                       lam_user=lam_user or 0.0)
    return oracle.run(P, oracle.prim_to_cons(P, t.W), t_end=t.t_end, record=False)


@pytest.mark.parametrize("chunk", [254, 1022, 2046, 3070])
def test_batch_matches_oracle_per_unit(chunk):
    """20 seeded tubes of 100..3000 cells; chunk 254 splits most into teams of up to
    12 workgroups (one team barrier per step), chunk 1022 into teams of up to 3;
    2046 (512 threads) and 3070 (768 threads) hold four cells per thread."""
    tubes = wl.tube_batch(20, seed=1, nmin=100, nmax=3000)
    B, _ = _batch(tubes, chunk)
    B.run(10**6)
    st = B.state()
    U = B.moments().cpu().numpy()
    worst = 0.0
    for b, t in enumerate(tubes):
        ref = _oracle_tube(t)
        err = float(np.max(np.abs(U[:, B.unit_slice(b)] - ref.U[:, 0, :])))
        worst = max(worst, err)
        assert st["status"][b] == 0 and ref.status == 0
        assert st["nsteps"][b] == ref.nsteps, (b, st["nsteps"][b], ref.nsteps)
        assert st["t"][b] == t.t_end
        assert err <= TOL, (b, err)
    report("batch vs oracle", chunk=chunk, units=len(tubes), worst=worst,
           teams=max(math.ceil(t.nx / chunk) for t in tubes))
    B.close()


def test_batch_mixed_models_sides_omega():
    """D1Q2 units on periodic domains with a different omega per unit."""
    tubes = wl.tube_batch(8, seed=3, nmin=150, nmax=900)
    for t in tubes:
        t.t_end = 0.05
    om = [0.6, 0.9, 1.2, 1.5, 1.0, 0.7, 1.3, 1.1]
    B, _ = _batch(tubes, 254, model=wl.D1Q2, omega=om, periodic=True)
    B.run(10**6)
    st = B.state()
    U = B.moments().cpu().numpy()
    for b, t in enumerate(tubes):
        ref = _oracle_tube(t, model=wl.D1Q2, omega=om[b], periodic=True)
        err = float(np.max(np.abs(U[:, B.unit_slice(b)] - ref.U[:, 0, :])))
        assert st["nsteps"][b] == ref.nsteps and err <= TOL, (b, err)
    B.close()


@pytest.mark.parametrize("chunk", [1022, 3070])
def test_batch_bitwise_equals_single_domain_runs(chunk):
    """Each unit of the batch equals the same problem run alone through lbrs_init /
    lbrs_step, bit for bit (same arithmetic, exact max reductions)."""
    tubes = wl.tube_batch(6, seed=5, nmin=300, nmax=6000)
    B, units = _batch(tubes, chunk)
    B.run(10**6)
    U = B.moments()
    for b, t in enumerate(tubes):
        sim = lbrs.Sim(t.model, t.nx, 1, domain=t.domain, gamma=t.gamma, omega=t.omega, cfl=t.cfl)
        sim.init_primitive(t.W)
        s = sim.run(t.t_end, chunk=20000)
        Us = sim.moments()[:, 0, :]
        same = torch.equal(Us, U[:, B.unit_slice(b)])
        report("batch vs single", chunk=chunk, unit=b, n=t.nx, steps=s["nsteps"], bitwise=same)
        assert same
        sim.close()
    B.close()


def test_batch_nonphysical_unit_is_isolated():
    """A unit driven non-physical (lattice speed far below the bound) is flagged
    with the oracle's failing step; the other units are unaffected."""
    tubes = wl.tube_batch(5, seed=7, nmin=200, nmax=700)
    for t in tubes:
        t.omega = 1.9
    B, _ = _batch(tubes, 254, lam_user={2: 0.2})
    B.run(10**6)
    st = B.state()
    assert st["rc"] == lbrs.LBRS_E_NONPHYSICAL
    ref = _oracle_tube(tubes[2], omega=1.9, lam_user=0.2)
    assert ref.status == oracle.NONPHYSICAL
    assert st["status"][2] & 1 and st["fail_step"][2] == ref.fail_step
    for b in (0, 1, 3, 4):
        assert st["status"][b] == 0 and st["t"][b] == tubes[b].t_end
    B.close()


@pytest.mark.parametrize("chunk", [1022, 2046, 3070])
def test_batch_full_configuration(chunk):
    """1024 tubes, cells log-uniform in [200, 20000] (seed 0), each to its own
    t_end in [0.1, 0.25], in the chunk sizes the benchmark tunes over: every unit
    finishes; the smallest units match the oracle and a sample of large ones
    matches single-domain runs bit for bit."""
    tubes = wl.tube_batch(1024, seed=0)
    B, _ = _batch(tubes, chunk)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    B.run(10**6)
    e1.record()
    st = B.state()
    ms = e0.elapsed_time(e1)
    lups = sum(st["nsteps"][b] * t.nx for b, t in enumerate(tubes))
    report("batch full", chunk=chunk, ms=ms, lups=lups, glups=lups / ms / 1e6, total_cells=B.total,
           max_steps=max(st["nsteps"]))
    assert st["rc"] == 0
    assert all(st["t"][b] == t.t_end for b, t in enumerate(tubes))
    U = B.moments()
    order = np.argsort([t.nx for t in tubes])
    for b in order[:4]:
        t = tubes[b]
        ref = _oracle_tube(t)
        err = float(np.max(np.abs(U[:, B.unit_slice(b)].cpu().numpy() - ref.U[:, 0, :])))
        assert st["nsteps"][b] == ref.nsteps and err <= TOL
    for b in order[[500, 900, 1023]]:
        t = tubes[b]
        sim = lbrs.Sim(t.model, t.nx, 1, domain=t.domain, gamma=t.gamma, omega=t.omega, cfl=t.cfl)
        sim.init_primitive(t.W)
        sim.run(t.t_end, chunk=50000)
        assert torch.equal(sim.moments()[:, 0, :], U[:, B.unit_slice(b)])
        sim.close()
    B.close()
