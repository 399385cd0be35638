"""The no-allocation entry point (lbrs_run_noalloc, static device time state)
against the ordinary one (lbrs_init + lbrs_step + lbrs_moments with a caller
scratch area), called through the C ABI: two calls in a row, the second on a
smaller grid (the static state keeps the first call's contents, so the
second shows that everything that must start at zero is cleared); results
bit for bit equal, state outputs equal.  Also: the oracle bar on the first
problem, and the rejected inputs."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

from helpers import TOL, report

pytestmark = pytest.mark.gpu


def _existing(w, t_end, fuse, max_steps):
    sim = lbrs.Sim(w.model, w.nx, w.ny, domain=w.domain, gamma=w.gamma, omega=w.omega, cfl=w.cfl,
                   bc=w.sides, layout=lbrs.LBRS_LAYOUT_ROWS)
    sim.init_primitive(w.W)
    if fuse >= 2:
        sim.set_fusion(fuse)
    sim.step(max_steps, t_end)
    U = sim.moments()
    st = sim.state()
    sim.close()
    return U, st


def _noalloc(w, t_end, fuse, max_steps):
    p = lbrs.make_params(w.model, w.nx, w.ny, w.domain, w.gamma, w.omega, w.cfl, w.sides,
                         layout=lbrs.LBRS_LAYOUT_ROWS)
    fb, ub, _ = lbrs.lbrs_query_sizes(p)
    W = torch.from_numpy(w.W).cuda()
    U0 = torch.empty_like(W)
    lbrs.lbrs_prim_to_cons(p, W, U0)
    f0 = torch.empty(fb // 8, dtype=torch.float64, device="cuda")
    f1 = torch.empty_like(f0)
    U = torch.empty_like(U0)
    state = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbrs.lbrs_run_noalloc(p, U0, f0, f1, max_steps, t_end, fuse, U, state)
    torch.cuda.synchronize()
    return U, state.cpu().numpy()


def test_noalloc_matches_the_existing_entry_point_twice():
    cases = [(wl.riemann2d(160), 0.06, 2), (wl.riemann2d(144), 0.05, 3),
             (wl.riemann2d(128), 0.05, 4), (wl.riemann2d(96), 0.04, 1)]
    for i, (w, t_end, fuse) in enumerate(cases):
        print(f"noalloc case {i}: {w.name} {w.nx}x{w.ny} fuse {fuse}", flush=True)
        U_ref, st = _existing(w, t_end, fuse, 10**4)
        U, state = _noalloc(w, t_end, fuse, 10**4)
        report("noalloc vs init/step", case=i, n=w.nx, steps=st["nsteps"], state=state.tolist(),
               bitwise=bool(torch.equal(U, U_ref)))
        assert st["rc"] == 0 and state[3] == 0.0 and state[4] == -1.0
        assert state[0] == st["t"] == t_end and int(state[1]) == st["nsteps"]
        assert state[2] == st["lambda"]
        assert torch.equal(U, U_ref)
        if i == 0:
            P = oracle.Problem(model=w.model, nx=w.nx, ny=w.ny, domain=w.domain, gamma=w.gamma,
                               omega=w.omega, cfl=w.cfl, sides=w.sides)
            ref = oracle.run(P, oracle.prim_to_cons(P, w.W), t_end=t_end)
            assert ref.nsteps == st["nsteps"]
            assert float(np.max(np.abs(U.cpu().numpy() - ref.U))) <= TOL


def test_noalloc_rejects_bodies_and_bad_arguments():
    w = wl.riemann2d(32)
    solid = np.zeros((32, 32), np.uint8)
    solid[10:14, 10:14] = 1
    p = lbrs.make_params(w.model, 32, 32, w.domain, bc=w.sides, solid=solid)
    buf = torch.empty(16 * 32 * 32, dtype=torch.float64, device="cuda")
    U = torch.empty(4 * 32 * 32, dtype=torch.float64, device="cuda")
    for kw in [dict(p=p, fuse=1), dict(p=lbrs.make_params(w.model, 32, 32, w.domain), fuse=5)]:
        with pytest.raises(lbrs.LBRSError) as e:
            lbrs.lbrs_run_noalloc(kw["p"], U, buf, torch.empty_like(buf), 5, 0.1, kw["fuse"], U)
        assert e.value.code == lbrs.LBRS_E_INVAL
