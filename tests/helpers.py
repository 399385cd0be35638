"""Shared test helpers: build the same problem for the oracle and the GPU library
from one seeded workload (the workload module holds data only)."""
from __future__ import annotations

import math

import numpy as np

import oracle

TOL = 1e-10  # max-abs parity bar on rho, rho u, (rho v,) rho E


def oracle_problem(w, lam_mode=oracle.LAM_PER_STEP, lam_user=0.0, sides=None, omega=None,
                   model=None):
    return oracle.Problem(model=w.model if model is None else model, nx=w.nx, ny=w.ny,
                          domain=w.domain, gamma=w.gamma,
                          omega=w.omega if omega is None else omega, cfl=w.cfl,
                          sides=tuple(w.sides if sides is None else sides), lam_mode=lam_mode,
                          lam_user=lam_user)


def gpu_sim(w, lam_mode=0, lam_user=0.0, sides=None, omega=None, model=None, layout=0):
    from paper_1504_07034_amd import lbrs
    return lbrs.Sim(w.model if model is None else model, w.nx, w.ny, domain=w.domain,
                    gamma=w.gamma, omega=w.omega if omega is None else omega, cfl=w.cfl,
                    bc=tuple(w.sides if sides is None else sides), lambda_mode=lam_mode,
                    lambda_user=lam_user, layout=layout)


def max_abs(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b))) if a.size else 0.0


def report(name, **kw):
    print(f"[{name}] " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def t_inf():
    return math.inf
