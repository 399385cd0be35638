"""LBRS oracle -- TEST INFRASTRUCTURE ONLY.

A ctypes front end to ``liblbrs_oracle.so``, the plain FP64 CPU implementation
of the Lattice Boltzmann Relaxation Scheme (arXiv 1504.07034, Sec. II) in
``lbrs_oracle.cpp``, plus an exact Riemann solver (``riemann.py``).  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the GPU library never does, and the two share no code.

Layouts (all numpy float64, C order):
  * conserved state U: SoA planes ``[K][ny][nx]`` -- K = 3 in 1D (rho, rho u,
    rho E), K = 4 in 2D (rho, rho u, rho v, rho E), K = 1 in the scalar mode;
  * primitive state W: ``[K][ny][nx]`` -- (rho, u, p) or (rho, u, v, p);
  * populations f: ``[Q][K][ny][nx]`` with the discrete velocities ordered as
    in the paper: D1Q2 (-, +), D1Q3 (-, 0, +), D2Q4 (-,-), (+,-), (+,+), (-,+).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbrs_oracle.cpp")
LIB_SERIAL = os.path.join(HERE, "liblbrs_oracle.so")
LIB_OMP = os.path.join(HERE, "liblbrs_oracle_omp.so")
LIB = LIB_SERIAL

D1Q2, D1Q3, D2Q4 = 0, 1, 2
FLUX_EULER, FLUX_LINEAR, FLUX_QUADRATIC = 0, 1, 2
TRANSMISSIVE, PERIODIC, WALL, DIRICHLET = 0, 1, 2, 3
LAM_PER_STEP, LAM_FROZEN, LAM_USER = 0, 1, 2
OK, INVAL, NONPHYSICAL = 0, -1, -4

NQ = {D1Q2: 2, D1Q3: 3, D2Q4: 4}


# The serial build the tests use, and the timing build (same source, OpenMP
# over cells, -O3 -march=native); neither contracts multiply-adds.
_FLAGS = {
    LIB_SERIAL: ["-O2"],
    LIB_OMP: ["-O3", "-march=native", "-fopenmp"],
}


def _compile(lib: str, force: bool) -> str:
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        tmp = lib + ".tmp"
        subprocess.check_call(["g++", *_FLAGS[lib], "-std=c++17", "-fPIC", "-shared",
                               "-ffp-contract=off", SRC, "-o", tmp])
        os.replace(tmp, lib)
    return lib


def build(force: bool = True) -> str:
    """Compile both builds of the oracle with g++; returns the serial one."""
    _compile(LIB_OMP, force)
    return _compile(LIB_SERIAL, force)


def use(variant: str = "serial", threads: int | None = None) -> int:
    """Select the build later calls load: "serial" (the default) or "omp"
    (OpenMP over cells; `threads` sets the thread count).  Returns the
    number of threads the selected build runs its cell loops with."""
    global LIB, _lib
    lib = LIB_OMP if variant == "omp" else LIB_SERIAL
    if lib != LIB:
        LIB, _lib = lib, None
    return _load().orc_threads(int(threads or 0))


class _Problem(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int), ("flux", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("cfl", ctypes.c_double),
        ("side", ctypes.c_int * 4),
        ("lam_mode", ctypes.c_int), ("lam_user", ctypes.c_double),
        ("adv_x", ctypes.c_double), ("adv_y", ctypes.c_double),
        ("dir", ctypes.POINTER(ctypes.c_double) * 4),
        ("q", ctypes.c_double * 4),
        ("solid", ctypes.POINTER(ctypes.c_ubyte)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if LIB in _FLAGS:
            _compile(LIB, force=False)
        lib = ctypes.CDLL(LIB)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.orc_flux.argtypes = [P, dp, dp, dp]
        lib.orc_flux.restype = None
        lib.orc_local_lambda.argtypes = [P, dp]
        lib.orc_local_lambda.restype = ctypes.c_double
        lib.orc_equilibria.argtypes = [P, dp, ctypes.c_double, dp]
        lib.orc_equilibria.restype = None
        lib.orc_prim_to_cons.argtypes = [P, dp, dp]
        lib.orc_prim_to_cons.restype = None
        lib.orc_initial_lattice_speed.argtypes = [P, dp]
        lib.orc_initial_lattice_speed.restype = ctypes.c_double
        lib.orc_run.argtypes = [P, dp, ctypes.c_double, ctypes.c_long, dp, dp, dp, dp, lp, dp, lp]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_step_fixed.argtypes = [P, dp, dp, ctypes.c_double, dp, dp]
        lib.orc_step_fixed.restype = ctypes.c_int
        lib.orc_run_tangent.argtypes = [P, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_long,
                                        dp, dp]
        lib.orc_run_tangent.restype = ctypes.c_int
        lib.orc_init_tangent.argtypes = [P, dp, dp, ctypes.c_double, dp, dp]
        lib.orc_init_tangent.restype = ctypes.c_int
        lib.orc_threads.argtypes = [ctypes.c_int]
        lib.orc_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Problem:
    model: int
    nx: int
    ny: int = 1
    domain: tuple = (0.0, 1.0, 0.0, 1.0)
    gamma: float = 1.4
    omega: float = 1.0
    cfl: float = 0.5
    sides: tuple = (TRANSMISSIVE, TRANSMISSIVE, TRANSMISSIVE, TRANSMISSIVE)
    lam_mode: int = LAM_PER_STEP
    lam_user: float = 0.0
    flux: int = FLUX_EULER
    adv: tuple = (0.0, 0.0)
    # Dirichlet data per side (xlo, xhi, ylo, yhi): conserved states [K][n],
    # n = ny for the x-sides, nx for the y-sides; None for other sides.
    dirichlet: tuple = (None, None, None, None)
    # FLUX_QUADRATIC: g1(u) = q0 u + q1 u^2/2, g2(u) = q2 u + q3 u^2/2
    quad: tuple = (0.0, 0.0, 0.0, 0.0)
    # Solid cells [ny][nx] (nonzero = solid) of a body in a D2Q4 Euler
    # domain, or None.
    solid: object = None

    @property
    def Q(self) -> int:
        return NQ[self.model]

    @property
    def K(self) -> int:
        if self.flux != FLUX_EULER:
            return 1
        return 4 if self.model == D2Q4 else 3

    @property
    def dx(self) -> float:
        return (self.domain[1] - self.domain[0]) / self.nx

    def c(self) -> _Problem:
        p = _Problem()
        p.model, p.flux, p.nx, p.ny = self.model, self.flux, self.nx, self.ny
        p.x0, p.x1, p.y0, p.y1 = self.domain
        p.gamma, p.omega, p.cfl = self.gamma, self.omega, self.cfl
        for i in range(4):
            p.side[i] = self.sides[i]
        p.lam_mode, p.lam_user = self.lam_mode, self.lam_user
        p.adv_x, p.adv_y = self.adv
        keep = []
        for i in range(4):
            d = self.dirichlet[i]
            if d is None:
                p.dir[i] = ctypes.POINTER(ctypes.c_double)()
            else:
                a = np.ascontiguousarray(d, dtype=np.float64)
                keep.append(a)
                p.dir[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p._keep = keep  # the arrays live as long as the struct
        for i in range(4):
            p.q[i] = float(self.quad[i])
        if self.solid is None:
            p.solid = ctypes.POINTER(ctypes.c_ubyte)()
        else:
            m = np.ascontiguousarray(self.solid, dtype=np.uint8).reshape(self.ny, self.nx)
            keep.append(m)
            p.solid = m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
        return p


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def flux(P: Problem, U):
    """Flux vectors (Gx, Gy) of one conserved state U (K values)."""
    U = _arr(U)
    Gx = np.zeros(P.K)
    Gy = np.zeros(P.K)
    _load().orc_flux(ctypes.byref(P.c()), _ptr(U), _ptr(Gx), _ptr(Gy))
    return Gx, Gy


def local_lambda(P: Problem, U) -> float:
    return _load().orc_local_lambda(ctypes.byref(P.c()), _ptr(_arr(U)))


def equilibria(P: Problem, U, lam: float):
    """Equilibria f^eq[i][k] of one state at lattice speed lam."""
    out = np.zeros((P.Q, P.K))
    _load().orc_equilibria(ctypes.byref(P.c()), _ptr(_arr(U)), lam, _ptr(out))
    return out


def prim_to_cons(P: Problem, W):
    W = _arr(W).reshape(P.K, P.ny, P.nx)
    U = np.zeros_like(W)
    _load().orc_prim_to_cons(ctypes.byref(P.c()), _ptr(W), _ptr(U))
    return U


def initial_lattice_speed(P: Problem, U0) -> float:
    return _load().orc_initial_lattice_speed(ctypes.byref(P.c()), _ptr(_arr(U0)))


@dataclass
class RunResult:
    status: int
    U: np.ndarray
    f: np.ndarray | None
    dt: np.ndarray
    lam: np.ndarray
    nsteps: int
    t: float
    fail_step: int


def run(P: Problem, U0, t_end: float = math.inf, max_steps: int = 10**9,
        want_f: bool = False, record: bool = True) -> RunResult:
    """Run the scheme from conserved U0 [K][ny][nx] to t_end (or max_steps)."""
    U0 = _arr(U0).reshape(P.K, P.ny, P.nx)
    U = np.zeros_like(U0)
    f = np.zeros((P.Q, P.K, P.ny, P.nx)) if want_f else None
    cap = int(min(max_steps, 10**7))
    if record and not math.isfinite(t_end) and max_steps > 10**7:
        raise ValueError("record=True needs a finite max_steps or t_end")
    if record and math.isfinite(t_end) and max_steps > 10**7:
        # generous cap for the recorded sequences (steps are bounded by t_end)
        cap = 4 * 10**6
    dts = np.zeros(cap if record else 0)
    lams = np.zeros(cap if record else 0)
    n = ctypes.c_long(0)
    t = ctypes.c_double(0.0)
    fail = ctypes.c_long(-1)
    st = _load().orc_run(ctypes.byref(P.c()), _ptr(U0), float(t_end), int(max_steps), _ptr(U),
                         _ptr(f), _ptr(dts) if record else None, _ptr(lams) if record else None,
                         ctypes.byref(n), ctypes.byref(t), ctypes.byref(fail))
    k = n.value
    return RunResult(st, U, f, dts[:k] if record else dts, lams[:k] if record else lams, k,
                     t.value, fail.value)


def step_fixed(P: Problem, f, lam: float, df=None):
    """One step at fixed lattice speed from populations f [Q][K][ny][nx].

    Returns (f_next, df_next); df_next is the exact tangent (forward-mode dual
    numbers) along df, or None when df is None."""
    f = _arr(f).reshape(P.Q, P.K, P.ny, P.nx)
    out = np.zeros_like(f)
    dout = np.zeros_like(f) if df is not None else None
    dfa = _arr(df).reshape(f.shape) if df is not None else None
    st = _load().orc_step_fixed(ctypes.byref(P.c()), _ptr(f), _ptr(dfa), float(lam), _ptr(out),
                                _ptr(dout))
    if st != OK:
        raise ValueError(f"orc_step_fixed failed: {st}")
    return out, dout


def run_tangent(P: Problem, W0, dW0, lam: float, nsteps: int, isentropic: bool = False):
    """Directional derivative of U(T) along dW0 (primitive), fixed lattice speed."""
    W0 = _arr(W0).reshape(P.K, P.ny, P.nx)
    dW0 = _arr(dW0).reshape(P.K, P.ny, P.nx)
    U = np.zeros_like(W0)
    dU = np.zeros_like(W0)
    st = _load().orc_run_tangent(ctypes.byref(P.c()), _ptr(W0), _ptr(dW0), int(isentropic),
                                 float(lam), int(nsteps), _ptr(U), _ptr(dU))
    if st != OK:
        raise ValueError(f"orc_run_tangent failed: {st}")
    return U, dU


def init_tangent(P: Problem, U0, dU0, lam: float):
    """f^0 = f^eq(U0) at lattice speed lam and its tangent along dU0."""
    U0 = _arr(U0).reshape(P.K, P.ny, P.nx)
    dU0 = _arr(dU0).reshape(P.K, P.ny, P.nx)
    f0 = np.zeros((P.Q, P.K, P.ny, P.nx))
    df0 = np.zeros_like(f0)
    st = _load().orc_init_tangent(ctypes.byref(P.c()), _ptr(U0), _ptr(dU0), float(lam), _ptr(f0),
                                  _ptr(df0))
    if st != OK:
        raise ValueError(f"orc_init_tangent failed: {st}")
    return f0, df0
