"""Thin Python binding of the LBRS C ABI (include/lbrs.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels of
``liblbrs.so``.  Functions carry the C names; tensors are torch float64 CUDA
tensors (device pointers), and work is enqueued on torch's current stream
unless a stream is given.  Loading fails loudly when the library is not built
or no GPU is visible -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbrs.so")

LBRS_OK, LBRS_E_INVAL, LBRS_E_NOMEM, LBRS_E_HIP, LBRS_E_NONPHYSICAL, LBRS_E_STATE = 0, -1, -2, -3, -4, -5
LBRS_D1Q2, LBRS_D1Q3, LBRS_D2Q4 = 0, 1, 2
LBRS_BC_TRANSMISSIVE, LBRS_BC_PERIODIC, LBRS_BC_WALL, LBRS_BC_DIRICHLET = 0, 1, 2, 3
LBRS_LAMBDA_PER_STEP, LBRS_LAMBDA_FROZEN_INIT, LBRS_LAMBDA_USER = 0, 1, 2
LBRS_LAYOUT_PLANAR, LBRS_LAYOUT_ROWS = 0, 1
LBRS_LAW_EULER, LBRS_LAW_SCALAR = 0, 1

# Every symbol include/lbrs.h declares (checked by the CPU test-suite).
EXPORTS = (
    "lbrs_query_sizes", "lbrs_prim_to_cons", "lbrs_init", "lbrs_step", "lbrs_get_state",
    "lbrs_moments", "lbrs_get_f", "lbrs_set_f", "lbrs_window_objective", "lbrs_step_tape",
    "lbrs_adjoint_step", "lbrs_adjoint_init", "lbrs_prim_to_cons_adjoint",
    "lbrs_isentropic_to_cons", "lbrs_isentropic_to_cons_adjoint", "lbrs_forward_checkpointed",
    "lbrs_backward_checkpointed", "lbrs_set_stream", "lbrs_set_tile", "lbrs_batch_query",
    "lbrs_batch_init", "lbrs_batch_run", "lbrs_batch_get_state", "lbrs_batch_moments",
    "lbrs_batch_destroy", "lbrs_batch2d_query", "lbrs_batch2d_init", "lbrs_batch2d_reset",
    "lbrs_batch2d_step", "lbrs_batch2d_step_tape", "lbrs_batch2d_adjoint_step",
    "lbrs_batch2d_adjoint_init", "lbrs_batch2d_set_window", "lbrs_batch2d_window_objective",
    "lbrs_batch2d_moments", "lbrs_batch2d_get_f", "lbrs_batch2d_set_f", "lbrs_batch2d_gradient",
    "lbrs_batch2d_get_state", "lbrs_batch2d_destroy", "lbrs_body_codes", "lbrs_strerror",
    "lbrs_destroy", "lbrs_set_fusion", "lbrs_batch2d_set_fusion", "lbrs_adjoint_step2",
    "lbrs_step_tape2", "lbrs_forward_taped", "lbrs_backward_taped", "lbrs_cfl_max",
    "lbrs_step_tapes", "lbrs_adjoint_steps",
    "lbrs_run_noalloc", "lbrs_pair_stats",
)


class lbrs_params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("cfl", ctypes.c_double),
        ("bc", ctypes.c_int * 4),
        ("lambda_mode", ctypes.c_int), ("lambda_user", ctypes.c_double),
        ("layout", ctypes.c_int),
        ("dirichlet", ctypes.c_void_p * 4),
        ("law", ctypes.c_int), ("scalar_flux", ctypes.c_double * 4),
        ("solid", ctypes.c_void_p),
    ]


class LBRSError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def load_library(path: str = LIB_PATH, require_gpu: bool = True):
    """Load liblbrs.so (raises if it is missing, or if no GPU is visible)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    if require_gpu and not torch.cuda.is_available():
        raise RuntimeError("the LBRS library needs a visible gfx950 GPU")
    lib = ctypes.CDLL(path)
    vp, dp, P = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(lbrs_params)
    szp = ctypes.POINTER(ctypes.c_size_t)
    i, d, ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "lbrs_query_sizes": (i, [P, szp, szp, szp]),
        "lbrs_prim_to_cons": (i, [P, vp, vp, vp]),
        "lbrs_init": (i, [ctypes.POINTER(vp), P, vp, vp, vp, vp, vp]),
        "lbrs_step": (i, [vp, i, d]),
        "lbrs_get_state": (i, [vp, dp, ctypes.POINTER(ll), dp, ctypes.POINTER(ctypes.c_uint),
                               ctypes.POINTER(ll)]),
        "lbrs_moments": (i, [vp, vp]),
        "lbrs_get_f": (i, [vp, vp]),
        "lbrs_set_f": (i, [vp, vp, d, ll]),
        "lbrs_window_objective": (i, [vp, i, i, i, i, vp, vp]),
        "lbrs_step_tape": (i, [vp, vp]),
        "lbrs_adjoint_step": (i, [vp, vp, vp, vp]),
        "lbrs_adjoint_init": (i, [vp, vp, vp, vp]),
        "lbrs_prim_to_cons_adjoint": (i, [P, vp, vp, vp, vp]),
        "lbrs_isentropic_to_cons": (i, [P, vp, vp, vp]),
        "lbrs_isentropic_to_cons_adjoint": (i, [P, vp, vp, vp, vp]),
        "lbrs_forward_checkpointed": (i, [vp, i, i, vp]),
        "lbrs_backward_checkpointed": (i, [vp, i, i, vp, vp, vp, vp]),
        "lbrs_set_stream": (i, [vp, vp]),
        "lbrs_set_tile": (i, [vp, i, i, i]),
        "lbrs_set_fusion": (i, [vp, i]),
        "lbrs_batch2d_set_fusion": (i, [vp, i]),
        "lbrs_adjoint_step2": (i, [vp, vp, vp, vp, vp]),
        "lbrs_step_tape2": (i, [vp, vp, vp]),
        "lbrs_step_tapes": (i, [vp, i, vp]),
        "lbrs_adjoint_steps": (i, [vp, i, vp, vp, vp]),
        "lbrs_forward_taped": (i, [vp, i, vp]),
        "lbrs_backward_taped": (i, [vp, i, vp, vp, vp]),
        "lbrs_batch_query": (i, [i, P, i, ctypes.POINTER(ll), szp]),
        "lbrs_batch_init": (i, [ctypes.POINTER(vp), i, P, dp, i, vp, vp, vp, vp]),
        "lbrs_batch_run": (i, [vp, i]),
        "lbrs_batch_get_state": (i, [vp, dp, ctypes.POINTER(ll), dp, ctypes.POINTER(ctypes.c_uint),
                                     ctypes.POINTER(ll)]),
        "lbrs_batch_moments": (i, [vp, vp]),
        "lbrs_batch_destroy": (None, [vp]),
        "lbrs_batch2d_query": (i, [i, P, ctypes.POINTER(ll), szp]),
        "lbrs_batch2d_init": (i, [ctypes.POINTER(vp), i, P, vp, vp, vp, vp, vp]),
        "lbrs_batch2d_reset": (i, [vp, vp]),
        "lbrs_batch2d_step": (i, [vp, i]),
        "lbrs_batch2d_step_tape": (i, [vp, vp]),
        "lbrs_batch2d_adjoint_step": (i, [vp, vp, vp, vp]),
        "lbrs_batch2d_adjoint_init": (i, [vp, vp, vp, vp]),
        "lbrs_batch2d_set_window": (i, [vp, d, d]),
        "lbrs_batch2d_window_objective": (i, [vp, vp, vp]),
        "lbrs_batch2d_moments": (i, [vp, vp]),
        "lbrs_batch2d_get_f": (i, [vp, vp]),
        "lbrs_batch2d_set_f": (i, [vp, vp, ll]),
        "lbrs_batch2d_gradient": (i, [vp, vp, i, i, vp, vp, vp, vp, vp, vp, i]),
        "lbrs_batch2d_get_state": (i, [vp, ctypes.POINTER(ll), dp, ctypes.POINTER(ctypes.c_uint)]),
        "lbrs_batch2d_destroy": (None, [vp]),
        "lbrs_body_codes": (i, [P, ctypes.POINTER(ctypes.c_ushort)]),
        "lbrs_strerror": (ctypes.c_char_p, [i]),
        "lbrs_cfl_max": (d, [i]),
        "lbrs_run_noalloc": (i, [P, vp, vp, vp, i, d, i, vp, vp, vp]),
        "lbrs_pair_stats": (i, [vp, ctypes.POINTER(ll), i]),
        "lbrs_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load_library(require_gpu=False).lbrs_strerror(code).decode()
    except Exception:  # pragma: no cover - message only
        return f"error {code}"


def _check(rc: int, where: str):
    if rc != LBRS_OK:
        raise LBRSError(rc, where)


def _dptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_params(model, nx, ny=1, domain=(0.0, 1.0, 0.0, 1.0), gamma=1.4, omega=1.0, cfl=0.5,
                bc=(0, 0, 0, 0), lambda_mode=LBRS_LAMBDA_PER_STEP, lambda_user=0.0,
                layout=LBRS_LAYOUT_PLANAR, dirichlet=(None, None, None, None),
                law=LBRS_LAW_EULER, scalar_flux=(0.0, 0.0, 0.0, 0.0),
                solid=None) -> lbrs_params:
    """dirichlet: per side, a device tensor of conserved states [K][n] (or None);
    law / scalar_flux: the conservation law (scalar: g1 = c0 u + c1 u^2/2,
    g2 = c2 u + c3 u^2/2); solid: a host uint8 array [ny][nx] (nonzero = solid
    cell of a body) or None -- the params keep a reference to it."""
    p = lbrs_params()
    p.model, p.nx, p.ny = int(model), int(nx), int(ny)
    p.x0, p.x1, p.y0, p.y1 = map(float, domain)
    p.gamma, p.omega, p.cfl = float(gamma), float(omega), float(cfl)
    for s in range(4):
        p.bc[s] = int(bc[s])
    p.lambda_mode, p.lambda_user = int(lambda_mode), float(lambda_user)
    p.layout = int(layout)
    for s in range(4):
        d = dirichlet[s]
        p.dirichlet[s] = None if d is None else d.data_ptr()
    p.law = int(law)
    for k in range(4):
        p.scalar_flux[k] = float(scalar_flux[k])
    if solid is None:
        p.solid = None
    else:
        m = np.ascontiguousarray(np.asarray(solid), dtype=np.uint8)
        if m.shape != (int(ny), int(nx)):
            raise ValueError(f"solid mask must be [ny][nx] = {(ny, nx)}, got {m.shape}")
        p._solid = m  # kept alive with the struct
        p.solid = m.ctypes.data
    return p


def lbrs_body_codes(p: lbrs_params):
    """Node codes of the body of p (host computation, no GPU needed):
    uint16 [ny][nx], the rule of population i in bits 3i..3i+2 and bit 15
    for a solid cell."""
    out = np.zeros((p.ny, p.nx), dtype=np.uint16)
    _check(load_library(require_gpu=False).lbrs_body_codes(
        ctypes.byref(p), out.ctypes.data_as(ctypes.POINTER(ctypes.c_ushort))), "lbrs_body_codes")
    return out


# ------------------------------------------------------------- C-named calls
def lbrs_query_sizes(p: lbrs_params):
    f, u, s = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().lbrs_query_sizes(ctypes.byref(p), ctypes.byref(f), ctypes.byref(u),
                                           ctypes.byref(s)), "lbrs_query_sizes")
    return f.value, u.value, s.value


def lbrs_cfl_max(model: int) -> float:
    """Largest admissible cfl of a model (host only)."""
    return load_library(require_gpu=False).lbrs_cfl_max(int(model))


def lbrs_run_noalloc(p: lbrs_params, U0, f0, f1, max_steps: int, t_end: float,
                     steps_per_launch: int, U, state=None, stream=None):
    """Whole run with the library's static time state (no allocation)."""
    _check(load_library().lbrs_run_noalloc(
        ctypes.byref(p), _dptr(U0), _dptr(f0), _dptr(f1), int(max_steps), float(t_end),
        int(steps_per_launch), _dptr(U), _dptr(state), _stream(stream)), "lbrs_run_noalloc")


def lbrs_prim_to_cons(p: lbrs_params, W: torch.Tensor, U: torch.Tensor, stream=None):
    _check(load_library().lbrs_prim_to_cons(ctypes.byref(p), _dptr(W), _dptr(U), _stream(stream)),
           "lbrs_prim_to_cons")


def lbrs_prim_to_cons_adjoint(p: lbrs_params, W, Ubar, Wbar, stream=None):
    _check(load_library().lbrs_prim_to_cons_adjoint(ctypes.byref(p), _dptr(W), _dptr(Ubar),
                                                    _dptr(Wbar), _stream(stream)),
           "lbrs_prim_to_cons_adjoint")


def lbrs_isentropic_to_cons(p: lbrs_params, rho, U, stream=None):
    _check(load_library().lbrs_isentropic_to_cons(ctypes.byref(p), _dptr(rho), _dptr(U),
                                                  _stream(stream)), "lbrs_isentropic_to_cons")


def lbrs_isentropic_to_cons_adjoint(p: lbrs_params, rho, Ubar, rhobar, stream=None):
    _check(load_library().lbrs_isentropic_to_cons_adjoint(ctypes.byref(p), _dptr(rho), _dptr(Ubar),
                                                          _dptr(rhobar), _stream(stream)),
           "lbrs_isentropic_to_cons_adjoint")


def lbrs_forward_checkpointed(ctx, nsteps: int, segment: int, ckpt):
    _check(load_library().lbrs_forward_checkpointed(ctx, int(nsteps), int(segment), _dptr(ckpt)),
           "lbrs_forward_checkpointed")


def lbrs_backward_checkpointed(ctx, nsteps: int, segment: int, ckpt, tape, fbar, work):
    _check(load_library().lbrs_backward_checkpointed(ctx, int(nsteps), int(segment), _dptr(ckpt),
                                                     _dptr(tape), _dptr(fbar), _dptr(work)),
           "lbrs_backward_checkpointed")


def lbrs_forward_taped(ctx, nsteps: int, tape):
    _check(load_library().lbrs_forward_taped(ctx, int(nsteps), _dptr(tape)), "lbrs_forward_taped")


def lbrs_backward_taped(ctx, nsteps: int, tape, fbar, work):
    _check(load_library().lbrs_backward_taped(ctx, int(nsteps), _dptr(tape), _dptr(fbar),
                                              _dptr(work)), "lbrs_backward_taped")


def lbrs_init(p: lbrs_params, U0, f0, f1, scratch, stream=None):
    ctx = ctypes.c_void_p()
    _check(load_library().lbrs_init(ctypes.byref(ctx), ctypes.byref(p), _dptr(U0), _dptr(f0),
                                    _dptr(f1), _dptr(scratch), _stream(stream)), "lbrs_init")
    return ctx


def lbrs_step(ctx, max_steps: int, t_end: float = math.inf):
    _check(load_library().lbrs_step(ctx, int(max_steps), float(t_end)), "lbrs_step")


def lbrs_get_state(ctx):
    t, lam = ctypes.c_double(), ctypes.c_double()
    n, fail = ctypes.c_longlong(), ctypes.c_longlong()
    st = ctypes.c_uint()
    rc = load_library().lbrs_get_state(ctx, ctypes.byref(t), ctypes.byref(n), ctypes.byref(lam),
                                       ctypes.byref(st), ctypes.byref(fail))
    if rc not in (LBRS_OK, LBRS_E_NONPHYSICAL):
        raise LBRSError(rc, "lbrs_get_state")
    return {"rc": rc, "t": t.value, "nsteps": n.value, "lambda": lam.value, "status": st.value,
            "fail_step": fail.value}


def lbrs_moments(ctx, U):
    _check(load_library().lbrs_moments(ctx, _dptr(U)), "lbrs_moments")


def lbrs_get_f(ctx, f):
    _check(load_library().lbrs_get_f(ctx, _dptr(f)), "lbrs_get_f")


def lbrs_set_f(ctx, f, t: float, n: int):
    _check(load_library().lbrs_set_f(ctx, _dptr(f), float(t), int(n)), "lbrs_set_f")


def lbrs_window_objective(ctx, ix0, ix1, iy0, iy1, J, fbar):
    _check(load_library().lbrs_window_objective(ctx, int(ix0), int(ix1), int(iy0), int(iy1),
                                                _dptr(J), _dptr(fbar)), "lbrs_window_objective")


def lbrs_step_tape(ctx, Utape):
    _check(load_library().lbrs_step_tape(ctx, _dptr(Utape)), "lbrs_step_tape")


def lbrs_adjoint_step(ctx, Utape, fbar_next, fbar):
    _check(load_library().lbrs_adjoint_step(ctx, _dptr(Utape), _dptr(fbar_next), _dptr(fbar)),
           "lbrs_adjoint_step")


def lbrs_step_tape2(ctx, Utape_n, Utape_n1):
    _check(load_library().lbrs_step_tape2(ctx, _dptr(Utape_n), _dptr(Utape_n1)), "lbrs_step_tape2")


def lbrs_step_tapes(ctx, k, Utape):
    _check(load_library().lbrs_step_tapes(ctx, int(k), _dptr(Utape)), "lbrs_step_tapes")


def lbrs_adjoint_steps(ctx, k, Utape, fbar_next, fbar):
    _check(load_library().lbrs_adjoint_steps(ctx, int(k), _dptr(Utape), _dptr(fbar_next),
                                             _dptr(fbar)), "lbrs_adjoint_steps")


def lbrs_adjoint_step2(ctx, Utape_n1, Utape_n, fbar_next2, fbar):
    _check(load_library().lbrs_adjoint_step2(ctx, _dptr(Utape_n1), _dptr(Utape_n),
                                             _dptr(fbar_next2), _dptr(fbar)), "lbrs_adjoint_step2")


def lbrs_adjoint_init(ctx, fbar0, U0, Ubar0):
    _check(load_library().lbrs_adjoint_init(ctx, _dptr(fbar0), _dptr(U0), _dptr(Ubar0)),
           "lbrs_adjoint_init")


def lbrs_set_stream(ctx, stream=None):
    _check(load_library().lbrs_set_stream(ctx, _stream(stream)), "lbrs_set_stream")


def lbrs_set_fusion(ctx, steps_per_launch: int):
    _check(load_library().lbrs_set_fusion(ctx, int(steps_per_launch)), "lbrs_set_fusion")


def lbrs_set_tile(ctx, rows_per_tile: int, waves_per_block: int = 4, alternate: int = 1):
    _check(load_library().lbrs_set_tile(ctx, int(rows_per_tile), int(waves_per_block),
                                        int(alternate)), "lbrs_set_tile")


def lbrs_destroy(ctx):
    if ctx:
        load_library().lbrs_destroy(ctx)


# ------------------------------------------------------------- convenience
class Sim:
    """One domain: owns its device buffers (torch), drives the C calls."""

    def __init__(self, model, nx, ny=1, domain=(0.0, 1.0, 0.0, 1.0), gamma=1.4, omega=1.0,
                 cfl=0.5, bc=(0, 0, 0, 0), lambda_mode=LBRS_LAMBDA_PER_STEP, lambda_user=0.0,
                 layout=LBRS_LAYOUT_PLANAR, device="cuda", dirichlet_W=(None, None, None, None),
                 law=LBRS_LAW_EULER, scalar_flux=(0.0, 0.0, 0.0, 0.0), solid=None):
        """dirichlet_W: per side, the prescribed primitive states [K][n] of a
        DIRICHLET side (n = ny for the x-sides, nx for the y-sides), converted
        to conserved states on the device and kept for the context's life;
        solid: host uint8 mask [ny][nx] of a body (2D Euler), or None."""
        load_library()
        self.layout = layout
        self.device = torch.device(device)
        self.law = law
        self.dirichlet = tuple(None if d is None else self._side_to_cons(d, gamma)
                               for d in dirichlet_W)
        self.p = make_params(model, nx, ny, domain, gamma, omega, cfl, bc, lambda_mode, lambda_user,
                             layout, self.dirichlet, law, scalar_flux, solid)
        self.body = solid is not None
        self.model, self.nx, self.ny = model, nx, ny
        self.Q = {0: 2, 1: 3, 2: 4}[model]
        self.K = 1 if law == LBRS_LAW_SCALAR else (4 if model == LBRS_D2Q4 else 3)
        fb, ub, sb = lbrs_query_sizes(self.p)
        self.f0 = torch.empty(fb // 8, dtype=torch.float64, device=self.device)
        self.f1 = torch.empty(fb // 8, dtype=torch.float64, device=self.device)
        self.scratch = torch.zeros(sb // 8, dtype=torch.float64, device=self.device)
        self.ctx = None
        self._tile = None   # launch shape and fusion, re-applied to every new context
        self._fuse = 1

    def _side_to_cons(self, Wside, gamma):
        """Conserved states of a side's primitive states [4][n] (2D Euler), by
        the library's conversion on a 3-row strip of unit cells."""
        W = torch.as_tensor(Wside, dtype=torch.float64).to(self.device)
        if self.law == LBRS_LAW_SCALAR:  # u is its own conserved variable
            return W.reshape(-1).contiguous()
        n = W.shape[1]
        Wg = W[:, None, :].expand(W.shape[0], 3, n).contiguous()
        U = torch.empty_like(Wg)
        lbrs_prim_to_cons(make_params(LBRS_D2Q4, n, 3, (0.0, float(n), 0.0, 3.0), gamma), Wg, U)
        return U[:, 0, :].contiguous()

    @property
    def blocked(self) -> bool:
        """The blocked 1D layout: the populations of each 64-cell block contiguous."""
        return self.layout == LBRS_LAYOUT_ROWS and self.model != LBRS_D2Q4

    @property
    def f_shape(self):
        """Shape of population-shaped tensors in this context's layout."""
        if self.blocked:
            return ((self.nx + 63) // 64, self.Q, self.K, 64)
        if self.layout == LBRS_LAYOUT_ROWS:
            return (self.ny, self.Q, self.K, self.nx)
        return (self.Q, self.K, self.ny, self.nx)

    def to_planar(self, f: torch.Tensor) -> torch.Tensor:
        """[Q][K][ny][nx] view/copy of a population tensor of this context."""
        if self.blocked:
            nb = (self.nx + 63) // 64
            g = f.reshape(nb, self.Q, self.K, 64).permute(1, 2, 0, 3).reshape(self.Q, self.K, -1)
            return g[:, :, :self.nx].reshape(self.Q, self.K, 1, self.nx).contiguous()
        if self.layout == LBRS_LAYOUT_ROWS:
            return f.reshape(self.ny, self.Q, self.K, self.nx).permute(1, 2, 0, 3).contiguous()
        return f.reshape(self.Q, self.K, self.ny, self.nx)

    def from_planar(self, f: torch.Tensor) -> torch.Tensor:
        if self.blocked:
            nb = (self.nx + 63) // 64
            g = torch.zeros((self.Q, self.K, nb * 64), dtype=f.dtype, device=f.device)
            g[:, :, :self.nx] = f.reshape(self.Q, self.K, self.nx)
            return g.reshape(self.Q, self.K, nb, 64).permute(2, 0, 1, 3).contiguous()
        if self.layout == LBRS_LAYOUT_ROWS:
            return f.reshape(self.Q, self.K, self.ny, self.nx).permute(2, 0, 1, 3).contiguous()
        return f.reshape(self.Q, self.K, self.ny, self.nx).contiguous()

    @property
    def u_shape(self):
        return (self.K, self.ny, self.nx)

    def prim_to_cons(self, W: torch.Tensor) -> torch.Tensor:
        W = W.to(self.device, torch.float64).contiguous()
        U = torch.empty(self.u_shape, dtype=torch.float64, device=self.device)
        lbrs_prim_to_cons(self.p, W, U)
        return U

    def init(self, U0: torch.Tensor):
        U0 = U0.to(self.device, torch.float64).contiguous()
        if self.ctx is not None:
            lbrs_destroy(self.ctx)
        self.ctx = lbrs_init(self.p, U0, self.f0, self.f1, self.scratch)
        if self._tile is not None:
            lbrs_set_tile(self.ctx, *self._tile)
        if self._fuse != 1:
            lbrs_set_fusion(self.ctx, self._fuse)
        return self

    def init_primitive(self, W):
        if not isinstance(W, torch.Tensor):
            W = torch.from_numpy(W)
        return self.init(self.prim_to_cons(W))

    def set_tile(self, rows_per_tile: int, waves_per_block: int = 4, alternate=None):
        """alternate: None = the default march (alternating, one way with a body).
        Kept for later contexts of this Sim (init creates a new one)."""
        if alternate is None:
            alternate = 0 if self.body else 1
        if self.ctx is not None:
            lbrs_set_tile(self.ctx, rows_per_tile, waves_per_block, alternate)
        self._tile = (rows_per_tile, waves_per_block, alternate)

    @property
    def fusable(self) -> bool:
        """Two fused steps per launch are available (2D Euler, no body, no
        Dirichlet side)."""
        return (self.model == LBRS_D2Q4 and self.law == LBRS_LAW_EULER and not self.body
                and all(d is None for d in self.dirichlet))

    @property
    def fusion(self) -> int:
        return self._fuse

    def set_fusion(self, steps_per_launch: int):
        """2: two fused steps per launch (2D Euler without body or Dirichlet sides).
        Kept for later contexts of this Sim."""
        if self.ctx is not None:
            lbrs_set_fusion(self.ctx, steps_per_launch)
        self._fuse = int(steps_per_launch)

    def step(self, max_steps: int, t_end: float = math.inf):
        lbrs_step(self.ctx, max_steps, t_end)

    def run(self, t_end: float, chunk: int = 1000, max_steps: int = 10**8):
        """Step until t_end (or max_steps); polls the device state every chunk steps."""
        done = 0
        while done < max_steps:
            k = min(chunk, max_steps - done)
            self.step(k, t_end)
            done += k
            s = self.state()
            if s["t"] >= t_end or s["rc"] != LBRS_OK or s["nsteps"] < done:
                return s
        return self.state()

    def state(self):
        return lbrs_get_state(self.ctx)

    PAIR_STATS = ("pairs", "rejected", "bound_only", "single", "predicted", "pred_hit",
                  "pred_miss", "evaluated", "pred_none", "listed", "overflow", "steps3",
                  "steps4", "enqueued")

    def pair_stats(self) -> dict:
        """Counters of the fused launches since init (lbrs_pair_stats)."""
        n = len(self.PAIR_STATS)
        out = (ctypes.c_longlong * n)()
        _check(load_library().lbrs_pair_stats(self.ctx, out, n), "lbrs_pair_stats")
        return dict(zip(self.PAIR_STATS, list(out)))

    def moments(self) -> torch.Tensor:
        U = torch.empty(self.u_shape, dtype=torch.float64, device=self.device)
        lbrs_moments(self.ctx, U)
        return U

    def get_f(self) -> torch.Tensor:
        f = torch.empty(self.f_shape, dtype=torch.float64, device=self.device)
        lbrs_get_f(self.ctx, f)
        return f

    def set_f(self, f: torch.Tensor, t: float, n: int):
        lbrs_set_f(self.ctx, f.contiguous(), t, n)

    def close(self):
        if self.ctx is not None:
            lbrs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- 1D batch
def lbrs_batch_query(units, chunk: int):
    n = len(units)
    arr = (lbrs_params * n)(*units)
    offs = (ctypes.c_longlong * (n + 1))()
    sb = ctypes.c_size_t()
    _check(load_library().lbrs_batch_query(n, arr, int(chunk), offs, ctypes.byref(sb)),
           "lbrs_batch_query")
    return list(offs), sb.value


def lbrs_batch_init(units, t_end, chunk, U0, f, scratch, stream=None):
    n = len(units)
    arr = (lbrs_params * n)(*units)
    te = (ctypes.c_double * n)(*[float(x) for x in t_end]) if t_end is not None else None
    b = ctypes.c_void_p()
    _check(load_library().lbrs_batch_init(ctypes.byref(b), n, arr, te, int(chunk), _dptr(U0),
                                          _dptr(f), ctypes.c_void_p(scratch.data_ptr()),
                                          _stream(stream)), "lbrs_batch_init")
    return b


def lbrs_batch_run(b, max_steps: int):
    _check(load_library().lbrs_batch_run(b, int(max_steps)), "lbrs_batch_run")


def lbrs_batch_get_state(b, nunits: int):
    t = (ctypes.c_double * nunits)()
    lam = (ctypes.c_double * nunits)()
    n = (ctypes.c_longlong * nunits)()
    st = (ctypes.c_uint * nunits)()
    fail = (ctypes.c_longlong * nunits)()
    rc = load_library().lbrs_batch_get_state(b, t, n, lam, st, fail)
    if rc not in (LBRS_OK, LBRS_E_NONPHYSICAL):
        raise LBRSError(rc, "lbrs_batch_get_state")
    return {"rc": rc, "t": list(t), "nsteps": list(n), "lambda": list(lam), "status": list(st),
            "fail_step": list(fail)}


def lbrs_batch_moments(b, U):
    _check(load_library().lbrs_batch_moments(b, _dptr(U)), "lbrs_batch_moments")


class Batch1D:
    """A ragged batch of 1D units in one persistent launch (pools owned here)."""

    def __init__(self, units, t_end=None, chunk: int = 1022, device="cuda"):
        load_library()
        self.units = list(units)
        self.n = len(self.units)
        self.Q = 2 if self.units[0].model == LBRS_D1Q2 else 3
        self.chunk = chunk
        self.offsets, sb = lbrs_batch_query(self.units, chunk)
        self.total = self.offsets[-1]
        self.device = torch.device(device)
        self.f = torch.empty((self.Q * 3, self.total), dtype=torch.float64, device=self.device)
        self.scratch = torch.zeros(max(sb, 256), dtype=torch.uint8, device=self.device)
        self.t_end = t_end
        self.b = None

    def init(self, U0: torch.Tensor):
        if self.b is not None:
            load_library().lbrs_batch_destroy(self.b)
        self.b = lbrs_batch_init(self.units, self.t_end, self.chunk, U0.contiguous(), self.f,
                                 self.scratch)
        return self

    def run(self, max_steps: int):
        lbrs_batch_run(self.b, max_steps)

    def state(self):
        return lbrs_batch_get_state(self.b, self.n)

    def moments(self) -> torch.Tensor:
        U = torch.empty((3, self.total), dtype=torch.float64, device=self.device)
        lbrs_batch_moments(self.b, U)
        return U

    def unit_slice(self, b: int):
        return slice(self.offsets[b], self.offsets[b + 1])

    def close(self):
        if self.b is not None:
            load_library().lbrs_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- 2D batch
class Batch2D:
    """Independent 2D domains stepped together (fixed lattice speeds); pools,
    checkpoint store and tape owned here.  Thin: every call is one C call."""

    def __init__(self, doms, device="cuda"):
        lib = load_library()
        self.doms = list(doms)
        self.n = len(self.doms)
        arr = (lbrs_params * self.n)(*self.doms)
        offs = (ctypes.c_longlong * (self.n + 1))()
        sb = ctypes.c_size_t()
        _check(lib.lbrs_batch2d_query(self.n, arr, offs, ctypes.byref(sb)), "lbrs_batch2d_query")
        self.offsets = list(offs)
        self.total = self.offsets[-1]
        self.device = torch.device(device)
        self.f0 = torch.empty(16 * self.total, dtype=torch.float64, device=self.device)
        self.f1 = torch.empty(16 * self.total, dtype=torch.float64, device=self.device)
        self.scratch = torch.zeros(max(sb.value, 256), dtype=torch.uint8, device=self.device)
        self._arr = arr
        self.b = None
        self._fuse = 1  # kept for later handles (init creates a new one)

    def init(self, U0: torch.Tensor, stream=None):
        lib = load_library()
        if self.b is not None:
            lib.lbrs_batch2d_destroy(self.b)
        self.U0 = U0.contiguous()
        b = ctypes.c_void_p()
        _check(lib.lbrs_batch2d_init(ctypes.byref(b), self.n, self._arr, _dptr(self.U0),
                                     _dptr(self.f0), _dptr(self.f1),
                                     ctypes.c_void_p(self.scratch.data_ptr()), _stream(stream)),
               "lbrs_batch2d_init")
        self.b = b
        if self._fuse != 1:
            self.set_fusion(self._fuse)
        return self

    def set_fusion(self, steps_per_launch: int):
        """k = 2 to 4: k fused steps per forward launch (lbrs_batch2d_set_fusion)."""
        self._fuse = int(steps_per_launch)
        if self.b is not None:
            _check(load_library().lbrs_batch2d_set_fusion(self.b, self._fuse),
                   "lbrs_batch2d_set_fusion")

    def reset(self, U0):
        _check(load_library().lbrs_batch2d_reset(self.b, _dptr(U0)), "lbrs_batch2d_reset")

    def step(self, n: int):
        _check(load_library().lbrs_batch2d_step(self.b, int(n)), "lbrs_batch2d_step")

    def step_tape(self, tape):
        _check(load_library().lbrs_batch2d_step_tape(self.b, _dptr(tape)), "lbrs_batch2d_step_tape")

    def adjoint_step(self, tape, gn, g):
        _check(load_library().lbrs_batch2d_adjoint_step(self.b, _dptr(tape), _dptr(gn), _dptr(g)),
               "lbrs_batch2d_adjoint_step")

    def adjoint_init(self, fb0, U0, Ub):
        _check(load_library().lbrs_batch2d_adjoint_init(self.b, _dptr(fb0), _dptr(U0), _dptr(Ub)),
               "lbrs_batch2d_adjoint_init")

    def set_window(self, lo: float, hi: float):
        _check(load_library().lbrs_batch2d_set_window(self.b, float(lo), float(hi)),
               "lbrs_batch2d_set_window")

    def window_objective(self, J, fbar):
        _check(load_library().lbrs_batch2d_window_objective(self.b, _dptr(J), _dptr(fbar)),
               "lbrs_batch2d_window_objective")

    def moments(self) -> torch.Tensor:
        U = torch.empty((4, self.total), dtype=torch.float64, device=self.device)
        _check(load_library().lbrs_batch2d_moments(self.b, _dptr(U)), "lbrs_batch2d_moments")
        return U

    def get_f(self) -> torch.Tensor:
        f = torch.empty(16 * self.total, dtype=torch.float64, device=self.device)
        _check(load_library().lbrs_batch2d_get_f(self.b, _dptr(f)), "lbrs_batch2d_get_f")
        return f

    def gradient(self, U0, nsteps: int, segment: int, ckpt, tape, fbar, work, J, Ubar0,
                 use_graph: bool = True):
        _check(load_library().lbrs_batch2d_gradient(
            self.b, _dptr(U0), int(nsteps), int(segment), _dptr(ckpt), _dptr(tape), _dptr(fbar),
            _dptr(work), _dptr(J), _dptr(Ubar0), int(use_graph)), "lbrs_batch2d_gradient")

    def state(self):
        n = ctypes.c_longlong()
        lam = (ctypes.c_double * self.n)()
        st = (ctypes.c_uint * self.n)()
        rc = load_library().lbrs_batch2d_get_state(self.b, ctypes.byref(n), lam, st)
        if rc not in (LBRS_OK, LBRS_E_NONPHYSICAL):
            raise LBRSError(rc, "lbrs_batch2d_get_state")
        return {"rc": rc, "nsteps": n.value, "lambda": list(lam), "status": list(st)}

    def unit_slice(self, d: int):
        return slice(self.offsets[d], self.offsets[d + 1])

    def close(self):
        if self.b is not None:
            load_library().lbrs_batch2d_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
