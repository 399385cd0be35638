"""Host logic of solid bodies (no GPU): the node codes the library builds for
the step kernel, and which masks it accepts.

Population order (D2Q4, Sec. II.D): 0 (-,-), 1 (+,-), 2 (+,+), 3 (-,+).
Rule per population in bits 3i..3i+2: 0 pulled, 1 face image across x,
2 face image across y, 3 concave corner, 4 convex corner tip; bit 15 solid.
The expected codes below are worked out by hand from the rules at chosen
nodes of the forward-facing step; the accepted masks are checked against the
oracle's independent implementation of the same admissibility condition."""
import numpy as np
import pytest
import torch

import oracle
from paper_1504_07034_amd import lbrs
from paper_1504_07034_amd import workloads as wl

T, P, W, D = 0, 1, 2, 3
PULL, FACE_X, FACE_Y, CONCAVE, TIP = 0, 1, 2, 3, 4


def lib_available():
    try:
        lbrs.load_library(require_gpu=False)
        return True
    except Exception:
        return False


pytestmark = pytest.mark.skipif(not lib_available(), reason="liblbrs.so is not built")


def code(**rules):
    """Code from {population index: rule}."""
    c = 0
    for i, r in rules.items():
        c |= r << (3 * int(i[1:]))
    return c


_SIDE_STATES = torch.zeros(4 * 64, dtype=torch.float64)  # never read by the host calls


def params(nx, ny, sides, solid, model=lbrs.LBRS_D2Q4, law=lbrs.LBRS_LAW_EULER):
    dirichlet = tuple(_SIDE_STATES if sides[s] == D else None for s in range(4))
    return lbrs.make_params(model, nx, ny, (0.0, nx / ny, 0.0, 1.0), bc=sides, solid=solid,
                            law=law, scalar_flux=(0.0, 1.0, 1.0, 0.0), dirichlet=dirichlet)


def test_forward_step_codes_by_hand():
    w = wl.forward_step()
    # the step: columns >= 48, rows <= 15 (centres x > 0.6, y < 0.2 at dx = 1/80)
    assert w.solid[:16, 48:].all() and not w.solid[16:, :].any() and not w.solid[:, :48].any()
    c = lbrs.lbrs_body_codes(params(w.nx, w.ny, (T, T, W, W), w.solid))
    assert c[5, 100] == 0x8000 and c[15, 48] == 0x8000            # solid cells
    assert c[40, 100] == 0                                        # open flow
    # top face of the step, node (60, 16): the upward populations 2 (+,+) and
    # 3 (-,+) come from row 15 (solid); their axis neighbours: across y only
    assert c[16, 60] == code(p2=FACE_Y, p3=FACE_Y)
    # front face, node (47, 8): populations 0 (-,-) and 3 (-,+) come from
    # column 48 (solid), across x only
    assert c[8, 47] == code(p0=FACE_X, p3=FACE_X)
    # the step's tip seen from node (47, 16): only population 3 (-,+) has a
    # solid source (48, 15), whose axis neighbours (48, 16) and (47, 15) are
    # fluid -- a convex corner tip
    assert c[16, 47] == code(p3=TIP)
    # the node above the tip column, (48, 16): population 3 from (49, 15)
    # across y; population 2 (+,+) from (47, 15), fluid
    assert c[16, 48] == code(p3=FACE_Y)
    # the step's foot, node (47, 0), with the bottom wall: population 3 from
    # (48, -1), both neighbours solid (concave); population 2 from (46, -1)
    # across y (the wall); population 0 from (48, 1) across x
    assert c[0, 47] == code(p0=FACE_X, p2=FACE_Y, p3=CONCAVE)
    # bottom wall away from the step, node (20, 0): across y; the top wall,
    # node (20, 79): populations 0 and 1 across y
    assert c[0, 20] == code(p2=FACE_Y, p3=FACE_Y)
    assert c[79, 20] == code(p0=FACE_Y, p1=FACE_Y)
    # inflow (Dirichlet-like, not a wall) side: node (0, 40) has no image
    assert c[40, 0] == 0


def test_wall_box_corner_codes():
    """Walls on all sides with an empty mask: every corner node is concave
    on its diagonal population and a face on the two others."""
    nx, ny = 9, 7
    c = lbrs.lbrs_body_codes(params(nx, ny, (W, W, W, W), np.zeros((ny, nx), np.uint8)))
    assert c[0, 0] == code(p1=FACE_X, p2=CONCAVE, p3=FACE_Y)
    assert c[0, nx - 1] == code(p0=FACE_X, p3=CONCAVE, p2=FACE_Y)
    assert c[ny - 1, 0] == code(p2=FACE_X, p1=CONCAVE, p0=FACE_Y)
    assert c[ny - 1, nx - 1] == code(p3=FACE_X, p0=CONCAVE, p1=FACE_Y)
    assert c[3, 4] == 0


def test_periodic_wrap_through_the_mask():
    """A body touching a periodic side is seen from the other side."""
    nx, ny = 12, 10
    m = np.zeros((ny, nx), np.uint8)
    m[3:7, 0:3] = 1
    c = lbrs.lbrs_body_codes(params(nx, ny, (P, P, P, P), m))
    # node (11, 4): populations 0 (-,-) and 3 (-,+) pull from column 12 = 0
    assert c[4, 11] == code(p0=FACE_X, p3=FACE_X)
    # with transmissive sides the same node sees no body (clamped to itself)
    c2 = lbrs.lbrs_body_codes(params(nx, ny, (T, T, T, T), m))
    assert c2[4, 11] == 0


def random_mask(rng, nx, ny):
    m = np.zeros((ny, nx), np.uint8)
    for _ in range(rng.integers(1, 6)):
        w, h = rng.integers(1, 5, size=2)
        x0, y0 = rng.integers(0, nx - w), rng.integers(0, ny - h)
        m[y0:y0 + h, x0:x0 + w] = 1
    return m


@pytest.mark.parametrize("sides", [(T, T, T, T), (P, P, W, W), (W, W, W, W), (D, T, W, W),
                                   (T, D, P, P)])
def test_admissibility_agrees_with_the_oracle(sides):
    """Random masks (thin gaps included): the library accepts exactly the
    masks the oracle accepts."""
    rng = np.random.default_rng(sum(sides))
    nx, ny = 16, 12
    U = np.zeros((4, ny, nx))
    U[0] = 1.0
    U[3] = 2.5
    dirichlet = [None] * 4
    for s in range(4):
        if sides[s] == D:
            n = ny if s < 2 else nx
            dirichlet[s] = np.tile(np.array([1.0, 0.0, 0.0, 2.5])[:, None], (1, n))
    seen = set()
    for _ in range(60):
        m = random_mask(rng, nx, ny)
        Po = oracle.Problem(model=oracle.D2Q4, nx=nx, ny=ny, domain=(0.0, nx / ny, 0.0, 1.0),
                            sides=sides, solid=m, dirichlet=tuple(dirichlet))
        ok_oracle = oracle.run(Po, U, max_steps=0).status == oracle.OK
        try:
            lbrs.lbrs_body_codes(params(nx, ny, sides, m))
            ok_lib = True
        except lbrs.LBRSError as e:
            assert e.code == lbrs.LBRS_E_INVAL
            ok_lib = False
        assert ok_lib == ok_oracle
        seen.add(ok_lib)
    assert seen == {True, False}


def test_body_params_rejected():
    m = np.zeros((8, 8), np.uint8)
    for p in (params(8, 8, (T, T, T, T), m, law=lbrs.LBRS_LAW_SCALAR),):
        with pytest.raises(lbrs.LBRSError):
            lbrs.lbrs_body_codes(p)
    p1 = lbrs.make_params(lbrs.LBRS_D1Q3, 8, 1)
    p1.solid = m.ctypes.data
    with pytest.raises(lbrs.LBRSError):
        lbrs.lbrs_body_codes(p1)
    with pytest.raises(ValueError):
        params(8, 8, (T, T, T, T), np.zeros((7, 8), np.uint8))
    # walls at a corner: only with a mask
    with pytest.raises(lbrs.LBRSError):
        lbrs.lbrs_query_sizes(lbrs.make_params(lbrs.LBRS_D2Q4, 8, 8, (0, 1, 0, 1), bc=(W, T, W, T)))
    f, u, s0 = lbrs.lbrs_query_sizes(params(8, 8, (W, T, W, T), m))
    _, _, s1 = lbrs.lbrs_query_sizes(lbrs.make_params(lbrs.LBRS_D2Q4, 8, 8, (0, 1, 0, 1)))
    # the codes (2 B per cell) come on top of the time state; a context with a
    # body never fuses launches, so it has no candidate list (16384 x 16 B)
    assert s0 >= s1 - 16384 * 16 + 2 * 64
