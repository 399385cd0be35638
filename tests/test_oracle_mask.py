"""Pins of the oracle's solid bodies (masks of solid cells).

The wall of a body runs through the fluid nodes next to it, and a population
whose pull source is solid takes the same-node specular image (the free-slip
principle of Sec. II.E; faces, concave corners and convex corner tips).  What
fixes these rules independently of the oracle's own code:

* flat faces and concave corners: the method of images.  A mirror-symmetric
  periodic domain without any body, restricted to one half (quarter), is the
  bounded problem with walls through the mirror node rows/columns;
* all rules, including the corner tip: a gas at rest stays exactly at rest
  around any body (a wrong sign or a wrong mirror population leaves momentum
  at the wall nodes);
* D4 symmetry around a square body and mirror symmetry around an off-centre
  rectangle;
* a body that only reproduces wall sides gives the wall-side result;
* the shock-diffraction case: far from the body the planar shock runs at the
  Rankine-Hugoniot speed.
"""
import numpy as np
import pytest

import oracle
from paper_1504_07034_amd import workloads as wl

from test_oracle_dirichlet import side_cons

pytestmark = pytest.mark.filterwarnings("ignore")


def smooth(rng, nx, ny, amp, modes=4):
    """Sum of a few random Fourier modes on an nx x ny grid of cell centres."""
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    out = np.zeros((ny, nx))
    for _ in range(modes):
        kx, ky = rng.integers(-2, 3, size=2)
        th = rng.uniform(0, 2 * np.pi)
        out += amp / modes * np.cos(2 * np.pi * (kx * X + ky * Y) + th)
    return out


def random_state(rng, nx, ny):
    """Primitive (rho, u, v, p) planes with smooth random structure."""
    W = np.empty((4, ny, nx))
    W[0] = 1.0 + smooth(rng, nx, ny, 0.2)
    W[1] = smooth(rng, nx, ny, 0.3)
    W[2] = smooth(rng, nx, ny, 0.3)
    W[3] = 1.0 + smooth(rng, nx, ny, 0.2)
    return W


def P2(nx, ny, sides, solid=None, omega=1.3):
    h = 1.0 / ny
    return oracle.Problem(model=oracle.D2Q4, nx=nx, ny=ny, domain=(0.0, nx * h, 0.0, 1.0),
                          sides=sides, omega=omega, solid=solid)


T, P, W = oracle.TRANSMISSIVE, oracle.PERIODIC, oracle.WALL


def on_walls(Wh, x=False, y=False):
    """The state with no normal velocity on the mirror rows (y) / columns (x):
    a node on a mirror line is its own image."""
    Wh = Wh.copy()
    if y:
        Wh[2][[0, -1], :] = 0.0
    if x:
        Wh[1][:, [0, -1]] = 0.0
    return Wh


def mirror_y(Wh):
    """Rows 0..H-1 -> periodic rows 0..2H-3, symmetric about rows 0 and H-1."""
    H = Wh.shape[1]
    lower = Wh[:, 1:H - 1][:, ::-1].copy()
    lower[2] *= -1.0
    return np.concatenate([Wh, lower], axis=1)


def mirror_x(Wh):
    Wt = Wh.transpose(0, 2, 1)[[0, 2, 1, 3]]
    return mirror_y(Wt)[[0, 2, 1, 3]].transpose(0, 2, 1)


@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_faces_y_method_of_images(omega):
    rng = np.random.default_rng(1)
    nx, H, a, b = 24, 14, 2, 3          # fluid rows a .. a+H-1, solid below/above
    ny = a + H + b
    Wh = on_walls(random_state(rng, nx, H), y=True)
    solid = np.zeros((ny, nx), np.uint8)
    solid[:a] = 1
    solid[a + H:] = 1
    Wm = np.zeros((4, ny, nx))
    Wm[0] = 1.0
    Wm[3] = 1.0
    Wm[:, a:a + H] = Wh
    Pm = P2(nx, ny, (P, P, T, T), solid, omega)
    rm = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=60)
    Wd = mirror_y(Wh)
    Pd = P2(nx, 2 * H - 2, (P, P, P, P), None, omega)
    rd = oracle.run(Pd, oracle.prim_to_cons(Pd, Wd), max_steps=60)
    assert rm.status == 0 and rd.status == 0
    assert np.max(np.abs(rm.U[:, a:a + H] - rd.U[:, :H])) <= 1e-12
    assert np.all(rm.U[:, :a] == 0.0) and np.all(rm.U[:, a + H:] == 0.0)
    # the same lattice speeds up to round-off (λ* is the same maximum)
    assert np.max(np.abs(rm.lam - rd.lam) / rd.lam) <= 1e-13


def test_faces_x_method_of_images():
    rng = np.random.default_rng(2)
    ny, H, a, b = 20, 13, 3, 2
    nx = a + H + b
    Wh = on_walls(random_state(rng, H, ny), x=True)
    solid = np.zeros((ny, nx), np.uint8)
    solid[:, :a] = 1
    solid[:, a + H:] = 1
    Wm = np.zeros((4, ny, nx))
    Wm[0] = 1.0
    Wm[3] = 1.0
    Wm[:, :, a:a + H] = Wh
    Pm = P2(nx, ny, (T, T, P, P), solid)
    rm = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=60)
    Wd = mirror_x(Wh)
    Pd = P2(2 * H - 2, ny, (P, P, P, P))
    rd = oracle.run(Pd, oracle.prim_to_cons(Pd, Wd), max_steps=60)
    assert rm.status == 0 and rd.status == 0
    assert np.max(np.abs(rm.U[:, :, a:a + H] - rd.U[:, :, :H])) <= 1e-12


@pytest.mark.parametrize("frame", ["mask", "sides"])
def test_box_concave_corners_method_of_images(frame):
    """A closed box: four faces and four concave corners, against the
    periodic domain mirrored about both axes."""
    rng = np.random.default_rng(3)
    Hx, Hy = 16, 12
    Wh = on_walls(random_state(rng, Hx, Hy), x=True, y=True)
    if frame == "mask":
        a = 2
        nx, ny = Hx + 2 * a, Hy + 2 * a
        solid = np.ones((ny, nx), np.uint8)
        solid[a:a + Hy, a:a + Hx] = 0
        Wm = np.zeros((4, ny, nx))
        Wm[0] = 1.0
        Wm[3] = 1.0
        Wm[:, a:a + Hy, a:a + Hx] = Wh
        Pm = P2(nx, ny, (T, T, T, T), solid)
        sl = (slice(None), slice(a, a + Hy), slice(a, a + Hx))
    else:
        # wall sides meeting at corners, with an all-fluid mask to enable the
        # corner rules
        Pm = P2(Hx, Hy, (W, W, W, W), np.zeros((Hy, Hx), np.uint8))
        Wm = Wh
        sl = (slice(None), slice(None), slice(None))
    rm = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=50)
    Wd = mirror_x(mirror_y(Wh))
    Pd = P2(2 * Hx - 2, 2 * Hy - 2, (P, P, P, P))
    rd = oracle.run(Pd, oracle.prim_to_cons(Pd, Wd), max_steps=50)
    assert rm.status == 0 and rd.status == 0
    assert np.max(np.abs(rm.U[sl] - rd.U[:, :Hy, :Hx])) <= 1e-12


def blocks_mask(nx, ny, seed, nblocks=6):
    """Random rectangles at least 2 cells across, gaps of at least 2 cells."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((ny, nx), np.uint8)
    placed = 0
    while placed < nblocks:
        w, h = rng.integers(2, 6, size=2)
        x0 = rng.integers(2, nx - w - 2)
        y0 = rng.integers(2, ny - h - 2)
        grown = solid[y0 - 2:y0 + h + 2, x0 - 2:x0 + w + 2]
        if grown.any():
            continue
        solid[y0:y0 + h, x0:x0 + w] = 1
        placed += 1
    return solid


@pytest.mark.parametrize("seed,sides", [(0, (T, T, W, W)), (1, (P, P, P, P)), (2, (W, W, W, W))])
def test_rest_state_around_bodies(seed, sides):
    """u = v = 0 stays exact and rho, p stay uniform to round-off for any
    body: every image rule maps the rest equilibrium onto itself."""
    nx, ny = 40, 32
    solid = blocks_mask(nx, ny, seed)
    Pm = P2(nx, ny, sides, solid, omega=1.7)
    Wm = np.zeros((4, ny, nx))
    Wm[0] = 1.3
    Wm[3] = 0.8
    r = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=40)
    assert r.status == 0
    fl = solid == 0
    assert np.max(np.abs(r.U[1][fl])) == 0.0
    assert np.max(np.abs(r.U[2][fl])) == 0.0
    assert np.max(np.abs(r.U[0][fl] - 1.3)) <= 1e-13
    assert np.max(np.abs(r.U[3][fl] - 0.8 / 0.4)) <= 1e-13
    assert np.all(r.U[:, ~fl] == 0.0)


def test_rest_state_detects_a_wrong_tip_sign():
    """The rest pin does see the convex tips: a body whose tips see a
    moving gas breaks it (sanity of the pin itself: a uniform flow is not a
    steady state around a square, so momentum changes next to the body)."""
    nx = ny = 24
    solid = np.zeros((ny, nx), np.uint8)
    solid[10:14, 10:14] = 1
    Pm = P2(nx, ny, (P, P, P, P), solid)
    Wm = np.zeros((4, ny, nx))
    Wm[0] = 1.0
    Wm[1] = 0.3
    Wm[3] = 1.0
    r = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=5)
    fl = solid == 0
    assert np.max(np.abs(r.U[2][fl])) > 1e-3


def test_square_body_d4_symmetry():
    """A ring pulse around a centred square body: the D4 symmetries of the
    setting hold to round-off (faces, concave-free convex tips)."""
    n = 40
    solid = np.zeros((n, n), np.uint8)
    solid[16:24, 16:24] = 1
    Pm = P2(n, n, (T, T, T, T), solid)
    x = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(x, x)
    R = np.hypot(X, Y)
    Wm = np.zeros((4, n, n))
    Wm[0] = 1.0 + 0.5 * np.exp(-((R - 0.28) / 0.06) ** 2)
    Wm[3] = 1.0 + 1.5 * np.exp(-((R - 0.28) / 0.06) ** 2)
    r = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=80)
    assert r.status == 0
    rho, m, q, e = r.U
    tol = 1e-13
    assert np.max(np.abs(rho - rho[:, ::-1])) <= tol
    assert np.max(np.abs(rho - rho[::-1, :])) <= tol
    assert np.max(np.abs(rho - rho.T)) <= tol
    assert np.max(np.abs(m + m[:, ::-1])) <= tol
    assert np.max(np.abs(q + q[::-1, :])) <= tol
    assert np.max(np.abs(m - q.T)) <= tol
    assert np.max(np.abs(e - e.T)) <= tol
    # the pulse has reached the body
    assert np.max(np.abs(m[15, 16:24])) > 1e-3


def test_rectangle_body_mirror_symmetry():
    """Uniform flow along x past an off-centre rectangle, symmetric about the
    channel's mid-line: mirror symmetry in y holds to round-off."""
    nx, ny = 48, 30
    solid = np.zeros((ny, nx), np.uint8)
    solid[11:19, 14:20] = 1
    Pm = P2(nx, ny, (T, T, W, W), solid)
    Wm = np.zeros((4, ny, nx))
    Wm[0] = 1.4
    Wm[1] = 0.8
    Wm[3] = 1.0
    solid_r = Pm.solid
    r = oracle.run(Pm, oracle.prim_to_cons(Pm, Wm), max_steps=70)
    assert r.status == 0
    rho, m, q, e = r.U
    assert np.max(np.abs(rho - rho[::-1])) <= 1e-13
    assert np.max(np.abs(m - m[::-1])) <= 1e-13
    assert np.max(np.abs(q + q[::-1])) <= 1e-13
    assert np.max(np.abs(e - e[::-1])) <= 1e-13
    assert np.max(np.abs(q[solid_r == 0])) > 1e-3


def test_body_free_mask_equals_wall_sides():
    rng = np.random.default_rng(5)
    nx, ny = 22, 18
    Wh = random_state(rng, nx, ny)
    Pa = P2(nx, ny, (T, P, W, W)[:0] + (P, P, W, W))
    Pb = P2(nx, ny, (P, P, W, W), np.zeros((ny, nx), np.uint8))
    ra = oracle.run(Pa, oracle.prim_to_cons(Pa, Wh), max_steps=40)
    rb = oracle.run(Pb, oracle.prim_to_cons(Pb, Wh), max_steps=40)
    assert ra.status == 0 and rb.status == 0
    assert np.array_equal(ra.U, rb.U)


def test_masks_rejected():
    nx, ny = 20, 16
    U = np.zeros((4, ny, nx))
    U[0] = 1.0
    U[3] = 2.5
    gap = np.zeros((ny, nx), np.uint8)
    gap[:, 4:8] = 1
    gap[:, 9:13] = 1                         # a channel one cell wide
    slot = np.zeros((ny, nx), np.uint8)
    slot[:7, 6:12] = 1
    slot[:7, 8] = 0                          # a slot one cell wide in a body
    full = np.ones((ny, nx), np.uint8)
    for m in (gap, slot, full):
        r = oracle.run(P2(nx, ny, (T, T, T, T), m), U, max_steps=1)
        assert r.status == oracle.INVAL
    # a plate one cell thick is a body (each side sees a face); the rest
    # state stays at rest around it
    thin = np.zeros((ny, nx), np.uint8)
    thin[5:11, 9] = 1
    r = oracle.run(P2(nx, ny, (T, T, T, T), thin), U, max_steps=20)
    assert r.status == oracle.OK
    assert np.max(np.abs(r.U[1:3][:, thin == 0])) == 0.0
    # bodies are for the D2Q4 Euler equations only
    Ps = P2(nx, ny, (T, T, T, T), np.zeros((ny, nx), np.uint8))
    Ps.flux = oracle.FLUX_QUADRATIC
    Ps.quad = (0.0, 1.0, 1.0, 0.0)
    assert oracle.run(Ps, np.ones((1, ny, nx)), max_steps=1).status == oracle.INVAL
    # corners of wall sides still need a mask
    assert oracle.run(P2(nx, ny, (W, T, W, T)), U, max_steps=1).status == oracle.INVAL
    assert oracle.run(P2(nx, ny, (W, T, W, T), np.zeros((ny, nx), np.uint8)), U,
                      max_steps=1).status == oracle.OK


def test_solid_cells_ignore_their_initial_state():
    """The state given in solid cells (even a non-physical one) plays no part."""
    nx, ny = 24, 20
    solid = np.zeros((ny, nx), np.uint8)
    solid[6:12, 8:15] = 1
    rng = np.random.default_rng(7)
    Wm = random_state(rng, nx, ny)
    Pm = P2(nx, ny, (T, T, T, T), solid)
    U0 = oracle.prim_to_cons(Pm, Wm)
    Ubad = U0.copy()
    Ubad[:, solid == 1] = np.nan
    ra = oracle.run(Pm, U0, max_steps=30)
    rb = oracle.run(Pm, Ubad, max_steps=30)
    assert ra.status == 0 and rb.status == 0
    assert np.array_equal(ra.U, rb.U)
    assert np.array_equal(ra.dt, rb.dt)


def test_diffraction_planar_shock_speed():
    """The Sec. III shock diffraction at 200 x 200 to t = 0.1: in the top rows,
    which no signal from the corner has reached, the shock found from the
    mass along the row (conservative scheme, post-shock inflow) is where the
    Mach 5.09 shock speed puts it, x = 0.2 + 5.09 t, within half a cell."""
    w = wl.shock_diffraction(200)
    Pr = oracle.Problem(model=oracle.D2Q4, nx=w.nx, ny=w.ny, domain=w.domain, sides=w.sides,
                        solid=w.solid)
    Pr.dirichlet = tuple(None if d is None else side_cons(Pr, d) for d in w.dirichlet_W)
    r = oracle.run(Pr, oracle.prim_to_cons(Pr, w.W), t_end=0.1, record=False)
    assert r.status == 0
    rho2 = w.meta["post"][0]
    for j in (-1, -2, -5):
        front = (r.U[0, j].mean() - 1.4) / (rho2 - 1.4)
        assert abs(front - (0.2 + 5.09 * 0.1)) <= 0.5 / w.nx


@pytest.mark.parametrize("omega", [0.7, 1.0, 1.6])
def test_convex_tip_method_of_images_about_a_diagonal(omega):
    """The convex-tip rule is the method of images about a 45-degree line.

    D2Q4 hops change x and y by one cell each, so the nodes with x + y even and
    those with x + y odd form two lattices that never exchange populations
    (away from clamped sides, with a fixed lattice speed).  Take the body
    {x + y <= N - 3} on an N x N grid (N odd): every fluid node of the even
    lattice on the line x + y = N - 1 sees a solid cell only across its
    (-1,-1) diagonal, never across an axis, i.e. a convex tip.  The mirror
    sigma(x, y) = (N-1-y, N-1-x) about that line maps the even lattice onto
    itself, the velocity (+,+) onto (-,-) and (m_x, m_y) onto (-m_y, -m_x).
    On the line a sigma-symmetric solution therefore has
    f_(+,+) = M f_(-,-) with M = that momentum map: the tip rule (opposite
    population, momenta swapped times -s_x s_y = -1).  So the body run equals
    the body-free run from sigma-symmetric data on the even lattice at and
    above the line, inside the region no clamped side reaches.  A bounce-back
    tip (both momenta negated without the swap) breaks the equality wherever
    m_x != m_y on the line."""
    N, steps = 41, 8
    rng = np.random.default_rng(11)
    A = random_state(rng, N, N)
    sig = lambda F: F[::-1, ::-1].T      # F(sigma(p)) for a [y][x] plane
    W = np.empty_like(A)
    W[0] = 0.5 * (A[0] + sig(A[0]))
    W[3] = 0.5 * (A[3] + sig(A[3]))
    W[1] = 0.5 * (A[1] - sig(A[2]))      # u(sigma p) = -v(p)
    W[2] = 0.5 * (A[2] - sig(A[1]))      # v(sigma p) = -u(p)
    assert np.array_equal(sig(W[0]), W[0]) and np.allclose(sig(W[1]), -W[2], atol=0)
    y, x = np.mgrid[0:N, 0:N]
    solid = ((x + y) <= N - 3).astype(np.uint8)
    free = P2(N, N, (T,) * 4, omega=omega)
    U0 = oracle.prim_to_cons(free, W)
    lam = 2.0 * oracle.initial_lattice_speed(free, U0)  # fixed speed: the lattices decouple
    for pr in (free,):
        pr.lam_mode, pr.lam_user = oracle.LAM_USER, lam
    body = P2(N, N, (T,) * 4, solid=solid, omega=omega)
    body.lam_mode, body.lam_user = oracle.LAM_USER, lam
    ref = oracle.run(free, U0, max_steps=steps)
    got = oracle.run(body, U0, max_steps=steps)
    assert ref.status == 0 and got.status == 0
    even_above = ((x + y) % 2 == (N - 1) % 2) & ((x + y) >= N - 1)
    inner = (x >= steps) & (y >= steps) & (x <= N - 1 - steps) & (y <= N - 1 - steps)
    sel = even_above & inner
    assert sel.sum() > 100
    on_line = sel & ((x + y) == N - 1)
    # the tip nodes carry tangential momentum, so a bounce-back tip would show
    assert np.max(np.abs(ref.U[1][on_line] - ref.U[2][on_line])) > 1e-2
    for k in range(4):
        np.testing.assert_allclose(got.U[k][sel], ref.U[k][sel], rtol=0, atol=1e-13)
