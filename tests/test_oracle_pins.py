"""Pins of the FP64 reference against what the paper and mathematics fix:
closed forms, invariants, brute force on tiny inputs, library routines.

CPU only.  Each test names the passage of arXiv 2511.17710 it follows.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import checks

HERE = os.path.dirname(os.path.abspath(__file__))
PI = np.pi


def golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------- metric
def test_cfl_paper_statement_2d_cartesian():
    """Sec. 2.4 (CFL paragraph): in 2D Cartesian with dx = dy, dx_min = dx/sqrt(2)."""
    fx = golden("paper_closed_forms.json")["cfl_2d_cartesian"]
    for dx in fx["dx"]:
        g = O.make_grid("cart", 2, (10, 10), (0, 0), (10 * dx, 10 * dx))
        assert O.dt_from_cfl(g, 1.0) == pytest.approx(dx / np.sqrt(2.0), rel=1e-15)
        g3 = O.make_grid("cart", 3, (4, 4, 4), (0, 0, 0), (4 * dx,) * 3)
        assert O.dt_from_cfl(g3, 1.0) == pytest.approx(dx / np.sqrt(3.0), rel=1e-15)


def _fd_jacobian(g, x, phi, h=1e-5):
    """Columns dX/dx^1, dX/dx^2, dX/dphi of the forward map, central differences."""
    cols = []
    for d in range(2):
        xp = np.array(x, dtype=float)
        xm = np.array(x, dtype=float)
        xp[d] += h
        xm[d] -= h
        cols.append((O.code_to_cart(g, xp, phi) - O.code_to_cart(g, xm, phi)) / (2 * h))
    cols.append((O.code_to_cart(g, x, phi + h) - O.code_to_cart(g, x, phi - h)) / (2 * h))
    return np.array(cols).T


@pytest.mark.parametrize("geom,vt,rmax", [("sph", 0.0, 20.0), ("qsph", 0.0, 20.0),
                                          ("qsph", 0.3, 50.0), ("qsph", 0.8, 50.0)])
def test_metric_is_jacobian_of_forward_map(geom, vt, rmax):
    """Sec. 2.4: for the diagonal metrics sqrt(h_ii) = |dX/dx^i| of the code ->
    Cartesian map, and the coordinate columns are orthogonal."""
    g = O.make_grid(geom, 2, (64, 32), (1.0, 0), (rmax, PI), vartheta=vt)
    rng = np.random.default_rng(1)
    for _ in range(25):
        x = np.array([rng.uniform(0.3, 63.7), rng.uniform(0.3, 31.7), 0.0])
        phi = rng.uniform(0, 2 * PI)
        Jm = _fd_jacobian(g, x, phi)
        h = O.sqrt_h(g, x)
        np.testing.assert_allclose(np.linalg.norm(Jm, axis=0), h, rtol=2e-8)
        G = Jm.T @ Jm
        off = G - np.diag(np.diag(G))
        assert np.max(np.abs(off)) < 1e-7 * np.max(np.diag(G))


def test_qsph_dtheta_dT_matches_finite_difference():
    """Sec. 2.4: d theta/d T = 1 + 2 vt + 12 vt (T/pi)(T/pi - 1) is the derivative of
    theta(T) = T + 2 vt T (1 - 2T/pi)(1 - T/pi)."""
    for vt in (0.05, 0.3, 0.9):
        g = O.make_grid("qsph", 2, (8, 8), (1.0, 0), (10.0, PI), vartheta=vt)
        for T in np.linspace(0.01, PI - 0.01, 23):
            h = 1e-6
            fd = (O.theta_of_T(g, T + h) - O.theta_of_T(g, T - h)) / (2 * h)
            # scale factor h22 / (dT r) is theta_T
            x2 = T / (PI / 8)
            hh = O.sqrt_h(g, [0.0, x2, 0.0])
            r = 1.0  # r at x1 = 0 (r0 = 0, r_min = 1)
            assert hh[1] / ((PI / 8) * r) == pytest.approx(fd, rel=1e-8)


def test_qsph_theta_fixed_points():
    """theta(T) fixes 0, pi/2 and pi for any vartheta (closed form of Sec. 2.4)."""
    for vt in (0.0, 0.3, 0.9):
        g = O.make_grid("qsph", 2, (8, 8), (1.0, 0), (10.0, PI), vartheta=vt)
        assert O.theta_of_T(g, 0.0) == 0.0
        assert O.theta_of_T(g, PI / 2) == pytest.approx(PI / 2, abs=1e-15)
        assert O.theta_of_T(g, PI) == pytest.approx(PI, abs=1e-15)


@pytest.mark.parametrize("vt", [1e-6, 0.05, 0.3, 0.4, 0.9])
def test_qsph_inverse_roundtrip(vt):
    """App. B: T(theta) inverts theta(T) on [0, pi] (depressed-cubic reading)."""
    g = O.make_grid("qsph", 2, (8, 8), (1.0, 0), (10.0, PI), vartheta=vt)
    for T in np.linspace(0.0, PI, 101):
        assert O.T_of_theta(g, O.theta_of_T(g, T)) == pytest.approx(T, abs=1e-13)


@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.0), ("qsph", 0.3)])
def test_coordinate_roundtrip(geom, vt):
    """Sec. 2.4 forward then backward maps return the code coordinates; phi in [0, 2pi)."""
    g = O.make_grid(geom, 2, (256, 128), (1.0, 0), (50.0, PI), vartheta=vt)
    rng = np.random.default_rng(2)
    for _ in range(200):
        x = np.array([rng.uniform(0, 256), rng.uniform(0.01, 127.99), 0.0])
        phi = rng.uniform(0, 2 * PI)
        X = O.code_to_cart(g, x, phi)
        xb, pb = O.cart_to_code(g, X)
        assert abs(xb[0] - x[0]) < 1e-11 and abs(xb[1] - x[1]) < 1e-11
        assert 0.0 <= pb < 2 * PI
        assert abs((pb - phi + PI) % (2 * PI) - PI) < 1e-12


# --------------------------------------------------------------------------- fields
def test_fields_from_tetrad_axis_and_scaling():
    """eq. tetradtrans (F^i = F^i_hat / sqrt(h_ii)) and the axis rule of Sec. 2.6
    (E3 = B2 = 0 on j = 0 and j = N2)."""
    g = O.make_grid("sph", 2, (16, 8), (1.0, 0), (5.0, PI))
    rng = np.random.default_rng(3)
    shp = (6,) + O.padded_shape(g)
    tet = rng.normal(size=shp)
    EB = O.fields_from_tetrad(g, tet, 1)
    for c in range(6):
        for (j, i) in [(2, 3), (5, 9), (0, 4), (9, 1)]:
            x = np.array([i - 2 + checks.STAG[c, 0], j - 2 + checks.STAG[c, 1], 0.0])
            on_axis = (c in (2, 4)) and (j - 2 in (0, 8))
            if on_axis:
                assert EB[c, 0, j, i] == 0.0
            else:
                h = O.sqrt_h(g, x)[c % 3]
                assert EB[c, 0, j, i] == pytest.approx(tet[c, 0, j, i] / h, rel=1e-14)


# --------------------------------------------------------------------------- interpolation
@pytest.mark.parametrize("dim", [2, 3])
def test_interp_equals_bruteforce_tent(dim):
    """Step 3 of Sec. 2.3 with the first-order shape: equal to a brute-force sum of
    tent-function weights over the whole Yee lattice of each component."""
    n = (5, 4, 3)[:dim] + (1,) * (3 - dim)
    g = O.make_grid("cart", dim, n, (0, 0, 0), n)
    rng = np.random.default_rng(4)
    EB = rng.normal(size=(6,) + O.padded_shape(g))
    P = 40
    cell = np.zeros((P, 3), dtype=np.int32)
    offs = np.zeros((P, 3))
    for d in range(dim):
        cell[:, d] = rng.integers(0, n[d], P)
        offs[:, d] = rng.random(P)
    offs[0, :dim] = 0.0
    offs[1, :dim] = 0.5
    a = O.interp(g, EB, cell, offs)
    b = checks.tent_interp(EB, n, dim, cell, offs)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


def test_interp_reproduces_linear_fields():
    """A field linear in code coordinates on each component's lattice is
    interpolated exactly (first-order shape); constants give a partition of unity."""
    g = O.make_grid("cart", 3, (6, 6, 6), (0, 0, 0), (6, 6, 6))
    shp = O.padded_shape(g)
    k, j, i = np.meshgrid(*[np.arange(s) - 2.0 for s in shp], indexing="ij")
    coef = np.array([[0.3, -1.1, 0.7, 2.0], [1.5, 0.2, -0.4, -1.0], [0.1, 0.9, 1.3, 0.5],
                     [-0.6, 0.4, 0.8, 3.0], [1.0, 1.0, -1.0, 0.0], [0.0, -2.0, 0.25, 1.0]])
    EB = np.zeros((6,) + shp)
    for c in range(6):
        s = checks.STAG[c]
        EB[c] = coef[c, 0] * (i + s[0]) + coef[c, 1] * (j + s[1]) + coef[c, 2] * (k + s[2]) + \
            coef[c, 3]
    rng = np.random.default_rng(5)
    P = 50
    cell = rng.integers(1, 5, size=(P, 3)).astype(np.int32)
    offs = rng.random((P, 3))
    out = O.interp(g, EB, cell, offs)
    x = cell + offs
    exp = x @ coef[:, :3].T + coef[:, 3]
    np.testing.assert_allclose(out, exp, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------- tetrad + rotation
@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.0), ("qsph", 0.3)])
def test_to_cart_is_contravariant_pushforward(geom, vt):
    """Step 4 (eq. tetradtrans + rotation): the global Cartesian vector of the
    contravariant components F^i is F^i dX/dx^i (x^3 = phi), with dX/dx^i taken
    from finite differences of the Sec. 2.4 forward map."""
    g = O.make_grid(geom, 2, (64, 32), (1.0, 0), (30.0, PI), vartheta=vt)
    rng = np.random.default_rng(6)
    P = 30
    cell = np.stack([rng.integers(0, 64, P), rng.integers(1, 31, P), np.zeros(P)], 1).astype(np.int32)
    offs = np.concatenate([rng.random((P, 2)), np.zeros((P, 1))], 1)
    phi = rng.uniform(0, 2 * PI, P)
    F6 = rng.normal(size=(P, 6))
    E, B = O.to_cart(g, cell, offs, phi, F6)
    for p in range(P):
        Jm = _fd_jacobian(g, cell[p] + offs[p], phi[p])
        np.testing.assert_allclose(E[p], Jm @ F6[p, :3], rtol=1e-7, atol=1e-7 * np.abs(Jm).max())
        np.testing.assert_allclose(B[p], Jm @ F6[p, 3:], rtol=1e-7, atol=1e-7 * np.abs(Jm).max())


def test_to_cart_cartesian_scales_by_cell_size():
    g = O.make_grid("cart", 3, (4, 4, 4), (0, 0, 0), (2.0, 8.0, 4.0))
    F6 = np.arange(1, 7, dtype=float).reshape(1, 6)
    E, B = O.to_cart(g, np.zeros((1, 3), np.int32), np.zeros((1, 3)), None, F6)
    np.testing.assert_array_equal(E[0], [0.5, 4.0, 3.0])
    np.testing.assert_array_equal(B[0], [2.0, 10.0, 6.0])


# --------------------------------------------------------------------------- Boris
def test_boris_pure_E_kick():
    """B = 0: u^{n+1/2} = u^{n-1/2} + 2 k E exactly."""
    rng = np.random.default_rng(7)
    E = rng.normal(size=(20, 3))
    u = rng.normal(size=(20, 3))
    out = O.boris(0.13, E, np.zeros((20, 3)), u)
    np.testing.assert_allclose(out, u + 2 * 0.13 * E, rtol=0, atol=1e-15)


def test_boris_pure_B_rotation_closed_form():
    """E = 0: one step is an exact rotation about B by -2 atan(k|B|/gamma)
    (clockwise for k > 0), and |u| is conserved."""
    rng = np.random.default_rng(8)
    for _ in range(50):
        B = rng.normal(size=3)
        u = rng.normal(size=3) * 3
        k = rng.uniform(-0.4, 0.4)
        out = O.boris(k, np.zeros(3), B, u)[0]
        gam = np.sqrt(1 + u @ u)
        alpha = -2 * np.arctan(k * np.linalg.norm(B) / gam)
        b = B / np.linalg.norm(B)
        rot = u * np.cos(alpha) + np.cross(b, u) * np.sin(alpha) + b * (b @ u) * (1 - np.cos(alpha))
        np.testing.assert_allclose(out, rot, rtol=0, atol=2e-14 * np.linalg.norm(u))
        assert np.linalg.norm(out) == pytest.approx(np.linalg.norm(u), rel=1e-15)


def test_boris_ExB_drift():
    """Uniform E x B with |E| < |B|: the time-averaged velocity is E x B / B^2."""
    E = np.array([0.1, 0.0, 0.0])
    B = np.array([0.0, 0.0, 1.0])
    k = 0.05
    u = np.zeros((1, 3))
    vs = []
    for _ in range(20000):
        u = O.boris(k, E, B, u)
        g = np.sqrt(1 + np.sum(u * u))
        vs.append(u[0] / g)
    v = np.mean(vs, axis=0)
    vd = np.cross(E, B) / (B @ B)
    assert np.linalg.norm(v - vd) / np.linalg.norm(vd) < 1e-3


# --------------------------------------------------------------------------- full step pins
def _one_species(cell, offs, u, q=1.0, m=1.0, w=None, phi=None):
    n = cell.shape[0]
    return dict(q=q, m=m, cell=cell, offs=offs, u=u, w=np.ones(n) if w is None else w,
                phi=phi, alive=np.ones(n, dtype=np.int32))


def test_larmor_orbit_full_pipeline():
    """Uniform B interpolates exactly, so the Cartesian pipeline reproduces the
    discrete Boris circle: radius dt |u_perp| / (2 gamma sin(alpha/2)) about a
    fixed centre, alpha = 2 atan(k|B|/gamma)."""
    n = 32
    g = O.make_grid("cart", 2, (n, n), (0, 0), (n, n))
    tet = np.zeros((6, 1, n, n))
    tet[5] = 1.0
    EB = O.fields_from_tetrad(g, tet, 0)
    dt = O.dt_from_cfl(g, 0.45)
    u0 = np.array([[0.7, 0.2, 0.1]])
    sp = [_one_species(np.array([[16, 16, 0]], np.int32), np.array([[0.3, 0.6, 0.0]]), u0)]
    pts = []
    for s in range(150):
        sp, _ = O.run(g, dt, 1, EB, sp)
        pts.append(sp[0]["cell"][0, :2] + sp[0]["offs"][0, :2])
    pts = np.array(pts)
    gam = np.sqrt(1 + u0[0] @ u0[0])
    k = dt / 2.0
    alpha = 2 * np.arctan(k / gam)
    R = dt * np.linalg.norm(u0[0, :2]) / (2 * gam * np.sin(alpha / 2))
    # centre from three points, then radius spread
    A = pts[0]
    Bp = pts[40]
    Cp = pts[80]
    M = np.array([[Bp[0] - A[0], Bp[1] - A[1]], [Cp[0] - A[0], Cp[1] - A[1]]]) * 2
    rhs = np.array([Bp @ Bp - A @ A, Cp @ Cp - A @ A])
    ctr = np.linalg.solve(M, rhs)
    rad = np.linalg.norm(pts - ctr, axis=1)
    assert np.max(np.abs(rad - R)) < 1e-12 * n
    assert np.all(np.abs(sp[0]["u"][0] - 0) < 10)


def test_free_streaming_cartesian():
    """E = B = 0: offsets advance by dt u / (gamma Delta) per step, cells wrap."""
    n = 8
    g = O.make_grid("cart", 3, (n, n, n), (0, 0, 0), (2.0 * n, n, 0.5 * n))
    EB = np.zeros((6,) + O.padded_shape(g))
    dt = O.dt_from_cfl(g, 0.45)
    rng = np.random.default_rng(9)
    P = 64
    cell = rng.integers(0, n, size=(P, 3)).astype(np.int32)
    offs = rng.random((P, 3))
    u = rng.normal(size=(P, 3)) * 2
    sp = [_one_species(cell, offs, u)]
    out, _ = O.run(g, dt, 5, EB, sp)
    gam = np.sqrt(1 + np.sum(u * u, 1))
    D = np.array([2.0, 1.0, 0.5])
    x_exp = cell + offs + 5 * dt * u / gam[:, None] / D
    x_got = out[0]["cell"] + out[0]["offs"]
    dx = (x_got - x_exp + n / 2) % n - n / 2
    assert np.max(np.abs(dx)) < 1e-13
    assert np.all((out[0]["offs"] >= 0) & (out[0]["offs"] < 1))
    np.testing.assert_array_equal(out[0]["u"], u)


@pytest.mark.parametrize("geom,vt,rmax", [("sph", 0.0, 20.0), ("qsph", 0.0, 20.0),
                                          ("qsph", 0.3, 50.0)])
def test_offset_relative_move_equals_literal(geom, vt, rmax):
    """Steps 6-7: x^{n+1} = backward(forward(x^n) + dt u/gamma).  The reference
    evaluates it in offset-relative form; it must agree with the literal
    composition of the Sec. 2.4 maps, including near the axis."""
    N1, N2 = 512, 256
    g = O.make_grid(geom, 2, (N1, N2), (1.0, 0), (rmax, PI), vartheta=vt)
    dt = O.dt_from_cfl(g, 0.45)
    rng = np.random.default_rng(10)
    P = 2000
    cell = np.stack([rng.integers(2, N1 - 2, P), rng.integers(0, N2, P), np.zeros(P)], 1).astype(np.int32)
    cell[:200, 1] = rng.integers(0, 2, 200)  # near theta = 0
    cell[200:400, 1] = N2 - 1 - rng.integers(0, 2, 200)  # near theta = pi
    offs = np.concatenate([rng.random((P, 2)), np.zeros((P, 1))], 1)
    cell[400:420, 1] = 0
    offs[400:420, 1] = 0.0  # exactly on the axis theta = 0
    phi = rng.uniform(0, 2 * PI, P)
    u = rng.normal(size=(P, 3)) * 3
    res = O.move(g, dt, cell, offs, phi, u)
    xl, pl = O.move_literal(g, dt, cell, offs, phi, u)
    x_rel = res["cell"][:, :2] + res["offs"][:, :2]
    err = np.abs(x_rel - xl[:, :2])
    assert np.max(err) < 1e-9, np.max(err)
    dph = np.abs((res["phi"] - pl + PI) % (2 * PI) - PI)
    rho = np.array([np.linalg.norm(O.code_to_cart(g, x_rel[p].tolist() + [0.0], 0.0)[:2])
                    for p in range(P)])
    assert np.max(dph * np.maximum(rho, 1e-300)) < 1e-9
    assert np.all((res["offs"][:, :2] >= 0) & (res["offs"][:, :2] < 1))
    assert np.all((res["cell"][:, 1] >= 0) & (res["cell"][:, 1] < N2))


def test_radial_exit_kills_after_depositing():
    """A particle leaving r_min or r_max deposits the whole step (ghost cells),
    then is dead and never pushed again (reading of the ABSORB and ATMOSPHERE particle boundaries, Sec. 5.1.2 and Sec. 5.2)."""
    g = O.make_grid("sph", 2, (16, 16), (1.0, 0), (3.0, PI))
    EB = np.zeros((6,) + O.padded_shape(g))
    dt = O.dt_from_cfl(g, 0.45)
    th = (8 + 0.5) * PI / 16
    cell = np.array([[0, 8, 0], [15, 8, 0]], np.int32)
    offs = np.array([[0.02, 0.5, 0], [0.98, 0.5, 0]])
    u = np.array([[-5 * np.sin(th), 0, -5 * np.cos(th)], [5 * np.sin(th), 0, 5 * np.cos(th)]])
    phi = np.zeros(2)
    sp = [_one_species(cell, offs, u, phi=phi)]
    out, J = O.run(g, dt, 1, EB, sp)
    assert list(out[0]["alive"]) == [0, 0]
    assert out[0]["cell"][0, 0] == -1 and out[0]["cell"][1, 0] == 16
    r = checks.continuity_residual(J, (16, 16, 1), 2, False, dt,
                                   (out[0]["cell_prev"], out[0]["offs_prev"]),
                                   (out[0]["cell"], out[0]["offs"]), np.ones(2))
    assert r < 1e-12
    out2, J2 = O.run(g, dt, 1, EB, out)
    assert np.all(J2 == 0)
    np.testing.assert_array_equal(out2[0]["cell"], out[0]["cell"])


# --------------------------------------------------------------------------- deposit
def _random_state(geom, dim, n, P, rng, vt=0.0, rmax=10.0, umax=4.0):
    if geom == "cart":
        g = O.make_grid("cart", dim, n, (0, 0, 0), n)
    else:
        g = O.make_grid(geom, 2, n, (1.0, 0), (rmax, PI), vartheta=vt)
    cell = np.zeros((P, 3), np.int32)
    offs = np.zeros((P, 3))
    for d in range(dim):
        lo = 0 if geom == "cart" or d == 1 else 0
        cell[:, d] = rng.integers(lo, n[d], P)
        offs[:, d] = rng.random(P)
    u = rng.normal(size=(P, 3)) * umax
    phi = rng.uniform(0, 2 * PI, P) if geom != "cart" else None
    q = rng.choice([-1.0, 1.0], P)
    w = rng.uniform(0.5, 2.0, P)
    return g, cell, offs, u, phi, q, w


@pytest.mark.parametrize("geom,dim,n,vt", [("cart", 2, (6, 5, 1), 0.0), ("cart", 3, (5, 4, 3), 0.0),
                                           ("sph", 2, (12, 10, 1), 0.0),
                                           ("qsph", 2, (12, 10, 1), 0.3)])
def test_deposit_charge_continuity(geom, dim, n, vt):
    """eq. chargecons-2: sum_s q_s sum_p [S(x - x^{n+1}) - S(x - x^n)]/dt + div J = 0
    at every node of the lattice (first-order shape, code coordinates)."""
    rng = np.random.default_rng(11)
    g, cell, offs, u, phi, q, w = _random_state(geom, dim, n, 400, rng, vt=vt)
    EB = rng.normal(size=(6,) + O.padded_shape(g)) * 0.3
    dt = O.dt_from_cfl(g, 0.45)
    species = []
    for qq in (-1.0, 1.0):
        sel = q == qq
        species.append(dict(q=qq, m=1.0, cell=cell[sel], offs=offs[sel], u=u[sel], w=w[sel],
                            phi=None if phi is None else phi[sel],
                            alive=np.ones(sel.sum(), np.int32)))
    out, J = O.run(g, dt, 1, EB, species)
    prev_c = np.concatenate([s["cell_prev"] for s in out])
    prev_o = np.concatenate([s["offs_prev"] for s in out])
    new_c = np.concatenate([s["cell"] for s in out])
    new_o = np.concatenate([s["offs"] for s in out])
    qw = np.concatenate([s["q"] * s["w"] for s in out])
    r = checks.continuity_residual(J, n, dim, geom == "cart", dt, (prev_c, prev_o), (new_c, new_o), qw)
    assert r < 1e-12, r
    # sum rules: sum J^d = sum_p q w dx^d / dt over the in-plane dims
    m = checks.unwrap_step(prev_c, new_c, n, dim, geom == "cart")
    dx = (new_c + m * 0 - prev_c) * 0  # placeholder for shape
    dx = m + new_o - prev_o
    for d in range(dim):
        assert np.sum(J[d]) == pytest.approx(np.sum(qw * dx[:, d]) / dt, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("geom,dim,n,vt", [("cart", 2, (5, 4, 1), 0.0), ("cart", 3, (4, 3, 3), 0.0),
                                           ("sph", 2, (8, 6, 1), 0.0), ("qsph", 2, (8, 6, 1), 0.3)])
def test_deposit_equals_umeda_absolute(geom, dim, n, vt):
    """Step 8 and the Sec. 3.2 footnote: the offset form of the zig-zag equals
    Umeda et al.'s scheme written on absolute positions (brute force, tiny grids)."""
    rng = np.random.default_rng(12)
    g, cell, offs, u, phi, q, w = _random_state(geom, dim, n, 60, rng, vt=vt)
    EB = rng.normal(size=(6,) + O.padded_shape(g)) * 0.3
    dt = O.dt_from_cfl(g, 0.45)
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=offs, u=u, w=w, phi=phi,
               alive=np.ones(len(w), np.int32))]
    out, J = O.run(g, dt, 1, EB, sp)
    s = out[0]
    if geom == "cart" and dim == 2:
        gam = np.sqrt(1 + np.sum(s["u"] ** 2, 1))
        dx3 = dt * s["u"][:, 2] / gam
    elif geom != "cart":
        dx3 = (s["phi"] - phi + PI) % (2 * PI) - PI
    else:
        dx3 = None
    Jb = checks.umeda_brute(n, dim, geom == "cart", dt, np.ones(len(w)), w, s["cell_prev"],
                            s["offs_prev"], s["cell"], s["offs"], dx3)
    scale = np.max(np.abs(Jb))
    np.testing.assert_allclose(J, Jb, rtol=0, atol=1e-13 * scale)


def test_2d_out_of_plane_sum_rule():
    """2D: sum J^3 = sum_p q w dx^3 / dt (reading of the out-of-plane current)."""
    rng = np.random.default_rng(13)
    g, cell, offs, u, phi, q, w = _random_state("cart", 2, (6, 6, 1), 300, rng)
    EB = np.zeros((6,) + O.padded_shape(g))
    dt = O.dt_from_cfl(g, 0.45)
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=offs, u=u, w=w, phi=None,
               alive=np.ones(len(w), np.int32))]
    out, J = O.run(g, dt, 1, EB, sp)
    gam = np.sqrt(1 + np.sum(u ** 2, 1))
    assert np.sum(J[2]) == pytest.approx(np.sum(w * u[:, 2] / gam), rel=1e-13)


def test_pure_B_energy_conserved_curvilinear():
    """Energy in pure B: |u| is constant per particle for any interpolated B."""
    from paper_2511_17710_amd import workloads as W
    wl = W.curvilinear("qsph", 32, 16, 20.0, 0.3, ppc=4, theta=0.5, density_power=0,
                       steps=5, omega=0.0, seed=7)
    g = O.make_grid("qsph", 2, wl.n, wl.lo, wl.hi, vartheta=0.3)
    EB = O.fields_from_tetrad(g, wl.fields_tetrad, 1)
    dt = O.dt_from_cfl(g, 0.45)
    u0 = [np.linalg.norm(s["u"], axis=1) for s in wl.species]
    out, _ = O.run(g, dt, 5, EB, wl.species)
    for s, a in zip(out, u0):
        alive = s["alive"] == 1
        np.testing.assert_allclose(np.linalg.norm(s["u"], axis=1)[alive], a[alive], rtol=1e-13)


# --------------------------------------------------------------------------- sort
def test_sort_matches_numpy_stable_argsort():
    rng = np.random.default_rng(14)
    keys = rng.integers(0, 50, 5000).astype(np.int32)
    keys[rng.random(5000) < 0.1] = np.iinfo(np.int32).max
    np.testing.assert_array_equal(O.sort_perm(keys), np.argsort(keys, kind="stable"))


def test_run_sorts_by_cell_and_dead_last():
    """Stable sort by cell in brick order (8x8 bricks in 2D, x fastest between
    and inside bricks), dead particles last; checked against numpy's stable
    argsort of the key written out here."""
    rng = np.random.default_rng(15)
    n = (20, 12, 1)
    g = O.make_grid("cart", 2, n, (0, 0, 0), n)
    P = 3000
    cell = np.stack([rng.integers(0, 20, P), rng.integers(0, 12, P), np.zeros(P)], 1).astype(np.int32)
    offs = np.concatenate([rng.random((P, 2)), np.zeros((P, 1))], 1)
    alive = (rng.random(P) > 0.2).astype(np.int32)
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=offs, u=np.zeros((P, 3)), w=np.arange(P, dtype=float),
               phi=None, alive=alive)]
    EB = np.zeros((6,) + O.padded_shape(g))
    out, _ = O.run(g, 0.1, 1, EB, sp, sort_every=1)
    nbx = 3  # ceil(20 / 8)
    brick = cell[:, 0] // 8 + nbx * (cell[:, 1] // 8)
    local = cell[:, 0] % 8 + 8 * (cell[:, 1] % 8)
    key = np.where(alive == 1, brick * 64 + local, np.iinfo(np.int32).max)
    perm = np.argsort(key, kind="stable")
    np.testing.assert_array_equal(out[0]["perm"], perm)
    np.testing.assert_array_equal(out[0]["w"], np.arange(P, dtype=float)[perm])


def test_sort_brick_order_3d():
    """3D: 4x4x4 bricks."""
    rng = np.random.default_rng(18)
    n = (9, 8, 6)
    g = O.make_grid("cart", 3, n, (0, 0, 0), n)
    P = 4000
    cell = np.stack([rng.integers(0, n[d], P) for d in range(3)], 1).astype(np.int32)
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=rng.random((P, 3)), u=np.zeros((P, 3)),
               w=np.ones(P), phi=None, alive=np.ones(P, np.int32))]
    out, _ = O.run(g, 0.1, 1, np.zeros((6,) + O.padded_shape(g)), sp, sort_every=1)
    nb = [3, 2, 2]
    b = cell // 4
    lc = cell % 4
    key = (b[:, 0] + nb[0] * (b[:, 1] + nb[1] * b[:, 2])) * 64 + lc[:, 0] + 4 * (lc[:, 1] + 4 * lc[:, 2])
    np.testing.assert_array_equal(out[0]["perm"], np.argsort(key, kind="stable"))


# --------------------------------------------------------------------------- adjoint
def _adj_case(geom, dim, n, P, K, seed, vt=0.0):
    rng = np.random.default_rng(seed)
    g, cell, offs, u, phi, q, w = _random_state(geom, dim, n, P, rng, vt=vt, umax=1.5)
    if geom != "cart":
        cell[:, 0] = rng.integers(3, n[0] - 3, P)
    EB = rng.normal(size=(6,) + O.padded_shape(g)) * 0.2
    if geom == "cart":
        # active region defines the fields; ghosts are periodic copies
        act = np.zeros_like(EB)
        sl = tuple([slice(None)] + [slice(2, 2 + n[d]) if d < dim else slice(None)
                                    for d in (2, 1, 0)])
        act[sl] = EB[sl]
        EB = act
    dt = O.dt_from_cfl(g, 0.45)
    species = [dict(q=-1.0, m=1.0, cell=cell, offs=offs, u=u, w=w, phi=phi,
                    alive=np.ones(P, np.int32)),
               dict(q=1.0, m=2.0, cell=cell.copy(), offs=offs.copy(), u=-u, w=w,
                    phi=phi, alive=np.ones(P, np.int32))]
    lamJ = rng.normal(size=(3,) + O.padded_shape(g))
    lam_u = [rng.normal(size=(P, 3)) for _ in species]
    return g, EB, dt, species, lamJ, lam_u, rng


def _active_mask(g):
    shp = O.padded_shape(g)
    mask = np.zeros((6,) + shp, bool)
    sl = [slice(None)]
    for d in (2, 1, 0):
        sl.append(slice(2, 2 + g.n[d]) if d < g.dim else slice(None))
    mask[tuple(sl)] = True
    return mask


@pytest.mark.parametrize("geom,dim,n,vt", [("cart", 2, (6, 6, 1), 0.0), ("cart", 3, (5, 4, 4), 0.0),
                                           ("sph", 2, (16, 12, 1), 0.0),
                                           ("qsph", 2, (16, 12, 1), 0.3)])
def test_adjoint_dot_product_with_jvp(geom, dim, n, vt):
    """<grad L, v> from the reverse sweep equals the forward-mode directional
    derivative of the same discrete K-step map (exact differentiation)."""
    K = 3
    g, EB, dt, species, lamJ, lam_u, rng = _adj_case(geom, dim, n, 30, K, 16, vt)
    res = O.adjoint(g, dt, K, EB, species, lamJ, lam_u=lam_u)
    vEB = rng.normal(size=EB.shape)
    if geom == "cart":
        vEB = vEB * _active_mask(g)
    vu = [rng.normal(size=(30, 3)) for _ in species]
    vd = [np.concatenate([rng.normal(size=(30, dim)), np.zeros((30, 3 - dim))], 1) * 0
          for _ in species]
    L, dL = O.jvp(g, dt, K, EB, vEB, species, vu, vd, lamJ, lam_u=lam_u)
    assert L == pytest.approx(res["loss"], rel=1e-13)
    ip = np.sum(res["dEB"] * vEB) + sum(np.sum(a * b) for a, b in zip(res["du0"], vu))
    assert ip == pytest.approx(dL, rel=1e-11, abs=1e-12)


def test_adjoint_matches_central_differences():
    """Central finite differences of the plain FP64 forward (no duals) along
    random directions of E/B and u0 (3D Cartesian, periodic)."""
    K = 4
    n = (6, 6, 6)
    g, EB, dt, species, lamJ, lam_u, rng = _adj_case("cart", 3, n, 40, K, 17)
    res = O.adjoint(g, dt, K, EB, species, lamJ, lam_u=lam_u)
    mask = _active_mask(g)

    def loss(EBx, sps):
        out, J = O.run(g, dt, K, EBx, sps)
        return np.sum(lamJ * J) + sum(np.sum(l * s["u"]) for l, s in zip(lam_u, out))

    assert loss(EB, species) == pytest.approx(res["loss"], rel=1e-12)
    for trial in range(3):
        vEB = rng.normal(size=EB.shape) * mask
        vu = [rng.normal(size=(40, 3)) for _ in species]
        h = 1e-6
        sp_p = [dict(s, u=s["u"] + h * v) for s, v in zip(species, vu)]
        sp_m = [dict(s, u=s["u"] - h * v) for s, v in zip(species, vu)]
        fd = (loss(EB + h * vEB, sp_p) - loss(EB - h * vEB, sp_m)) / (2 * h)
        ip = np.sum(res["dEB"] * vEB) + sum(np.sum(a * b) for a, b in zip(res["du0"], vu))
        assert ip == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_sort_keys_export_orders_like_run():
    """The exported key function orders particles exactly as the sorts of a
    run do (the per-step GPU tests sort the GPU's own state with it)."""
    rng = np.random.default_rng(21)
    n = (12, 9, 7)
    g = O.make_grid("cart", 3, n, (0, 0, 0), n)
    P = 3000
    cell = np.stack([rng.integers(0, n[d], P) for d in range(3)], 1).astype(np.int32)
    alive = (rng.random(P) > 0.1).astype(np.int32)
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=rng.random((P, 3)), u=np.zeros((P, 3)),
               w=np.ones(P), phi=None, alive=alive)]
    out, _ = O.run(g, 0.1, 1, np.zeros((6,) + O.padded_shape(g)), sp, sort_every=1)
    np.testing.assert_array_equal(O.sort_perm(O.sort_keys(g, cell, alive)), out[0]["perm"])


@pytest.mark.parametrize("geom,dim,n,vt", [("cart", 2, (6, 5, 1), 0.0), ("cart", 3, (5, 4, 3), 0.0),
                                           ("qsph", 2, (12, 10, 1), 0.3)])
def test_fast_telescoped_continuity_checker(geom, dim, n, vt):
    """The FP64 bincount form of the telescoped charge change equals the
    extended-precision one, and gives a residual at round-off for the
    reference's own step."""
    rng = np.random.default_rng(12)
    g, cell, offs, u, phi, q, w = _random_state(geom, dim, n, 400, rng, vt=vt)
    EB = rng.normal(size=(6,) + O.padded_shape(g)) * 0.3
    dt = O.dt_from_cfl(g, 0.45)
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=offs, u=u, w=w * q, phi=phi,
               alive=np.ones(len(w), np.int32))]
    out, J = O.run(g, dt, 1, EB, sp)
    s = out[0]
    prev, new = (s["cell_prev"], s["offs_prev"]), (s["cell"], s["offs"])
    a = checks.drho_nodes(n, dim, geom == "cart", prev, new, s["w"])
    b = checks.drho_nodes_fast(n, dim, geom == "cart", prev, new, s["w"])
    assert np.max(np.abs(np.asarray(a, dtype=np.float64) - b)) <= 1e-14 * np.max(np.abs(b))
    r = checks.continuity_residual_telescoped(J, n, dim, geom == "cart", dt, prev, new, s["w"])
    assert r < 1e-12, r
