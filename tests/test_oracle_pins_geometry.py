"""Pins of the FP64 reference's grid constants, time step, edge branches of
the move and the curvilinear adjoint, against quantities computed here
without the reference's own formulas.

The forward maps below are written from the coordinate definitions of
arXiv 2511.17710 Sec. 2.4 (spherical: uniform r and theta; quasi-spherical:
r = r0 + exp(R), theta(T) of App. B) with the cell sizes derived from the
grid's endpoints, and the metric scale factors are taken as the column norms
of their central-difference Jacobian: a wrong cell size, endpoint or scale
factor inside the reference changes its metric, its time step and its
code -> Cartesian map, and fails these tests.

CPU only.
"""
import numpy as np
import pytest

from oracle import oracle as O

PI = np.pi


# ----------------------------------------------------------------------------- independent maps
def _forward_np(geom, n, rmin, rmax, r0, vt, x1, x2, phi):
    """(x1, x2, phi) -> global Cartesian X, from Sec. 2.4: r spans [rmin, rmax]
    over N1 cells, theta spans [0, pi] over N2 cells (through T for the
    quasi-spherical grid)."""
    N1, N2 = n
    if geom == "sph":
        r = rmin + (rmax - rmin) * x1 / N1
        th = PI * x2 / N2
    else:
        Rlo, Rhi = np.log(rmin - r0), np.log(rmax - r0)
        r = r0 + np.exp(Rlo + (Rhi - Rlo) * x1 / N1)
        T = PI * x2 / N2
        th = T + 2 * vt * T * (1 - 2 * T / PI) * (1 - T / PI)
    return np.stack([r * np.sin(th) * np.cos(phi), r * np.sin(th) * np.sin(phi), r * np.cos(th)],
                    axis=-1)


def _scale_factors_np(geom, n, rmin, rmax, r0, vt, x1, x2, h=1e-3):
    """|dX/dx^1|, |dX/dx^2|, |dX/dphi| by central differences (4th order)."""
    def F(a, b, p):
        return _forward_np(geom, n, rmin, rmax, r0, vt, a, b, p)

    phi = np.full_like(x1, 0.7)

    def d(fp, fm, fp2, fm2, step):
        return (8 * (fp - fm) - (fp2 - fm2)) / (12 * step)

    c1 = d(F(x1 + h, x2, phi), F(x1 - h, x2, phi), F(x1 + 2 * h, x2, phi), F(x1 - 2 * h, x2, phi), h)
    c2 = d(F(x1, x2 + h, phi), F(x1, x2 - h, phi), F(x1, x2 + 2 * h, phi), F(x1, x2 - 2 * h, phi), h)
    c3 = d(F(x1, x2, phi + h), F(x1, x2, phi - h), F(x1, x2, phi + 2 * h), F(x1, x2, phi - 2 * h), h)
    return np.stack([np.linalg.norm(c, axis=-1) for c in (c1, c2, c3)], axis=-1)


GRIDS = [  # (geom, n, rmin, rmax, r0, vartheta)
    ("sph", (1024, 512), 1.0, 20.0, 0.0, 0.0),     # the uniform-r spherical workload
    ("qsph", (1024, 512), 1.0, 20.0, 0.0, 0.0),    # log-r, uniform theta
    ("qsph", (2048, 1024), 1.0, 50.0, 0.0, 0.3),   # log-r, theta stretched
    ("qsph", (96, 40), 2.0, 30.0, 0.5, -0.25),     # r0 != 0, stretching toward the equator
]


@pytest.mark.parametrize("geom,n,rmin,rmax,r0,vt", GRIDS)
def test_grid_endpoints(geom, n, rmin, rmax, r0, vt):
    """Sec. 2.4: code coordinate x1 = 0 is r_min and x1 = N1 is r_max;
    x2 = 0 is the axis theta = 0 and x2 = N2 the axis theta = pi."""
    g = O.make_grid(geom, 2, n, (rmin, 0), (rmax, PI), r0=r0, vartheta=vt)
    N1, N2 = n
    for x2 in (0.3 * N2, 0.5 * N2, 0.77 * N2):
        for x1, rr in ((0.0, rmin), (float(N1), rmax)):
            X = O.code_to_cart(g, [x1, x2, 0.0], 1.1)
            assert np.linalg.norm(X) == pytest.approx(rr, rel=1e-14)
    for x1 in (0.0, 0.4 * N1, float(N1)):
        top = O.code_to_cart(g, [x1, 0.0, 0.0], 0.4)
        bot = O.code_to_cart(g, [x1, float(N2), 0.0], 0.4)
        r = np.linalg.norm(top)
        assert np.hypot(top[0], top[1]) <= 1e-15 * r and top[2] > 0       # theta = 0
        assert np.hypot(bot[0], bot[1]) <= 1e-14 * r and bot[2] < 0       # theta = pi
        assert np.linalg.norm(bot) == pytest.approx(r, rel=1e-14)


@pytest.mark.parametrize("geom,n,rmin,rmax,r0,vt", GRIDS)
def test_metric_against_independent_map(geom, n, rmin, rmax, r0, vt):
    """sqrt(h_ii) of the reference equals the column norms of the Jacobian of
    the independently written forward map (this fixes the cell sizes dr,
    dtheta, dR, dT and the endpoints, which the reference's own maps share
    with its metric)."""
    g = O.make_grid(geom, 2, n, (rmin, 0), (rmax, PI), r0=r0, vartheta=vt)
    rng = np.random.default_rng(3)
    x1 = rng.uniform(0.5, n[0] - 0.5, 40)
    x2 = rng.uniform(0.5, n[1] - 0.5, 40)
    ref = _scale_factors_np(geom, n, rmin, rmax, r0, vt, x1, x2)
    for k in range(40):
        h = O.sqrt_h(g, [x1[k], x2[k], 0.0])
        np.testing.assert_allclose(h, ref[k], rtol=1e-8)
        X = O.code_to_cart(g, [x1[k], x2[k], 0.0], 0.7)
        np.testing.assert_allclose(X, _forward_np(geom, n, rmin, rmax, r0, vt, x1[k], x2[k], 0.7),
                                   rtol=1e-13, atol=1e-13 * rmax)


@pytest.mark.parametrize("geom,n,rmin,rmax,r0,vt", GRIDS)
def test_timestep_bruteforce(geom, n, rmin, rmax, r0, vt):
    """Sec. 2.4 CFL paragraph: dt = CFL * min over cell centres of
    (sum_i 1/h_ii)^(-1/2) over the two poloidal directions, evaluated here by
    brute force over every cell centre with the independent scale factors."""
    N1, N2 = n
    g = O.make_grid(geom, 2, n, (rmin, 0), (rmax, PI), r0=r0, vartheta=vt)
    i, j = np.meshgrid(np.arange(N1) + 0.5, np.arange(N2) + 0.5, indexing="ij")
    h = _scale_factors_np(geom, n, rmin, rmax, r0, vt, i.ravel(), j.ravel())
    dxmin = np.min((1.0 / h[:, 0] ** 2 + 1.0 / h[:, 1] ** 2) ** -0.5)
    assert O.dt_from_cfl(g, 0.45) == pytest.approx(0.45 * dxmin, rel=1e-9)


def test_timestep_cartesian_bruteforce():
    """Sec. 2.4: anisotropic 3D Cartesian cells, (sum 1/dx_i^2)^(-1/2)."""
    g = O.make_grid("cart", 3, (8, 5, 4), (0, -1, 2), (4.0, 4.0, 10.0))
    d = np.array([4.0 / 8, 5.0 / 5, 8.0 / 4])
    assert O.dt_from_cfl(g, 0.3) == pytest.approx(0.3 * np.sum(1 / d ** 2) ** -0.5, rel=1e-15)


# ----------------------------------------------------------------------------- move edge branches
def test_offset_rounding_to_one_goes_to_next_cell():
    """Sec. 3.1 (cell index + offset in [0,1)) and reading 8: a step that
    lands a hair below a cell face, so that y - floor(y) rounds to 1, gives
    the upper cell with offset 0 (never an offset equal to 1)."""
    g = O.make_grid("cart", 2, (8, 8), (0, 0), (8.0, 8.0))
    eps = 2.0 ** -60
    cell = np.array([[3, 5, 0], [0, 2, 0]], np.int32)
    offs = np.array([[3 * eps, 0.5, 0.0], [3 * eps, 0.25, 0.0]])
    # dt = 1, cell size 1, gamma = 1 to the last bit: the x step is u_x itself
    u = np.array([[-4 * eps, 0.0, 0.0], [-4 * eps, 0.0, 0.0]])
    assert np.sqrt(1 + u[0, 0] ** 2) == 1.0
    r = O.move(g, 1.0, cell, offs, None, u)
    # y = -eps: floor(y) = -1 and y - floor(y) = 1 - eps rounds to 1
    np.testing.assert_array_equal(r["cell"][:, 0], [3, 0])
    np.testing.assert_array_equal(r["offs"][:, 0], [0.0, 0.0])
    np.testing.assert_array_equal(r["m"][:, 0], [0, 0])
    assert np.all(r["offs"] < 1.0)
    # the deposit of that step carries exactly the (tiny) displacement
    sp = [dict(q=1.0, m=1.0, cell=cell, offs=offs, u=u, w=np.ones(2), phi=None,
               alive=np.ones(2, np.int32))]
    EB = np.zeros((6,) + O.padded_shape(g))
    out, J = O.run(g, 1.0, 1, EB, sp)
    np.testing.assert_array_equal(out[0]["cell"][:, 0], [3, 0])
    assert np.sum(J[0]) == pytest.approx(-2 * 3 * eps, rel=1e-12)


def _u_for_displacement(D, dt):
    """Four-velocity whose step dt u / gamma is the Cartesian displacement D."""
    v = np.asarray(D) / dt
    return v / np.sqrt(1.0 - np.sum(v * v, axis=-1, keepdims=True))


@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.0), ("qsph", 0.3)])
def test_theta_clamp_at_the_axes(geom, vt):
    """Reading 19 (Sec. 2.4 maps, theta in [0, pi]): a particle carried exactly
    onto the axis theta = 0 ends in cell 0 with an offset >= 0 (offset 0 if
    rounding took it below the axis); one carried onto theta = pi ends in cell
    N2 - 1 with the largest offset below 1 when x2 reaches N2; particles
    crossing the axis stay in [0, N2) and agree with the literal composition
    of the maps."""
    N1, N2 = 64, 32
    g = O.make_grid(geom, 2, (N1, N2), (1.0, 0), (20.0, PI), vartheta=vt)
    dt = O.dt_from_cfl(g, 0.45)
    rng = np.random.default_rng(21)
    P = 400
    for pole in (0, 1):
        cell = np.zeros((P, 3), np.int32)
        # next to r_min, within a third of a cell of the axis: the time step
        # (set by the smallest cell, r_min dtheta) reaches the axis from there
        cell[:, 0] = 0
        cell[:, 1] = 0 if pole == 0 else N2 - 1
        offs = np.zeros((P, 3))
        offs[:, 0] = rng.uniform(0.0, 0.1, P)
        offs[:, 1] = rng.uniform(0.02, 0.3, P) if pole == 0 else rng.uniform(0.7, 0.98, P)
        phi = rng.uniform(0, 2 * PI, P)
        X = np.array([O.code_to_cart(g, cell[k] + offs[k], phi[k]) for k in range(P)])
        rho = np.hypot(X[:, 0], X[:, 1])
        # exactly onto the axis (cylindrical radius to 0), some beyond it
        frac = np.where(np.arange(P) < P // 2, 1.0, rng.uniform(1.0, 1.3, P))
        D = np.zeros((P, 3))
        D[:, 0] = -frac * X[:, 0]
        D[:, 1] = -frac * X[:, 1]
        ok = np.linalg.norm(D, axis=1) < 0.9 * dt  # |v| < 1 at this dt
        cell, offs, phi, D = cell[ok], offs[ok], phi[ok], D[ok]
        assert ok.sum() > 50, "too few steps short enough for this grid"
        u = _u_for_displacement(D, dt)
        r = O.move(g, dt, cell, offs, phi, u)
        assert np.all((r["cell"][:, 1] >= 0) & (r["cell"][:, 1] < N2))
        assert np.all((r["offs"][:, 1] >= 0) & (r["offs"][:, 1] < 1))
        xl, _ = O.move_literal(g, dt, cell, offs, phi, u)
        lit = np.clip(xl[:, 1], 0.0, N2 - 2.0 ** -40)
        got = r["cell"][:, 1] + r["offs"][:, 1]
        np.testing.assert_allclose(got, lit, atol=1e-9)
        onto = slice(0, int(np.sum(np.arange(P)[ok] < P // 2)))
        if pole == 0:
            assert np.all(r["cell"][onto, 1] == 0)
            assert np.all(r["offs"][onto, 1] <= 1e-12)
            # rounding puts about half of them at or below the axis: offset 0
            assert np.sum(r["offs"][onto, 1] == 0.0) > 10
        else:
            assert np.all(r["cell"][onto, 1] == N2 - 1)
            assert np.all(r["offs"][onto, 1] >= 1 - 1e-12)
            # those whose x2 reached N2 get the largest offset below 1
            assert np.sum(r["offs"][onto, 1] == np.nextafter(1.0, 0.0)) > 10


# ----------------------------------------------------------------------------- curvilinear adjoint
@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.3)])
def test_curvilinear_adjoint_central_differences(geom, vt):
    """The reverse sweep on (quasi-)spherical grids against central finite
    differences of the plain FP64 forward map (no dual numbers) along random
    directions of the fields and the initial four-velocities."""
    N1, N2, P, K = 16, 12, 40, 3
    g = O.make_grid(geom, 2, (N1, N2), (1.0, 0), (6.0, PI), vartheta=vt)
    rng = np.random.default_rng(23)
    cell = np.zeros((P, 3), np.int32)
    cell[:, 0] = rng.integers(3, N1 - 3, P)
    cell[:, 1] = rng.integers(0, N2, P)
    cell[:8, 1] = rng.integers(0, 2, 8)           # next to theta = 0
    cell[8:16, 1] = N2 - 1 - rng.integers(0, 2, 8)  # next to theta = pi
    offs = np.concatenate([rng.random((P, 2)), np.zeros((P, 1))], 1)
    phi = rng.uniform(0, 2 * PI, P)
    u = rng.normal(size=(P, 3))
    w = rng.uniform(0.5, 1.5, P)
    EB = rng.normal(size=(6,) + O.padded_shape(g)) * 0.2
    dt = O.dt_from_cfl(g, 0.45)
    species = [dict(q=-1.0, m=1.0, cell=cell, offs=offs, u=u, w=w, phi=phi,
                    alive=np.ones(P, np.int32)),
               dict(q=1.0, m=3.0, cell=cell.copy(), offs=offs.copy(), u=-u, w=w, phi=phi.copy(),
                    alive=np.ones(P, np.int32))]
    lamJ = rng.normal(size=(3,) + O.padded_shape(g))
    lam_u = [rng.normal(size=(P, 3)) for _ in species]
    res = O.adjoint(g, dt, K, EB, species, lamJ, lam_u=lam_u)

    def loss(EBx, sps):
        out, J = O.run(g, dt, K, EBx, sps)
        return np.sum(lamJ * J) + sum(np.sum(lu * s["u"]) for lu, s in zip(lam_u, out))

    assert loss(EB, species) == pytest.approx(res["loss"], rel=1e-12)
    for _ in range(3):
        vEB = rng.normal(size=EB.shape)
        vu = [rng.normal(size=(P, 3)) for _ in species]
        h = 1e-6
        sp_p = [dict(s, u=s["u"] + h * v) for s, v in zip(species, vu)]
        sp_m = [dict(s, u=s["u"] - h * v) for s, v in zip(species, vu)]
        fd = (loss(EB + h * vEB, sp_p) - loss(EB - h * vEB, sp_m)) / (2 * h)
        ip = np.sum(res["dEB"] * vEB) + sum(np.sum(a * b) for a, b in zip(res["du0"], vu))
        assert ip == pytest.approx(fd, rel=1e-6, abs=1e-8)
