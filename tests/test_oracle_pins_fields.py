"""Pins of the reference field solver (App. A: discretized Faraday and
Ampere laws; Sec. 2.6: the polar axis; Sec. 2.5: the current filter) against
discrete identities and closed forms that do not reuse its formulas:
- div(sqrt(h) B) is unchanged by Faraday's law (a discrete divergence of a
  discrete curl vanishes identically);
- Gauss's law: Ampere's law changes div(sqrt(h) E) by coupling times the
  charge change of a charge-conserving deposit (nodes away from the axis and
  the radial edges);
- vacuum: every Fourier mode of E on a periodic Cartesian grid follows the
  Yee recurrence E^{n+1} + E^{n-1} = (2 - 4 dt^2 sum_d sin^2(k_d D_d/2)/D_d^2) E^n;
- the polar area A(x1) of the integrated axis update equals a quadrature of
  sqrt(h) over the half cell next to the axis;
- the filter: the binomial kernel of a unit impulse, constants and sums kept
  on periodic grids, and the axis mirror conditions.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import checks

NG = 2
STAG = checks.STAG


def _grid(geom, dim, n, vt=0.0, cell=1.0):
    if geom == "cart":
        return O.make_grid("cart", dim, n, (0, 0, 0), tuple(cell * x for x in n))
    return O.make_grid(geom, 2, n, (1.0, 0, 0), (6.0, np.pi, 1), vartheta=vt)


def _sqrt_h_at(g, x1, x2):
    """(sqrt h11, sqrt h22, sqrt h33) at arrays of code coordinates."""
    out = np.zeros(x1.shape + (3,))
    for idx in np.ndindex(x1.shape):
        out[idx] = O.sqrt_h(g, (x1[idx], x2[idx], 0.0))
    return out


def _coords(g, c):
    """Code coordinates of every element of component c of a padded array."""
    shp = O.padded_shape(g)
    k, j, i = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
    x1 = i - NG + STAG[c][0]
    x2 = j - NG + STAG[c][1]
    return x1.astype(float), x2.astype(float)


def _random_fields(g, rng):
    EB = rng.normal(size=(6,) + O.padded_shape(g))
    if g.geom == 0:
        # periodic ghosts consistent with the active region
        act = EB.copy()
        for c in range(6):
            act[c] = _wrap(g, EB[c])
        EB = act
    else:
        EB[2, :, [NG, NG + g.n[1]], :] = 0.0  # E3 on the axis
        EB[4, :, [NG, NG + g.n[1]], :] = 0.0  # B2 on the axis
    return EB


def _wrap(g, A):
    """Fill the periodic ghosts of one padded component from its active region."""
    out = A.copy()
    dims = [g.n[d] if d < g.dim else 1 for d in range(3)]
    for ax, d in ((2, 0), (1, 1), (0, 2)):
        if d >= g.dim:
            continue
        idx = (np.arange(out.shape[ax]) - NG) % dims[d] + NG
        out = np.take(out, idx, axis=ax)
    return out


def _div_sqrt_h(g, F, comps):
    """sum_a Delta_a (sqrt(h) F^a) at cell centres (B-like, comps at the
    cell faces) or nodes (E-like); returns a padded-shaped array (valid where
    the neighbours exist)."""
    out = np.zeros(O.padded_shape(g))
    for a, c in enumerate(comps):
        if a >= g.dim:
            continue
        x1, x2 = _coords(g, c)
        h = _sqrt_h_at(g, x1, x2)
        w = h[..., 0] * h[..., 1] * h[..., 2] * F[c - comps[0]]
        ax = 2 - a
        sh = np.zeros_like(w)
        if STAG[c][a] == 0.0:  # face values at integer points: cell centre i+1/2 uses i+1 - i
            sl_a = [slice(None)] * 3
            sl_b = [slice(None)] * 3
            sl_a[ax] = slice(0, -1)
            sl_b[ax] = slice(1, None)
            sh[tuple(sl_a)] = w[tuple(sl_b)] - w[tuple(sl_a)]
        else:  # half-integer values: node i uses (i+1/2) - (i-1/2)
            sl_a = [slice(None)] * 3
            sl_b = [slice(None)] * 3
            sl_a[ax] = slice(1, None)
            sl_b[ax] = slice(0, -1)
            sh[tuple(sl_a)] = w[tuple(sl_a)] - w[tuple(sl_b)]
        out += sh
    return out


@pytest.mark.parametrize("geom,dim,n,vt", [("cart", 2, (9, 7, 1), 0.0), ("cart", 3, (6, 5, 4), 0.0),
                                           ("sph", 2, (10, 8, 1), 0.0),
                                           ("qsph", 2, (10, 8, 1), 0.3)])
def test_faraday_keeps_div_B(geom, dim, n, vt):
    rng = np.random.default_rng(1)
    g = _grid(geom, dim, n, vt, cell=1.3)
    EB = _random_fields(g, rng)
    new = O.faraday(g, EB, 0.37)
    assert not np.allclose(new[3:], EB[3:])
    d0 = _div_sqrt_h(g, EB[3:], (3, 4, 5))
    d1 = _div_sqrt_h(g, new[3:], (3, 4, 5))
    # cells whose faces the solver updated
    sl = [slice(None)] * 3
    for d in range(dim):
        sl[2 - d] = slice(NG, NG + n[d])
    diff = (d1 - d0)[tuple(sl)]
    assert np.max(np.abs(diff)) <= 1e-12 * np.max(np.abs(d0[tuple(sl)])), np.max(np.abs(diff))


@pytest.mark.parametrize("geom,dim,n,vt", [("cart", 2, (8, 7, 1), 0.0), ("cart", 3, (5, 5, 4), 0.0),
                                           ("sph", 2, (12, 10, 1), 0.0),
                                           ("qsph", 2, (12, 10, 1), 0.3)])
def test_ampere_keeps_gauss_law_with_the_deposit(geom, dim, n, vt):
    """Ampere's law with the current of a particle step changes
    div(sqrt(h) E) by coupling times the change of the deposited charge."""
    rng = np.random.default_rng(2)
    g = _grid(geom, dim, n, vt)
    EB = _random_fields(g, rng) * 0.2
    dt = O.dt_from_cfl(g, 0.45)
    P = 400
    cell = np.stack([rng.integers(2 if geom != "cart" else 0, n[d] - (2 if geom != "cart" else 0), P)
                     if d < dim else np.zeros(P, int) for d in range(3)], 1).astype(np.int32)
    offs = np.concatenate([rng.random((P, dim)), np.zeros((P, 3 - dim))], 1)
    sp = [dict(q=-1.0, m=1.0, cell=cell, offs=offs, u=rng.normal(size=(P, 3)),
               w=rng.uniform(0.5, 2, P), phi=rng.uniform(0, 2 * np.pi, P) if geom != "cart" else None,
               alive=np.ones(P, np.int32))]
    out, J = O.run(g, dt, 1, EB, sp)
    s = out[0]
    coupling = 4 * np.pi
    new = O.ampere(g, EB, J, dt, coupling)
    d0 = _div_sqrt_h(g, EB[:3], (0, 1, 2))
    d1 = _div_sqrt_h(g, new[:3], (0, 1, 2))
    qw = s["q"] * s["w"]
    drho = checks.drho_nodes(n, dim, geom == "cart", (s["cell_prev"], s["offs_prev"]),
                             (s["cell"], s["offs"]), qw).astype(float)
    sl = [slice(None)] * 3
    for d in range(dim):
        if geom == "cart":
            sl[2 - d] = slice(NG, NG + n[d])
        else:  # interior nodes: away from the axis and the radial edges
            sl[2 - d] = slice(NG + 1, NG + n[d])
    lhs = (d1 - d0)[tuple(sl)]
    rhs = coupling * drho[tuple(sl)]
    assert np.max(np.abs(rhs)) > 0
    assert np.max(np.abs(lhs - rhs)) <= 1e-11 * np.max(np.abs(rhs)), np.max(np.abs(lhs - rhs))


@pytest.mark.parametrize("dim,n,kvec,cell", [(2, (16, 12, 1), (3, 2, 0), 1.0),
                                             (3, (8, 10, 6), (1, 2, 1), 0.7)])
def test_vacuum_modes_follow_the_yee_recurrence(dim, n, kvec, cell):
    g = _grid("cart", dim, n, cell=cell)
    dt = O.dt_from_cfl(g, 0.45)
    # one Fourier mode in every E component, B = 0; the leap-frog loop of the
    # paper with no particles: Faraday dt/2 twice, Ampere dt
    k = [2 * np.pi * kvec[d] / n[d] for d in range(3)]  # per code cell
    EB = np.zeros((6,) + O.padded_shape(g))
    amp = [1.0, -0.4, 0.7]
    for c in range(3):
        x1, x2 = _coords(g, c)
        x3 = np.zeros_like(x1)
        if dim == 3:
            shp = O.padded_shape(g)
            x3 = (np.arange(shp[0])[:, None, None] - NG + STAG[c][2]) * np.ones_like(x1)
        EB[c] = amp[c] * np.cos(k[0] * x1 + k[1] * x2 + k[2] * x3 + 0.3)
    J = np.zeros((3,) + O.padded_shape(g))
    series = []
    probe = (0, 0, NG + 3, NG + 2) if dim == 2 else (0, NG + 1, NG + 3, NG + 2)
    for _ in range(12):
        series.append(EB[probe])
        EB = O.faraday(g, EB, dt / 2)
        EB = O.faraday(g, EB, dt / 2)
        EB = O.ampere(g, EB, J, dt, 4 * np.pi)
    a = np.array(series)
    s2 = sum((np.sin(k[d] / 2) / cell) ** 2 for d in range(dim))
    c2 = 2 - 4 * dt * dt * s2
    # the recurrence holds for the transverse part; a longitudinal part stays
    # constant (curl of a gradient vanishes), which the recurrence does not
    # move either only if it is absent: remove it by the two-step difference
    lhs = a[2:] + a[:-2] - c2 * a[1:-1]
    # the longitudinal (curl-free) part is static: it adds (2 - c2) * E_L
    EL = lhs[0] / (2 - c2) if abs(2 - c2) > 0 else 0.0
    np.testing.assert_allclose(lhs, (2 - c2) * EL, rtol=0, atol=1e-12)


def test_vacuum_transverse_mode_2d_exact():
    """2D, E3 only (purely transverse): the recurrence holds with nothing static."""
    n = (20, 16, 1)
    g = _grid("cart", 2, n)
    dt = O.dt_from_cfl(g, 0.45)
    k = (2 * np.pi * 3 / n[0], 2 * np.pi * 5 / n[1])
    EB = np.zeros((6,) + O.padded_shape(g))
    x1, x2 = _coords(g, 2)
    EB[2] = np.sin(k[0] * x1 + k[1] * x2)
    J = np.zeros((3,) + O.padded_shape(g))
    vals = []
    for _ in range(30):
        vals.append(EB[2, 0, NG + 4, NG + 7])
        EB = O.faraday(g, EB, dt)
        EB = O.ampere(g, EB, J, dt, 4 * np.pi)
    a = np.array(vals)
    c2 = 2 - 4 * dt * dt * (np.sin(k[0] / 2) ** 2 + np.sin(k[1] / 2) ** 2)
    np.testing.assert_allclose(a[2:] + a[:-2], c2 * a[1:-1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.0), ("qsph", 0.3), ("qsph", -0.4)])
def test_polar_area_is_the_half_cell_integral(geom, vt):
    g = _grid(geom, 2, (16, 12, 1), vt)
    xs, ws = np.polynomial.legendre.leggauss(40)
    for x1 in (0.5, 3.5, 15.5):
        # integral over x2 in [0, 1/2] of sqrt(h11) sqrt(h22) sqrt(h33)
        pts = 0.25 * (xs + 1.0)
        vals = [np.prod(O.sqrt_h(g, (x1, x2, 0.0))) for x2 in pts]
        quad = 0.25 * np.dot(ws, vals)
        assert O.polar_area(g, x1) == pytest.approx(quad, rel=1e-12)


def test_filter_impulse_response_and_sums():
    g = _grid("cart", 3, (7, 6, 5))
    J = np.zeros((3,) + O.padded_shape(g))
    J[1, NG + 2, NG + 3, NG + 4] = 1.0
    out = O.filter_current(g, J, 1)
    w1 = np.array([0.25, 0.5, 0.25])
    kern = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    np.testing.assert_allclose(out[1, NG + 1:NG + 4, NG + 2:NG + 5, NG + 3:NG + 6], kern,
                               rtol=0, atol=1e-16)
    assert np.sum(np.abs(out[1])) == pytest.approx(1.0)
    rng = np.random.default_rng(3)
    J = rng.normal(size=(3,) + O.padded_shape(g))
    act = (slice(None), slice(NG, NG + 5), slice(NG, NG + 6), slice(NG, NG + 7))
    out = O.filter_current(g, J, 3)
    np.testing.assert_allclose(out[act].sum(axis=(1, 2, 3)), J[act].sum(axis=(1, 2, 3)), rtol=1e-12)
    const = np.full_like(J, 2.5)
    np.testing.assert_allclose(O.filter_current(g, const, 2)[act], 2.5, rtol=1e-15)


@pytest.mark.parametrize("geom", ["sph", "qsph"])
def test_filter_axis_mirrors(geom):
    """Near theta = 0 and pi the filter acts on the array extended by the
    mirror conditions: J1 even about the axis node, J2 odd about it, J3 zero
    on it; built here explicitly and filtered with the plain kernel."""
    n1, n2 = 9, 8
    g = _grid(geom, 2, (n1, n2, 1), 0.2 if geom == "qsph" else 0.0)
    rng = np.random.default_rng(4)
    J = rng.normal(size=(3,) + O.padded_shape(g))
    out = O.filter_current(g, J, 1)
    w = np.array([0.25, 0.5, 0.25])
    K = np.outer(w, w)  # [dj, di]
    for c in range(3):
        A = J[c, 0]  # [j, i] padded
        for i in range(1, n1 - 1):
            for jn in (0, 1, n2 - 1, n2) if c != 1 else (0, n2 - 1):
                acc = 0.0
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        jj = jn + dj
                        if c == 0:
                            jj = -jj if jj < 0 else (2 * n2 - jj if jj > n2 else jj)
                            v = A[jj + NG, i + di + NG]
                        elif c == 1:
                            if jj < 0:
                                v = -A[-1 - jj + NG, i + di + NG]
                            elif jj >= n2:
                                v = -A[2 * n2 - 1 - jj + NG, i + di + NG]
                            else:
                                v = A[jj + NG, i + di + NG]
                        else:
                            v = 0.0 if jj in (0, n2) else A[(-jj if jj < 0 else (2 * n2 - jj if jj > n2 else jj)) + NG, i + di + NG]
                        acc += K[dj + 1, di + 1] * v
                if c == 2 and jn in (0, n2):
                    acc = 0.0
                assert out[c, 0, jn + NG, i + NG] == pytest.approx(acc, rel=1e-13, abs=1e-15), (c, jn, i)


@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.3), ("cart", 0.0)])
def test_discrete_gradients_are_static(geom, vt):
    """A field whose covariant components are the discrete gradient of a
    scalar has no discrete curl: E_i = -Delta_i Phi (Phi on the nodes) leaves
    B unchanged under Faraday's law, B_i = Delta_i psi (psi at the cell
    centres) leaves E unchanged under Ampere's law without current.  The
    covariant components are formed here with h_ii at each component's own
    Yee point, which pins where the solver evaluates the metric."""
    n = (10, 8, 1)
    g = _grid(geom, 2, n, vt, cell=1.3)
    rng = np.random.default_rng(5)
    shp = O.padded_shape(g)
    Phi = rng.normal(size=shp)
    psi = rng.normal(size=shp)
    if geom == "cart":  # periodic scalars
        Phi, psi = _wrap(g, Phi), _wrap(g, psi)
    EB = np.zeros((6,) + shp)
    # E_1 at (i+1/2, j) = -(Phi(i+1, j) - Phi(i, j)); E_2 at (i, j+1/2) likewise
    cE = [np.zeros(shp), np.zeros(shp)]
    cE[0][:, :, :-1] = -(Phi[:, :, 1:] - Phi[:, :, :-1])
    cE[1][:, :-1, :] = -(Phi[:, 1:, :] - Phi[:, :-1, :])
    # B_1 at (i, j+1/2) = psi(i+1/2, j+1/2) - psi(i-1/2, j+1/2); B_2 at (i+1/2, j)
    cB = [np.zeros(shp), np.zeros(shp)]
    cB[0][:, :, 1:] = psi[:, :, 1:] - psi[:, :, :-1]
    cB[1][:, 1:, :] = psi[:, 1:, :] - psi[:, :-1, :]
    for a, c in ((0, 0), (1, 1)):
        x1, x2 = _coords(g, c)
        with np.errstate(divide="ignore", invalid="ignore"):
            EB[c] = cE[a] / _sqrt_h_at(g, x1, x2)[..., a] ** 2
    for a, c in ((0, 3), (1, 4)):
        x1, x2 = _coords(g, c)
        with np.errstate(divide="ignore", invalid="ignore"):
            EB[c] = cB[a] / _sqrt_h_at(g, x1, x2)[..., a] ** 2
    EB[~np.isfinite(EB)] = 0.0  # ghost points at r = 0 (no stencil here reaches them)
    if geom != "cart":
        EB[4, :, [NG, NG + n[1]], :] = 0.0  # B2 on the axis
    else:
        EB = np.stack([_wrap(g, EB[c]) for c in range(6)])
    newB = O.faraday(g, EB, 0.3)
    sl = (slice(None), slice(NG, NG + n[1]), slice(NG, NG + n[0]))
    np.testing.assert_allclose(newB[5][sl], EB[5][sl], rtol=0, atol=1e-12 * np.abs(EB[3:]).max())
    J = np.zeros((3,) + shp)
    newE = O.ampere(g, EB, J, 0.3, 4 * np.pi)
    # E3 at (i, j): Delta_i B_2 - Delta_j B_1 = 0 away from the axis nodes
    sl3 = (slice(None), slice(NG + (1 if geom != "cart" else 0), NG + n[1]), slice(NG + 1, NG + n[0]))
    np.testing.assert_allclose(newE[2][sl3], EB[2][sl3], rtol=0, atol=1e-12 * np.abs(EB[:3]).max())


@pytest.mark.parametrize("geom,vt", [("sph", 0.0), ("qsph", 0.3)])
def test_axis_line_current_is_static(geom, vt):
    """The field of a current along the polar axis: B_3 (= r sin(theta)
    B_phi_hat) the same at every half node in theta, and the axial current
    2 B_3 / coupling in the radial conformal current of both axis nodes
    (outward at theta = 0, inward at theta = pi) -- the half-cell share of
    the current that the bulk update balances against a jump of B_3 -- keep
    E constant, the integrated axis update included."""
    n = (10, 8, 1)
    g = _grid(geom, 2, n, vt)
    shp = O.padded_shape(g)
    EB = np.zeros((6,) + shp)
    K = 0.7
    x1, x2 = _coords(g, 5)
    EB[5] = K / _sqrt_h_at(g, x1, x2)[..., 2] ** 2  # B^3 with B_3 = K
    J = np.zeros((3,) + shp)
    coupling = 4 * np.pi
    J[0, 0, NG, :] = 2 * K / coupling
    J[0, 0, NG + n[1], :] = -2 * K / coupling
    new = O.ampere(g, EB, J, 0.2, coupling)
    act = (slice(None), slice(NG, NG + n[1] + 1), slice(NG, NG + n[0]))
    np.testing.assert_allclose(new[0][act], 0.0, atol=1e-13)
