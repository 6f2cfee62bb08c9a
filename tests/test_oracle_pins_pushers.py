"""Pins of the reference's alternative pushers (Sec. 2.2: Vay 2008 beside
Boris 1970; Sec. 5.2: the hybrid with the guiding-centre approximation),
against the defining equations and closed forms, not the reference's own
formulas."""
import numpy as np
import pytest

from oracle import oracle as O

NG = 2


def _rng(seed):
    return np.random.default_rng(seed)


def test_vay_solves_its_implicit_equation():
    """Vay (2008): u_new = u + (q dt/m)(E + (v_old + v_new)/2 x B); in code units
    u_new = u + 2kE + k (v_old + v_new) x B.  The closed-form root must satisfy
    the implicit equation itself."""
    r = _rng(1)
    n = 2000
    u = r.normal(size=(n, 3)) * 3.0
    E = r.normal(size=(n, 3)) * 0.5
    B = r.normal(size=(n, 3)) * 2.0
    k = 0.37
    un = O.vay(k, E, B, u)
    v0 = u / np.sqrt(1 + np.sum(u * u, 1))[:, None]
    v1 = un / np.sqrt(1 + np.sum(un * un, 1))[:, None]
    res = un - u - 2 * k * E - k * np.cross(v0 + v1, B)
    assert np.max(np.abs(res)) <= 1e-13 * np.max(np.abs(un))


def test_vay_pure_E_kick():
    r = _rng(2)
    u = r.normal(size=(100, 3))
    E = r.normal(size=(100, 3))
    k = 0.2
    np.testing.assert_allclose(O.vay(k, E, np.zeros_like(E), u), u + 2 * k * E, rtol=0,
                               atol=1e-15)


def test_vay_pure_B_rotation_closed_form():
    """E = 0: |u| is kept and u turns about B by 2 atan(k|B|/gamma) (the
    implicit midpoint rotation), clockwise for k > 0."""
    r = _rng(3)
    u = r.normal(size=(200, 3)) * 2
    B = r.normal(size=(200, 3))
    k = 0.3
    un = O.vay(k, np.zeros_like(B), B, u)
    np.testing.assert_allclose(np.linalg.norm(un, axis=1), np.linalg.norm(u, axis=1), rtol=1e-14)
    g = np.sqrt(1 + np.sum(u * u, 1))
    bn = np.linalg.norm(B, axis=1)
    b = B / bn[:, None]
    ang = -2 * np.arctan(k * bn / g)
    par = np.sum(u * b, 1)[:, None] * b
    perp = u - par
    rot = par + perp * np.cos(ang)[:, None] + np.cross(b, perp) * np.sin(ang)[:, None]
    np.testing.assert_allclose(un, rot, rtol=0, atol=1e-13)


def test_vay_keeps_relativistic_ExB_drift_exactly_boris_does_not():
    """A particle moving at the E x B drift (E perpendicular to B, |E| < |B|)
    feels no force; Vay's pusher keeps it there to round-off over many steps,
    Boris's does not (its known relativistic E x B defect)."""
    B = np.array([[0.0, 0.0, 1.0]])
    E = np.array([[0.0, 0.6, 0.0]])
    vd = np.cross(E, B) / 1.0  # E x B / B^2
    gd = 1 / np.sqrt(1 - np.sum(vd * vd))
    ud = gd * vd
    k = 0.4
    uv, ub = ud.copy(), ud.copy()
    for _ in range(1000):
        uv = O.vay(k, E, B, uv)
        ub = O.boris(k, E, B, ub)
    assert np.max(np.abs(uv - ud)) <= 1e-13 * np.max(np.abs(ud))
    assert np.max(np.abs(ub - ud)) > 1e-6 * np.max(np.abs(ud))


def test_gca_drifts_at_ExB_with_parallel_kick():
    """Guiding-centre update: the velocity perpendicular to B is exactly
    E x B / B^2, the parallel four-velocity gains 2k E.b, and the Lorentz
    factor is that of the resulting velocity."""
    r = _rng(4)
    n = 500
    B = r.normal(size=(n, 3))
    bn = np.linalg.norm(B, axis=1)
    b = B / bn[:, None]
    # fields with |E_perp| < |B|
    Ep = np.cross(b, r.normal(size=(n, 3)))
    Ep *= (0.8 * bn * r.random(n) / np.maximum(np.linalg.norm(Ep, axis=1), 1e-12))[:, None]
    E = Ep + b * r.normal(size=(n, 1)) * 0.3
    u = r.normal(size=(n, 3)) * 2
    k = 0.25
    un = O.gca(k, E, B, u)
    gn = np.sqrt(1 + np.sum(un * un, 1))
    v = un / gn[:, None]
    vE = np.cross(E, B) / (bn * bn)[:, None]
    vpar = np.sum(v * b, 1)
    np.testing.assert_allclose(v - vpar[:, None] * b, vE, rtol=0, atol=1e-14)
    upar = np.sum(u * b, 1) + 2 * k * np.sum(E * b, 1)
    np.testing.assert_allclose(np.sum(un * b, 1), upar, rtol=1e-13, atol=1e-14)


def _uniform_fields(g, E, B):
    """Contravariant fields of a uniform Cartesian E, B on a periodic grid
    with unit cells (F^i = F_hat^i / Delta_i)."""
    EB = np.zeros((6,) + O.padded_shape(g))
    for c in range(3):
        EB[c] = E[c]
        EB[3 + c] = B[c]
    return EB


def test_gca_particle_moves_with_its_guiding_centre():
    """Full pipeline, 2D Cartesian with unit cells: a particle in the
    guiding-centre regime in uniform E perpendicular to B advances its
    in-plane position by dt * E x B / B^2 every step (offsets exact)."""
    n = (16, 16, 1)
    g = O.make_grid("cart", 2, n, (0, 0, 0), n)
    E, B = np.array([0.0, 0.3, 0.0]), np.array([0.0, 0.0, 1.0])
    EB = _uniform_fields(g, E, B)
    dt = O.dt_from_cfl(g, 0.45)
    sp = [dict(q=-1.0, m=1.0, cell=np.array([[5, 7, 0]], np.int32),
               offs=np.array([[0.25, 0.5, 0.0]]), u=np.array([[0.3, -0.2, 0.1]]),
               w=np.ones(1), phi=None, alive=np.ones(1, np.int32), pusher=2, e_ovr=0.9,
               larmor_max=10.0)]
    out, _ = O.run(g, dt, 8, EB, sp)
    vE = np.cross(E, B)
    x0 = np.array([5.25, 7.5])
    x8 = out[0]["cell"][0, :2] + out[0]["offs"][0, :2]
    # the in-plane motion is the drift from the first step on; the parallel
    # four-velocity (0.1 along z) is kept, E.b = 0
    np.testing.assert_allclose(x8 - x0, 8 * dt * vE[:2], rtol=0, atol=1e-13)
    gam = np.sqrt((1 + 0.1 ** 2) / (1 - vE @ vE))
    np.testing.assert_allclose(out[0]["u"][0], gam * vE + np.array([0, 0, 0.1]), rtol=1e-14)


@pytest.mark.parametrize("vay", [0, 1])
def test_hybrid_regime_switch(vay):
    """Outside the guiding-centre regime (gyroradius above the critical one,
    or |E| >= e_ovr |B|) the hybrid runs the conventional pusher unchanged."""
    n = (12, 10, 1)
    g = O.make_grid("cart", 2, n, (0, 0, 0), n)
    r = _rng(5)
    EB = np.zeros((6,) + O.padded_shape(g))
    EB[:3] = r.uniform(-0.1, 0.1, size=EB[:3].shape)
    EB[5] = 1.0
    dt = O.dt_from_cfl(g, 0.45)
    P = 300
    base = dict(q=1.0, m=1.0, cell=np.stack([r.integers(0, 12, P), r.integers(0, 10, P),
                                              np.zeros(P, int)], 1).astype(np.int32),
                offs=np.concatenate([r.random((P, 2)), np.zeros((P, 1))], 1),
                u=r.normal(size=(P, 3)), w=np.ones(P), phi=None, alive=np.ones(P, np.int32))
    plain, _ = O.run(g, dt, 3, EB, [dict(base, pusher=vay)])
    # critical gyroradius far below every particle's: never guiding centre
    tiny, _ = O.run(g, dt, 3, EB, [dict(base, pusher=vay + 2, larmor_max=1e-9)])
    np.testing.assert_array_equal(tiny[0]["u"], plain[0]["u"])
    # |E| < e_ovr |B| never holds: never guiding centre
    strict, _ = O.run(g, dt, 3, EB, [dict(base, pusher=vay + 2, e_ovr=0.0, larmor_max=1e9)])
    np.testing.assert_array_equal(strict[0]["u"], plain[0]["u"])
    # every particle in the guiding-centre regime: u perpendicular to B
    # is the drift alone
    gc, _ = O.run(g, dt, 1, EB, [dict(base, pusher=vay + 2, larmor_max=1e9)])
    assert not np.array_equal(gc[0]["u"], plain[0]["u"])
