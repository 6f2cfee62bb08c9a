"""ctypes front end of the FP64 reference library liboracle.so.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.

Particle state is a dict of numpy arrays:
  cell  int32 (n,3)   per-dimension cell index (unused dims 0)
  offs  float64 (n,3) in-cell offsets in [0,1)
  u     float64 (n,3) four-velocity, global Cartesian basis
  w     float64 (n,)  weight
  phi   float64 (n,)  azimuth (axisymmetric grids) or None
  alive int32 (n,)
Field arrays are padded [6][np3][np2][np1] float64, currents [3][...].
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

GEOM = {"cart": 0, "sph": 1, "qsph": 2}
NG = 2


class OrcGrid(C.Structure):
    _fields_ = [("geom", C.c_int32), ("dim", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("r0", C.c_double),
                ("vartheta", C.c_double), ("periodic", C.c_int32 * 3), ("rho0", C.c_double)]


class OrcSpecies(C.Structure):
    _fields_ = [("n", C.c_int64), ("cell", C.POINTER(C.c_int32)),
                ("offs", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
                ("alive", C.POINTER(C.c_int32)), ("cell_prev", C.POINTER(C.c_int32)),
                ("offs_prev", C.POINTER(C.c_double)), ("perm", C.POINTER(C.c_int32))]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle.build import build_oracle
            build_oracle()
        _LIB = C.CDLL(path)
        _LIB.orc_dt_from_cfl.restype = C.c_double
        _LIB.orc_theta_of_T.restype = C.c_double
        _LIB.orc_T_of_theta.restype = C.c_double
        _LIB.orc_field_points.restype = C.c_int64
        _LIB.orc_polar_area.restype = C.c_double
    return _LIB


def _p(a, ctype):
    if a is None:
        return C.POINTER(ctype)()
    return a.ctypes.data_as(C.POINTER(ctype))


def make_grid(geom, dim, n, lo, hi, r0=0.0, vartheta=0.0, periodic=(1, 1, 1), rho0=1.0):
    g = OrcGrid()
    g.geom = GEOM[geom] if isinstance(geom, str) else int(geom)
    g.dim = int(dim)
    n = list(n) + [1] * (3 - len(n))
    lo = list(lo) + [0.0] * (3 - len(lo))
    hi = list(hi) + [1.0] * (3 - len(hi))
    for d in range(3):
        g.n[d] = int(n[d])
        g.lo[d] = float(lo[d])
        g.hi[d] = float(hi[d])
        g.periodic[d] = int(periodic[d])
    g.r0 = float(r0)
    g.vartheta = float(vartheta)
    g.rho0 = float(rho0)
    return g


def padded_shape(g):
    dims = [g.n[d] + 2 * NG if d < g.dim else 1 for d in range(3)]
    return (dims[2], dims[1], dims[0])


def dt_from_cfl(g, cfl):
    return lib().orc_dt_from_cfl(C.byref(g), C.c_double(cfl))


def sqrt_h(g, x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))
    h = np.zeros(3)
    lib().orc_sqrt_h(C.byref(g), _p(x, C.c_double), _p(h, C.c_double))
    return h


def theta_of_T(g, T):
    return lib().orc_theta_of_T(C.byref(g), C.c_double(T))


def T_of_theta(g, th):
    return lib().orc_T_of_theta(C.byref(g), C.c_double(th))


def code_to_cart(g, x, phi=0.0):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))
    X = np.zeros(3)
    lib().orc_code_to_cart(C.byref(g), _p(x, C.c_double), C.c_double(phi), _p(X, C.c_double))
    return X


def cart_to_code(g, X):
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(3))
    x = np.zeros(3)
    ph = C.c_double(0.0)
    lib().orc_cart_to_code(C.byref(g), _p(X, C.c_double), _p(x, C.c_double), C.byref(ph))
    return x, ph.value


def fields_from_tetrad(g, arr, includes_ghosts):
    arr = np.ascontiguousarray(arr, dtype=np.float64)
    out = np.zeros((6,) + padded_shape(g))
    rc = lib().orc_fields_from_tetrad(C.byref(g), _p(arr, C.c_double), C.c_int32(includes_ghosts),
                                      _p(out, C.c_double))
    assert rc == 0
    return out


def interp(g, EB, cell, offs):
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.float64)
    n = cell.shape[0]
    out = np.zeros((n, 6))
    lib().orc_interp(C.byref(g), _p(EB, C.c_double), C.c_int64(n), _p(cell, C.c_int32),
                     _p(offs, C.c_double), _p(out, C.c_double))
    return out


def to_cart(g, cell, offs, phi, F6):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.float64)
    F6 = np.ascontiguousarray(F6, dtype=np.float64)
    phi = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
    n = cell.shape[0]
    E = np.zeros((n, 3))
    B = np.zeros((n, 3))
    lib().orc_to_cart(C.byref(g), C.c_int64(n), _p(cell, C.c_int32), _p(offs, C.c_double),
                      _p(phi, C.c_double), _p(F6, C.c_double), _p(E, C.c_double),
                      _p(B, C.c_double))
    return E, B


def boris(k, E, B, u):
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(-1, 3)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1, 3)
    u = np.array(u, dtype=np.float64).reshape(-1, 3)
    lib().orc_boris(C.c_int64(u.shape[0]), C.c_double(k), _p(E, C.c_double), _p(B, C.c_double),
                    _p(u, C.c_double))
    return u


def vay(k, E, B, u):
    """Vay (2008) push of u (n,3) with E, B (n,3); returns the new u."""
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(-1, 3)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1, 3)
    out = np.array(u, dtype=np.float64).reshape(-1, 3).copy()
    lib().orc_vay(C.c_int64(out.shape[0]), C.c_double(k), _p(E, C.c_double), _p(B, C.c_double),
                  _p(out, C.c_double))
    return out


def gca(k, E, B, u):
    """Guiding-centre update of u (n,3); returns the new u."""
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(-1, 3)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1, 3)
    out = np.array(u, dtype=np.float64).reshape(-1, 3).copy()
    lib().orc_gca(C.c_int64(out.shape[0]), C.c_double(k), _p(E, C.c_double), _p(B, C.c_double),
                  _p(out, C.c_double))
    return out


def move(g, dt, cell, offs, phi, u):
    cell = np.array(cell, dtype=np.int32)
    offs = np.array(offs, dtype=np.float64)
    phi = None if phi is None else np.array(phi, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = cell.shape[0]
    alive = np.ones(n, dtype=np.int32)
    m3 = np.zeros((n, 3), dtype=np.int32)
    dx3 = np.zeros(n)
    lib().orc_move(C.byref(g), C.c_double(dt), C.c_int64(n), _p(cell, C.c_int32),
                   _p(offs, C.c_double), _p(phi, C.c_double), _p(u, C.c_double),
                   _p(alive, C.c_int32), _p(m3, C.c_int32), _p(dx3, C.c_double))
    return dict(cell=cell, offs=offs, phi=phi, alive=alive, m=m3, dx3=dx3)


def move_literal(g, dt, cell, offs, phi, u):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.float64)
    phi = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = cell.shape[0]
    xn = np.zeros((n, 3))
    pn = np.zeros(n)
    lib().orc_move_literal(C.byref(g), C.c_double(dt), C.c_int64(n), _p(cell, C.c_int32),
                           _p(offs, C.c_double), _p(phi, C.c_double), _p(u, C.c_double),
                           _p(xn, C.c_double), _p(pn, C.c_double))
    return xn, pn


def sort_perm(keys):
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    perm = np.zeros(keys.shape[0], dtype=np.int32)
    lib().orc_sort_perm(C.c_int64(keys.shape[0]), _p(keys, C.c_int32), _p(perm, C.c_int32))
    return perm


def sort_keys(g, cell, alive):
    """The key every sort of run() orders a species by (int32 per particle)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32).reshape(-1, 3)
    alive = np.ascontiguousarray(alive, dtype=np.int32).reshape(-1)
    keys = np.zeros(cell.shape[0], dtype=np.int32)
    rc = lib().orc_sort_keys(C.byref(g), C.c_int64(cell.shape[0]), _p(cell, C.c_int32),
                             _p(alive, C.c_int32), _p(keys, C.c_int32))
    if rc != 0:
        raise RuntimeError(f"orc_sort_keys failed rc={rc}")
    return keys


def faraday(g, EB, f):
    """B -= f curl E / sqrt(h) on a copy of the padded fields (App. A)."""
    out = np.array(EB, dtype=np.float64, copy=True, order="C")
    rc = lib().orc_faraday(C.byref(g), _p(out, C.c_double), C.c_double(f))
    if rc:
        raise RuntimeError("orc_faraday")
    return out


def ampere(g, EB, J, dt, coupling):
    """E += dt curl B / sqrt(h) - coupling dt J / sqrt(h), with the axis rules."""
    out = np.array(EB, dtype=np.float64, copy=True, order="C")
    J = np.ascontiguousarray(J, dtype=np.float64)
    rc = lib().orc_ampere(C.byref(g), _p(out, C.c_double), _p(J, C.c_double), C.c_double(dt),
                          C.c_double(coupling))
    if rc:
        raise RuntimeError("orc_ampere")
    return out


def filter_current(g, J, passes=1):
    out = np.array(J, dtype=np.float64, copy=True, order="C")
    rc = lib().orc_filter(C.byref(g), _p(out, C.c_double), C.c_int32(passes))
    if rc:
        raise RuntimeError("orc_filter")
    return out


def polar_area(g, x1):
    return lib().orc_polar_area(C.byref(g), C.c_double(x1))


def _species_struct(g, st, with_prev=False):
    """Make contiguous FP64 copies of a particle dict and a matching OrcSpecies."""
    n = st["cell"].shape[0]
    s = dict(
        cell=np.array(st["cell"], dtype=np.int32).reshape(n, 3).copy(),
        offs=np.array(st["offs"], dtype=np.float64).reshape(n, 3).copy(),
        u=np.array(st["u"], dtype=np.float64).reshape(n, 3).copy(),
        w=np.array(st["w"], dtype=np.float64).reshape(n).copy(),
        phi=(np.array(st["phi"], dtype=np.float64).reshape(n).copy()
             if (g.geom != 0 and st.get("phi") is not None) else None),
        alive=np.array(st.get("alive", np.ones(n)), dtype=np.int32).reshape(n).copy(),
    )
    if with_prev:
        s["cell_prev"] = np.zeros((n, 3), dtype=np.int32)
        s["offs_prev"] = np.zeros((n, 3))
        s["perm"] = np.arange(n, dtype=np.int32)
    o = OrcSpecies()
    o.n = n
    o.cell = _p(s["cell"], C.c_int32)
    o.offs = _p(s["offs"], C.c_double)
    o.u = _p(s["u"], C.c_double)
    o.w = _p(s["w"], C.c_double)
    o.phi = _p(s["phi"], C.c_double)
    o.alive = _p(s["alive"], C.c_int32)
    o.cell_prev = _p(s.get("cell_prev"), C.c_int32)
    o.offs_prev = _p(s.get("offs_prev"), C.c_double)
    o.perm = _p(s.get("perm"), C.c_int32)
    return s, o


def run(g, dt, nsteps, EB, species, sort_every=0, step0=0):
    """Advance every species nsteps; returns (new species dicts, J of the last step).

    species: list of dicts with keys q, m and the particle arrays.
    """
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    keep, structs = [], []
    for st in species:
        s, o = _species_struct(g, st, with_prev=True)
        keep.append(s)
        structs.append(o)
    arr = (OrcSpecies * len(structs))(*structs)
    q = np.array([s["q"] for s in species], dtype=np.float64)
    m = np.array([s["m"] for s in species], dtype=np.float64)
    J = np.zeros((3,) + padded_shape(g))
    # pusher per species: "pusher" 0 Boris, 1 Vay, +2 guiding-centre hybrid
    # with thresholds "e_ovr" and "larmor_max" (defaults: Boris)
    push = np.array([int(s.get("pusher", 0)) for s in species], dtype=np.int32)
    eov = np.array([float(s.get("e_ovr", 0.9)) for s in species], dtype=np.float64)
    lmax = np.array([float(s.get("larmor_max", 0.0)) for s in species], dtype=np.float64)
    rc = lib().orc_run_pushers(C.byref(g), C.c_double(dt), C.c_int32(nsteps),
                               C.c_int32(sort_every), C.c_int64(step0), _p(EB, C.c_double),
                               C.c_int32(len(structs)), _p(q, C.c_double), _p(m, C.c_double),
                               _p(push, C.c_int32), _p(eov, C.c_double), _p(lmax, C.c_double),
                               arr, _p(J, C.c_double))
    if rc != 0:
        raise RuntimeError(f"orc_run failed rc={rc}")
    out = []
    for st, s in zip(species, keep):
        d = dict(s)
        d["q"], d["m"] = st["q"], st["m"]
        out.append(d)
    return out, J


def _ptr_array(arrs):
    P = C.POINTER(C.c_double)
    return (P * len(arrs))(*[_p(a, C.c_double) for a in arrs])


def adjoint(g, dt, K, EB, species, lamJ, lam_u=None, lam_d=None):
    """Reverse-mode gradient of L = <lamJ, J_final> + sum lam_u.u_K + sum lam_d.delta_K."""
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    lamJ = np.ascontiguousarray(lamJ, dtype=np.float64)
    keep, structs = [], []
    for st in species:
        s, o = _species_struct(g, st)
        keep.append(s)
        structs.append(o)
    arr = (OrcSpecies * len(structs))(*structs)
    q = np.array([s["q"] for s in species], dtype=np.float64)
    m = np.array([s["m"] for s in species], dtype=np.float64)
    ns = len(species)
    lu = [np.ascontiguousarray(a, dtype=np.float64) for a in lam_u] if lam_u else None
    ld = [np.ascontiguousarray(a, dtype=np.float64) for a in lam_d] if lam_d else None
    du0 = [np.zeros((s["cell"].shape[0], 3)) for s in keep]
    dd0 = [np.zeros((s["cell"].shape[0], 3)) for s in keep]
    dEB = np.zeros_like(EB)
    loss = C.c_double(0.0)
    rc = lib().orc_adjoint(C.byref(g), C.c_double(dt), C.c_int32(K), _p(EB, C.c_double),
                           C.c_int32(ns), _p(q, C.c_double), _p(m, C.c_double), arr,
                           _p(lamJ, C.c_double), _ptr_array(lu) if lu else None,
                           _ptr_array(ld) if ld else None, _p(dEB, C.c_double),
                           _ptr_array(du0), _ptr_array(dd0), C.byref(loss))
    if rc != 0:
        raise RuntimeError(f"orc_adjoint failed rc={rc}")
    return dict(loss=loss.value, dEB=dEB, du0=du0, dd0=dd0)


def jvp(g, dt, K, EB, vEB, species, vu0, vd0, lamJ, lam_u=None, lam_d=None):
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    vEB = None if vEB is None else np.ascontiguousarray(vEB, dtype=np.float64)
    lamJ = np.ascontiguousarray(lamJ, dtype=np.float64)
    keep, structs = [], []
    for st in species:
        s, o = _species_struct(g, st)
        keep.append(s)
        structs.append(o)
    arr = (OrcSpecies * len(structs))(*structs)
    q = np.array([s["q"] for s in species], dtype=np.float64)
    m = np.array([s["m"] for s in species], dtype=np.float64)
    vu = [np.ascontiguousarray(a, dtype=np.float64) for a in vu0] if vu0 else None
    vd = [np.ascontiguousarray(a, dtype=np.float64) for a in vd0] if vd0 else None
    lu = [np.ascontiguousarray(a, dtype=np.float64) for a in lam_u] if lam_u else None
    ld = [np.ascontiguousarray(a, dtype=np.float64) for a in lam_d] if lam_d else None
    loss = C.c_double(0.0)
    dloss = C.c_double(0.0)
    rc = lib().orc_jvp(C.byref(g), C.c_double(dt), C.c_int32(K), _p(EB, C.c_double),
                       _p(vEB, C.c_double), C.c_int32(len(species)), _p(q, C.c_double),
                       _p(m, C.c_double), arr, _ptr_array(vu) if vu else None,
                       _ptr_array(vd) if vd else None, _p(lamJ, C.c_double),
                       _ptr_array(lu) if lu else None, _ptr_array(ld) if ld else None,
                       C.byref(loss), C.byref(dloss))
    if rc != 0:
        raise RuntimeError(f"orc_jvp failed rc={rc}")
    return loss.value, dloss.value
