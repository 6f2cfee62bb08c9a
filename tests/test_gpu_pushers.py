"""GPU parity of the alternative pushers (Sec. 2.2: Vay 2008; Sec. 5.2: the
guiding-centre hybrid) against the FP64 reference, one step from common
seeded inputs, species pushed differently in one launch.  Bars as for the
Boris step: FP64 cells bit-exact and momenta <= 1e-12; FP32 momenta <= 1e-5,
current <= 1e-5, continuity <= 1e-6.  The hybrid's regime thresholds are
placed in the widest gap of the particles' values near the middle of their
range, so no particle's regime hangs on rounding."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import parity_util as U

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "cart2d_16": lambda: W.cart2d(n=16, ppc=8, theta=0.5, steps=1, seed=91, shuffle=True),
        "cart3d_8": lambda: W.cart3d(n=8, ppc=4, steps=1, nwaves=8, seed=92, shuffle=True),
        "qsph_s_64x32": lambda: W.curvilinear("qsph", 64, 32, 50.0, 0.3, ppc=4, theta=0.5,
                                              density_power=0, steps=1, seed=93, shuffle=True),
    }


def _gap_threshold(v, lo_q=0.3, hi_q=0.7):
    """The midpoint of the widest relative gap between sorted values inside
    the [lo_q, hi_q] quantile range."""
    v = np.sort(v[np.isfinite(v)])
    a, b = int(lo_q * len(v)), int(hi_q * len(v))
    seg = v[a:b + 1]
    rel = (seg[1:] - seg[:-1]) / np.maximum(seg[1:], 1e-300)
    i = int(np.argmax(rel))
    return 0.5 * (seg[i] + seg[i + 1]), float(rel[i])


def _set_pushers(wl, prec, codes):
    """codes: pusher code per species; thresholds of the hybrid from the
    particles' initial fields and momenta."""
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    for sp, code in zip(wl.species, codes):
        sp["pusher"] = code
        if not code & 2:
            continue
        F = O.interp(g, EB, sp["cell"], sp["offs"])
        E, B = O.to_cart(g, sp["cell"], sp["offs"], sp.get("phi"), F)
        k = sp["q"] * dt / (2 * sp["m"] * wl.rho0)
        eb = np.linalg.norm(E, axis=1) / np.linalg.norm(B, axis=1)
        ratio = eb.max() * 1.5 if eb.max() < 0.6 else None
        if ratio:
            e_ovr = min(ratio, 0.95)
        else:
            e_ovr, egap = _gap_threshold(eb, 0.5, 0.9)
            assert egap > 1e-4, egap
        rl = np.linalg.norm(sp["u"], axis=1) * dt / (2 * abs(k) * np.linalg.norm(B, axis=1))
        lmax, gap = _gap_threshold(rl[eb < e_ovr])
        assert gap > 1e-4, gap
        sp["e_ovr"], sp["larmor_max"] = float(e_ovr), float(lmax)
        sp["_gca_count"] = int(np.sum((eb < e_ovr) & (rl < lmax)))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("codes", [(1, 2), (3, 1)], ids=["vay+boris_gca", "vay_gca+vay"])
@pytest.mark.parametrize("name", list(_cases()))
def test_pushers_one_step(name, codes, prec):
    wl = _cases()[name]()
    if prec == "f32":
        W.round_to_f32(wl)
    _set_pushers(wl, prec, codes)
    ngc = [sp.get("_gca_count", 0) for sp in wl.species]
    tol = U.TOL[prec]
    ref, Jref, gpu, Jg, dt, ctx = U.run_both(wl, prec, 1, sort_every=1,
                                             print_case=f"[pushers] {name} {codes} {prec}")
    g, EB = U.oracle_fields(wl, prec)
    ks = U.kick_scale(wl, g, EB, dt)
    for s, (r, q) in enumerate(zip(ref, gpu)):
        perm = r["perm"]
        np.testing.assert_array_equal(q["perm"], perm)
        np.testing.assert_array_equal(q["alive"], r["alive"])
        err_u = U.momentum_error(r, q, wl.species[s]["u"][perm], ks[s][perm])
        same = np.all(q["cell"] == r["cell"], axis=1)
        if prec == "f64":
            assert same.all(), f"{(~same).sum()} cell mismatches"
        else:
            bad = ~same & ~U.near_face(r["offs"][:, :wl.dim], 1e-5)
            assert not bad.any(), f"{bad.sum()} cell mismatches away from faces"
        doff = np.abs(q["offs"] - r["offs"])[same]
        print(f"  species {s} (pusher {codes[s]}, {ngc[s]} guiding centres): u err {err_u:.2e}, "
              f"offsets {doff.max(initial=0):.2e}", flush=True)
        assert err_u <= tol["u"], err_u
        assert doff.max(initial=0) <= tol["offs"], doff.max()
    eJ = U.rel_l2(Jg, Jref)
    cres = U.continuity_of(wl, Jg, gpu, dt)
    print(f"  J relL2={eJ:.3e} continuity={cres:.3e}", flush=True)
    assert eJ <= tol["J"], eJ
    assert cres <= tol["cont"], cres
    assert sum(ngc) > 0


def test_pusher_arguments_and_adjoint_refusal():
    import torch

    from paper_2511_17710_amd import picstep as P
    wl = W.cart2d(n=8, ppc=2, steps=1, seed=95)
    ctx = P.from_workload(wl, prec="f64", sort_every=0)
    with pytest.raises(P.PicError):
        ctx.species_set_pusher(0, "vay", gca=True, e_ovr=1.5, larmor_max=1.0)
    with pytest.raises(P.PicError):
        ctx.species_set_pusher(0, "boris", gca=True, e_ovr=0.5, larmor_max=0.0)
    with pytest.raises(P.PicError):
        ctx.species_set_pusher(5, "vay")
    ctx.species_set_pusher(1, "vay")
    with pytest.raises(P.PicError) as e:
        ctx.forward_checkpointed(ctx.timestep_from_cfl(wl.cfl), 2, 1)
    assert e.value.status == P.PIC_E_UNSUPPORTED
    ctx.species_set_pusher(1, "boris")
    ctx.forward_checkpointed(ctx.timestep_from_cfl(wl.cfl), 2, 1)
    torch.cuda.synchronize()
