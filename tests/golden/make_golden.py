"""Writes oracle_regression.json: a few outputs of the FP64 reference on tiny
seeded cases, so that later edits of the reference show up as test failures.
Calls only oracle/ (and the input generators)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2511_17710_amd import workloads as W  # noqa: E402


def cases():
    yield "cart2d_8", W.cart2d(n=8, ppc=2, steps=3, seed=101), 3
    yield "cart3d_4", W.cart3d(n=4, ppc=2, steps=2, nwaves=4, seed=102), 2
    yield "qsph_16x8", W.curvilinear("qsph", 16, 8, 20.0, 0.3, ppc=2, theta=0.5,
                                     density_power=0, steps=3, seed=103), 3
    yield "sph_16x8", W.curvilinear("sph", 16, 8, 20.0, 0.0, ppc=2, theta=0.5,
                                    density_power=2, steps=3, seed=104), 3


def compute():
    out = {}
    for name, wl, steps in cases():
        g = O.make_grid(wl.geom, wl.dim, wl.n, wl.lo, wl.hi, r0=wl.r0, vartheta=wl.vartheta,
                        periodic=wl.periodic, rho0=wl.rho0)
        EB = O.fields_from_tetrad(g, wl.fields_tetrad, wl.fields_includes_ghosts)
        dt = O.dt_from_cfl(g, wl.cfl)
        sp, J = O.run(g, dt, steps, EB, wl.species, sort_every=2)
        out[name] = dict(
            dt=dt,
            J_sum=[float(np.sum(J[c])) for c in range(3)],
            J_l2=float(np.linalg.norm(J)),
            u0=[float(v) for v in sp[0]["u"][0]],
            offs0=[float(v) for v in sp[0]["offs"][0]],
            cell0=[int(v) for v in sp[0]["cell"][0]],
            perm_head=[int(v) for v in sp[1]["perm"][:8]],
        )
    return out


if __name__ == "__main__":
    data = compute()
    data["_source"] = "written by tests/golden/make_golden.py from the FP64 reference"
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("wrote", len(data) - 1, "cases")
