"""Write the oracle's results for the two full-size workloads (test infrastructure).

Calls only the FP64 oracle (its OpenMP build, which gives the same bits as the
single-threaded one) and the input generators:

  static_droplet_512x512_50k.json   the 512 x 512 static droplet (shaped Peng-Robinson,
                                    Tr = 0.5, R = 80) after 50,000 steps
  drop_impact_2048x1024_2k.json     the 2048 x 1024 droplet impact on a film between walls
                                    (shaped Peng-Robinson, Tr = 0.47) after its first 2,000 steps

Each file holds the density and forced velocity on a regular grid of sample nodes and
along one full row and one full column, the far-field vapor and liquid densities
(``fullsize.regions``), the largest |u| and the FP64 mass.  Usage:

    python tests/golden/make_fullsize_goldens.py [static|impact|all]

(about 20 minutes for the droplet and 6 for the impact on 8 cores).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from fullsize import FILES, regions  # noqa: E402
from lbm_inputs import (DROP_IMPACT_2048, STATIC_DROPLET_512, drop_impact_fields, drop_impact_tau,  # noqa: E402
                        static_droplet_fields)

STATIC_FILE = os.path.join(HERE, FILES["static_droplet_512"])
IMPACT_FILE = os.path.join(HERE, FILES["drop_impact_2048"])


def _grid(a: np.ndarray, stride: int) -> list:
    return [[float("%.17g" % v) for v in row] for row in a[::stride, ::stride]]


def _line(a) -> list:
    return [float("%.17g" % v) for v in a]


def _summary(m: dict, stride_rho: int, stride_u: int, row: int, col: int) -> dict:
    rho, ux, uy = m["rho"], m["ux"], m["uy"]
    return {
        "stride_rho": stride_rho, "stride_u": stride_u,
        "rho": _grid(rho, stride_rho), "ux": _grid(ux, stride_u), "uy": _grid(uy, stride_u),
        "row": row, "rho_row": _line(rho[row]), "ux_row": _line(ux[row]), "uy_row": _line(uy[row]),
        "col": col, "rho_col": _line(rho[:, col]), "ux_col": _line(ux[:, col]), "uy_col": _line(uy[:, col]),
        "max_abs_u": float(np.sqrt(ux * ux + uy * uy).max()),
        "mass": float(rho.sum()),
    }


def static_droplet() -> dict:
    r = STATIC_DROPLET_512
    eo, so = O.eos_build(O.make_eos(**r["eos"]))
    rho0 = static_droplet_fields(r, eo.rho_v, eo.rho_l)
    L = O.Lattice(O.make_params(r["nx"], r["ny"], eo, sigma=so, tau=r["tau"]), omp=True)
    L.init_eq(rho0)
    mass0 = float(rho0.sum())
    t0 = time.perf_counter()
    L.run(r["steps"])
    dt = time.perf_counter() - t0
    m = L.macros()
    rv, rl = regions("static_droplet_512", m["rho"], eo.rho_v)
    c = r["nx"] // 2
    out = {
        "_source": "written by tests/golden/make_fullsize_goldens.py: FP64 oracle (OpenMP build, %d threads, "
                   "%.0f s) on lbm_inputs.STATIC_DROPLET_512" % (L.threads, dt),
        "recipe": r, "steps": r["steps"], "rho_v_maxwell": eo.rho_v, "rho_l_maxwell": eo.rho_l,
        "mass0": mass0, "rho_v": rv, "rho_l": rl,
    }
    out.update(_summary(m, 8, 16, c, c))
    return out


def drop_impact() -> dict:
    r = DROP_IMPACT_2048
    eo, so = O.eos_build(O.make_eos(**r["eos"]))
    rho0, ux0, uy0 = drop_impact_fields(r, eo.rho_v, eo.rho_l)
    P = O.make_params(r["nx"], r["ny"], eo, sigma=so, tau=drop_impact_tau(r), walls=True,
                      rho_wall_lo=eo.rho_l, rho_wall_hi=eo.rho_v)
    L = O.Lattice(P, omp=True)
    L.init_eq(rho0, ux0, uy0)
    mass0 = float(rho0.sum())
    t0 = time.perf_counter()
    L.run(r["parity_steps"])
    dt = time.perf_counter() - t0
    m = L.macros()
    rv, rl = regions("drop_impact_2048", m["rho"], eo.rho_v)
    out = {
        "_source": "written by tests/golden/make_fullsize_goldens.py: FP64 oracle (OpenMP build, %d threads, "
                   "%.0f s) on lbm_inputs.DROP_IMPACT_2048" % (L.threads, dt),
        "recipe": r, "steps": r["parity_steps"], "rho_v_maxwell": eo.rho_v, "rho_l_maxwell": eo.rho_l,
        "mass0": mass0, "rho_v": rv, "rho_l": rl,
    }
    out.update(_summary(m, 16, 32, 20, r["nx"] // 2))
    return out


def main(which: str) -> None:
    if which in ("impact", "all"):
        res = drop_impact()
        with open(IMPACT_FILE, "w") as fh:
            json.dump(res, fh)
        print("wrote", IMPACT_FILE, res["_source"], flush=True)
    if which in ("static", "all"):
        res = static_droplet()
        with open(STATIC_FILE, "w") as fh:
            json.dump(res, fh)
        print("wrote", STATIC_FILE, res["_source"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
