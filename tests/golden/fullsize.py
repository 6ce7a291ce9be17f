"""The oracle's stored results for the two full-size workloads, and how a run is compared
with them (test infrastructure: read by the GPU tests and by bench.py's parity leg).

The stored files are written by ``make_fullsize_goldens.py`` in this folder, which calls
only the FP64 oracle.  Each holds the density and the forced velocity u = (j + F/2)/rho on
a regular grid of sample nodes and along one full row and one full column, the far-field
vapor and liquid densities (``regions``), the largest |u| and the mass.
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = {
    "static_droplet_512": "static_droplet_512x512_50k.json",
    "drop_impact_2048": "drop_impact_2048x1024_2k.json",
}


def path(name: str) -> str:
    return os.path.join(HERE, FILES[name])


def load(name: str) -> dict:
    with open(path(name)) as fh:
        return json.load(fh)


def regions(name: str, rho: np.ndarray, rho_v_maxwell: float) -> tuple[float, float]:
    """Measured (rho_v, rho_l) of a density field of workload `name`.

    Static droplet: vapor = mean over the four 32 x 32 corner blocks (the nodes farthest from
    the droplet), liquid = mean over the 32 x 32 block at the centre.  Drop impact: vapor = mean
    over the nodes below twice the Maxwell vapor density in the box around the impact, rows
    40..339 and columns 624..1423 (the vapor the splash stirs; the vapor farther up is still the
    initial state at 2,000 steps); liquid = mean over film rows 8..31 in the 256 columns at each end
    of the lattice (away from the impact)."""
    if name == "static_droplet_512":
        c = rho.shape[1] // 2
        corners = np.concatenate([rho[:32, :32].ravel(), rho[:32, -32:].ravel(), rho[-32:, :32].ravel(),
                                  rho[-32:, -32:].ravel()])
        return float(corners.mean()), float(rho[c - 16:c + 16, c - 16:c + 16].mean())
    box = rho[40:340, 624:1424]
    vap = box[box < 2.0 * rho_v_maxwell]
    film = np.concatenate([rho[8:32, :256].ravel(), rho[8:32, -256:].ravel()])
    return float(vap.mean()), float(film.mean())


def compare(name: str, g: dict, rho: np.ndarray, ux: np.ndarray, uy: np.ndarray, mass0: float | None = None) -> dict:
    """Errors of full fields rho, ux, uy [ny][nx] against the stored oracle result g.

    rho_v_rel_err / rho_l_rel_err: the measured far-field densities (``regions``);
    rho_vapor_nodes_max_rel_err / rho_liquid_nodes_max_rel_err: the largest relative density
    error over the stored nodes below / above the mid density (rho_v + rho_l)/2 of Maxwell;
    u_linf: the largest |u - u_oracle| over the stored nodes (either component);
    max_abs_u_rel_err: relative error of the largest |u| over the whole field."""
    sr, su = g["stride_rho"], g["stride_u"]
    mid = 0.5 * (g["rho_v_maxwell"] + g["rho_l_maxwell"])
    ro = np.concatenate([np.asarray(g["rho"]).ravel(), g["rho_row"], g["rho_col"]])
    rg = np.concatenate([rho[::sr, ::sr].ravel(), rho[g["row"]], rho[:, g["col"]]])
    rel = np.abs(rg - ro) / ro
    vap = ro < mid
    uo = np.concatenate([np.asarray(g["ux"]).ravel(), np.asarray(g["uy"]).ravel(), g["ux_row"], g["uy_row"],
                         g["ux_col"], g["uy_col"]])
    ug = np.concatenate([ux[::su, ::su].ravel(), uy[::su, ::su].ravel(), ux[g["row"]], uy[g["row"]],
                         ux[:, g["col"]], uy[:, g["col"]]])
    rv, rl = regions(name, rho, g["rho_v_maxwell"])
    out = {
        "steps": g["steps"],
        "rho_v_rel_err": abs(rv - g["rho_v"]) / g["rho_v"],
        "rho_l_rel_err": abs(rl - g["rho_l"]) / g["rho_l"],
        "rho_vapor_nodes_max_rel_err": float(rel[vap].max()) if vap.any() else 0.0,
        "rho_liquid_nodes_max_rel_err": float(rel[~vap].max()) if (~vap).any() else 0.0,
        "u_linf": float(np.abs(ug - uo).max()),
        "max_abs_u": float(np.sqrt(ux * ux + uy * uy).max()),
        "max_abs_u_oracle": g["max_abs_u"],
        "rho_v": rv, "rho_l": rl, "rho_v_oracle": g["rho_v"], "rho_l_oracle": g["rho_l"],
        "sampled_nodes": int(ro.size),
    }
    out["max_abs_u_rel_err"] = abs(out["max_abs_u"] - g["max_abs_u"]) / g["max_abs_u"]
    if mass0 is not None:
        out["mass_drift"] = abs(float(rho.sum()) - mass0) / mass0
    return out
