"""Throughput of the fused shaped-EOS pseudopotential D2Q9 step on one MI355X.

Headline workload: droplet impact on a liquid film between walls (Sec. IV.B), 2048 x 1024,
droplet R = 100 at V = 0.072 onto a film of height 40 = 0.2 D, Re = 300 (tau_l = 0.644),
shaped Peng-Robinson EOS (a = 2/49, b = 2/21, omega = 0.344) at Tr = 0.47 (density ratio
3.07e4) with the Smooth loop (alpha = 0.3), raised vapor slope (k_vap = 4), EOS scale 0.25,
Li forcing with sigma from eps; FP32-shifted storage (rho_ref = rho_v) with FP64
mass/momentum reductions.  One "step" is one time step of the whole hot path.  Inputs are
resident in HBM before the timed region starts.  The same workload in FP64, and the
512 x 512 static droplet in both precisions, are secondary legs.

The roofline figure times the step kernel alone, with HIP events on the stream it is
launched on.  achieved = algorithmic bytes per launch (80 B per cell update in FP32-shifted,
144 B in FP64, times the cell updates one launch makes) / average launch time;
measured_GB/s = the HBM bytes per launch that the committed PMC summary (profiles/) gives
for that kernel and workload, over the same launch time.

Further legs (in the same JSON line): per-case parity of both full-size workloads against
the FP64 oracle's stored results, an HBM sweep of larger lattices, the batched planar sweep,
the finite-difference reference solver, the adjoint of the droplet loss (cost against the
forward, agreement with central differences), a plain device-copy calibration and the FP64
CPU oracle on a bounded sample of the headline workload (one thread and all cores).

Prints ONE JSON line (rank 0).  --gpus N with N > 1 exits: the library runs the hot path on one GPU.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS + HBM GB/s (%roofline), FP32-shifted vs FP64 D2Q9; adjoint/fwd time"
# algorithmic bytes per cell update: 8 moving populations read + written, rest population FP64 read + written
BYTES = {"fp32": 8 * 4 * 2 + 8 * 2, "fp64": 9 * 8 * 2}
STREAM_BYTES = 64 << 20  # the library streams its stores when both population buffers take at most this
LEGS = ("c3", "c2", "parity", "sweep", "aa", "batched", "fd", "adjoint", "cpu")


def _prec_name(prec_id, lbm):
    return "fp32" if prec_id == lbm.FP32_SHIFTED else "fp64"


# two-step tile height per precision (lbm_params.tile_rows) of the benchmark's lattices: -1 = the
# fastest of the library's candidates, timed when a lattice is created (--tile-rows sets others)
TILE_ROWS = {"fp32": -1, "fp64": -1}


def _tile_rows(lbm, prec, tile_rows):
    return TILE_ROWS[_prec_name(prec, lbm)] if tile_rows is None else tile_rows


def kernel_name(lbm, P, shape=None):
    """Name of the step kernel (as rocprofv3 prints it) that advances lattice P, and its steps per launch.
    shape: (tile rows, wavefronts) of the two-step tile a lattice runs (Lattice.tile_shape()); by default
    the one lbm_describe reports for P."""
    var, rows, waves = lbm.describe(P)
    if shape is not None and var == lbm.VARIANT_BLOCK2:
        rows, waves = shape
    t = "float" if P.prec == lbm.FP32_SHIFTED else "double"
    if var == lbm.VARIANT_MARCH:
        return "k_step<%s, 0>" % t, 1
    if var == lbm.VARIANT_BLOCK:
        return "k_step_blk<%s, 0>" % t, 1
    if var == lbm.VARIANT_AA:
        return "k_aa_step<%s, false, 0>" % t, 1  # with k_aa_psi, and the odd-step instances
    nt = 2 * lbm.layout(P)[1] <= STREAM_BYTES
    # one row per wavefront: tiles of waves - 6 rows; two: up to 2 waves - 6
    kern = "k_step2_rows2" if rows > waves - 6 else "k_step2_blk"
    return "%s<%s, 0, %s, %s>" % (kern, t, "true" if P.walls else "false", "true" if nt else "false"), 2


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def tiles_of(lbm, L):
    """'58xH tiles' of a two-step lattice, else ''."""
    if lbm.describe(L.P)[0] != lbm.VARIANT_BLOCK2:
        return ""
    return "58x%d tiles" % L.tile_shape()[0]


def drop_impact_lattice(lbm, prec, reduce_every, variant=0, tile_rows=None):
    """The headline workload (lbm_inputs.DROP_IMPACT_2048); tile_rows None: TILE_ROWS."""
    from lbm_inputs import DROP_IMPACT_2048 as R, drop_impact_fields, drop_impact_tau

    e, s = lbm.eos_build(lbm.make_eos(**R["eos"]))
    rho, ux, uy = drop_impact_fields(R, e.rho_v, e.rho_l)
    P = lbm.make_params(R["nx"], R["ny"], e, sigma=s, tau=drop_impact_tau(R), prec=prec, walls=True,
                        rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v, reduce_every=reduce_every, kernel_variant=variant,
                        tile_rows=_tile_rows(lbm, prec, tile_rows))
    return lbm.Lattice(P, rho, ux, uy, device="cuda:0"), e


def drop_impact_name(e=None):
    from lbm_inputs import DROP_IMPACT_2048 as R

    ratio = "" if e is None else " (density ratio %.3g)" % (e.rho_l / e.rho_v)
    return ("droplet impact on a film between walls %dx%d, R=%d, film %d, V=%g, Re=300, shaped PR Tr=0.47%s "
            "(Smooth alpha=0.3, k_vap=4, scale 0.25), Li forcing" % (R["nx"], R["ny"], R["R"], R["h"], R["V"], ratio))


def droplet_lattice(lbm, n, prec, reduce_every, R=None, variant=0, tile_rows=None):
    """Static droplet on an n x n periodic lattice (the 512 x 512 workload, or the roofline sweep with R = n/6)."""
    from lbm_inputs import STATIC_DROPLET_512 as S, droplet_density

    e, s = lbm.eos_build(lbm.make_eos(**S["eos"]))
    R = n // 6 if R is None else R
    rho0 = droplet_density(n, n, e.rho_v, e.rho_l, R=R, W=S["W"])
    P = lbm.make_params(n, n, e, sigma=s, tau=S["tau"], prec=prec, reduce_every=reduce_every, kernel_variant=variant,
                        tile_rows=_tile_rows(lbm, prec, tile_rows))
    return lbm.Lattice(P, rho0, device="cuda:0"), e


def droplet_name(n, R):
    return ("static droplet %dx%d periodic, R=%d, shaped PR Tr=0.5 (Smooth alpha=0.3, k_vap=4, scale 0.25), "
            "MRT tau_nu=0.7, Li forcing" % (n, n, R))


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------
def time_steps(L, steps, warmup):
    """Seconds for `steps` steps after `warmup` untimed ones, by HIP events on the lattice's stream."""
    import torch

    L.step(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(L.stream)
    L.step(steps)
    ev1.record(L.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


def reduce_schedule(steps, warmup, every=100):
    """Reduction interval for a timed window [warmup, warmup + steps): `every`, shortened to the
    window length when the window is shorter, so that the window always holds a reducing step; and
    the number of reducing steps (t % interval == 0) inside it."""
    re = max(1, min(every, steps))
    n = (warmup + steps - 1) // re - (warmup - 1) // re if warmup > 0 else (steps - 1) // re + 1
    return re, n


def traffic_rows():
    """Machine-readable PMC rows of every committed summary: {(kernel, workload, prec): (bytes, sha256)}."""
    rows = {}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if line.startswith("| traffic |"):
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                # | traffic | kernel | workload | prec | bytes/launch | sources sha256 |
                if len(cells) >= 6:
                    rows[(cells[1], cells[2], cells[3])] = (float(cells[4]), cells[5])
    return rows


def sources_digest() -> str:
    """SHA-256 over the sources of the step kernels (a PMC summary is valid only for these)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("lbm_device.h", "lbm_step.hip"):
        with open(os.path.join(ROOT, "paper_2107_06355_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, prec):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC summaries, or None when
    there is none or the kernel sources changed since the counters were taken."""
    row = traffic_rows().get((kernel, workload, prec))
    if row is None or row[1] != sources_digest():
        return None
    return row[0]


def workload_leg(lbm, make, prec, steps, warmup, kernel_steps):
    """One workload in one precision: the whole hot path over the timed window (reductions
    included), then the step kernel alone over `kernel_steps` steps for the roofline."""
    import torch

    re, nred = reduce_schedule(steps, warmup)
    L, e = make(prec, re)
    sec, wall = time_steps(L, steps, warmup)
    L.check()
    hist = L.history()
    mass = hist[:, 1]
    cells = L.nx * L.ny
    tiles = tiles_of(lbm, L)
    shape = L.tile_shape() if tiles else None
    L.close()
    del L
    # the step kernel alone, in the tile shape the window ran
    L, e = make(prec, 0, shape[0] if shape else 0)
    kname, spl = kernel_name(lbm, L.P, shape)
    ksteps = max(spl, kernel_steps - kernel_steps % spl)
    ksec, _ = time_steps(L, ksteps, 20)
    L.check()
    L.close()
    del L
    torch.cuda.empty_cache()
    pn = _prec_name(prec, lbm)
    launch_us = ksec * 1e6 / (ksteps // spl)
    alg = BYTES[pn] * cells * spl  # algorithmic bytes of one launch
    out = {"MLUPS": cells * steps / sec / 1e6, "ms_per_step": sec * 1e3 / steps, "wall_s": wall,
           "reduce_every": re, "reductions_in_window": nred,
           "mass_drift_over_run": float(abs(mass / mass[0] - 1).max()) if len(mass) else None,
           "kernel": kname, "tiles": tiles, "steps_per_launch": spl,
           "kernel_steps_timed": ksteps,
           "avg_launch_us": launch_us, "kernel_us_per_step": launch_us / spl,
           "algorithmic_bytes_per_launch": alg, "kernel_GB/s": alg / launch_us / 1e3,
           "frac_hbm_peak": alg / launch_us / 1e3 / HBM_PEAK_GBS}
    return out


def roofline(r, workload, prec, calib):
    t = measured_traffic(r["kernel"], workload + (", " + r["tiles"] if r.get("tiles") else ""), prec)
    out = {"bound": "hbm", "achieved": r["kernel_GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": r["kernel_GB/s"] / HBM_PEAK_GBS, "traffic": t,
           "kernel": r["kernel"], "tiles": r.get("tiles", ""), "bytes_per_cell_update": BYTES[prec],
           "cell_updates_per_launch": r["algorithmic_bytes_per_launch"] // BYTES[prec],
           "steps_per_launch": r["steps_per_launch"], "avg_launch_us": r["avg_launch_us"],
           "basis": "achieved = %d B per cell update x cell updates per launch / avg launch time (one-step "
                    "equivalent: a two-step launch moves the populations through HBM once for two updates)"
                    % BYTES[prec],
           "copy_ceiling_frac": r["kernel_GB/s"] / calib["GB/s"]}
    if t is not None:
        out["measured_GB/s"] = t / r["avg_launch_us"] / 1e3
        out["measured_frac"] = out["measured_GB/s"] / HBM_PEAK_GBS
        out["traffic_over_algorithmic"] = t / r["algorithmic_bytes_per_launch"]
    return out


def copy_bandwidth(nbytes=1 << 31, reps=20):
    """Read+write bandwidth of a plain device copy (torch's copy kernel) of `nbytes`."""
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * nbytes, "GB/s": 2 * nbytes / sec / 1e9, "us": sec * 1e6}


# ---------------------------------------------------------------------------
# per-case parity against the oracle's stored results
# ---------------------------------------------------------------------------
def parity_leg(lbm):
    """Both full-size workloads from their initial state to the oracle's stored step count, in both
    precisions, compared with the FP64 oracle's stored fields (tests/golden/)."""
    import numpy as np
    import torch

    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import fullsize

    out = {"targets": {"rho_v_rel_err": 1e-3, "rho_l_rel_err": 1e-5, "u_linf": 1e-5, "mass_drift": 1e-10,
                       "applies_to": "fp32"}}
    cases = (("static_droplet_512", lambda prec: droplet_lattice(lbm, 512, prec, 100, R=80)),
             ("drop_impact_2048", lambda prec: drop_impact_lattice(lbm, prec, 100)))
    for name, make in cases:
        if not os.path.exists(fullsize.path(name)):
            out[name] = None
            continue
        g = fullsize.load(name)
        res = {"workload": droplet_name(512, 80) if name == "static_droplet_512" else drop_impact_name(),
               "steps": g["steps"]}
        for prec in (lbm.FP32_SHIFTED, lbm.FP64):
            L, e = make(prec)
            L.step(g["steps"])
            L.check()
            m = L.macros()
            rho, ux, uy = (m[k].cpu().numpy() for k in ("rho", "ux", "uy"))
            h = L.history()
            r = fullsize.compare(name, g, rho, ux, uy, mass0=g["mass0"])
            r["mass_drift_history"] = float(np.abs(h[:, 1] / h[0, 1] - 1).max())
            res[_prec_name(prec, lbm)] = r
            L.close()
            del L
            torch.cuda.empty_cache()
        out[name] = res
        f = res["fp32"]
        print("# parity %s fp32 vs oracle after %d steps: rho_v %.1e rho_l %.1e u_linf %.1e (vapor nodes %.1e); "
              "fp64 rho %.1e u %.1e" % (name, g["steps"], f["rho_v_rel_err"], f["rho_l_rel_err"], f["u_linf"],
                                        f["rho_vapor_nodes_max_rel_err"],
                                        max(res["fp64"]["rho_vapor_nodes_max_rel_err"],
                                            res["fp64"]["rho_liquid_nodes_max_rel_err"]), res["fp64"]["u_linf"]),
              file=sys.stderr, flush=True)
    return out


# ---------------------------------------------------------------------------
# CPU baseline
# ---------------------------------------------------------------------------
def cpu_baseline(steps_one, steps_all):
    """The FP64 oracle on a bounded sample of the headline workload: `steps_one` time steps single-threaded
    and `steps_all` with the oracle's OpenMP build on every core this process may use."""
    import oracle as O
    from lbm_inputs import DROP_IMPACT_2048 as R, drop_impact_fields, drop_impact_tau

    eo, so = O.eos_build(O.make_eos(**R["eos"]))
    rho, ux, uy = drop_impact_fields(R, eo.rho_v, eo.rho_l)
    P = O.make_params(R["nx"], R["ny"], eo, sigma=so, tau=drop_impact_tau(R), walls=True, rho_wall_lo=eo.rho_l,
                      rho_wall_hi=eo.rho_v)
    cells = R["nx"] * R["ny"]
    legs = {}
    for omp, steps in ((False, steps_one), (True, steps_all)):
        L = O.Lattice(P, omp=omp)
        L.init_eq(rho, ux, uy)
        t0 = time.perf_counter()
        L.run(steps)
        dt = time.perf_counter() - t0
        legs[omp] = {"value": cells * steps / dt / 1e6, "unit": "MLUPS", "cores": L.threads, "kind": "oracle",
                     "sample": "%s, first %d time steps (FP64, %s, %.1f s)" % (
                         drop_impact_name(), steps, "%d threads (OpenMP build)" % L.threads if omp else "single thread",
                         dt)}
        del L
    out = dict(legs[True])
    out["host"] = _host_cpu()
    out["single_thread"] = legs[False]
    print("# cpu baseline (oracle): %.2f MLUPS on %d threads, %.2f MLUPS on one" % (
        out["value"], out["cores"], legs[False]["value"]), file=sys.stderr, flush=True)
    return out


def _host_cpu() -> str:
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return "%s, %d CPUs available" % (model, len(os.sched_getaffinity(0)))


# ---------------------------------------------------------------------------
# secondary legs
# ---------------------------------------------------------------------------
def sweep_leg(lbm, sides, steps, only=""):
    out = []
    for side in sides:
        for prec in (lbm.FP32_SHIFTED, lbm.FP64):
            pn = _prec_name(prec, lbm)
            if only and pn != only:
                continue
            L, e = droplet_lattice(lbm, side, prec, 0)
            tiles = tiles_of(lbm, L)
            kname, spl = kernel_name(lbm, L.P, L.tile_shape() if tiles else None)
            n = max(spl, steps - steps % spl)
            sec, _ = time_steps(L, n, 20)
            L.check()
            cells = side * side
            gbs = BYTES[pn] * cells * n / sec / 1e9
            launch_us = sec * 1e6 / (n // spl)
            row = {"n": side, "prec": pn, "kernel": kname, "tiles": tiles, "MLUPS": cells * n / sec / 1e6, "GB/s": gbs,
                   "frac_hbm_peak": gbs / HBM_PEAK_GBS, "us_per_step": sec * 1e6 / n, "avg_launch_us": launch_us,
                   "steps_per_launch": spl}
            t = measured_traffic(kname, "droplet %dx%d" % (side, side) + (", " + tiles if tiles else ""), pn)
            if t is not None:
                row["measured_GB/s"] = t / launch_us / 1e3
                row["measured_frac"] = row["measured_GB/s"] / HBM_PEAK_GBS
            out.append(row)
            print("# sweep %s %dx%d: %.0f MLUPS, %.0f GB/s algorithmic (%.1f%%), %.2f us per launch (%s, %s)" % (
                pn, side, side, row["MLUPS"], gbs, 100 * gbs / HBM_PEAK_GBS, launch_us, kname, tiles),
                file=sys.stderr, flush=True)
            L.close()
            del L
            import torch

            torch.cuda.empty_cache()
    return out


def adjoint_leg(lbm, n=512, R=80, W0=20.0, steps=4000, K=200, fd_check=True):
    """Adjoint of the static-droplet loss (far-field vapor density + interface width): cost against the
    plain forward, and, in FP64, agreement with central differences of the same forward (h = 1e-6)."""
    import torch
    from lbm_inputs import STATIC_DROPLET_512 as S, droplet_density
    from paper_2107_06355_amd.rollout import vapor_width_loss

    e, s = lbm.eos_build(lbm.make_eos(**S["eos"]))
    rho0 = droplet_density(n, n, e.rho_v, e.rho_l, R=R, W=W0)

    def loss_grad(rho):
        r = rho.detach().clone().requires_grad_(True)
        L = vapor_width_loss(r, e.rho_v, R, W0)
        L.backward()
        return float(L.detach()), r.grad

    def run(prec, mode=None, ee=e, G=-1.0, sig=s):
        P = lbm.make_params(n, n, ee, G=G, sigma=sig, tau=S["tau"], prec=prec, reduce_every=0)
        lat = lbm.Lattice(P, rho0, device="cuda:0")
        if mode in ("checkpoint", "checkpoint_one_stream"):
            # two record segments: the next segment's recomputation overlaps the current one's
            # transposed steps on a second stream; one segment: both on the lattice's stream
            lat.enable_checkpointing(K, steps, overlap=mode == "checkpoint")
        elif mode == "record":
            lat.enable_recording(steps)
        return lat

    out = {"workload": "static droplet %dx%d R=%d W0=%g, shaped PR Tr=0.5, %d steps; the forward checkpoints every "
                       "%d steps and the adjoint recomputes each segment (the specified mode; the next segment's "
                       "recomputation overlaps the current one's transposed steps on a second stream, or runs on "
                       "the lattice's stream: checkpoint_one_stream), or the forward records every step"
                       % (n, n, R, W0, steps, K)}
    for prec, name in ((lbm.FP32_SHIFTED, "fp32"), (lbm.FP64, "fp64")):
        plain = run(prec)
        plain.step(50)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(plain.stream)
        plain.step(steps)
        ev[1].record(plain.stream)
        plain.check()
        plain.close()
        torch.cuda.synchronize()
        t_fwd = ev[0].elapsed_time(ev[1])
        res = {"forward_ms": t_fwd}
        for mode in ("checkpoint", "checkpoint_one_stream", "record"):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            lat = run(prec, mode)
            ev[0].record(lat.stream)
            lat.step(steps)
            ev[1].record(lat.stream)
            lat.check()
            L0, g = loss_grad(lat.macros()["rho"])
            ev[2].record(lat.stream)
            grads = lat.adjoint(g)
            ev[3].record(lat.stream)
            torch.cuda.synchronize()
            t_f, t_adj = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
            res[mode] = {"forward_ms": t_f, "adjoint_ms": t_adj, "adjoint_over_forward": t_adj / t_fwd,
                         # what gradients cost on top of a plain forward, in plain forwards
                         "extra_over_forward": (t_f - t_fwd + t_adj) / t_fwd, "grad": grads}
            res["loss"] = L0
            print("# adjoint %s (%s): forward %.1f ms (plain %.1f), adjoint %.1f ms -> %.2fx the plain forward, "
                  "%.2fx extra in all" % (name, mode, t_f, t_fwd, t_adj, t_adj / t_fwd,
                                          res[mode]["extra_over_forward"]), file=sys.stderr, flush=True)
            lat.close()
            del lat
            torch.cuda.empty_cache()
        # the specified mode (checkpoint every K steps) is the headline; the recorded one is a variant
        res["grad"] = res["checkpoint"]["grad"]
        res["adjoint_over_forward"] = res["checkpoint"]["adjoint_over_forward"]
        res["adjoint_over_forward_recorded"] = res["record"]["adjoint_over_forward"]
        res["record_vs_checkpoint_max_rel_diff"] = max(
            abs(res["record"]["grad"][k] - res["checkpoint"]["grad"][k]) / max(abs(res["checkpoint"]["grad"][k]), 1e-300)
            for k in res["record"]["grad"])
        out[name] = res
    out["adjoint_over_forward_checkpointed"] = {k: out[k]["adjoint_over_forward"] for k in ("fp32", "fp64")}
    out["adjoint_over_forward_recorded"] = {k: out[k]["adjoint_over_forward_recorded"] for k in ("fp32", "fp64")}
    if fd_check:
        base = [e.rho_max, e.p_max, e.rho_min, e.p_min]

        def L_of(knots=None, G=-1.0, sig=s):
            ee = lbm.eos_set_knots(e, *knots) if knots is not None else e
            lat = run(lbm.FP64, None, ee, G, sig)
            lat.step(steps)
            lat.check()
            val = loss_grad(lat.macros()["rho"])[0]
            lat.close()
            return val

        fd = {}
        for j, nm in enumerate(("rho_max", "p_max", "rho_min", "p_min")):
            h = 1e-6 * abs(base[j])
            kp, km = list(base), list(base)
            kp[j] += h
            km[j] -= h
            fd[nm] = (L_of(kp) - L_of(km)) / (2 * h)
        fd["G"] = (L_of(G=-1.0 + 1e-6) - L_of(G=-1.0 - 1e-6)) / 2e-6
        fd["sigma"] = (L_of(sig=s * (1 + 1e-6)) - L_of(sig=s * (1 - 1e-6))) / (2e-6 * s)
        out["fd_fp64"] = fd
        for name in ("fp64", "fp32"):
            g = out[name]["grad"]
            out["rel_err_%s_vs_fd" % name] = {k: abs(g[k] - fd[k]) / max(abs(fd[k]), 1e-300) for k in fd}
        print("# adjoint vs FD (fp64, checkpointed): max rel err %.2e" % max(out["rel_err_fp64_vs_fd"].values()),
              file=sys.stderr, flush=True)
    return out


def aa_leg(lbm, steps=1000, big_steps=20):
    """The in-place AA variant (one population buffer, two launches per step) on the drop-impact
    lattice and on the 8192^2 droplet: time per step, the one-step-equivalent algorithmic rate,
    and the device memory of populations + workspace against the two-buffer default."""
    import torch

    out = []
    for wl, make, n in (("drop impact 2048x1024", lambda prec: drop_impact_lattice(lbm, prec, 0, variant=lbm.VARIANT_AA),
                         steps),
                        ("droplet 8192x8192", lambda prec: droplet_lattice(lbm, 8192, prec, 0, variant=lbm.VARIANT_AA),
                         big_steps)):
        for prec in (lbm.FP32_SHIFTED, lbm.FP64):
            pn = _prec_name(prec, lbm)
            L, e = make(prec)
            sec, _ = time_steps(L, n, 10)
            L.check()
            cells = L.nx * L.ny
            gbs = BYTES[pn] * cells * n / sec / 1e9
            _, pop, ws = lbm.layout(L.P)
            q = lbm.make_params(L.nx, L.ny, e, prec=prec)
            _, pop2, ws2 = lbm.layout(q)
            row = {"workload": wl, "prec": pn, "us_per_step": sec * 1e6 / n, "MLUPS": cells * n / sec / 1e6,
                   "GB/s": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS, "device_bytes": pop + ws,
                   "device_bytes_two_buffer": 2 * pop2 + ws2}
            out.append(row)
            print("# aa %s %s: %.2f us/step, %.0f MLUPS, %.0f GB/s algorithmic (%.1f%%); %.2f GB of device memory "
                  "against %.2f GB with two buffers" % (wl, pn, row["us_per_step"], row["MLUPS"], gbs,
                                                       100 * gbs / HBM_PEAK_GBS, row["device_bytes"] / 1e9,
                                                       row["device_bytes_two_buffer"] / 1e9),
                  file=sys.stderr, flush=True)
            L.close()
            del L
            torch.cuda.empty_cache()
    return out


def batched_leg(lbm, steps=20000, n_lattices=64, seed=0):
    """Uneven batched planar sweep: 64 lattices L_b x 4 (L_b = 4 U{32..512}), Tr ~ U(0.35, 0.95), shaped PR,
    FP32-shifted, in the library's automatic launch mode; aggregate MLUPS and coexistence error against Maxwell."""
    import torch
    from lbm_inputs import SHAPED_PR, batched_planar_recipe, planar_density

    lengths, trs = batched_planar_recipe(n_lattices=n_lattices, seed=seed)
    P, rhos, eos = [], [], []
    for L, Tr in zip(lengths, trs):
        e, s = lbm.eos_build(lbm.make_eos(**dict(SHAPED_PR, Tr=Tr)))
        P.append(lbm.make_params(L, 4, e, sigma=s, tau=[1.0] * 9, prec=lbm.FP32_SHIFTED))
        rhos.append(planar_density(L, 4, e.rho_v, e.rho_l, W=20, axis=0))
        eos.append(e)
    B = lbm.Batch(P, rhos, device="cuda:0")
    B.step(100)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(B.stream)
    B.step(steps)
    ev[1].record(B.stream)
    torch.cuda.synchronize()
    B.check()
    sec = ev[0].elapsed_time(ev[1]) / 1e3
    cells = sum(4 * L for L in lengths)
    got = B.macros()
    ev_v = [abs(got[b]["rho"][0, 0] - eos[b].rho_v) / eos[b].rho_v for b in range(n_lattices)]
    ev_l = [abs(got[b]["rho"][0, lengths[b] // 2] - eos[b].rho_l) / eos[b].rho_l for b in range(n_lattices)]
    B.close()
    out = {"workload": "%d planar lattices 4 x L, L in [%d, %d], Tr in [%.2f, %.2f], shaped PR, FP32-shifted, %d steps"
                       % (n_lattices, min(lengths), max(lengths), min(trs), max(trs), steps + 100),
           "cells": cells, "steps": steps, "seconds": sec, "MLUPS": cells * steps / sec / 1e6,
           "us_per_step": sec * 1e6 / steps,
           "vapor_rel_err_vs_maxwell": {"max": max(ev_v), "mean": sum(ev_v) / n_lattices},
           "liquid_rel_err_vs_maxwell": {"max": max(ev_l), "mean": sum(ev_l) / n_lattices}}
    print("# batched %d lattices (%d cells): %.1f us/step, %.0f MLUPS; vapor error vs Maxwell max %.2f%% mean %.2f%%"
          % (n_lattices, cells, out["us_per_step"], out["MLUPS"], 100 * max(ev_v), 100 * sum(ev_v) / n_lattices),
          file=sys.stderr, flush=True)
    return out


def fd_leg(lbm, n=512, steps=2000, dt=0.2):
    """Finite-difference reference solver (MacCormack, FP64) on an n x n periodic droplet: C-S a=0.387 at
    Tr=0.6 with eps of the Li scheme (the paper's FD case), h = 1.  Algorithmic bytes per node and step:
    the state (rho, u, v) read once and written once = 48 B (one launch per step; the predicted state,
    psi and p_EOS live in LDS)."""
    import torch
    from lbm_inputs import droplet_density

    e, s = lbm.eos_build(lbm.make_eos(base=0, a=0.387, b=4.0, R=1.0, Tr=0.6))
    F = lbm.FdSolver(lbm.make_fd_params(n, n, e, h=1.0, dt=dt, eps=e.eps),
                     droplet_density(n, n, e.rho_v, e.rho_l, R=n // 6, W=8), device="cuda:0")
    F.step(100)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(F.stream)
    F.step(steps)
    ev[1].record(F.stream)
    torch.cuda.synchronize()
    F.check()
    sec = ev[0].elapsed_time(ev[1]) / 1e3
    F.close()
    gbs = 48.0 * n * n * steps / sec / 1e9
    out = {"workload": "FD MacCormack %dx%d periodic droplet, C-S a=0.387 Tr=0.6, h=1, dt=%g, FP64" % (n, n, dt),
           "us_per_step": sec * 1e6 / steps, "Mnode_steps_per_s": n * n * steps / sec / 1e6, "GB/s": gbs,
           "frac_hbm_peak": gbs / HBM_PEAK_GBS, "bytes_per_node_step": 48, "launches_per_step": 1}
    print("# FD solver %dx%d: %.2f us/step, %.0f Mnode-steps/s, %.0f GB/s algorithmic" % (
        n, n, out["us_per_step"], out["Mnode_steps_per_s"], gbs), file=sys.stderr, flush=True)
    return out


def drop_impact_variants_leg(lbm, steps=400):
    """The headline workload on each step-kernel decomposition, both precisions (time per step)."""
    import torch

    out = {"workload": drop_impact_name()}
    for prec in (lbm.FP32_SHIFTED, lbm.FP64):
        for variant, vname in ((1, "row_march"), (2, "row_block"), (3, "two_step")):
            L, e = drop_impact_lattice(lbm, prec, 0, variant)
            sec, _ = time_steps(L, steps, 20)
            L.check()
            us = sec * 1e6 / steps
            out["%s_%s_us_per_step" % (_prec_name(prec, lbm), vname)] = us
            print("# drop impact %s %s: %.2f us/step" % (_prec_name(prec, lbm), vname, us), file=sys.stderr, flush=True)
            L.close()
            del L
            torch.cuda.empty_cache()
    return out


def stability_leg(lbm, steps=3000):
    """Sec. IV stability map: width calibration (batched planar lattices) and 3 EOS x 9 Tr x 12 v_r
    droplet impacts (600 x 250, FP32-shifted); the largest stable simulated density ratio per EOS."""
    import torch
    from paper_2107_06355_amd import stability as S

    t0 = time.perf_counter()
    table = S.calibrate()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    smap, best = S.stability_map(table, steps=steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    runs = sum(len(v) for v in smap.values())
    out = {"calibration_s": t1 - t0, "map_s": t2 - t1, "impact_runs": runs, "steps_per_run": steps,
           "best": {k: (None if v is None else {"ratio": v[0], "Tr": v[1], "vr": v[2]}) for k, v in best.items()},
           "map": {k: {"%.2f" % Tr: "".join("S" if m[(Tr, vr)] else "." for vr in S.VRS) for Tr in S.TRS}
                   for k, m in smap.items()},
           "vr": list(S.VRS)}
    print("# stability map: calibration %.1f s, %d impacts in %.1f s" % (t1 - t0, runs, t2 - t1),
          file=sys.stderr, flush=True)
    return out


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed steps of each workload leg")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--kernel-steps", type=int, default=2000, help="steps over which the step kernel is timed alone")
    ap.add_argument("--legs", default=",".join(LEGS), help="comma list of: " + ", ".join(LEGS))
    ap.add_argument("--only", default="", help="fp32 | fp64: time one precision of the workload legs")
    ap.add_argument("--sweep", default="2048,4096,8192,16384", help="lattice sides of the HBM sweep")
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--batched-steps", type=int, default=20000, help="timed steps of the batched leg")
    ap.add_argument("--aa-steps", type=int, default=1000, help="timed steps of the AA leg on the impact lattice")
    ap.add_argument("--tile-rows", default="-1,-1",
                    help="two-step tile height FP32,FP64 (lbm_params.tile_rows): -1 timed at lattice creation, "
                         "0 the library's rule, 10..18 / 5..10 a fixed height")
    # about 10 s of host work each (2048 x 1024 FP64 oracle: ~0.36 s per step on one core,
    # ~0.03 s on 16)
    ap.add_argument("--cpu-steps", type=int, default=30, help="oracle steps of the single-threaded CPU leg")
    ap.add_argument("--cpu-omp-steps", type=int, default=360, help="oracle steps of the all-core CPU leg")
    ap.add_argument("--adjoint-steps", type=int, default=4000)
    ap.add_argument("--no-adjoint-fd", action="store_true", help="skip the finite-difference check of the adjoint")
    ap.add_argument("--stability-map", action="store_true", help="add the Sec. IV stability-map leg (~1 min)")
    ap.add_argument("--drop-impact-variants", action="store_true",
                    help="add the headline workload on each step-kernel decomposition")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs the hot path on ONE GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    try:
        TILE_ROWS["fp32"], TILE_ROWS["fp64"] = (int(v) for v in args.tile_rows.split(","))
    except ValueError:
        print("bench.py: --tile-rows takes two integers, FP32,FP64", file=sys.stderr)
        sys.exit(2)
    legs = [v.strip() for v in args.legs.split(",") if v.strip()]
    bad = [v for v in legs if v not in LEGS]
    if bad:
        ap.error("unknown legs %s" % bad)

    import torch

    from paper_2107_06355_amd import lbm

    lbm.load()
    torch.cuda.set_device(0)
    calib = copy_bandwidth()
    print("# device copy: %.0f GB/s (read+write, %d MiB buffers)" % (calib["GB/s"], calib["bytes_moved"] >> 21),
          file=sys.stderr, flush=True)
    precs = [p for p in (lbm.FP32_SHIFTED, lbm.FP64) if not args.only or _prec_name(p, lbm) == args.only]
    out = {}
    res = {}
    for leg, make, wname in (
            ("c3", lambda prec, re, h=None: drop_impact_lattice(lbm, prec, re, tile_rows=h), "drop impact 2048x1024"),
            ("c2", lambda prec, re, h=None: droplet_lattice(lbm, 512, prec, re, R=80, tile_rows=h),
             "droplet 512x512")):
        if leg not in legs:
            continue
        res[leg] = {}
        for prec in precs:
            pn = _prec_name(prec, lbm)
            r = workload_leg(lbm, make, prec, args.steps, args.warmup, args.kernel_steps)
            r["roofline"] = roofline(r, wname, pn, calib)
            res[leg][pn] = r
            print("# %s %s: %.1f MLUPS (%.2f us/step, %d reductions in the window); step kernel %.2f us per launch "
                  "of %d steps = %.0f GB/s algorithmic (%.1f%% of 8 TB/s; %s, %s)%s" % (
                      wname, pn, r["MLUPS"], r["ms_per_step"] * 1e3, r["reductions_in_window"], r["avg_launch_us"],
                      r["steps_per_launch"], r["kernel_GB/s"], 100 * r["frac_hbm_peak"], r["kernel"], r["tiles"],
                      "" if r["roofline"].get("measured_GB/s") is None else
                      ", %.0f GB/s measured (%.1f%%)" % (r["roofline"]["measured_GB/s"],
                                                        100 * r["roofline"]["measured_frac"])),
                  file=sys.stderr, flush=True)
    head_leg = "c3" if "c3" in res else ("c2" if "c2" in res else None)
    if head_leg is not None:
        pn = "fp32" if "fp32" in res[head_leg] else "fp64"
        r = res[head_leg][pn]
        tiles = {"tiles": r["tiles"], "tile_rows_mode": TILE_ROWS[pn]}
        if head_leg == "c3":
            from lbm_inputs import DROP_IMPACT_2048

            e, _ = lbm.eos_build(lbm.make_eos(**DROP_IMPACT_2048["eos"]))
            cfg = {"workload": drop_impact_name(e), "lattice": [2048, 1024], "walls": "top and bottom",
                   "storage": pn, "reduce_every": r["reduce_every"],
                   "reductions_in_window": r["reductions_in_window"], **tiles}
        else:
            cfg = {"workload": droplet_name(512, 80), "lattice": [512, 512], "storage": pn,
                   "reduce_every": r["reduce_every"], "reductions_in_window": r["reductions_in_window"], **tiles}
        out.update({
            "metric": METRIC, "value": r["MLUPS"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if pn == "fp32" else "f64", "data": "synthetic", "config": cfg,
            "roofline": r["roofline"]})
    if "c3" in res:
        out["drop_impact_2048x1024"] = res["c3"]
    if "c2" in res:
        out["static_droplet_512x512"] = res["c2"]
    if "parity" in legs:
        out["parity"] = parity_leg(lbm)
    if "sweep" in legs:
        out["sweep"] = sweep_leg(lbm, [int(v) for v in args.sweep.split(",") if v.strip()], args.sweep_steps, args.only)
    if "aa" in legs:
        out["aa"] = aa_leg(lbm, steps=args.aa_steps, big_steps=max(2, args.aa_steps // 50))
    if "batched" in legs:
        out["batched"] = batched_leg(lbm, steps=args.batched_steps)
    if "fd" in legs:
        out["fd"] = fd_leg(lbm)
        out["fd_4096"] = fd_leg(lbm, n=4096, steps=50)
    if args.drop_impact_variants:
        out["drop_impact_variants"] = drop_impact_variants_leg(lbm)
    if args.stability_map:
        out["stability"] = stability_leg(lbm)
    if "adjoint" in legs:
        out["adjoint"] = adjoint_leg(lbm, steps=args.adjoint_steps, fd_check=not args.no_adjoint_fd)
    out["copy_calibration"] = calib
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, args.cpu_omp_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
