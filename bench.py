"""Throughput of the fused shaped-EOS pseudopotential D2Q9 step on one MI355X.

Default workload: static droplet (R=80, tanh rim of width 20) on a 512x512 periodic lattice,
shaped Peng-Robinson EOS (a=2/49, b=2/21, omega=0.344) at Tr=0.5 with the Smooth vdW-loop
replacement (alpha=0.3), raised vapor sound speed (k_vap=4), EOS scale 0.25, MRT with
tau_nu=0.7 and Li forcing with sigma from eps; FP32-shifted storage (rho_ref = rho_v) with
FP64 mass/momentum reductions every 100 steps, 50k steps; the same in FP64.  One "step" is
one time step of the whole hot path.  Inputs are resident in HBM before the timed region
starts.  The roofline figure times the step kernel alone on the stream it is launched on.

Further legs (in the same JSON line): an HBM sweep of larger lattices, the adjoint of the
droplet loss (cost against the forward, agreement with central differences), a plain
device-copy calibration and the FP64 CPU oracle on a bounded sample.

Prints ONE JSON line (rank 0).  --gpus N with N > 1 exits: the library runs the hot path on one GPU.
"""
from __future__ import annotations

import argparse
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
# step kernel of each decomposition (lbm_variant): row march, row block, two-step block
KERNEL_NAME = {1: "k_step<%s, 0>", 2: "k_step_blk<%s, 0>", 3: "k_step2_blk<%s, 0, false, %s>"}
STREAM_BYTES = 64 << 20  # the library streams its stores when both population buffers take at most this


def kernel_name(lbm, var, prec, P):
    """Name of the step kernel (as rocprofv3 prints it) that advances lattice P in this precision."""
    t = "float" if prec == "fp32" else "double"
    if var != lbm.VARIANT_BLOCK2:
        return KERNEL_NAME[var] % t
    return KERNEL_NAME[var] % (t, "true" if 2 * lbm.layout(P)[1] <= STREAM_BYTES else "false")

EOS_KW = dict(base=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, Tr=0.5, scale=0.25, shape=1, alpha=0.3, k_vap=4.0)
TAU = [1, 1, 1, 1, 1, 1, 1, 0.7, 0.7]


def workload_name(n, R):
    return ("static droplet %dx%d periodic, R=%d, shaped PR Tr=0.5 (Smooth alpha=0.3, k_vap=4, scale 0.25), "
            "MRT tau_nu=0.7, Li forcing" % (n, n, R))


def make_lattice(lbm, n, prec, R=None, reduce_every=100, band_rows=0, variant=0):
    """Static droplet on an n x n periodic lattice; R defaults to n/6 (the roofline sweep)."""
    from lbm_inputs import droplet_density

    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    R = n // 6 if R is None else R
    rho0 = droplet_density(n, n, e.rho_v, e.rho_l, R=R, W=20)
    P = lbm.make_params(n, n, e, sigma=s, tau=TAU, prec=lbm.FP32_SHIFTED if prec == "fp32" else lbm.FP64,
                        reduce_every=reduce_every, band_rows=band_rows, kernel_variant=variant)
    return lbm.Lattice(P, rho0, device="cuda:0"), e, s, rho0


def time_steps(L, steps, warmup):
    import torch

    L.step(warmup)
    torch.cuda.synchronize()
    stream = L.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    L.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


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


def sources_digest() -> str:
    """SHA-256 over the sources of the step kernels (a PMC summary is valid only for these)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("lbm_device.h", "lbm_step.hip"):
        with open(os.path.join(ROOT, "paper_2107_06355_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, n, prec):
    """HBM bytes per launch of `kernel` at n x n from the committed PMC summary, or None when there is
    none for this kernel/size or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_step_droplet_pmc_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    want = "%s n=%d %s" % (kernel, n, prec)
    digest = sources_digest()
    for line in open(path):
        if line.startswith("| traffic |"):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            # | traffic | kernel n=.. prec | bytes/launch | sources sha256 |
            if len(cells) >= 4 and cells[1] == want and cells[3] == digest:
                return float(cells[2])
    return None


def cpu_baseline(n, steps, R):
    """The FP64 oracle on a bounded sample of the same workload (single thread)."""
    import oracle as O
    from lbm_inputs import droplet_density

    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    rho0 = droplet_density(n, n, eo.rho_v, eo.rho_l, R=R, W=20)
    L = O.Lattice(O.make_params(n, n, eo, sigma=so, tau=TAU))
    L.init_eq(rho0)
    t0 = time.perf_counter()
    L.run(steps)
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%dx%d droplet, %d time steps from the same initial state (FP64, single thread, %.1f s)"
                      % (n, n, steps, dt), "host": _host_cpu()}


def _host_cpu() -> str:
    """CPU model and the CPUs this process may run on (the oracle uses one of them)."""
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return "%s, %d CPUs available" % (model, len(os.sched_getaffinity(0)))


def adjoint_leg(lbm, n=512, R=80, W0=20.0, steps=4000, K=200, fd_check=True):
    """Adjoint of the static-droplet loss (far-field vapor density + interface width): cost against the
    plain forward, and, in FP64, agreement with central differences of the same forward (h = 1e-6)."""
    import torch
    from lbm_inputs import droplet_density
    from paper_2107_06355_amd.rollout import vapor_width_loss

    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    rho0 = droplet_density(n, n, e.rho_v, e.rho_l, R=R, W=W0)

    def loss_grad(rho):
        r = rho.detach().clone().requires_grad_(True)
        L = vapor_width_loss(r, e.rho_v, R, W0)
        L.backward()
        return float(L.detach()), r.grad

    def run(prec, mode=None, ee=e, G=-1.0, sig=s):
        P = lbm.make_params(n, n, ee, G=G, sigma=sig, tau=TAU, prec=prec, reduce_every=0)
        lat = lbm.Lattice(P, rho0, device="cuda:0")
        if mode == "checkpoint":
            lat.enable_checkpointing(K, steps)
        elif mode == "record":
            lat.enable_recording(steps)
        return lat

    out = {"workload": "static droplet %dx%d R=%d W0=%g, shaped PR Tr=0.5, %d steps; the forward records every "
                       "step (primary) or checkpoints every %d steps and recomputes" % (n, n, R, W0, steps, K)}
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
        for mode in ("record", "checkpoint"):
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
        res["grad"] = res["record"]["grad"]
        res["adjoint_over_forward"] = res["record"]["adjoint_over_forward"]
        res["record_vs_checkpoint_max_rel_diff"] = max(
            abs(res["record"]["grad"][k] - res["checkpoint"]["grad"][k]) / max(abs(res["checkpoint"]["grad"][k]), 1e-300)
            for k in res["record"]["grad"])
        out[name] = res
    if fd_check:
        # central differences of the FP64 forward, relative step 1e-6
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
        g64 = out["fp64"]["grad"]
        out["fd_fp64"] = fd
        out["rel_err_fp64_vs_fd"] = {k: abs(g64[k] - fd[k]) / max(abs(fd[k]), 1e-300) for k in fd}
        g32 = out["fp32"]["grad"]
        out["rel_err_fp32_vs_fd"] = {k: abs(g32[k] - fd[k]) / max(abs(fd[k]), 1e-300) for k in fd}
        print("# adjoint vs FD (fp64): max rel err %.2e" % max(out["rel_err_fp64_vs_fd"].values()),
              file=sys.stderr, flush=True)
    return out


def batched_leg(lbm, steps=20000, n_lattices=64, seed=0):
    """Uneven batched planar sweep: 64 lattices L_b x 4 (L_b = 4 U{32..512}), Tr ~ U(0.35, 0.95), shaped PR,
    FP32-shifted, in the library's automatic launch mode (grouped: one launch per step over every lattice's
    rows); aggregate MLUPS and coexistence error against Maxwell."""
    import torch
    from lbm_inputs import batched_planar_recipe, planar_density

    lengths, trs = batched_planar_recipe(n_lattices=n_lattices, seed=seed)
    P, rhos, eos = [], [], []
    for L, Tr in zip(lengths, trs):
        e, s = lbm.eos_build(lbm.make_eos(**dict(EOS_KW, Tr=Tr)))
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


def drop_impact_leg(lbm, steps=400):
    """Droplet impact on a film between walls, 2048 x 1024 (R = 100, film 40, V = 0.072, Re = 300, v_r = 1),
    shaped Peng-Robinson at Tr = 0.47 (density ratio 3.07e4, rims of width 16): time per step of each
    step-kernel decomposition in both precisions."""
    import torch
    from lbm_inputs import droplet_on_film

    nx, ny, tau_l = 2048, 1024, 0.644
    e, s = lbm.eos_build(lbm.make_eos(**dict(EOS_KW, Tr=0.47)))
    rho, ux, uy = droplet_on_film(nx, ny, e.rho_v, e.rho_l, R=100, h=40, gap=4, V=0.072, W=16)
    out = {"workload": "drop impact %dx%d with walls, shaped PR Tr=0.47 (ratio %.3g), Re=300, %d steps"
                       % (nx, ny, e.rho_l / e.rho_v, steps)}
    for prec, name in ((lbm.FP32_SHIFTED, "fp32"), (lbm.FP64, "fp64")):
        for variant, vname in ((1, "row_march"), (2, "row_block"), (3, "two_step")):
            P = lbm.make_params(nx, ny, e, sigma=s, tau=[1] * 7 + [tau_l] * 2, prec=prec, walls=True,
                                rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v, reduce_every=0, kernel_variant=variant)
            L = lbm.Lattice(P, rho, ux, uy, device="cuda:0")
            L.step(20)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(L.stream)
            L.step(steps)
            ev[1].record(L.stream)
            torch.cuda.synchronize()
            L.check()
            us = ev[0].elapsed_time(ev[1]) * 1e3 / steps
            out["%s_%s_us_per_step" % (name, vname)] = us
            print("# drop impact %s %s: %.2f us/step, %.0f MLUPS" % (name, vname, us, nx * ny / us),
                  file=sys.stderr, flush=True)
            L.close()
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
    print("# stability map: calibration %.1f s, %d impacts in %.1f s; best ratio %s" % (
        t1 - t0, runs, t2 - t1, {k: (None if v is None else round(v[0])) for k, v in best.items()}),
        file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--n", type=int, default=512, help="lattice side of the timed workload")
    ap.add_argument("--radius", type=int, default=80, help="droplet radius of the timed workload")
    ap.add_argument("--sweep", default="2048,4096,8192,16384",
                    help="extra lattice sides for the HBM roofline ('' = none)")
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default="", help="fp32 | fp64: time just one precision of the main workload")
    ap.add_argument("--band-rows", type=int, default=0, help="rows per wave band (0 = the library's choice)")
    ap.add_argument("--sweep-band-rows", default="", help="comma list of band heights to time in the sweep")
    ap.add_argument("--calib-only", action="store_true", help="only measure the plain copy bandwidth")
    ap.add_argument("--variant", type=int, default=0, help="step-kernel decomposition: 0 auto, 1 row march, 2 row block")
    ap.add_argument("--sweep-variants", default="", help="comma list of kernel variants for the sweep")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost / gradient leg")
    ap.add_argument("--adjoint-only", action="store_true")
    ap.add_argument("--no-adjoint-fd", action="store_true", help="skip the finite-difference check of the adjoint")
    ap.add_argument("--adjoint-steps", type=int, default=4000)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-lattice sweep leg")
    ap.add_argument("--batched-only", action="store_true")
    ap.add_argument("--stability-map", action="store_true", help="add the Sec. IV stability-map leg (~1 min)")
    ap.add_argument("--drop-impact", action="store_true", help="add the walled drop-impact timing leg (seconds)")
    ap.add_argument("--no-fd", action="store_true", help="skip the finite-difference reference-solver leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs the hot path on ONE GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2107_06355_amd import lbm

    lbm.load()
    torch.cuda.set_device(0)
    calib = copy_bandwidth()
    print("# device copy: %.0f GB/s (read+write, %d MiB buffers)" % (calib["GB/s"], calib["bytes_moved"] >> 21),
          file=sys.stderr, flush=True)
    if args.calib_only:
        print(json.dumps({"copy": calib}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(lbm)}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(lbm, steps=args.adjoint_steps, fd_check=not args.no_adjoint_fd)}), flush=True)
        return
    n = args.n
    res = {}
    for prec in ("fp32", "fp64"):
        if args.only and prec != args.only:
            continue
        # the metric: the whole hot path, FP64 mass/momentum reductions every 100 steps
        L, e, s, _ = make_lattice(lbm, n, prec, R=args.radius, band_rows=args.band_rows, variant=args.variant)
        var, rows, waves = lbm.describe(L.P)
        sec, wall = time_steps(L, args.steps, args.warmup)
        L.check()
        L.close()
        del L
        # the roofline: the step kernel alone (no reduction launches in the timed region)
        L, e, s, _ = make_lattice(lbm, n, prec, R=args.radius, reduce_every=0, band_rows=args.band_rows,
                                  variant=args.variant)
        ksec, _ = time_steps(L, args.steps, args.warmup)
        L.check()
        cells = n * n
        spl = 2 if var == lbm.VARIANT_BLOCK2 else 1  # time steps per launch of the step kernel
        mlups = cells * args.steps / sec / 1e6
        kgbs = BYTES[prec] * cells * args.steps / ksec / 1e9
        res[prec] = {"MLUPS": mlups, "GB/s_step": BYTES[prec] * cells * args.steps / sec / 1e9,
                     "ms_per_step": sec * 1e3 / args.steps, "wall_s": wall,
                     "kernel_GB/s": kgbs, "frac_hbm_peak": kgbs / HBM_PEAK_GBS,
                     "avg_launch_us": ksec * 1e6 / (args.steps / spl), "steps_per_launch": spl,
                     "kernel": kernel_name(lbm, var, prec, L.P),
                     "rows_per_block": rows, "waves": waves}
        print("# %s %dx%d: %.1f MLUPS (%.2f us/step with reductions); step kernel %.2f us = %.1f GB/s "
              "algorithmic (%.1f%% of 8 TB/s)" % (prec, n, n, mlups, sec * 1e6 / args.steps, ksec * 1e6 / args.steps,
                                                   kgbs, 100 * kgbs / HBM_PEAK_GBS), file=sys.stderr, flush=True)
        L.close()
        del L
        torch.cuda.empty_cache()

    sweep = []
    bands = [int(v) for v in args.sweep_band_rows.split(",") if v.strip()] or [0]
    variants = [int(v) for v in args.sweep_variants.split(",") if v.strip()] or [args.variant]
    combos = [(v, b) for v in variants for b in (bands if v == 1 else [0])]
    for side in [int(v) for v in args.sweep.split(",") if v.strip()]:
        for prec in ("fp32", "fp64"):
            if args.only and prec != args.only:
                continue
            for variant, band in combos:
                L, e, s, _ = make_lattice(lbm, side, prec, reduce_every=0, band_rows=band, variant=variant)
                sec, wall = time_steps(L, args.sweep_steps, 20)
                L.check()
                cells = side * side
                gbs = BYTES[prec] * cells * args.sweep_steps / sec / 1e9
                sweep.append({"n": side, "prec": prec, "variant": variant, "band_rows": band,
                              "MLUPS": cells * args.sweep_steps / sec / 1e6,
                              "GB/s": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
                              "avg_launch_us": sec * 1e6 / args.sweep_steps})
                print("# sweep %s %dx%d variant=%d band=%d: %.0f MLUPS, %.0f GB/s (%.1f%%), %.2f us/step" % (
                    prec, side, side, variant, band, sweep[-1]["MLUPS"], gbs, 100 * gbs / HBM_PEAK_GBS,
                    sweep[-1]["avg_launch_us"]), file=sys.stderr, flush=True)
                L.close()
                del L
                torch.cuda.empty_cache()

    main_prec = "fp32" if "fp32" in res else "fp64"
    r = res[main_prec]
    out = {
        "metric": METRIC,
        "value": r["MLUPS"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(n, args.radius), "lattice": [n, n], "storage": main_prec,
                   "reduce_every": 100},
        "roofline": {"bound": "hbm", "achieved": r["kernel_GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["kernel_GB/s"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(r["kernel"], n, main_prec),
                     "kernel": r["kernel"], "bytes_per_cell": BYTES[main_prec],
                     "cell_updates_per_launch": n * n * r["steps_per_launch"],
                     "steps_per_launch": r["steps_per_launch"], "avg_launch_us": r["avg_launch_us"],
                     "copy_ceiling_frac": r["kernel_GB/s"] / calib["GB/s"]},
        "fp64": res.get("fp64"),
        "fp32": res.get("fp32"),
        "sweep": sweep,
        "copy_calibration": calib,
    }
    if not args.no_batched:
        out["batched"] = batched_leg(lbm)
    if args.stability_map:
        out["stability"] = stability_leg(lbm)
    if args.drop_impact:
        out["drop_impact"] = drop_impact_leg(lbm)
    if not args.no_fd:
        out["fd"] = fd_leg(lbm)
        out["fd_4096"] = fd_leg(lbm, n=4096, steps=50)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(lbm, steps=args.adjoint_steps, fd_check=not args.no_adjoint_fd)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_steps, args.radius)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
