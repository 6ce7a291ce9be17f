"""torch.autograd front end of lbm_adjoint.

``LbmRollout.apply(knots, G, sigma, rho0, spec)`` runs ``spec.steps`` fused steps from
f^eq(rho0, u = 0) and returns rho(T) and u(T) as float64 tensors on the lattice's device (``rollout``
keeps rho only); its backward calls lbm_adjoint_fields and returns dL/d(knots), dL/dG, dL/dsigma and dL/drho0.  With ``spec.K = None``
the forward records every step in HBM (16 B per node and step in FP32) and the backward runs
only the transposed steps; with an integer K it checkpoints every K steps and recomputes each
segment.  knots = (rho_max, p_max, rho_min, p_min) are the
four interior points of the Smooth loop (Sec. III.D), treated as free parameters with the
ellipse coefficients refitted to them; sigma is the Eq. LiFS coefficient, independent of G.
All arithmetic runs in liblbm; this module only marshals tensors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import lbm


@dataclass
class RolloutSpec:
    eos: lbm.LbmEos                      # a built Smooth / Modified Smooth EOS (lbm.eos_build)
    nx: int
    ny: int
    steps: int
    K: int | None = 200                  # None: record every step instead of checkpointing
    prec: int = lbm.FP32_SHIFTED
    params: dict = field(default_factory=dict)   # extra lbm.make_params keywords (tau, walls, ...)
    device: str = "cuda:0"


def _f(x) -> float:
    return float(x.detach().cpu().item()) if hasattr(x, "detach") else float(x)


def _autograd_function():
    import torch

    class LbmRollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, knots, G, sigma, rho0, spec: RolloutSpec):
            ctx.set_materialize_grads(False)
            k = [float(v) for v in knots.detach().cpu().double().tolist()]
            e = lbm.eos_set_knots(spec.eos, *k)
            P = lbm.make_params(spec.nx, spec.ny, e, G=_f(G), sigma=_f(sigma), prec=spec.prec, **spec.params)
            lat = lbm.Lattice(P, rho0.detach(), device=spec.device)
            if spec.K is None:
                lat.enable_recording(spec.steps)
            else:
                lat.enable_checkpointing(spec.K, spec.steps)
            lat.step(spec.steps)
            lat.check()
            m = lat.macros()
            ctx.lat = lat
            ctx.meta = (knots.dtype, knots.device, rho0.dtype, rho0.device)
            return m["rho"], m["ux"], m["uy"]

        @staticmethod
        def backward(ctx, g_rho, g_ux, g_uy):
            lat = ctx.lat
            kd, kdev, rd, rdev = ctx.meta
            prep = lambda g: g.detach().to(torch.float64).contiguous() if g is not None else None
            if g_rho is None and g_ux is None and g_uy is None:
                g_rho = torch.zeros((lat.ny, lat.nx), dtype=torch.float64, device=lat.device)
            g = lat.adjoint(prep(g_rho), want_rho0=ctx.needs_input_grad[3], dL_dux=prep(g_ux), dL_duy=prep(g_uy))
            ctx.lat = None
            lat.close()
            need = ctx.needs_input_grad
            # a position whose forward input was not a tensor needing grad (a Python float G, say)
            # gets None, as autograd requires
            gk = torch.tensor([g[n] for n in lbm.GRAD_NAMES[:4]], dtype=kd, device=kdev) if need[0] else None
            gG = torch.tensor(g["G"], dtype=torch.float64) if need[1] else None
            gs = torch.tensor(g["sigma"], dtype=torch.float64) if need[2] else None
            gr = g["rho0"].to(dtype=rd, device=rdev) if need[3] and "rho0" in g else None
            return gk, gG, gs, gr, None

    return LbmRollout


_FN = None


def rollout_fields(knots, G, sigma, rho0, spec: RolloutSpec):
    """(rho(T), u_x(T), u_y(T)) with gradients flowing to knots, G, sigma and rho0 (torch tensors);
    u is the forced velocity (j + F/2)/rho of Eq. Momentum."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(knots, G, sigma, rho0, spec)


def rollout(knots, G, sigma, rho0, spec: RolloutSpec):
    """rho(T) with gradients flowing to knots, G, sigma and rho0 (torch tensors)."""
    return rollout_fields(knots, G, sigma, rho0, spec)[0]


def knots_of(e: lbm.LbmEos) -> np.ndarray:
    return np.array([e.rho_max, e.p_max, e.rho_min, e.p_min])


def vapor_width_loss(rho, rho_v_ref: float, R0: float, W0: float, center=None, lam_w: float = 0.01):
    """Squared relative error of the mean far-field vapor density plus an interface-width penalty.

    rho_bar_v averages rho over |x - x_c| > R0 + 2 W0.  W_eff = 4.6 drho^2 2 pi R0 / (3 sum |grad rho|^2)
    is the width of a tanh profile of the droplet-initialisation form with the same gradient energy
    (central differences, periodic), drho = rho_l - rho_v taken from the field's max and the vapor mean.
    """
    import torch

    ny, nx = rho.shape
    cy, cx = (ny / 2, nx / 2) if center is None else center
    yy, xx = torch.meshgrid(torch.arange(ny, dtype=rho.dtype, device=rho.device),
                            torch.arange(nx, dtype=rho.dtype, device=rho.device), indexing="ij")
    far = ((xx - cx) ** 2 + (yy - cy) ** 2).sqrt() > R0 + 2 * W0
    rv = rho[far].mean()
    gx = 0.5 * (torch.roll(rho, -1, 1) - torch.roll(rho, 1, 1))
    gy = 0.5 * (torch.roll(rho, -1, 0) - torch.roll(rho, 1, 0))
    drho = rho.max() - rv
    w_eff = 4.6 * drho ** 2 * 2 * np.pi * R0 / (3 * (gx ** 2 + gy ** 2).sum())
    return ((rv - rho_v_ref) / rho_v_ref) ** 2 + lam_w * ((w_eff - W0) / W0) ** 2
