"""Laplace's law on the GPU path: static droplets of the 512x512 shaped Peng-Robinson workload.

In 2-D the pressure jump across a circular interface of radius R is gamma/R.  Droplets with
R = 40 ... 120 are run to near equilibrium; the slope of the pressure jump against 1/R is
compared with gamma of a planar interface of the same fluid from Eq. SurfaceTension, and the
intercept must vanish.
"""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import STATIC_DROPLET_512, droplet_density, planar_density

pytestmark = pytest.mark.gpu

EOS_KW = STATIC_DROPLET_512["eos"]
TAU = [1, 1, 1, 1, 1, 1, 1, 0.7, 0.7]
N = 512
RADII = (40, 60, 80, 100, 120)


def _planar_gamma(lbm, e, s, prec):
    ny = 400
    P = lbm.make_params(4, ny, e, sigma=s, tau=TAU, prec=prec)
    lat = lbm.Lattice(P, planar_density(4, ny, e.rho_v, e.rho_l, W=20, axis=1), device="cuda:0")
    lat.step(60000)
    lat.check()
    psi = lat.macros()["psi"].cpu().numpy()[:, 0]
    return O.surface_tension_planar(psi, -1.0)


def _droplet_jump(lbm, e, s, R, prec, steps):
    P = lbm.make_params(N, N, e, sigma=s, tau=TAU, prec=prec)
    rho0 = droplet_density(N, N, e.rho_v, e.rho_l, R=R, W=20)
    lat = lbm.Lattice(P, rho0, device="cuda:0")
    lat.step(steps)
    lat.check()
    m = lat.macros()
    rho, p = m["rho"].cpu().numpy(), m["p"].cpu().numpy()
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    r = np.hypot(x - N / 2, y - N / 2)
    core, far = r < 0.5 * R, r > R + 60
    rin, rout = rho[core].mean(), rho[far].mean()
    Re = np.sqrt((rho - rout).sum() / (np.pi * (rin - rout)))   # equimolar radius
    umax = float(np.hypot(m["ux"].cpu().numpy(), m["uy"].cpu().numpy()).max())
    return p[core].mean() - p[far].mean(), Re, umax


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_laplace_law_static_droplets(gpu_lib, prec_name):
    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    gamma = _planar_gamma(lbm, e, s, prec)
    rows = [_droplet_jump(lbm, e, s, R, prec, 150000) for R in RADII]  # the stiff liquid core rings for ~1e5 steps
    dp = np.array([r[0] for r in rows])
    inv = 1.0 / np.array([r[1] for r in rows])
    slope, icpt = np.polyfit(inv, dp, 1)
    fit = slope * inv + icpt
    print("gamma planar %.4e, Laplace slope %.4e, intercept %.3e, dp %s, R_e %s, max |u| %s" % (
        gamma, slope, icpt, dp, 1 / inv, [r[2] for r in rows]), flush=True)
    assert np.abs(fit - dp).max() <= 0.02 * dp.max()            # dp linear in 1/R
    assert abs(icpt) <= 0.03 * dp.max()                         # no jump for a flat interface
    assert slope == pytest.approx(gamma, rel=0.10)              # same gamma as the planar interface
