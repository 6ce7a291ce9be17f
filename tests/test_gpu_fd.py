"""Finite-difference reference solver (appendix "Finite Difference Method") on the GPU path.

Parity with the oracle's MacCormack step on a periodic droplet and on a droplet falling onto a
film between the appendix's wall layers (FP64, elementwise), the exact discrete decay of a
shear wave (periodic, and the sine mode the wall layers admit), and convergence of a planar
interface toward the Maxwell densities under mesh refinement (the purpose the paper gives the
solver).
"""
import math

import numpy as np
import pytest

import oracle as O
from lbm_inputs import droplet_density, droplet_on_film, planar_density

pytestmark = pytest.mark.gpu


def _cs(Tr):
    kw = dict(base=0, a=0.5, b=4.0, R=1.0, Tr=Tr)
    return kw


@pytest.mark.parametrize("shape", [(45, 38), (130, 70)], ids=["45x38", "130x70"])
@pytest.mark.parametrize("var_tau", [False, True])
def test_fd_droplet_matches_oracle(gpu_lib, var_tau, shape):
    lbm = gpu_lib
    kw = _cs(0.7)
    e, s = lbm.eos_build(lbm.make_eos(**kw))
    eo, so = O.eos_build(O.make_eos(**kw))
    (nx, ny), steps = shape, 150
    rho0 = droplet_density(nx, ny, e.rho_v, e.rho_l, R=10, W=8)
    rng = np.random.default_rng(3)
    u0, v0 = 1e-3 * rng.standard_normal((ny, nx)), 1e-3 * rng.standard_normal((ny, nx))
    tk = dict(var_tau=var_tau, tau_l=0.7, tau_v=1.3, tau_e=1.1, tau_nu=0.9)
    F = lbm.FdSolver(lbm.make_fd_params(nx, ny, e, h=1.0, dt=0.15, eps=e.eps, **tk), rho0, u0, v0, device="cuda:0")
    F.step(steps)
    F.check()
    r, u, v = (a.cpu().numpy() for a in F.fields())
    OF = O.FdSolver(O.make_fd_params(nx, ny, eo, h=1.0, dt=0.15, eps=eo.eps, **tk))
    OF.set(rho0, u0, v0)
    OF.run(steps)
    ro, uo, vo = OF.get()
    assert np.abs(r - ro).max() <= 1e-12 * np.abs(ro).max()
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max()) <= 1e-12 * max(np.abs(uo).max(), np.abs(vo).max())


def test_fd_shear_wave_exact_discrete_decay(gpu_lib):
    """Uniform density: u = A sin(k y) decays by g = 1 - l dt + (l dt)^2/2 per step with
    l = nu (2 sin(k h / 2) / h)^2 (central second difference, predictor-corrector), nu = (tau - 1/2)/3."""
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**_cs(0.7)))
    nx, ny, h, dt, tau, n, A = 4, 32, 0.5, 0.05, 0.8, 800, 1e-4
    y = np.arange(ny) * h
    k = 2 * np.pi / (ny * h)
    u0 = np.repeat((A * np.sin(k * y))[:, None], nx, axis=1)
    F = lbm.FdSolver(lbm.make_fd_params(nx, ny, e, h=h, dt=dt, tau_nu=tau), np.full((ny, nx), e.rho_l), u0,
                     device="cuda:0")
    F.step(n)
    F.check()
    r, u, v = (a.cpu().numpy() for a in F.fields())
    amp = 2 * (u[:, 0] * np.sin(k * y)).sum() / ny
    nu = (tau - 0.5) / 3
    lam = nu * (2 / h * math.sin(k * h / 2)) ** 2
    assert amp / A == pytest.approx((1 - lam * dt + (lam * dt) ** 2 / 2) ** n, rel=1e-12)
    assert np.abs(r - e.rho_l).max() == 0.0 and np.abs(v).max() < 1e-18


def test_fd_planar_converges_to_maxwell_at_second_order(gpu_lib):
    """Refining the mesh (fixed physical length 100, h = 1, 1/2, 1/4, dt = 0.2 h^2) the planar vapor
    density approaches the Maxwell value (eps of Eq. VaporLiqEq makes the continuum equilibrium the
    Maxwell one) with errors shrinking four-fold per halving of h."""
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**_cs(0.8)))
    E = []
    for h in (1.0, 0.5, 0.25):
        ny = int(round(100 / h))
        dt = 0.2 * h * h
        rho0 = planar_density(3, ny, e.rho_v, e.rho_l, W=10 / h, axis=1)
        F = lbm.FdSolver(lbm.make_fd_params(3, ny, e, h=h, dt=dt, eps=e.eps), rho0, device="cuda:0")
        F.step(int(round(3000 / dt)))
        F.check()
        r = F.fields()[0].cpu().numpy()[:, 0]
        E.append((r[0] - e.rho_v) / e.rho_v)
        F.close()
    assert abs(E[2]) < 2e-3
    assert 3.6 < E[0] / E[1] < 4.6 and 3.6 < E[1] / E[2] < 4.6


@pytest.mark.parametrize("var_tau", [False, True])
def test_fd_walls_droplet_on_film_matches_oracle(gpu_lib, var_tau):
    """45 x 38 mesh (two 32-wide tiles with a ragged tail, five 8-high tiles): a droplet at
    V = 0.05 above a film on the bottom wall, psi_l of Eq. B2 in the solid layer, reflexive top."""
    lbm = gpu_lib
    kw = _cs(0.7)
    e, s = lbm.eos_build(lbm.make_eos(**kw))
    eo, so = O.eos_build(O.make_eos(**kw))
    nx, ny, steps = 45, 38, 200
    rho0, u0, v0 = droplet_on_film(nx, ny, e.rho_v, e.rho_l, R=8, h=5, gap=3, V=0.05, W=5)
    tk = dict(var_tau=var_tau, tau_l=0.7, tau_v=1.3, tau_e=1.1, tau_nu=0.9, walls=True)
    F = lbm.FdSolver(lbm.make_fd_params(nx, ny, e, h=1.0, dt=0.15, eps=e.eps, **tk), rho0, u0, v0, device="cuda:0")
    F.step(steps)
    F.check()
    r, u, v = (a.cpu().numpy() for a in F.fields())
    OF = O.FdSolver(O.make_fd_params(nx, ny, eo, h=1.0, dt=0.15, eps=eo.eps, **tk))
    OF.set(rho0, u0, v0)
    OF.run(steps)
    ro, uo, vo = OF.get()
    assert np.abs(r - ro).max() <= 1e-12 * np.abs(ro).max()
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max()) <= 1e-12 * max(np.abs(uo).max(), np.abs(vo).max())


def test_fd_walls_shear_mode_exact_decay(gpu_lib):
    """u = 0 on b1 and the reflexive top make sin(pi (j+1)/ny) an exact discrete eigenmode of the
    central second difference: amplitude (1 - l dt + (l dt)^2/2)^n, l = nu (2 sin(k h/2)/h)^2, k = pi/(ny h)."""
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**_cs(0.7)))
    nx, ny, h, dt, tau, n, A = 4, 37, 0.5, 0.05, 0.8, 800, 1e-4
    j = np.arange(ny)
    mode = np.sin(np.pi * (j + 1) / ny)
    F = lbm.FdSolver(lbm.make_fd_params(nx, ny, e, h=h, dt=dt, tau_nu=tau, walls=True), np.full((ny, nx), e.rho_l),
                     np.repeat((A * mode)[:, None], nx, axis=1), device="cuda:0")
    F.step(n)
    F.check()
    r, u, v = (a.cpu().numpy() for a in F.fields())
    amp = (u[:, 0] * mode).sum() / (mode * mode).sum()
    k = np.pi / (ny * h)
    lam = (tau - 0.5) / 3 * (2 / h * math.sin(k * h / 2)) ** 2
    assert amp / A == pytest.approx((1 - lam * dt + (lam * dt) ** 2 / 2) ** n, rel=1e-11)
    assert np.abs(r - e.rho_l).max() < 1e-15 and np.abs(v).max() < 1e-18
