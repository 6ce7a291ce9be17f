"""The complex-step reference (oracle/complex_step.py) against the C oracle.

Its real part must be the C oracle's forward map, and its derivatives must match central
differences of the C oracle, so that it can stand in as the machine-precision reference for
the discrete adjoint.
"""
import numpy as np
import pytest

import oracle as O
from oracle import complex_step as CS
from lbm_inputs import droplet_density, droplet_on_film

SMOOTH = dict(Tr=0.6, a=0.387, shape=1, alpha=0.834, k_vap=2 / 0.387)
TAU = [1.0, 1.1, 1.2, 1.0, 1.1, 1.0, 1.1, 0.8, 0.8]


def _case(kind, nx=21, ny=17):
    e, s = O.eos_build(O.make_eos(**SMOOTH))
    if kind == "droplet":
        rho0 = droplet_density(nx, ny, e.rho_v, e.rho_l, R=5, W=4)
        walls = {}
    else:
        rho0, _, _ = droplet_on_film(nx, ny, e.rho_v, e.rho_l, R=4, h=4, gap=2, V=0.0, W=4)
        walls = dict(walls=True, rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v)
    rng = np.random.default_rng(3)
    w = (rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx)))
    return e, s, nx, ny, rho0, w, walls


def _c_loss(e, s, nx, ny, rho0, w, steps, walls, G=-1.0, sigma=None, knots=None):
    ee = O.eos_set_knots(e, *knots) if knots is not None else e
    L = O.Lattice(O.make_params(nx, ny, ee, G=G, sigma=s if sigma is None else sigma, tau=TAU, **walls))
    L.init_eq(rho0)
    L.run(steps)
    m = L.macros()
    return float((w[0] * m["rho"]).sum() + (w[1] * m["ux"]).sum() + (w[2] * m["uy"]).sum()), m


@pytest.mark.parametrize("kind", ["droplet", "walls"])
def test_real_part_is_the_c_oracle_map(kind):
    e, s, nx, ny, rho0, w, walls = _case(kind)
    steps = 12
    _, m = _c_loss(e, s, nx, ny, rho0, w, steps, walls)
    L = CS.Lattice(CS.Eos(e), nx, ny, -1.0, s, TAU, **walls)
    L.init_eq(rho0)
    L.run(steps)
    rho, ux, uy, ps = L.fields()[:4]
    for a in (rho, ux, uy, ps):
        assert np.abs(a.imag).max() == 0.0
    np.testing.assert_allclose(rho.real, m["rho"], rtol=1e-13, atol=0)
    scale = np.abs(m["ux"]).max() + np.abs(m["uy"]).max()
    assert np.abs(ux.real - m["ux"]).max() <= 1e-11 * scale
    assert np.abs(uy.real - m["uy"]).max() <= 1e-11 * scale
    np.testing.assert_allclose(ps.real, m["psi"], rtol=1e-13, atol=0)


def test_eos_matches_c_oracle_on_every_branch():
    e, _ = O.eos_build(O.make_eos(**SMOOTH))
    r = np.concatenate([np.linspace(0.2 * e.rho_v, e.rho_v, 7), np.linspace(e.rho_v, e.rho_max, 9),
                        np.linspace(e.rho_max, e.rho_min, 9), np.linspace(e.rho_min, e.rho_l, 9),
                        np.linspace(e.rho_l, 1.1 * e.rho_l, 5)])
    got = CS.Eos(e).p(r)
    np.testing.assert_allclose(got.real, O.eos_p(e, r), rtol=1e-12, atol=1e-18)
    # d p / d rho by complex step against the C oracle's analytic slope, away from the knots
    h = 1e-30
    rr = np.concatenate([np.linspace(0.3 * e.rho_v, 0.99 * e.rho_v, 4),
                         e.rho_v + (e.rho_max - e.rho_v) * np.array([0.2, 0.5, 0.8]),
                         e.rho_max + (e.rho_min - e.rho_max) * np.array([0.2, 0.5, 0.8]),
                         e.rho_min + (e.rho_l - e.rho_min) * np.array([0.2, 0.5, 0.8]),
                         np.linspace(1.01 * e.rho_l, 1.1 * e.rho_l, 3)])
    d = CS.Eos(e).p(rr + 1j * h).imag / h
    np.testing.assert_allclose(d, O.eos_dp(e, rr), rtol=1e-10, atol=0)


@pytest.mark.parametrize("kind", ["droplet", "walls"])
def test_complex_step_matches_central_differences_of_the_c_oracle(kind):
    e, s, nx, ny, rho0, w, walls = _case(kind)
    steps = 10
    nodes = [(ny // 2, nx // 2), (ny // 2, nx // 2 + 5), (1, 2)]
    g, d0 = CS.gradients(e, nx, ny, rho0, w, steps, -1.0, s, TAU, nodes=nodes, **walls)
    k = [e.rho_max, e.p_max, e.rho_min, e.p_min]
    fd = []
    for j in range(4):
        h = 1e-5 * abs(k[j])
        kp, km = list(k), list(k)
        kp[j] += h
        km[j] -= h
        fd.append((_c_loss(e, s, nx, ny, rho0, w, steps, walls, knots=kp)[0]
                   - _c_loss(e, s, nx, ny, rho0, w, steps, walls, knots=km)[0]) / (2 * h))
    h = 1e-5
    fd.append((_c_loss(e, s, nx, ny, rho0, w, steps, walls, G=-1 + h)[0]
               - _c_loss(e, s, nx, ny, rho0, w, steps, walls, G=-1 - h)[0]) / (2 * h))
    h = 1e-5 * s
    fd.append((_c_loss(e, s, nx, ny, rho0, w, steps, walls, sigma=s + h)[0]
               - _c_loss(e, s, nx, ny, rho0, w, steps, walls, sigma=s - h)[0]) / (2 * h))
    fd = np.array(fd)
    for n, a, b in zip(("rho_max", "p_max", "rho_min", "p_min", "G", "sigma"), g, fd):
        assert abs(a - b) <= 1e-5 * abs(b) + 1e-9 * np.abs(fd).max(), (kind, n, a, b)
    for (y, x), a in zip(nodes, d0):
        h = 1e-6 * rho0[y, x]
        rp, rm = rho0.copy(), rho0.copy()
        rp[y, x] += h
        rm[y, x] -= h
        b = (_c_loss(e, s, nx, ny, rp, w, steps, walls)[0] - _c_loss(e, s, nx, ny, rm, w, steps, walls)[0]) / (2 * h)
        assert abs(a - b) <= 1e-6 * abs(b) + 1e-8, (kind, y, x, a, b)


@pytest.mark.parametrize("kind", ["droplet", "walls"])
def test_complex_step_G_sigma_scaling_identity(kind):
    """psi^2 ~ 1/G makes F = psi F~ independent of G and |F~|^2 ~ G, so the map depends on G and
    sigma only through sigma G: G dL/dG = sigma dL/dsigma, to rounding with complex steps."""
    e, s, nx, ny, rho0, w, walls = _case(kind)
    g, _ = CS.gradients(e, nx, ny, rho0, w, 10, -1.0, s, TAU, **walls)
    assert abs(-1.0 * g[4] - s * g[5]) <= 1e-12 * abs(s * g[5])
