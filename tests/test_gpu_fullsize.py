"""Parity at the benchmark's sizes, in the launch configurations bench.py times.

512x512 (the timed workload, row-block kernel): the whole field after one step against the
oracle's step from the same populations.  8192x8192 (the HBM sweep, row-march kernel):
sampled nodes.  One step moves information at most two nodes (the pull, then psi of the
neighbours in Eq. ShanChenForce), so the next-step populations at x depend only on the
current populations within distance 2 of x.  For each sampled x the oracle steps a 7x7
periodic window centred on x, whose wrap-around cannot reach the centre, and its centre
must equal the GPU result at x.  Samples cover the 62-column strip edges, band edges,
the lattice corners (periodic wrap) and random nodes.
"""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import droplet_density

pytestmark = pytest.mark.gpu

EOS_KW = dict(base=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, Tr=0.5, scale=0.25, shape=1, alpha=0.3, k_vap=4.0)
TAU = [1, 1, 1, 1, 1, 1, 1, 0.7, 0.7]
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _bound(lbm, prec, f_o, rho_v):
    if prec == lbm.FP64:
        return 1e-12 * np.abs(f_o).max()
    return 2e-6 * np.abs(f_o - W9.reshape((9,) + (1,) * (f_o.ndim - 1)) * rho_v).max()


def _lattice(lbm, n, R, prec, steps):
    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    rho0 = droplet_density(n, n, e.rho_v, e.rho_l, R=R, W=20)
    P = lbm.make_params(n, n, e, sigma=s, tau=TAU, prec=prec, reduce_every=100)
    L = lbm.Lattice(P, rho0, device="cuda:0")
    L.step(steps)
    L.check()
    return L, e


@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_512_droplet_whole_field_one_step(gpu_lib, prec_name):
    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    L, e = _lattice(lbm, 512, 80, prec, 300)
    assert lbm.describe(L.P)[0] == lbm.VARIANT_BLOCK  # the kernel bench.py times at this size
    f_t = L.populations().cpu().numpy()
    L.step(1)
    f_g = L.populations().cpu().numpy()
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    OL = O.Lattice(O.make_params(512, 512, eo, sigma=so, tau=TAU))
    OL.set_f(f_t)
    OL.run(1)
    f_o = OL.get_f()
    assert np.abs(f_g - f_o).max() <= _bound(lbm, prec, f_o, e.rho_v)


def _samples(n, rng):
    xs = {0, 1, 2, 60, 61, 62, 63, 64, 123, 124, 125, n - 63, n - 62, n - 2, n - 1}
    ys = {0, 1, 3, 4, 5, 7, 8, 9, n // 2, n - 5, n - 4, n - 1}
    pts = [(y, x) for y in (0, n - 1, n // 2) for x in sorted(xs)]
    pts += [(y, x) for y in sorted(ys) for x in (0, 62, n // 2 + 7, n - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, n, size=2)) for _ in range(40)]
    # nodes on the droplet rim (all EOS branches)
    R = n // 6
    for k in range(24):
        a = 2 * np.pi * k / 24
        for dr in (-12, -4, 0, 4, 12):
            pts.append((int(n / 2 + (R + dr) * np.sin(a)) % n, int(n / 2 + (R + dr) * np.cos(a)) % n))
    return sorted(set(pts))


@pytest.mark.parametrize("n,prec_name", [(8192, "fp32"), (8192, "fp64"), (16384, "fp32")])
def test_large_droplet_sampled_nodes_one_step(gpu_lib, n, prec_name):
    """8192^2 (the HBM sweep) and 16384^2 (the largest size of the roofline sweep: 21 GB of
    FP32 populations, 64-bit plane offsets with 32-bit in-plane offsets)."""
    import torch

    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    L, e = _lattice(lbm, n, n // 6, prec, 20)
    assert lbm.describe(L.P)[0] == lbm.VARIANT_MARCH  # the kernel bench.py times at this size
    pts = _samples(n, np.random.default_rng(7))
    win = np.arange(-3, 4)
    ys = torch.tensor([[(y + dy) % n for dy in win] for y, _ in pts], device="cuda:0")
    xs = torch.tensor([[(x + dx) % n for dx in win] for _, x in pts], device="cuda:0")

    def windows():
        f = L.populations()  # (9, n, n) float64 on the device
        w = f[:, ys[:, :, None], xs[:, None, :]]  # (9, npts, 7, 7)
        del f
        torch.cuda.empty_cache()
        return w.cpu().numpy()

    f_t = windows()
    L.step(1)
    f_g = windows()[:, :, 3, 3]
    L.close()
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    P = O.make_params(7, 7, eo, sigma=so, tau=TAU)
    f_o = np.empty_like(f_g)
    for k in range(len(pts)):
        OL = O.Lattice(P)
        OL.set_f(np.ascontiguousarray(f_t[:, k]))
        OL.run(1)
        f_o[:, k] = OL.get_f()[:, 3, 3]
    err = np.abs(f_g - f_o)
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= _bound(lbm, prec, f_o, e.rho_v), (pts[worst[1]], err.max())
