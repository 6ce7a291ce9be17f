"""Parity at the benchmark's sizes, in the launch configurations bench.py times.

512x512 (the timed workload): the whole field after one two-step launch (the kernel the
benchmark times) and after one single step (the row-block kernel that runs the reduction
steps), each against the oracle from the same populations.  8192x8192 and 16384x16384
(the roofline sweep): sampled nodes.  One step moves information at most two nodes (the
pull, then psi of the neighbours in Eq. ShanChenForce), so after s steps the populations
at x depend only on the populations within distance 2s of x.  For each sampled x the
oracle steps a (4s+3)-wide periodic window centred on x, whose wrap-around cannot reach
the centre (edge nodes the cut makes unphysical carry NaN, which would show at the centre
if it could), and its centre must equal the GPU result at x.  Samples cover the edges of the
62-column strips and 58-column tiles, band and tile-row edges, the lattice corners
(periodic wrap), the droplet rim and random nodes.
"""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import STATIC_DROPLET_512, droplet_density

pytestmark = pytest.mark.gpu

EOS_KW = STATIC_DROPLET_512["eos"]
TAU = [1, 1, 1, 1, 1, 1, 1, 0.7, 0.7]
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _bound(lbm, prec, f_o, rho_v, steps=1):
    if prec == lbm.FP64:
        return 1e-12 * np.abs(f_o).max()
    return steps * 2e-6 * np.abs(f_o - W9.reshape((9,) + (1,) * (f_o.ndim - 1)) * rho_v).max()


# FP32-shifted: relative density error per step allowed on vapor nodes.  The whole-field bound above
# is set by the liquid's deviations from w rho_v; this one looks at the vapor alone.  A vapor node's
# populations deviate little from w rho_v, so their FP32 rounding (2^-24 of the deviation) is far
# below 1e-7 of rho_v; what reaches the vapor density is the FP32 rounding of psi near the interface
# entering the force, of order 2^-24 |G| psi^2 per step, which stays below 1e-6 of rho_v.
VAPOR_REL_PER_STEP = 1e-6


def _check_vapor(lbm, prec, f_g, f_o, e, steps):
    """Relative density error on the vapor nodes (rho below the Maxwell mid density)."""
    if prec == lbm.FP64:
        return
    rg, ro = f_g.sum(axis=0), f_o.sum(axis=0)
    vap = ro < 0.5 * (e.rho_v + e.rho_l)
    err = (np.abs(rg - ro) / ro)[vap].max()
    assert err <= min(1e-3, VAPOR_REL_PER_STEP * steps), err


def _lattice(lbm, n, R, prec, steps, variant=0):
    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    rho0 = droplet_density(n, n, e.rho_v, e.rho_l, R=R, W=20)
    P = lbm.make_params(n, n, e, sigma=s, tau=TAU, prec=prec, reduce_every=100, kernel_variant=variant)
    L = lbm.Lattice(P, rho0, device="cuda:0")
    L.step(steps)
    L.check()
    return L, e


@pytest.mark.parametrize("steps", [2, 1], ids=["two-step-launch", "one-step-launch"])
@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_512_droplet_whole_field(gpu_lib, prec_name, steps):
    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    L, e = _lattice(lbm, 512, 80, prec, 300)
    assert lbm.describe(L.P)[0] == lbm.VARIANT_BLOCK2  # the kernel bench.py times at this size
    f_t = L.populations().cpu().numpy()
    L.step(steps)  # two steps: one k_step2_blk launch; one step: one k_step_blk launch
    L.check()
    f_g = L.populations().cpu().numpy()
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    OL = O.Lattice(O.make_params(512, 512, eo, sigma=so, tau=TAU))
    OL.set_f(f_t)
    OL.run(steps)
    f_o = OL.get_f()
    assert np.abs(f_g - f_o).max() <= _bound(lbm, prec, f_o, e.rho_v, steps)
    _check_vapor(lbm, prec, f_g, f_o, e, steps)


@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_512_droplet_whole_field_100_steps(gpu_lib, prec_name):
    """The bench's 512^2 droplet from its initial state through 100 steps as bench.py runs them (a
    reduction at step 0, 49 two-step launches, then a two-step launch whose second step reduces),
    whole field against 100 oracle steps from the same initial populations."""
    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    L, e = _lattice(lbm, 512, 80, prec, 0)
    f0 = L.populations().cpu().numpy()
    L.step(101)
    L.check()
    f_g = L.populations().cpu().numpy()
    assert L.history().shape[0] == 2  # steps 0 and 100 reduced
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    OL = O.Lattice(O.make_params(512, 512, eo, sigma=so, tau=TAU))
    OL.set_f(f0)
    OL.run(101)
    f_o = OL.get_f()
    assert np.abs(f_g - f_o).max() <= _bound(lbm, prec, f_o, e.rho_v, 101)
    _check_vapor(lbm, prec, f_g, f_o, e, 101)


def _samples(n, rng):
    xs = {0, 1, 2, 57, 58, 60, 61, 62, 63, 64, 115, 116, 123, 124, 125, n - 63, n - 62, n - 2, n - 1}
    ys = {0, 1, 3, 4, 5, 7, 8, 9, 10, 11, 19, 20, n // 2, n - 5, n - 4, n - 1}
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


@pytest.mark.parametrize("n,prec_name,variant,steps", [(8192, "fp32", 0, 2), (8192, "fp64", 0, 2),
                                                      (16384, "fp32", 0, 2), (8192, "fp32", 1, 1)],
                         ids=["8192-fp32", "8192-fp64", "16384-fp32", "8192-fp32-march"])
def test_large_droplet_sampled_nodes(gpu_lib, n, prec_name, variant, steps):
    """8192^2 (the HBM sweep) and 16384^2 (the largest size of the roofline sweep: 21 GB of
    FP32 populations, 64-bit plane offsets with 32-bit in-plane offsets) after one launch of
    the two-step kernel the sweep times, and one row-march step (the large walled lattices)."""
    import torch

    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    L, e = _lattice(lbm, n, n // 6, prec, 20, variant)
    assert lbm.describe(L.P)[0] == (lbm.VARIANT_BLOCK2 if variant == 0 else variant)
    pts = _samples(n, np.random.default_rng(7))
    rad = 2 * steps + 1
    win = np.arange(-rad, rad + 1)
    ys = torch.tensor([[(y + dy) % n for dy in win] for y, _ in pts], device="cuda:0")
    xs = torch.tensor([[(x + dx) % n for dx in win] for _, x in pts], device="cuda:0")

    def windows():
        f = L.populations()  # (9, n, n) float64 on the device
        w = f[:, ys[:, :, None], xs[:, None, :]]  # (9, npts, 7, 7)
        del f
        torch.cuda.empty_cache()
        return w.cpu().numpy()

    f_t = windows()
    L.step(steps)
    L.check()
    f_g = windows()[:, :, rad, rad]
    L.close()
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    P = O.make_params(len(win), len(win), eo, sigma=so, tau=TAU)
    f_o = np.empty_like(f_g)
    for k in range(len(pts)):
        OL = O.Lattice(P)
        OL.set_f(np.ascontiguousarray(f_t[:, k]))
        OL.run_window(steps)  # the cut may make edge nodes unphysical; they cannot reach the centre
        f_o[:, k] = OL.get_f()[:, rad, rad]
    assert np.isfinite(f_o).all()
    err = np.abs(f_g - f_o)
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= _bound(lbm, prec, f_o, e.rho_v, steps), (pts[worst[1]], err.max())
    _check_vapor(lbm, prec, f_g, f_o, e, steps)


# Lattices whose two-step tiles run in 8 x 8-tile patches (more than 1024 tiles, at least 16 strips
# and 16 bands) with a ragged last patch column and patch row: 1000 x 1100 periodic has 18 strips
# (last patch column 2 strips wide) and 110 FP32 bands (last patch row 6 bands); 986 x 1203 with
# walls has 17 strips (last column 1 strip wide) and 121 FP32 / 201 FP64 bands (last patch row
# 1 band).  Every tile must be updated exactly once per launch: the whole field after four
# two-step launches against eight oracle steps from the same populations.
# FP64 runs these in tiles of two rows per wavefront (9 or 10 rows); FP32 in one-row tiles on the first two,
# and in two-row tiles on 2100 x 2000 periodic (37 strips, last patch column 5 wide; 17-row tiles:
# 118 bands, the last 11 rows tall) and 2090 x 2030 with walls (37 strips; 17-row tiles, 120 bands).
@pytest.mark.parametrize("case", [(1000, 1100, False), (986, 1203, True), (2100, 2000, False), (2090, 2030, True)],
                         ids=["periodic-1000x1100", "walls-986x1203", "periodic-2100x2000", "walls-2090x2030"])
@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_patch_ordered_lattice_whole_field(gpu_lib, prec_name, case):
    lbm = gpu_lib
    nx, ny, walls = case
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    rho0 = droplet_density(nx, ny, e.rho_v, e.rho_l, R=150, W=20)
    # vapor ghosts on both walls: the bulk next to them is vapor (a liquid ghost beside vapor
    # makes psi^2 < 0 at the first step, in the oracle as well)
    kw = dict(walls=True, rho_wall_lo=e.rho_v, rho_wall_hi=e.rho_v) if walls else {}
    P = lbm.make_params(nx, ny, e, sigma=s, tau=TAU, prec=prec, reduce_every=0, **kw)
    L = lbm.Lattice(P, rho0, device="cuda:0")
    v, rows, waves = lbm.describe(P)
    assert v == lbm.VARIANT_BLOCK2
    # one-row FP32 tiles of 10 rows below 2048 columns here; two-row tiles otherwise, their height
    # chosen per lattice (at most 18 rows FP32, 10 FP64)
    if prec == lbm.FP32_SHIFTED and nx < 2048:
        assert (rows, waves) == (10, 16), (rows, waves)
    else:
        hmax, w = (18, 12) if prec == lbm.FP32_SHIFTED else (10, 8)
        assert waves == w and hmax // 2 <= rows <= hmax, (rows, waves)
    L.step(20)
    f_t = L.populations().cpu().numpy()
    L.step(8)
    L.check()
    f_g = L.populations().cpu().numpy()
    L.close()
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    okw = dict(walls=True, rho_wall_lo=eo.rho_v, rho_wall_hi=eo.rho_v) if walls else {}
    OL = O.Lattice(O.make_params(nx, ny, eo, sigma=so, tau=TAU, **okw), omp=True)
    OL.set_f(f_t)
    OL.run(8)
    f_o = OL.get_f()
    assert np.abs(f_g - f_o).max() <= _bound(lbm, prec, f_o, e.rho_v, 8)
    _check_vapor(lbm, prec, f_g, f_o, e, 8)


# Every two-row tile height runs the same per-node arithmetic; the height only changes which
# workgroup updates a node and which nodes it recomputes as its halo.  On a lattice whose bands are
# ragged for every height (1000 x 1100 periodic, 986 x 1203 between walls) the populations after
# four two-step launches are bitwise equal across heights, and the tallest against the oracle.
@pytest.mark.parametrize("case", [(1000, 1100, False), (986, 1203, True)], ids=["periodic-1000x1100", "walls-986x1203"])
@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_tile_heights_give_identical_populations(gpu_lib, prec_name, case):
    lbm = gpu_lib
    nx, ny, walls = case
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    heights = (18, 17, 15, 12, 11) if prec == lbm.FP32_SHIFTED else (10, 9, 7, 5)
    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    rho0 = droplet_density(nx, ny, e.rho_v, e.rho_l, R=150, W=20)
    kw = dict(walls=True, rho_wall_lo=e.rho_v, rho_wall_hi=e.rho_v) if walls else {}
    out = {}
    for h in heights:
        P = lbm.make_params(nx, ny, e, sigma=s, tau=TAU, prec=prec, reduce_every=0, tile_rows=h, **kw)
        L = lbm.Lattice(P, rho0, device="cuda:0")
        assert L.tile_shape() == (h, 12 if prec == lbm.FP32_SHIFTED else 8)
        if h == heights[0]:
            L.step(20)
            f_t = L.populations().cpu().numpy()
            L.step(8)
        else:
            L.step(28)
        L.check()
        out[h] = L.populations().cpu().numpy()
        L.close()
    for h in heights[1:]:
        d = np.argwhere(out[h] != out[heights[0]])
        assert d.size == 0, (h, d[:4])
    eo, so = O.eos_build(O.make_eos(**EOS_KW))
    okw = dict(walls=True, rho_wall_lo=eo.rho_v, rho_wall_hi=eo.rho_v) if walls else {}
    OL = O.Lattice(O.make_params(nx, ny, eo, sigma=so, tau=TAU, **okw), omp=True)
    OL.set_f(f_t)
    OL.run(8)
    f_o = OL.get_f()
    assert np.abs(out[heights[0]] - f_o).max() <= _bound(lbm, prec, f_o, e.rho_v, 8)
    _check_vapor(lbm, prec, out[heights[0]], f_o, e, 8)


# tile_rows = -1: lbm_init times the candidate tile shapes on the lattice's own run from its initial
# state, keeps the fastest and writes the initial state again; the 2048 x 1024 drop impact (the
# benchmark's lattice) must then match a lattice built with that height explicitly, bit for bit, after
# 100 steps with a reduction every 10 steps.
@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_timed_tile_shape_matches_the_explicit_one(gpu_lib, prec_name):
    from lbm_inputs import DROP_IMPACT_2048, drop_impact_fields, drop_impact_tau

    lbm = gpu_lib
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    r = DROP_IMPACT_2048
    e, s = lbm.eos_build(lbm.make_eos(**r["eos"]))
    rho, ux, uy = drop_impact_fields(r, e.rho_v, e.rho_l)
    res = {}
    shape = None
    for h in (-1, None):
        P = lbm.make_params(r["nx"], r["ny"], e, sigma=s, tau=drop_impact_tau(r), prec=prec, walls=True,
                            rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v, reduce_every=10,
                            tile_rows=h if h is not None else shape[0])
        L = lbm.Lattice(P, rho, ux, uy, device="cuda:0")
        if h == -1:
            shape = L.tile_shape()
            print("# %s timed tile shape: %d rows, %d wavefronts" % (prec_name, *shape))
            if prec == lbm.FP32_SHIFTED:
                assert shape in [(10, 16)] + [(k, 12) for k in range(14, 19)], shape
            else:
                assert shape in [(k, 8) for k in range(7, 11)], shape
        else:
            assert L.tile_shape() == shape
        L.step(100)
        L.check()
        res[h] = (L.populations().cpu().numpy(), L.history())
        L.close()
    assert np.array_equal(res[-1][0], res[None][0])
    # same tiles, same order of the partial sums: the reductions agree bit for bit as well
    assert np.array_equal(res[-1][1], res[None][1])


@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_two_step_reductions_past_one_launch_match_one_step(gpu_lib, prec_name):
    """A reducing two-step launch leaves one FP64 partial per tile; up to 16384 of them are summed in
    one launch, more in two passes.  On an 8192 x 2304 lattice (18,176 FP32 tiles of 58 x 18, 32,802
    FP64 tiles of 58 x 10: the two-pass path) the history rows equal those of one-step launches (per-wave
    partials, another summation order) to the bounds of the small-lattice test."""
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**EOS_KW))
    nx, ny = 8192, 2304
    rho0 = droplet_density(nx, ny, e.rho_v, e.rho_l, R=600, W=20)
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    h = []
    for variant in (lbm.VARIANT_BLOCK2, lbm.VARIANT_BLOCK):
        P = lbm.make_params(nx, ny, e, sigma=s, tau=TAU, prec=prec, reduce_every=2, kernel_variant=variant)
        L = lbm.Lattice(P, rho0, device="cuda:0")
        if variant == lbm.VARIANT_BLOCK2:
            rows, _ = L.tile_shape()
            assert -(-nx // 58) * -(-ny // rows) > 16384, rows
        L.step(5)
        L.check()
        h.append(L.history())
        L.close()
    assert h[0].shape == h[1].shape == (3, 4)
    np.testing.assert_array_equal(h[0][:, 0], [0, 2, 4])
    np.testing.assert_array_equal(h[1][:, 0], [0, 2, 4])
    m = h[1][0, 1]
    tol = 1e-13 if prec == lbm.FP64 else 1e-9
    assert np.abs(h[0][:, 1] - h[1][:, 1]).max() <= tol * m, h[0][:, 1] - h[1][:, 1]
    assert np.abs(h[0][:, 2:] - h[1][:, 2:]).max() <= (1e-12 if prec == lbm.FP64 else 1e-8) * m
