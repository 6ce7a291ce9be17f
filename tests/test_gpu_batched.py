"""Batched lattices against the oracle, in both launch modes: persistent (one workgroup per
lattice looping over the steps) and grouped (one launch per step over every lattice's rows)."""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import batched_planar_recipe, droplet_density, droplet_on_film, planar_density

pytestmark = pytest.mark.gpu

PR = dict(base=1, a=2 / 49, b=2 / 21, omega=0.344, scale=0.25, shape=1, alpha=0.3, k_vap=4.0)


def _cases():
    """Mixed sizes, EOS, walls and relaxation: (eos kwargs, nx, ny, extra params, rho0, u0)."""
    out = []
    out.append((dict(Tr=0.7), 256, 4, {}, "planar-x"))
    out.append((dict(Tr=0.6, a=0.387, shape=1, alpha=0.834, k_vap=2 / 0.387), 130, 37, {}, "droplet"))
    out.append((dict(PR, Tr=0.5), 70, 5, {}, "planar-x"))
    out.append((dict(Tr=0.6), 64, 40, {"walls": True, "var_tau": True}, "film"))
    out.append((dict(PR, Tr=0.8), 2, 200, {}, "planar-y"))
    return out


def _rho0(kind, e, nx, ny):
    if kind == "planar-x":
        return planar_density(nx, ny, e.rho_v, e.rho_l, W=8, axis=0), None, None
    if kind == "planar-y":
        return planar_density(nx, ny, e.rho_v, e.rho_l, W=8, axis=1), None, None
    if kind == "droplet":
        return droplet_density(nx, ny, e.rho_v, e.rho_l, R=10, W=6), None, None
    return droplet_on_film(nx, ny, e.rho_v, e.rho_l, R=8, h=6, gap=3, V=0.0, W=6)


def _params(lbm, e, s, nx, ny, extra, prec):
    tau = [1.0, 1.1, 1.2, 1.0, 1.1, 1.0, 1.1, 0.8, 0.8]
    kw = {}
    if extra.get("walls"):
        kw.update(walls=True, rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v)
    if extra.get("var_tau"):
        kw.update(var_tau=True, tau_l=0.8, tau_v=0.5 + 3 * 0.3)
    return lbm.make_params(nx, ny, e, sigma=s, tau=tau, prec=prec, **kw), tau, kw


def _oracle(kw_eos, nx, ny, extra, tau, kw, rho0, steps):
    eo, so = O.eos_build(O.make_eos(**kw_eos))
    OP = O.make_params(nx, ny, eo, sigma=so, tau=tau, **kw)
    L = O.Lattice(OP)
    L.init_eq(rho0)
    L.run(steps)
    return L.macros()


MODES = [("persistent", 1), ("grouped", 2)]


@pytest.mark.parametrize("mode", [m for _, m in MODES], ids=[n for n, _ in MODES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_mixed_lattices_match_oracle(gpu_lib, prec, mode):
    lbm = gpu_lib
    P, rhos, meta = [], [], []
    pr = lbm.FP64 if prec == "fp64" else lbm.FP32_SHIFTED
    for kw_eos, nx, ny, extra, kind in _cases():
        e, s = lbm.eos_build(lbm.make_eos(**kw_eos))
        p, tau, kw = _params(lbm, e, s, nx, ny, extra, pr)
        r0, _, _ = _rho0(kind, e, nx, ny)
        P.append(p)
        rhos.append(r0)
        meta.append((kw_eos, nx, ny, extra, tau, kw))
    Bt = lbm.Batch(P, rhos, device="cuda:0")
    Bt.set_mode(mode)
    steps = 200
    Bt.step(25)
    Bt.step(35)  # a second, different launch (new graph)
    Bt.step(140)  # grouped: two 64-step graph replays and 12 direct launches
    Bt.check()
    got = Bt.macros()
    for b, (kw_eos, nx, ny, extra, tau, kw) in enumerate(meta):
        m = _oracle(kw_eos, nx, ny, extra, tau, kw, rhos[b], steps)
        err = np.abs(got[b]["rho"] - m["rho"]).max() / m["rho"].max()
        uerr = max(np.abs(got[b]["ux"] - m["ux"]).max(), np.abs(got[b]["uy"] - m["uy"]).max())
        if prec == "fp64":
            assert err < 1e-12, (b, err)
            assert uerr < 1e-12, (b, uerr)
        else:
            assert err < 2e-5, (b, err)
            assert uerr < 1e-5, (b, uerr)


@pytest.mark.parametrize("mode", [m for _, m in MODES], ids=[n for n, _ in MODES])
def test_batched_graph_replay_is_deterministic(gpu_lib, mode):
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**dict(PR, Tr=0.6)))
    P = [lbm.make_params(n, 4, e, sigma=s, prec=lbm.FP32_SHIFTED) for n in (128, 300, 62, 63)]
    rhos = [planar_density(p.nx, 4, e.rho_v, e.rho_l, W=10, axis=0) for p in P]
    a = lbm.Batch(P, rhos, device="cuda:0")
    b = lbm.Batch(P, rhos, device="cuda:0")
    a.set_mode(mode)
    b.set_mode(mode)
    if mode == 1:
        for _ in range(3):
            a.step(71)       # replayed graph, odd step count (buffer parity flips)
        b.step(213)
    else:
        for n in (128, 128, 7):  # the 128-step graph captured, then replayed; 3 two-step + 1 one-step launches
            a.step(n)
        b.step(263)              # the same launches: two graph replays, then the same tail
    ma, mb = a.macros(), b.macros()
    for x, y in zip(ma, mb):
        assert np.array_equal(x["rho"], y["rho"]) and np.array_equal(x["ux"], y["ux"])


FULL_SHAPES = {
    # the tallest lattice picks the workgroup's LDS size: 4, 8 or 16 rows
    "rows4": [(130, 3), (7, 1), (200, 4), (59, 2)],
    "rows8": [(130, 3), (61, 8), (7, 5), (200, 1)],
    "rows16": [(130, 3), (61, 16), (7, 5), (200, 1), (59, 4)],
}


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
@pytest.mark.parametrize("rows", sorted(FULL_SHAPES))
def test_batched_short_periodic_lattices_full_height(gpu_lib, rows, prec_name):
    """Batches of periodic lattices no taller than 16 rows run two steps per launch with whole
    columns per workgroup (rows wrap inside it): 1 to 16 rows, ragged strips, odd step counts
    (a final one-step launch), against the oracle."""
    lbm = gpu_lib
    shapes = FULL_SHAPES[rows]
    prec = lbm.FP64 if prec_name == "fp64" else lbm.FP32_SHIFTED
    kw = dict(Tr=0.7)
    e, s = lbm.eos_build(lbm.make_eos(**kw))
    tau = [1.0, 1.1, 1.2, 1.0, 1.1, 1.0, 1.1, 0.8, 0.8]
    P = [lbm.make_params(nx, ny, e, sigma=s, tau=tau, prec=prec) for nx, ny in shapes]
    rhos = [planar_density(nx, ny, e.rho_v, e.rho_l, W=6, axis=0) * (1 + 0.01 * np.sin(np.arange(ny)[:, None] + 0.3 * np.arange(nx)[None, :]))
            for nx, ny in shapes]
    Bt = lbm.Batch(P, rhos, device="cuda:0")
    Bt.set_mode(2)
    for n in (1, 2, 131):
        Bt.step(n)
    Bt.check()
    got = Bt.macros()
    for b, (nx, ny) in enumerate(shapes):
        m = _oracle(kw, nx, ny, {}, tau, {}, rhos[b], 134)
        err = np.abs(got[b]["rho"] - m["rho"]).max() / m["rho"].max()
        assert err < (1e-12 if prec == lbm.FP64 else 2e-5), (nx, ny, err)


def test_batched_modes_agree(gpu_lib):
    """The two launch modes (and the automatic choice, grouped here: the 2044 x 4 lattice gives its
    persistent workgroup 33 strips x 4 rows per step) run the same node arithmetic (FP64)."""
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**dict(PR, Tr=0.6)))
    P = [lbm.make_params(n, 4, e, sigma=s) for n in (2044, 130, 8)]
    rhos = [planar_density(p.nx, 4, e.rho_v, e.rho_l, W=10, axis=0) for p in P]
    out = []
    for mode in (1, 2, 0):
        Bt = lbm.Batch(P, rhos, device="cuda:0")
        Bt.set_mode(mode)
        Bt.step(150)
        Bt.check()
        out.append(Bt.macros())
    for b in range(len(P)):
        for k in ("rho", "ux", "uy"):
            scale = np.abs(out[0][b][k]).max() + 1e-300
            assert np.abs(out[0][b][k] - out[1][b][k]).max() <= 1e-13 * scale, (b, k)
            assert np.array_equal(out[1][b][k], out[2][b][k]), (b, k)


def test_batched_coexistence_sweep(gpu_lib):
    """A reduced version of the uneven batched sweep: shaped PR, Tr in [0.35, 0.95], FP32-shifted."""
    lbm = gpu_lib
    lengths, trs = batched_planar_recipe(n_lattices=12, seed=0, L_lo=32, L_hi=128)
    P, rhos, eos = [], [], []
    for L, Tr in zip(lengths, trs):
        e, s = lbm.eos_build(lbm.make_eos(**dict(PR, Tr=Tr)))
        P.append(lbm.make_params(L, 4, e, sigma=s, prec=lbm.FP32_SHIFTED))
        rhos.append(planar_density(L, 4, e.rho_v, e.rho_l, W=20, axis=0))
        eos.append(e)
    Bt = lbm.Batch(P, rhos, device="cuda:0")
    Bt.step(3000)
    Bt.check()
    got = Bt.macros()
    for b, (L, Tr) in enumerate(zip(lengths, trs)):
        m = _oracle(dict(PR, Tr=Tr), L, 4, {}, [1.0] * 9, {}, rhos[b], 3000)
        rv_g, rv_o = got[b]["rho"][0, 0], m["rho"][0, 0]
        rl_g, rl_o = got[b]["rho"][0, L // 2], m["rho"][0, L // 2]
        assert abs(rv_g - rv_o) / rv_o <= 1e-3, (b, Tr, rv_g, rv_o)
        assert abs(rl_g - rl_o) / rl_o <= 1e-5, (b, Tr, rl_g, rl_o)


def test_batched_reports_the_unstable_lattice(gpu_lib):
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(Tr=0.7))
    ep, _ = lbm.eos_build(lbm.make_eos(base=1, a=2 / 49, b=2 / 21, omega=0.344, Tr=0.5))
    P = [lbm.make_params(64, 4, e, sigma=s), lbm.make_params(8, 8, ep), lbm.make_params(64, 4, e, sigma=s)]
    rhos = [planar_density(64, 4, e.rho_v, e.rho_l, W=8, axis=0), np.full((8, 8), 1.1 * ep.rho_l),
            planar_density(64, 4, e.rho_v, e.rho_l, W=8, axis=0)]
    Bt = lbm.Batch(P, rhos, device="cuda:0")
    Bt.step(3)
    with pytest.raises(lbm.LbmError) as ei:
        Bt.check()
    assert ei.value.code == lbm.LBM_EUNSTABLE
    assert "lattice 1" in str(ei.value)
