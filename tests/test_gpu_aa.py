"""The in-place AA variant (LBM_VARIANT_AA): one population buffer, even steps in the natural
layout, odd steps in the swapped one.  Element-wise parity with the oracle runs in
test_gpu_parity.py (ragged and 1-wide lattices, walls, every EOS branch, odd step counts) and
at full length in test_gpu_fullsize_parity.py; here: what is specific to the in-place update.
"""
import numpy as np
import pytest

from lbm_inputs import droplet_density, droplet_on_film

pytestmark = pytest.mark.gpu

TAU = [1.0, 1.1, 1.2, 1.0, 1.1, 1.0, 1.1, 0.8, 0.8]


def _case(lbm, walls, nx=150, ny=44):
    e, s = lbm.eos_build(lbm.make_eos(base=0, a=0.387, Tr=0.6, shape=1, alpha=0.834, k_vap=2 / 0.387))
    if walls:
        rho0, ux0, uy0 = droplet_on_film(nx, ny, e.rho_v, e.rho_l, R=9, h=6, gap=3, V=0.05, W=4)
        extra = dict(walls=True, rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v)
    else:
        rho0, ux0, uy0 = droplet_density(nx, ny, e.rho_v, e.rho_l, R=12, W=4), None, None
        extra = {}
    return e, s, rho0, ux0, uy0, extra


@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "walls"])
@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_aa_equals_pull_variant(gpu_lib, walls, prec_name):
    """The same node arithmetic as the two-buffer row-block variant, so after 1, 2 and 61 steps the
    populations, the macroscopic fields and the FP64 reduction history agree with it up to FMA
    contraction: 1e-13 of the largest population in FP64; in FP32-shifted storage 1e-6 per step of
    the largest deviation from w rho_v (a few roundings of 2^-24), and the mass history to 1e-12."""
    lbm = gpu_lib
    prec = lbm.FP32_SHIFTED if prec_name == "fp32" else lbm.FP64
    e, s, rho0, ux0, uy0, extra = _case(lbm, walls)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    for steps in (1, 2, 61):
        out = {}
        for v in (lbm.VARIANT_BLOCK, lbm.VARIANT_AA):
            P = lbm.make_params(150, 44, e, sigma=s, tau=TAU, prec=prec, reduce_every=7, kernel_variant=v, **extra)
            L = lbm.Lattice(P, rho0, ux0, uy0, device="cuda:0")
            L.step(steps)
            L.check()
            m = L.macros()
            out[v] = (L.populations().cpu().numpy(), m["rho"].cpu().numpy(), m["ux"].cpu().numpy(), L.history())
            L.close()
        fb, fa = out[lbm.VARIANT_BLOCK][0], out[lbm.VARIANT_AA][0]
        if prec == lbm.FP64:
            bound = 1e-13 * np.abs(fb).max()
        else:
            bound = steps * 1e-6 * np.abs(fb - w * e.rho_v).max()
        assert np.abs(fa - fb).max() <= bound, (steps, np.abs(fa - fb).max(), bound)
        hb, ha = out[lbm.VARIANT_BLOCK][3], out[lbm.VARIANT_AA][3]
        assert hb.shape == ha.shape and np.array_equal(hb[:, 0], ha[:, 0])
        assert np.abs(ha[:, 1] / hb[:, 1] - 1).max() <= 1e-12


@pytest.mark.parametrize("t_save", [6, 7], ids=["even", "odd"])
def test_aa_save_and_load_keep_the_layout(gpu_lib, t_save):
    """lbm_save copies the buffer as it lies (natural layout after an even step count, swapped after
    an odd one) and lbm_load with the same step continues bit for bit."""
    lbm = gpu_lib
    e, s, rho0, ux0, uy0, extra = _case(lbm, True)
    P = lbm.make_params(150, 44, e, sigma=s, tau=TAU, prec=lbm.FP32_SHIFTED, kernel_variant=lbm.VARIANT_AA, **extra)
    L = lbm.Lattice(P, rho0, ux0, uy0, device="cuda:0")
    L.step(t_save)
    buf, step = L.save()
    assert step == t_save and L.state()[1] == 0
    L.step(9)
    a = L.populations().cpu().numpy()
    L.load_state(buf, step)
    L.step(9)
    L.check()
    assert np.array_equal(a, L.populations().cpu().numpy())
    L.close()


def test_aa_has_one_buffer_and_no_adjoint(gpu_lib):
    """The AA lattice holds one population buffer; recording and checkpointing (the adjoint's
    inputs) are refused with LBM_EINVAL."""
    lbm = gpu_lib
    e, s, rho0, _, _, _ = _case(lbm, False, 64, 32)
    P = lbm.make_params(64, 32, e, sigma=s, tau=TAU, kernel_variant=lbm.VARIANT_AA)
    L = lbm.Lattice(P, rho0, device="cuda:0")
    assert len(L.f) == 1
    for enable in (lambda: L.enable_checkpointing(4, 8), lambda: L.enable_recording(8)):
        with pytest.raises(lbm.LbmError) as ei:
            enable()
        assert ei.value.code == lbm.LBM_EINVAL
    L.step(3)
    L.check()
    L.close()
