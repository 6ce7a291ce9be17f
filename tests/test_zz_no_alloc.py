"""lbm_init_static (the entry point that allocates nothing) against lbm_init with a caller workspace.

Both contexts run the same kernels, so the populations and the FP64 reduction history agree bit
for bit.  Two calls in a row: a 300 x 200 walled droplet-on-film lattice in FP64 with reductions,
then a smaller 130 x 70 periodic droplet in FP32-shifted (the second call re-initialises the
device's static context and reuses its workspace).  A lattice whose workspace exceeds the static
array is refused before anything runs.
"""
import ctypes as C

import numpy as np
import pytest

from lbm_inputs import droplet_density, droplet_on_film

pytestmark = pytest.mark.gpu

SMOOTH = dict(base=0, a=0.5, b=4.0, R=1.0, Tr=0.6, shape=1, alpha=0.6, k_vap=4.0)


def _pair(lbm, P, rho, ux=None, uy=None, steps=57):
    ref = lbm.Lattice(P, rho, ux, uy, device="cuda:0")
    ref.step(steps)
    ref.check()
    st = lbm.Lattice(P, rho, ux, uy, device="cuda:0", static_workspace=True)
    assert st.ws is None
    st.step(steps)
    st.check()
    out = (ref.populations().cpu().numpy(), st.populations().cpu().numpy(), ref.history(), st.history(),
           ref.macros()["mass_mom"], st.macros()["mass_mom"])
    ref.close()
    st.close()
    return out


def test_static_workspace_matches_caller_workspace_two_calls(gpu_lib):
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**SMOOTH))
    # first call: walls, FP64, reductions every 10 steps (partials, block sums and history in the scratch)
    nx, ny = 300, 200
    rho, ux, uy = droplet_on_film(nx, ny, e.rho_v, e.rho_l, R=30, h=20, gap=3, V=0.05, W=6)
    P = lbm.make_params(nx, ny, e, sigma=s, prec=lbm.FP64, walls=True, rho_wall_lo=e.rho_l, rho_wall_hi=e.rho_v,
                        reduce_every=10)
    f_ref, f_st, h_ref, h_st, mm_ref, mm_st = _pair(lbm, P, rho, ux, uy)
    assert np.array_equal(f_ref, f_st)
    assert h_ref.shape[0] == 6 and np.array_equal(h_ref, h_st)
    assert mm_ref == mm_st
    # second call, smaller lattice, FP32-shifted, reductions every 7 steps
    nx, ny = 130, 70
    rho = droplet_density(nx, ny, e.rho_v, e.rho_l, R=15, W=5)
    P = lbm.make_params(nx, ny, e, sigma=s, prec=lbm.FP32_SHIFTED, reduce_every=7)
    f_ref, f_st, h_ref, h_st, mm_ref, mm_st = _pair(lbm, P, rho)
    assert np.array_equal(f_ref, f_st)
    assert h_ref.shape[0] == 9 and np.array_equal(h_ref, h_st)
    assert mm_ref == mm_st


def test_static_workspace_refuses_a_lattice_beyond_its_size(gpu_lib):
    lbm = gpu_lib
    e, s = lbm.eos_build(lbm.make_eos(**SMOOTH))
    P = lbm.make_params(8192, 8192, e, sigma=s, prec=lbm.FP32_SHIFTED)
    assert lbm.layout(P)[2] > 16 << 20
    import torch

    h = C.c_void_p(0)
    # refused on the size check before anything runs: the buffers are never touched
    a, b, r = (torch.empty(64, dtype=torch.float64, device="cuda:0") for _ in range(3))
    code = lbm.load().lbm_init_static(C.byref(h), C.byref(P), a.data_ptr(), b.data_ptr(), r.data_ptr(), None, None,
                                      None)
    torch.cuda.synchronize()
    assert code == lbm.LBM_EINVAL and not h.value
    assert b"16777216" in lbm.load().lbm_last_error()
