"""Host-side checks of the droplet loss used with the adjoint (no GPU)."""
import math

import numpy as np
import pytest

from lbm_inputs import droplet_density


def test_width_estimate_recovers_tanh_width():
    torch = pytest.importorskip("torch")
    from paper_2107_06355_amd.rollout import vapor_width_loss

    rv, rl = 0.01, 1.0
    for W in (14.0, 20.0, 28.0):
        rho = torch.tensor(droplet_density(256, 256, rv, rl, R=60, W=W))
        # with the exact vapor density and the true width the loss vanishes to discretisation error
        L = vapor_width_loss(rho, rv, 60, W, lam_w=1.0).item()
        assert L < 1e-3, (W, L)
        # a wrong reference vapor density shows up in the first term only
        L2 = vapor_width_loss(rho, 1.1 * rv, 60, W, lam_w=0.0).item()
        assert L2 == pytest.approx((1 / 1.1 - 1) ** 2, rel=1e-5)
