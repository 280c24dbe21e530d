"""Pin of the oracle's analytic gradient at the autograd workload's scale:
200k Gaussians (SH degree 3) on a 100 m city patch, 800x800 view.  For 64
seeded Gaussians, every parameter's derivative of L = sum(w * I) is
compared with central differences (h = 1e-4) of the oracle's own FP64
forward (a quantity defined without the backward), skipping components
whose two evaluations take a different blend decision."""
import numpy as np

import oracle
from gen import scenes

import fd_util as F


def test_oracle_gradient_matches_central_differences_at_c3_scale():
    g, cam = scenes.config3()
    pick, valid, rect = F.pick_gaussians(g, cam, 64, seed=33)
    w = F.loss_weights(g, cam, pick, rect, seed=34)
    fd, skipped = F.central_differences(g, cam, pick, valid, rect, w)
    assert skipped <= 0.05 * 64 * 59
    ys, xs = np.nonzero((w != 0).any(0))
    rb = oracle.backward(g, cam, w, xs.astype(np.int32), ys.astype(np.int32))
    got, want = F.gather(rb, fd)
    for k in F.PARAMS:
        scale = np.abs(want[k]).max()
        np.testing.assert_allclose(got[k], want[k], rtol=1e-5, atol=1e-6 * scale, err_msg=k)
