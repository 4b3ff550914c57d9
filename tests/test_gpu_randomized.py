"""Randomized receivers with Hessian reuse on the GPU: the multipliers of a
selection equal the oracle's for a survey on exactly those receivers, reused
factors give bitwise the same result as a fresh build, and a new selection is
built only every ``reuse`` iterations."""
import numpy as np
import pytest
import torch

import synth
from oracle import fd, hessian, solve

from parity import check  # noqa: E402

pytestmark = pytest.mark.gpu


def test_selection_matches_oracle_and_reuse_is_exact():
    from paper_2512_16642_amd import ehi, randomized as rz
    ehi.lib()
    s = synth.tiny()
    v = s.velocity()
    vel = torch.from_numpy(v).cuda()
    R = torch.from_numpy(s.residuals()).cuda()          # all 16 receivers
    h = rz.RandomizedHessian(s, n_subsets=5, reuse=3, seed=11)
    outs = []
    for it in range(6):
        idx, X = h.deblur(it, vel, R)
        outs.append((tuple(idx), X.cpu().numpy()))
    assert h.builds == 2
    assert outs[0][0] == outs[1][0] == outs[2][0] and outs[3][0] == outs[4][0]
    for it in (1, 2):
        np.testing.assert_array_equal(outs[it][1], outs[0][1])
    # oracle on the selected receivers of the first draw
    idx = np.array(outs[0][0])
    sub = h.subset_spec(idx)
    G = fd.green_dft(sub, v)
    H = hessian.hessian_r1(G)
    mu = 1e-3 * solve.lambda_max(H)
    Rs = s.residuals()[:, :, idx].astype(np.complex128)
    Xr = solve.multipliers(H, mu, Rs)
    X = outs[0][1]
    check(X, Xr, 1e-5, 1e-5, 2e-5, f"randomized selection {list(idx)} multipliers")
    h.close()
