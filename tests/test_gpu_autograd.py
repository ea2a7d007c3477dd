"""The torch.autograd.Function over rods_rollout / rods_backward: gradients
from loss.backward() equal the library's backward called directly with the
same loss gradient."""
import numpy as np
import pytest
import torch

from synth import make_workload
from tests.gpukit import to_dev

pytestmark = pytest.mark.gpu


def test_autograd_function_matches_direct_backward():
    from paper_2606_04206_amd import RodsHandle, RodsRollout
    n, K = 4, 2
    wl = make_workload(3, steps=n)
    sub = wl.subset(list(wl.oracle_rods[:4]))
    h = RodsHandle(sub, max_steps=n, ckpt_every=K)
    leaf = lambda a: to_dev(a).requires_grad_()
    x0, v0, U = leaf(sub.x0), leaf(sub.v0), leaf(sub.actions)
    b, sig = leaf(sub.rod_params[:, 2]), leaf(sub.rod_params[:, 3])
    tgt = to_dev(sub.target)
    counts = np.diff(sub.vert_offsets)
    w = to_dev(np.repeat(1.0 / (sub.n_rods * counts), counts))[:, None]
    xT = RodsRollout.apply(h, n, x0, v0, U, b, sig)
    loss = (w * (xT - tgt) ** 2).sum()
    loss.backward()
    # the same pass through the handle directly, with the same loss gradient
    gx = (2.0 * w * (xT.detach() - tgt)).contiguous()
    h.set_params(b.detach(), sig.detach())
    h.set_state(x0.detach(), v0.detach())
    xT2 = h.tensor(sub.n_vert, 3)
    h.rollout(n, U.detach(), record=True, x_final=xT2)
    assert torch.equal(xT.detach(), xT2)
    g = h.backward(gx, n_steps=n)
    for leafv, key in ((x0, "x0"), (v0, "v0"), (U, "u"), (b, "b"), (sig, "sigma")):
        assert leafv.grad is not None, key
        torch.testing.assert_close(leafv.grad, g[key], rtol=1e-6, atol=1e-12)
    assert float(loss) > 0 and torch.isfinite(x0.grad).all()
