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


def test_autograd_function_with_moving_spheres():
    """With the spheres' start state as an input: its gradient equals the
    library's body adjoint from the same loss gradient (zero cotangent on
    the spheres' final state), and a second call starts from body0 again."""
    from paper_2606_04206_amd import RodsHandle, RodsRollout
    n, K = 4, 2
    wl = make_workload(7, steps=n)
    sub = wl.subset(list(wl.oracle_rods[:4]))
    h = RodsHandle(sub, max_steps=n, ckpt_every=K)
    leaf = lambda a: to_dev(a).requires_grad_()
    body = np.zeros((len(sub.prim_type), 9))
    body[:, :3] = sub.prim_a
    body[:, 5] = 0.2
    x0, v0, U = leaf(sub.x0), leaf(sub.v0), leaf(sub.actions)
    b, sig, b0 = leaf(sub.rod_params[:, 2]), leaf(sub.rod_params[:, 3]), leaf(body)
    tgt = to_dev(sub.target)
    counts = np.diff(sub.vert_offsets)
    w = to_dev(np.repeat(1.0 / (sub.n_rods * counts), counts))[:, None]
    xT = RodsRollout.apply(h, n, x0, v0, U, b, sig, None, b0)
    loss = (w * (xT - tgt) ** 2).sum()
    loss.backward()
    assert b0.grad is not None and b0.grad.abs().max() > 0
    gx = (2.0 * w * (xT.detach() - tgt)).contiguous()
    h.set_params(b.detach(), sig.detach())
    h.set_state(x0.detach(), v0.detach())
    h.set_bodies(b0.detach())
    h.set_body_adjoint(None)
    xT2 = h.tensor(sub.n_vert, 3)
    h.rollout(n, U.detach(), record=True, x_final=xT2)
    assert torch.equal(xT.detach(), xT2)
    g = h.backward(gx, n_steps=n)
    torch.testing.assert_close(b0.grad, h.get_body_adjoint(), rtol=1e-6, atol=1e-12)
    for leafv, key in ((x0, "x0"), (U, "u"), (b, "b")):
        torch.testing.assert_close(leafv.grad, g[key], rtol=1e-6, atol=1e-12)
    # a second call restarts the spheres from body0
    xT3 = RodsRollout.apply(h, n, x0, v0, U, b, sig, None, b0)
    assert torch.equal(xT3.detach(), xT.detach())
