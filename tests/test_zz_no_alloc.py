"""The allocation-free forward pass of the warm-start network against the
ordinary one, through the C ABI (needs an MI355X).

gmot_mlp_forward_static keeps its activations in a static device workspace
instead of the network's own buffers; it runs the same kernels on the same
inputs, so its outputs must equal gmot_mlp_forward_dev's bit for bit.  Two
calls in a row (the second with a smaller batch, so stale rows of the first
stay in the workspace), a second network of another shape on the same
workspace, and a batch too large for the workspace (refused with a message).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def _run(net, x, static):
    y = torch.full((x.shape[0], net.widths[-1]), float("nan"), dtype=torch.float32, device="cuda")
    if static:
        net.forward_static(x, y)
    else:
        net.forward(x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_static_forward_equals_forward_twice_then_smaller(ctx):
    from paper_2406_10849_amd import MLP
    net = MLP(ctx, [8192, 512, 512, 512, 8192], seed=11)
    rng = np.random.default_rng(11)
    for batch in (256, 40):
        x = torch.from_numpy(rng.normal(size=(batch, 8192)).astype(np.float32)).cuda()
        ref = _run(net, x, static=False)
        got = _run(net, x, static=True)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)


def test_static_forward_other_shape_same_workspace(ctx):
    from paper_2406_10849_amd import MLP
    net = MLP(ctx, [96, 64, 40, 72], seed=12)
    rng = np.random.default_rng(12)
    x = torch.from_numpy(rng.normal(size=(24, 96)).astype(np.float32)).cuda()
    assert np.array_equal(_run(net, x, static=True), _run(net, x, static=False))


def test_static_forward_refuses_a_batch_that_does_not_fit(ctx):
    from paper_2406_10849_amd import MLP, GmotError, GMOT_EINVAL
    net = MLP(ctx, [8192, 512, 512, 512, 8192], seed=13)
    x = torch.zeros((1024, 8192), dtype=torch.float32, device="cuda")
    y = torch.zeros((1024, 8192), dtype=torch.float32, device="cuda")
    with pytest.raises(GmotError) as ei:
        net.forward_static(x, y)
    assert ei.value.code == GMOT_EINVAL
    assert "rows fit" in str(ei.value)
