"""The CPU MLP reference: gradient pinned by central finite differences,
bfloat16 rounding pinned by torch's own float32 -> bfloat16 conversion."""
import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_central_differences():
    widths = [7, 6, 5, 4]
    rng = np.random.default_rng(0)
    p = mlp.init_params(widths, seed=1) + rng.normal(0, 0.01, mlp.num_params(widths))
    x = rng.normal(size=(5, 7))
    t = rng.normal(size=(5, 4))
    loss, g = mlp.loss_and_grad(p, widths, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.shape[0]):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(p + e, widths, x, t)[0] - mlp.loss_and_grad(p - e, widths, x, t)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
    assert loss > 0


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.normal(size=10000) * 10 ** rng.uniform(-8, 8, size=10000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0])])
    ours = mlp.bf16_round(a)
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_quantized_forward_close_to_exact():
    widths = [16, 8, 8, 4]
    rng = np.random.default_rng(4)
    p = mlp.init_params(widths, seed=2)
    x = rng.normal(size=(3, 16))
    y0, _ = mlp.forward(p, widths, x, quantize=False)
    y1, _ = mlp.forward(p, widths, x, quantize=True)
    assert np.max(np.abs(y0 - y1)) <= 0.05 * max(1.0, np.max(np.abs(y0)))
    assert not np.array_equal(y0, y1)
