"""FP64 CPU reference of the warm-start MLP (test infrastructure only).

Network: h_0 = x; z_l = W_l h_{l-1} + b_l; h_l = relu(z_l) for hidden layers;
the last layer is linear.  Loss: mean squared error over batch and outputs,
L = sum (y - t)^2 / (B * n_out).  Parameters are laid out layer by layer as
W_l (n_l x n_{l-1}, row-major) followed by b_l.

With ``quantize=True`` every GEMM input (weights, activations, output
gradients) is rounded to bfloat16 with round-to-nearest-even, exactly where a
BF16-input / FP32-accumulate device GEMM rounds them; everything else stays
in float64.  With ``quantize=False`` the network is the plain FP64 function,
whose gradient is pinned by central finite differences in the tests.

The warm-start network itself is not in the paper; it initialises the
potentials of the scaling iteration (Section 3), which still decides
convergence.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round-to-nearest-even on the float32 value), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray, widths: List[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    out = []
    o = 0
    for l in range(1, len(widths)):
        n_in, n_out = widths[l - 1], widths[l]
        W = params[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = params[o:o + n_out]
        o += n_out
        out.append((np.asarray(W, dtype=np.float64), np.asarray(b, dtype=np.float64)))
    if o != params.shape[0]:
        raise ValueError("parameter vector has the wrong length")
    return out


def num_params(widths: List[int]) -> int:
    return sum(widths[l] * widths[l - 1] + widths[l] for l in range(1, len(widths)))


def forward(params, widths, x, quantize=False):
    """Returns (y, cache) with cache holding pre-activations and GEMM inputs."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params, widths)
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        hin = q(h)
        Wq = q(W)
        z = hin @ Wq.T + b
        cache.append((hin, Wq, z))
        h = np.maximum(z, 0.0) if l < len(layers) - 1 else z
        if quantize:
            h = h.astype(np.float32).astype(np.float64)
    return h, cache


def loss_and_grad(params, widths, x, t, quantize=False):
    """MSE loss and its gradient with respect to the flat parameter vector."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    y, cache = forward(params, widths, x, quantize)
    B, n_out = y.shape
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.sum(r * r) / (B * n_out))
    dz = 2.0 * r / (B * n_out)
    grads = []
    L = len(cache)
    for l in range(L - 1, -1, -1):
        hin, Wq, z = cache[l]
        if l < L - 1:
            dz = dz * (z > 0)
        dzq = q(dz)
        dW = dzq.T @ hin
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if l > 0:
            dz = dzq @ Wq
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def init_params(widths: List[int], seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(1, len(widths)):
        n_in, n_out = widths[l - 1], widths[l]
        lim = np.sqrt(6.0 / n_in)
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
