"""Pins for oracle/mlp.py: central finite differences against the analytic
backward, and the factor gradient against eq. (5) on the core computed with
the FFCP oracle's compressed MTTKRP and Gram identity."""

import numpy as np

from oracle import mlp as M
from oracle import ffcp as F
from oracle.tensor import hadamard_grams


def _tiny():
    g = np.random.default_rng(31)
    core = (2, 3, 2)
    R = 2
    dims = [int(np.prod(core)), 7, 5, sum(core) * R]
    params = M.init_params(g, dims)
    for k in ("b1", "b2", "b3"):
        params[k] = 0.1 * g.standard_normal(params[k].shape)
    G = g.standard_normal((3,) + core)
    G = G / np.linalg.norm(G.reshape(3, -1), axis=1)[:, None, None, None]
    return params, G


def test_backward_matches_central_differences():
    params, G = _tiny()
    _, grads = M.loss_and_backward(params, G)
    h = 1e-6
    for k in params:
        flat = params[k].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 9)):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = M.loss_and_backward(params, G)
            flat[idx] = old - h
            lm, _ = M.loss_and_backward(params, G)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, idx, fd, an)


def test_factor_gradient_is_eq5_on_core():
    g = np.random.default_rng(32)
    G = g.standard_normal((3, 4, 2))
    V = [g.standard_normal((s, 3)) for s in G.shape]
    loss, grads = M.cp_loss_and_grad(G, V)
    # loss against the dense reconstruction
    from oracle.tensor import kruskal_full
    assert abs(loss - np.sum((G - kruskal_full(V)) ** 2)) <= 1e-10
    for n in range(3):
        H = F.mttkrp_core(G, V, n)
        T = hadamard_grams(V, n)
        np.testing.assert_allclose(grads[n], 2.0 * (V[n] @ T - H),
                                   rtol=1e-12, atol=1e-12)


def test_gelu_grad_central_differences():
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    # closed values: gelu(0) = 0, gelu(x) -> x for large x
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert abs(M.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step is -lr * g / (|g| + eps')."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    st = {}
    M.adam_step(p, g, st, lr=0.1, eps=0.0)
    np.testing.assert_allclose(p["w"], [0.9, -1.9, 2.9], rtol=1e-12)
