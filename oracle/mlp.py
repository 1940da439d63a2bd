"""Learned FFCP initializer: a 3-layer MLP that maps a normalized Tucker core
to CP factors of that core, trained by the CP reconstruction loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; the network is an addition that serves
Alg. 1's initialization step.  Its training loss is the CP objective of the
core, and its gradient with respect to the predicted factors is eq. (5)
applied to the core (eq. (17) shows FFCP on an orthonormal Tucker format is
CP of the core):

  x      = vec(G) / ||G||                        (row-major, length prod R_n)
  h1     = gelu(x W1 + b1)        gelu(z) = z Phi(z)   (exact, erf form)
  h2     = gelu(h1 W2 + b2)
  y      = h2 W3 + b3             y = [vec V_1, ..., vec V_N], V_n: R_n x R
  loss   = || G/||G|| - [[V_1..V_N]] ||^2         (per sample; batch mean)
  dL/dV_n = 2 (V_n (hadamard_{p!=n} V_p^T V_p) - Ghat_(n) KR_{p!=n} V_p)

The initial factors handed to FFCP are V_n ||G||^(1/N) and A_n = U_n V_n.

``bf16`` (optional) is a rounding function applied where the GPU rounds:
every operand of a BF16 matrix product (weights, the activations, and in the
backward pass the output gradient and the pre-activation gradients), so a
GPU comparison consumes the same rounded values.

Pins: tests/test_oracle_mlp.py (central finite differences of the loss vs
the analytic backward; dL/dV equal to eq. (5) computed with the FFCP
oracle's MTTKRP and Gram identity).
"""

import math

import numpy as np

from .tensor import unfold, khatri_rao


def _erf(x):
    v = np.vectorize(math.erf, otypes=[np.float64])
    return v(x)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def cp_loss_and_grad(Ghat, V):
    """loss = ||Ghat - [[V]]||^2 and dloss/dV_n (eq. 5 on the core)."""
    N = Ghat.ndim
    R = V[0].shape[1]
    grams = [v.T @ v for v in V]
    H = [unfold(Ghat, n) @ khatri_rao([V[p] for p in range(N) if p != n])
         for n in range(N)]
    had = np.ones((R, R))
    for g in grams:
        had = had * g
    loss = float(np.sum(Ghat * Ghat) - 2.0 * np.sum(H[0] * V[0]) + np.sum(had))
    grads = []
    for n in range(N):
        T = np.ones((R, R))
        for p in range(N):
            if p != n:
                T = T * grams[p]
        grads.append(2.0 * (V[n] @ T - H[n]))
    return loss, grads


def init_params(rng, dims):
    """He-style init: W ~ N(0, 2/fan_in), b = 0.  dims = [d0, d1, d2, d3]."""
    params = {}
    for k in range(3):
        fan_in, fan_out = dims[k], dims[k + 1]
        params[f"W{k + 1}"] = rng.standard_normal((fan_in, fan_out)) * \
            math.sqrt(2.0 / fan_in)
        params[f"b{k + 1}"] = np.zeros(fan_out)
    return params


def forward(params, X, bf16=None):
    """X: batch x d0 (already normalized).  Returns (Y, cache)."""
    r = (lambda a: a) if bf16 is None else bf16
    W1, W2, W3 = (r(params[k]) for k in ("W1", "W2", "W3"))
    X = np.asarray(X, dtype=np.float64)
    z1 = r(X) @ W1 + params["b1"]
    h1 = gelu(z1)
    z2 = r(h1) @ W2 + params["b2"]
    h2 = gelu(z2)
    Y = r(h2) @ W3 + params["b3"]
    return Y, (X, z1, h1, z2, h2)


def split_factors(y, core_shape, R):
    V, off = [], 0
    for Rn in core_shape:
        V.append(y[off:off + Rn * R].reshape(Rn, R))
        off += Rn * R
    return V


def loss_and_backward(params, Ghats, bf16=None):
    """Mean loss over the batch and gradients of every parameter.
    Ghats: batch x R_1 x ... x R_N normalized cores."""
    Ghats = np.asarray(Ghats, dtype=np.float64)
    B = Ghats.shape[0]
    core_shape = Ghats.shape[1:]
    R = params["W3"].shape[1] // sum(core_shape)
    X = Ghats.reshape(B, -1)
    Y, (X, z1, h1, z2, h2) = forward(params, X, bf16)
    dY = np.zeros_like(Y)
    total = 0.0
    for b in range(B):
        V = split_factors(Y[b], core_shape, R)
        loss, grads = cp_loss_and_grad(Ghats[b], V)
        total += loss
        dY[b] = np.concatenate([g.reshape(-1) for g in grads]) / B
    r = (lambda a: a) if bf16 is None else bf16
    W2, W3 = r(params["W2"]), r(params["W3"])
    g = {}
    g["W3"] = r(h2).T @ r(dY)
    g["b3"] = dY.sum(axis=0)
    dh2 = r(dY) @ W3.T
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = r(h1).T @ r(dz2)
    g["b2"] = dz2.sum(axis=0)
    dh1 = r(dz2) @ W2.T
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = r(X).T @ r(dz1)
    g["b1"] = dz1.sum(axis=0)
    return total / B, g


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1.0 - beta1) * grads[k]
        v[...] = beta2 * v + (1.0 - beta2) * grads[k] * grads[k]
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params
