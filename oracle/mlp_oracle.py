"""FP64 CPU reference of the learned support proposal (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library neither imports nor links it, and it imports nothing
from the GPU package.  Plain numpy float64, no blocking or fusion.

The proposal is not part of the paper.  The paper's method accepts any
starting active set and keeps the warm start from one outer iteration to the
next (Algorithm 1, step 5, and the warm-start remark of Section III), and the
natural stopping condition (Eq. (9)) certifies whatever the start was; the
network only chooses that start.  What is computed here:

  embedding   z = (A P)^T b scaled to unit root-mean-square, P a fixed random
              m x d projection, so z = P^T (A^T b) up to a positive factor (the
              LASSO support under the relative lambda rule does not depend on
              the scale of b, so the factor loses nothing);
  network     h1 = gelu(W1 z + b1), h2 = gelu(W2 h1 + b2), s = W3 h2 + b3,
              gelu(u) = u Phi(u) with the exact normal CDF;
  loss        binary cross-entropy with logits and a positive-class weight w,
              summed over the m atoms and averaged over the batch:
              l(s, y) = w y log(1 + e^-s) + (1 - y) log(1 + e^s);
  gradient    the chain rule through the three layers, written out below;
  update      Adam (Kingma and Ba, 2015) with bias correction;
  proposal    the k atoms with the largest scores, ties to the lower index.

Flat parameter layout (row-major blocks, in this order):
  W1 [h][d], b1 [h], W2 [h][h], b2 [h], W3 [m][h], b3 [m].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def param_count(d: int, h: int, m: int) -> int:
    return h * d + h + h * h + h + m * h + m


def unpack(params: np.ndarray, d: int, h: int, m: int) -> dict:
    """Views of the six blocks of the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == param_count(d, h, m)
    out, o = {}, 0
    for name, shape in (("W1", (h, d)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (m, h)), ("b3", (m,))):
        size = int(np.prod(shape))
        out[name] = p[o:o + size].reshape(shape)
        o += size
    return out


def pack(blocks: dict) -> np.ndarray:
    return np.concatenate([np.asarray(blocks[k], dtype=np.float64).ravel()
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def gelu(u: np.ndarray) -> np.ndarray:
    """u * Phi(u), Phi the standard normal CDF."""
    return u * 0.5 * (1.0 + erf(u / SQRT2))


def gelu_prime(u: np.ndarray) -> np.ndarray:
    """d/du [u Phi(u)] = Phi(u) + u phi(u)."""
    return 0.5 * (1.0 + erf(u / SQRT2)) + u * INV_SQRT_2PI * np.exp(-0.5 * u * u)


def projected_dictionary(At: np.ndarray, P: np.ndarray) -> np.ndarray:
    """(A P)^T as a d x n array; At is the m x n atom-major dictionary, P is m x d."""
    return np.asarray(P, dtype=np.float64).T @ np.asarray(At, dtype=np.float64)


def embed(APt: np.ndarray, Bt: np.ndarray) -> np.ndarray:
    """Rows z_i = (A P)^T b_i, each scaled to unit root-mean-square (a zero row stays zero)."""
    Z = np.asarray(Bt, dtype=np.float64) @ np.asarray(APt, dtype=np.float64).T
    d = Z.shape[1]
    nrm = np.sqrt((Z * Z).sum(axis=1, keepdims=True))
    scale = np.where(nrm > 0.0, math.sqrt(d) / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    return Z * scale


def forward(params: np.ndarray, X0: np.ndarray, d: int, h: int, m: int) -> dict:
    """Pre-activations, activations and scores for a batch of embeddings X0 (rows)."""
    w = unpack(params, d, h, m)
    X0 = np.asarray(X0, dtype=np.float64)
    U1 = X0 @ w["W1"].T + w["b1"]
    H1 = gelu(U1)
    U2 = H1 @ w["W2"].T + w["b2"]
    H2 = gelu(U2)
    S = H2 @ w["W3"].T + w["b3"]
    return {"U1": U1, "H1": H1, "U2": U2, "H2": H2, "S": S}


def labels(supports, m: int) -> np.ndarray:
    """Dense 0/1 targets from per-signal support lists."""
    Y = np.zeros((len(supports), m), dtype=np.float64)
    for i, s in enumerate(supports):
        Y[i, np.asarray(s, dtype=np.int64)] = 1.0
    return Y


def softplus(x: np.ndarray) -> np.ndarray:
    """log(1 + e^x) without overflow."""
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x: np.ndarray) -> np.ndarray:
    e = np.exp(-np.abs(x))
    return np.where(x >= 0.0, 1.0 / (1.0 + e), e / (1.0 + e))


def loss(S: np.ndarray, Y: np.ndarray, pos_weight: float) -> float:
    """Mean over the batch of the summed weighted binary cross-entropy."""
    per = pos_weight * Y * softplus(-S) + (1.0 - Y) * softplus(S)
    return float(per.sum() / S.shape[0])


def loss_and_grad(params: np.ndarray, X0: np.ndarray, Y: np.ndarray, pos_weight: float,
                  d: int, h: int, m: int) -> tuple[float, np.ndarray]:
    """Loss and its gradient with respect to the flat parameters."""
    w = unpack(params, d, h, m)
    X0 = np.asarray(X0, dtype=np.float64)
    f = forward(params, X0, d, h, m)
    B = X0.shape[0]
    # d l / d s = sigma(s) (w y + 1 - y) - w y, then the batch mean
    dS = (sigmoid(f["S"]) * (pos_weight * Y + 1.0 - Y) - pos_weight * Y) / B
    g = {"W3": dS.T @ f["H2"], "b3": dS.sum(axis=0)}
    dU2 = (dS @ w["W3"]) * gelu_prime(f["U2"])
    g["W2"] = dU2.T @ f["H1"]
    g["b2"] = dU2.sum(axis=0)
    dU1 = (dU2 @ w["W2"]) * gelu_prime(f["U1"])
    g["W1"] = dU1.T @ X0
    g["b1"] = dU1.sum(axis=0)
    return loss(f["S"], Y, pos_weight), pack(g)


def adam(params, m1, m2, grad, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (t counts from 1).  Returns the new parameters and moments."""
    m1 = beta1 * np.asarray(m1, dtype=np.float64) + (1.0 - beta1) * grad
    m2 = beta2 * np.asarray(m2, dtype=np.float64) + (1.0 - beta2) * grad * grad
    mh = m1 / (1.0 - beta1 ** t)
    vh = m2 / (1.0 - beta2 ** t)
    return np.asarray(params, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m1, m2


def propose(S: np.ndarray, k: int) -> np.ndarray:
    """Per row, the k largest scores' atom indices (ties to the lower index), ascending by index."""
    S = np.asarray(S)
    out = np.empty((S.shape[0], k), dtype=np.int64)
    for i in range(S.shape[0]):
        order = np.lexsort((np.arange(S.shape[1]), -S[i]))   # by score desc, then index asc
        out[i] = np.sort(order[:k])
    return out
