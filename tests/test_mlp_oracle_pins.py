"""Pins of the FP64 reference of the learned support proposal (oracle/mlp_oracle.py).

Each test fixes the reference to something other than itself: textbook values
of the normal CDF, the identity gelu(x) - gelu(-x) = x, central finite
differences of its own forward pass (so a dropped or mis-signed term in the
hand-written chain rule fails), PyTorch's float64 CPU autograd, loss and Adam
as independent library routines, and brute-force ordering for the top-k
proposal.
"""
import math

import numpy as np
import pytest
import torch

import bmpl_inputs as bi
from oracle import mlp_oracle as mo


def _tiny(seed=0, d=4, h=5, m=6, B=3, k=2):
    rng = np.random.default_rng(seed)
    params = rng.standard_normal(mo.param_count(d, h, m)) * 0.7
    X0 = rng.standard_normal((B, d))
    sup = [rng.choice(m, size=k, replace=False) for _ in range(B)]
    return params, X0, mo.labels(sup, m), (d, h, m)


def test_gelu_textbook_values():
    # Phi(1) and Phi(-1) from the standard normal table; gelu(x) = x Phi(x)
    phi1 = 0.8413447460685429
    assert mo.gelu(np.array([1.0]))[0] == pytest.approx(phi1, rel=1e-15)
    assert mo.gelu(np.array([-1.0]))[0] == pytest.approx(-(1.0 - phi1), rel=1e-14)
    assert mo.gelu(np.array([0.0]))[0] == 0.0
    x = np.linspace(-6, 6, 97)
    np.testing.assert_allclose(mo.gelu(x) - mo.gelu(-x), x, rtol=0, atol=1e-15)
    # derivative against central differences of the function itself
    e = 1e-6
    np.testing.assert_allclose(mo.gelu_prime(x), (mo.gelu(x + e) - mo.gelu(x - e)) / (2 * e), rtol=1e-8, atol=1e-9)
    # derivative at 0 is Phi(0) = 1/2
    assert mo.gelu_prime(np.array([0.0]))[0] == 0.5


def test_forward_and_loss_match_torch_float64():
    params, X0, Y, (d, h, m) = _tiny(1)
    w = mo.unpack(params, d, h, m)
    f = mo.forward(params, X0, d, h, m)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in w.items()}
    x = torch.from_numpy(X0)
    h1 = torch.nn.functional.gelu(torch.nn.functional.linear(x, t["W1"], t["b1"]), approximate="none")
    h2 = torch.nn.functional.gelu(torch.nn.functional.linear(h1, t["W2"], t["b2"]), approximate="none")
    s = torch.nn.functional.linear(h2, t["W3"], t["b3"])
    np.testing.assert_allclose(f["S"], s.numpy(), rtol=1e-13, atol=1e-14)
    pw = 7.5
    ref = torch.nn.functional.binary_cross_entropy_with_logits(
        s, torch.from_numpy(Y), pos_weight=torch.full((m,), pw, dtype=torch.float64), reduction="sum") / X0.shape[0]
    assert mo.loss(f["S"], Y, pw) == pytest.approx(float(ref), rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_against_central_differences(seed):
    params, X0, Y, (d, h, m) = _tiny(seed)
    pw = 3.0
    _, g = mo.loss_and_grad(params, X0, Y, pw, d, h, m)
    num = np.empty_like(params)
    e = 1e-6
    for i in range(params.size):
        a = params.copy(); a[i] += e
        b = params.copy(); b[i] -= e
        num[i] = (mo.loss(mo.forward(a, X0, d, h, m)["S"], Y, pw) - mo.loss(mo.forward(b, X0, d, h, m)["S"], Y, pw)) / (2 * e)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-8)


def test_gradient_against_torch_autograd():
    params, X0, Y, (d, h, m) = _tiny(3, d=8, h=6, m=9, B=5, k=3)
    pw = 11.0
    loss, g = mo.loss_and_grad(params, X0, Y, pw, d, h, m)
    p = torch.tensor(params, requires_grad=True)
    w = {}
    o = 0
    for name, shape in (("W1", (h, d)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (m, h)), ("b3", (m,))):
        size = int(np.prod(shape))
        w[name] = p[o:o + size].reshape(shape)
        o += size
    x = torch.from_numpy(X0)
    h1 = torch.nn.functional.gelu(x @ w["W1"].T + w["b1"], approximate="none")
    h2 = torch.nn.functional.gelu(h1 @ w["W2"].T + w["b2"], approximate="none")
    s = h2 @ w["W3"].T + w["b3"]
    L = torch.nn.functional.binary_cross_entropy_with_logits(
        s, torch.from_numpy(Y), pos_weight=torch.full((m,), pw, dtype=torch.float64), reduction="sum") / X0.shape[0]
    L.backward()
    assert loss == pytest.approx(L.item(), rel=1e-13)
    np.testing.assert_allclose(g, p.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) for _ in range(4)]
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m1, m2 = p0.copy(), np.zeros(40), np.zeros(40)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m1, m2 = mo.adam(p, m1, m2, g, t, 3e-3)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_propose_brute_force_and_ties():
    rng = np.random.default_rng(7)
    S = np.round(rng.standard_normal((6, 40)), 1)      # rounding creates many ties
    S[0, :] = 0.25                                      # all tied: lowest indices win
    for k in (1, 5, 17, 40):
        got = mo.propose(S, k)
        for i in range(S.shape[0]):
            # brute force: a set T of size k is the answer iff every member beats every non-member
            # under (score desc, index asc)
            order = sorted(range(S.shape[1]), key=lambda j: (-S[i, j], j))
            assert list(got[i]) == sorted(order[:k])
    assert list(mo.propose(S[:1], 5)[0]) == [0, 1, 2, 3, 4]


def test_embedding_is_projected_correlation_direction():
    """z is P^T (A^T b) up to a positive factor, with unit root-mean-square."""
    P = bi.tiny_gaussian(64, 200, 5, 6, 0.01, seed=4)
    Pm = bi.projection(P.m, 128, seed=1)
    APt = mo.projected_dictionary(P.At, Pm)
    Z = mo.embed(APt, P.Bt)
    direct = (Pm.astype(np.float64).T @ (P.At.astype(np.float64) @ P.Bt.astype(np.float64).T)).T
    for i in range(P.p):
        c = Z[i] @ direct[i] / (np.linalg.norm(Z[i]) * np.linalg.norm(direct[i]))
        assert c == pytest.approx(1.0, abs=1e-12)
        assert math.sqrt(np.mean(Z[i] ** 2)) == pytest.approx(1.0, rel=1e-12)
    # scale invariance in b
    np.testing.assert_allclose(mo.embed(APt, 3.5 * P.Bt.astype(np.float64)), Z, rtol=1e-12, atol=1e-12)
    assert np.all(mo.embed(APt, np.zeros((1, P.n))) == 0.0)


def test_loss_decreases_under_plain_gradient_descent():
    """A property that holds for any correct gradient: small steps along -g lower the loss."""
    params, X0, Y, (d, h, m) = _tiny(9, d=6, h=7, m=8, B=4)
    loss0, g = mo.loss_and_grad(params, X0, Y, 2.0, d, h, m)
    for lr in (1e-3, 1e-2):
        l1 = mo.loss(mo.forward(params - lr * g, X0, d, h, m)["S"], Y, 2.0)
        assert l1 < loss0
        # first-order prediction
        assert (loss0 - l1) == pytest.approx(lr * g @ g, rel=0.05)


def test_src_classification_reference():
    """Class-residual rule: exact single-class reconstructions, the empty support, ties, relabelling."""
    from oracle import src_oracle as so
    rng = np.random.default_rng(2)
    n, per, classes = 30, 4, 5
    A = rng.standard_normal((classes * per, n))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    A[9] = 0.0
    A[9, 0] = 1.0                           # two exactly representable atoms for an exact tie
    A[17] = 0.0
    A[17, 1] = 1.0
    cls = np.repeat(np.arange(classes), per)
    X = np.zeros((4, classes * per))
    X[0, 4:6] = [1.0, -2.0]                 # class 1 only: b reconstructed exactly
    X[1, [1, 13]] = [3.0, 0.1]              # mostly class 0, a little class 3
    X[2, 9] = 1.0                           # two classes explain b equally well (see below)
    X[2, 17] = 1.0
    B = X @ A
    B[1] += 0.01 * rng.standard_normal(n)
    B[2] = A[9] + A[17]                     # b = a_9 + a_17: both single-class residuals have norm 1
    lab, res = so.classify(A, B, X, cls)
    assert lab[0] == 1 and res[0] < 1e-12
    assert lab[1] == 0
    assert lab[2] == 2 and abs(res[2] - 1.0) < 1e-12      # tie between classes 2 and 4 -> the lower
    assert lab[3] == -1 and np.isnan(res[3])               # empty support
    # relabelling classes permutes the labels the same way
    perm = np.array([3, 0, 4, 1, 2])
    lab2, _ = so.classify(A, B, X, perm[cls])
    assert lab2[0] == perm[1] and lab2[1] == perm[0] and lab2[3] == -1
