"""GPU parity of the learned support proposal (bmpl_mlp_* through the C ABI) against
the FP64 reference oracle/mlp_oracle.py.

Precision and tolerances.  The GPU multiplies bfloat16 weights and bfloat16
activations with float32 accumulation; the reference runs in float64 on the
same bfloat16-valued weights (rounded here with PyTorch's round-to-nearest-even
conversion, the rounding the library applies) and keeps every activation in
float64.  Each rounding to bfloat16 perturbs a value by at most u = 2^-9
relative.  The forward pass rounds five vectors on the way to the scores (the
signal, (A P)^T, the embedding, h1, h2); with layer gains near one and the
GELU's Lipschitz constant 1.13 the scores' row-wise relative error stays below
5 u 1.13^2 = 6.4 u, tested at 8 u.  The backward pass adds the roundings of
dl/ds, dl/du2 and dl/du1 and evaluates gelu' at perturbed pre-activations;
gradient blocks are tested norm-wise at 16 u.  A structural mistake (a missing
gelu', a transposed factor, a wrong sign) moves a block by O(1), far outside
these bands.  The top-k selection is an integer decision: it is compared
exactly against the reference's selection on the GPU's own float32 scores.
"""
import time

import numpy as np
import pytest

import bmpl_inputs as bi
import oracle
from oracle import mlp_oracle as mo
from tests.parity import check_batch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -9


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_5010_amd as pk
    return pk


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def bf16_values(x: np.ndarray) -> np.ndarray:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def oracle_params(params32: np.ndarray, d: int, h: int, m: int) -> np.ndarray:
    """Weights as the GPU multiplies them (bfloat16 values), biases in float32."""
    w = mo.unpack(params32.astype(np.float64), d, h, m)
    for k in ("W1", "W2", "W3"):
        w[k] = bf16_values(w[k].astype(np.float32))
    return mo.pack(w)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _small(seed=0, n=200, m=700, d=128, h=192, p=150, k=12):
    P = bi.tiny_gaussian(n, m, p, k, 0.01, seed=seed)
    Pm = bi.projection(m, d, seed=seed)
    params = bi.mlp_init(d, h, m, seed=seed, prior=k / m)
    # a less trivial operating point than the initialisation: perturb the biases
    rng = np.random.default_rng(seed)
    params = params + (0.3 * rng.standard_normal(params.size)).astype(np.float32) * (np.abs(params) == 0)
    return P, Pm, params.astype(np.float32), (d, h, m)


# ---------------------------------------------------------------------------
# Selection kernel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rows,L,k", [(37, 20000, 256), (64, 700, 12), (5, 100, 256), (9, 4099, 1), (3, 38912, 200)])
def test_topk_matches_reference_selection(rows, L, k):
    pk = _lib()
    rng = np.random.default_rng(L + k)
    S = np.round(rng.standard_normal((rows, L)), 2).astype(np.float32)   # many ties
    S[0, :] = 0.5                                                        # all tied
    if rows > 2:
        S[1, ::7] = np.nan                                              # NaN ranks lowest
        S[2, :] = -0.0
        S[2, 3::5] = 0.0                                                # signed zeros compare equal
    got = pk.topk(to_dev(S), k).cpu().numpy()
    kk = min(k, L)
    ref = mo.propose(S.astype(np.float64), kk)
    np.testing.assert_array_equal(got[:, :kk], ref)
    assert np.all(got[:, kk:] == -1)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

def test_embedding_and_forward_within_bfloat16_bands():
    pk = _lib()
    P, Pm, params, (d, h, m) = _small(1)
    net = pk.ProposalNet(to_dev(P.At), to_dev(Pm), h, max_batch=64)   # p = 150: three chunks
    net.set_params(to_dev(params))
    Z = net.embed(to_dev(P.Bt)).cpu().numpy().astype(np.float64)
    Zr = mo.embed(mo.projected_dictionary(P.At, Pm), P.Bt)
    for i in range(P.p):
        assert rel(Z[i], Zr[i]) <= 4 * U, i
    S = net.forward(to_dev(P.Bt)).cpu().numpy().astype(np.float64)
    Sr = mo.forward(oracle_params(params, d, h, m), Zr, d, h, m)["S"]
    errs = [rel(S[i], Sr[i]) for i in range(P.p)]
    assert max(errs) <= 8 * U, max(errs)


@pytest.mark.parametrize("seed,p", [(2, 150), (3, 64), (4, 1)])
def test_loss_and_gradient_against_reference(seed, p):
    pk = _lib()
    P, Pm, params, (d, h, m) = _small(seed, p=p)
    net = pk.ProposalNet(to_dev(P.At), to_dev(Pm), h, max_batch=160)
    net.set_params(to_dev(params))
    L = max(len(s) for s in P.supports)
    supp = np.full((p, L + 3), -1, dtype=np.int32)
    lens = np.zeros(p, dtype=np.int32)
    for i, s in enumerate(P.supports):
        supp[i, :len(s)] = s
        lens[i] = len(s)
    pw = 9.0
    loss, g = net.loss_grad(to_dev(P.Bt), to_dev(supp), to_dev(lens), pw)
    loss = float(loss.item())
    g = g.cpu().numpy().astype(np.float64)
    Zr = mo.embed(mo.projected_dictionary(P.At, Pm), P.Bt)
    loss_r, g_r = mo.loss_and_grad(oracle_params(params, d, h, m), Zr, mo.labels(P.supports, m), pw, d, h, m)
    assert abs(loss - loss_r) <= 8 * U * loss_r
    gb, rb = mo.unpack(g, d, h, m), mo.unpack(g_r, d, h, m)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert rel(gb[name], rb[name]) <= 16 * U, (name, rel(gb[name], rb[name]))


def mlp_tile(M: int, N: int) -> int:
    """Edge of the square output tile the network's matrix products use for an M x N output (the size rule
    of the library's launcher: 256 when there are at least 1024 such tiles, 128 when there are at least 512
    of 128, else 64)."""
    if -(-M // 256) * -(-N // 256) >= 1024:
        return 256
    if -(-M // 128) * -(-N // 128) >= 512:
        return 128
    return 64


def _full_width(p, seed):
    """The benchmark's network shape: n = 1024, m = 20000 atoms, d = h = 2048, random initial weights with
    perturbed biases (a non-trivial operating point)."""
    n, m, d, h = 1024, 20000, 2048, 2048
    P = bi.tiny_gaussian(n, m, p, 10, 0.01, seed=seed)
    Pm = bi.projection(m, d, seed=seed)
    params = bi.mlp_init(d, h, m, seed=seed, prior=10.0 / m)
    rng = np.random.default_rng(seed)
    params = params + (0.3 * rng.standard_normal(params.size)).astype(np.float32) * (np.abs(params) == 0)
    return P, Pm, params.astype(np.float32), (d, h, m)


def test_forward_large_tiles_full_width():
    """Inference as the benchmark runs it: chunks of 4096 signals through the 2048 / 2048 / 20000 network.
    A 4096-row chunk runs the hidden layers (bias + GELU epilogue) on 128 x 128 tiles and the output layer
    (bias epilogue, 20000 = 78 x 256 + 32: a ragged edge tile) on 256 x 256 tiles; the 96-row tail chunk on
    64 x 64 tiles.  Sampled rows (tile edges of both chunks) against the float64 reference, 8 u row-wise."""
    pk = _lib()
    p = 4096 + 96
    P, Pm, params, (d, h, m) = _full_width(p, seed=11)
    assert mlp_tile(4096, h) == 128 and mlp_tile(4096, m) == 256
    assert mlp_tile(96, h) == 64 and mlp_tile(96, m) == 64
    net = pk.ProposalNet(to_dev(P.At), to_dev(Pm), h, max_batch=4096)
    net.set_params(to_dev(params))
    S = net.forward(to_dev(P.Bt))
    torch.cuda.synchronize()
    rows = [0, 1, 127, 128, 255, 256, 1000, 2047, 2048, 3839, 3840, 4095, 4096, 4150, p - 1]
    S = S[rows].cpu().numpy().astype(np.float64)
    Zr = mo.embed(mo.projected_dictionary(P.At, Pm), P.Bt[rows])
    Sr = mo.forward(oracle_params(params, d, h, m), Zr, d, h, m)["S"]
    errs = [rel(S[q], Sr[q]) for q in range(len(rows))]
    assert max(errs) <= 8 * U, errs
    # the ragged last output tile (atoms 19968 .. 19999) on its own
    assert max(rel(S[q, 19968:], Sr[q, 19968:]) for q in range(len(rows))) <= 8 * U


def test_loss_and_gradient_training_shape():
    """One training batch as the benchmark runs it: 1024 signals, the 2048 / 2048 / 20000 network.  The
    output layer's forward product and dW3 = dS^T H2 run on 128 x 128 tiles (the other products on
    64 x 64); loss within 8 u and every gradient block within 16 u norm-wise of the float64 reference."""
    pk = _lib()
    p = 1024
    P, Pm, params, (d, h, m) = _full_width(p, seed=12)
    assert mlp_tile(p, m) == 128 and mlp_tile(m, h) == 128
    assert mlp_tile(p, h) == 64 and mlp_tile(h, h) == 64
    net = pk.ProposalNet(to_dev(P.At), to_dev(Pm), h, max_batch=p)
    net.set_params(to_dev(params))
    supp = np.full((p, 12), -1, dtype=np.int32)
    lens = np.zeros(p, dtype=np.int32)
    for i, sp in enumerate(P.supports):
        supp[i, :len(sp)] = sp
        lens[i] = len(sp)
    pw = 20.0
    loss, g = net.loss_grad(to_dev(P.Bt), to_dev(supp), to_dev(lens), pw)
    loss = float(loss.item())
    g = g.cpu().numpy().astype(np.float64)
    Zr = mo.embed(mo.projected_dictionary(P.At, Pm), P.Bt)
    loss_r, g_r = mo.loss_and_grad(oracle_params(params, d, h, m), Zr, mo.labels(P.supports, m), pw, d, h, m)
    assert abs(loss - loss_r) <= 8 * U * loss_r
    gb, rb = mo.unpack(g, d, h, m), mo.unpack(g_r, d, h, m)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert rel(gb[name], rb[name]) <= 16 * U, (name, rel(gb[name], rb[name]))


def test_adam_step_against_reference():
    pk = _lib()
    P, Pm, params, (d, h, m) = _small(5, p=32)
    net = pk.ProposalNet(to_dev(P.At), to_dev(Pm), h, max_batch=32)
    net.set_params(to_dev(params))
    rng = np.random.default_rng(11)
    p_ref = params.astype(np.float64)
    m1 = np.zeros_like(p_ref)
    m2 = np.zeros_like(p_ref)
    for t in range(1, 4):
        g = (rng.standard_normal(params.size) * 10.0 ** rng.uniform(-4, 0, params.size)).astype(np.float32)
        net.adam_step(2e-3, grad=to_dev(g))
        p_new, m1, m2 = mo.adam(p_ref, m1, m2, g.astype(np.float64), t, 2e-3)
        got = net.get_params().cpu().numpy().astype(np.float64)
        # float32 arithmetic on a handful of operations, then one rounding of the parameter.  The
        # update's error scales with lr, not with the update: when the first moment nearly cancels,
        # the update is tiny while the rounding of its terms is not; |m_hat| <= sqrt(v_hat) up to
        # O(1), and float32's beta2 = 0.999 alone shifts 1 - beta2 by 1.3e-5 relative.
        bound = 2.0 ** -22 * np.abs(p_new) + 2e-5 * 2e-3 + 1e-12
        assert np.all(np.abs(got - p_new) <= bound), np.max(np.abs(got - p_new) / bound)
        p_ref = got     # continue from the GPU's float32 state, as the GPU does


def test_full_size_forward_sampled():
    """The configured network (2048 -> 2048 -> 2048 -> 20000) on the face-like dictionary."""
    pk = _lib()
    P = bi.face_like(indices=range(40))
    d = h = 2048
    Pm = bi.projection(P.m, d, seed=0)
    params = bi.mlp_init(d, h, P.m, seed=0, prior=10 / P.m)
    net = pk.ProposalNet(to_dev(P.At), to_dev(Pm), h, max_batch=32)
    net.set_params(to_dev(params))
    S = net.forward(to_dev(P.Bt)).cpu().numpy().astype(np.float64)
    rows = [0, 17, 31, 32, 39]       # both chunks
    Zr = mo.embed(mo.projected_dictionary(P.At, Pm), P.Bt[rows])
    Sr = mo.forward(oracle_params(params, d, h, P.m), Zr, d, h, P.m)["S"]
    for q, i in enumerate(rows):
        assert rel(S[i], Sr[q]) <= 8 * U, (i, rel(S[i], Sr[q]))
    idx = net.propose(to_dev(P.Bt), 256).cpu().numpy()
    np.testing.assert_array_equal(idx, mo.propose(S.astype(np.float32).astype(np.float64), 256))


# ---------------------------------------------------------------------------
# Training on BMPL's own supports, and what the proposal gains
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_learned_proposal_gain_face_like():
    """Train on the supports BMPL produced for 65536 signals of a distinct seed stream (256 Adam
    steps); on 4096 test signals the top-256 proposal must recall the supports, every warm-started
    solve must converge and meet the parity rules on a sample, and the outer iterations must drop.
    Wall times are printed, not asserted: on this workload the plain BF16-screened solve is already
    a few microseconds per signal, and the gain is in iterations."""
    pk = _lib()
    from paper_1302_5010_amd import learned as ln
    P = bi.face_like(indices=range(4096))
    At = to_dev(P.At)
    Bt = to_dev(P.Bt)
    solver = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, screen="bf16", graph=True)
    T = bi.face_like(p=65536, stream=2)
    Bt_tr = to_dev(T.Bt)
    lab = ln.label_supports(solver, Bt_tr)
    assert bool(ln.converged(lab).all())
    d = h = 2048
    net = pk.ProposalNet(At, to_dev(bi.projection(P.m, d, seed=0)), h, max_batch=4096)
    net.set_params(to_dev(bi.mlp_init(d, h, P.m, seed=0, prior=10 / P.m)))
    losses = ln.train_proposal(net, Bt_tr, lab["x_idx"], lab["supp_len"], epochs=4, batch=1024, lr=1e-3,
                               pos_weight=20.0, record_every=16)
    losses = [float(v.item()) for v in losses]
    assert np.mean(losses[-4:]) < 0.2 * losses[0], losses
    del Bt_tr, lab

    plain = solver.solve(Bt)
    warm = ln.solve_with_proposal(solver, net, Bt, 256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = solver.solve(Bt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    warm = ln.solve_with_proposal(solver, net, Bt, 256)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for out in (plain, warm):
        st = out["status"].cpu().numpy()
        assert np.all(st & pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    xi, sl, pr = plain["x_idx"].cpu().numpy(), plain["supp_len"].cpu().numpy(), warm["proposal"].cpu().numpy()
    recall = np.mean([np.isin(xi[i, :sl[i]], pr[i]).mean() for i in range(P.p) if sl[i] > 0])
    it_plain = plain["iters"].cpu().numpy().mean()
    it_warm = warm["iters"].cpu().numpy().mean()
    fallback = np.mean((warm["status"].cpu().numpy() & pk.BMPL_SIG_FALLBACK) > 0)
    print(f"recall@256 {recall:.4f}  iters plain {it_plain:.2f} learned {it_warm:.2f}  fallback {fallback:.3f}  "
          f"solve s plain {t1 - t0:.4f} learned (incl. proposal) {t2 - t1:.4f}")
    assert recall >= 0.95
    assert it_warm < 0.6 * it_plain
    rows = list(range(5, P.p, 128))
    lam = P.lambda_rel * np.abs(P.At.astype(np.float64) @ P.Bt[rows].astype(np.float64).T).max(axis=0)
    ref = oracle.solve(P.At, P.Bt[rows], lam, P.rho)
    check_batch(P.At, P.Bt, lam, warm, ref, rows=range(len(rows)), gpu_rows=rows)
