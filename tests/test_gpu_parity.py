"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Kernel-level tests compare the correlation product with a float64 matmul
within float32's deterministic error bound and the selection with a CPU sort;
solver-level tests apply the parity rules of tests/parity.py to whole solves
on seeded workloads, from small ragged shapes up to the 2048 x 16384 x 1024
compressive-sensing workload in the benchmark's configuration (sampled signals).
"""
import numpy as np
import pytest

import bmpl_inputs as bi
import oracle
from tests.parity import check_batch, dense_from_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_5010_amd as pk
    return pk


def lam_rel(At, Bt, c):
    return c * np.abs(At.astype(np.float64) @ Bt.astype(np.float64).T).max(axis=0)


def lam_bound(At, Bt, c):
    """Deterministic float32 error bound of c * max_j |a_j^T b| computed by the float32 product."""
    n = At.shape[1]
    return c * 2 * n * 2.0 ** -24 * (np.abs(At.astype(np.float64)) @ np.abs(Bt.astype(np.float64)).T).max(axis=0)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


# ---------------------------------------------------------------------------
# Kernel level
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,p", [(96, 1000, 200), (128, 512, 16), (2048, 16384, 130), (1024, 300, 1)])
def test_correlate_within_float32_bound(n, m, p):
    pk = _lib()
    rng = np.random.default_rng(n + m + p)
    At = rng.standard_normal((m, n)).astype(np.float32)
    Rt = rng.standard_normal((p, n)).astype(np.float32)
    s = pk.Solver(to_dev(At), 0.1)
    G = s.correlate(to_dev(Rt)).cpu().numpy().astype(np.float64)
    A64, R64 = At.astype(np.float64), Rt.astype(np.float64)
    ref = R64 @ A64.T
    bound = 2 * n * 2.0 ** -24 * (np.abs(R64) @ np.abs(A64).T) + 1e-30
    err = np.abs(G - ref)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound):.3f}"


@pytest.mark.parametrize("screen", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("shape", range(15))
def test_correlate_every_tile_shape(shape, screen):
    """Every tile shape within the precision's bound, entry by entry, and bit-identical to shape 0 (every
    shape feeds each output's accumulator the same k chunks in the same order; shapes 8-10, bfloat16
    only, read the dictionary from its fragment-ordered copy; shapes 11-14 copy both operand tiles
    straight into swizzled LDS buffers)."""
    pk = _lib()
    rng = np.random.default_rng(shape)
    n, m = 160, 1500
    At = rng.standard_normal((m, n)).astype(np.float32)
    s = pk.Solver(to_dev(At), 0.1, screen=screen)
    if 8 <= shape <= 10 and screen != "bf16":
        with pytest.raises(pk.BmplError):
            s.set_tuning([shape, shape, shape])
        return
    s0 = pk.Solver(to_dev(At), 0.1, screen=screen)
    s0.set_tuning([0, 0, 0])
    s.set_tuning([shape, shape, shape])
    A64 = At.astype(np.float64)
    for p in (1, 37, 600):                 # one row, a ragged tile, several tiles in the >= 512 bucket
        Rt = rng.standard_normal((p, n)).astype(np.float32)
        Gd = s.correlate(to_dev(Rt))
        assert torch.equal(Gd, s0.correlate(to_dev(Rt))), (shape, p)
        G = Gd.cpu().numpy().astype(np.float64)
        R64 = Rt.astype(np.float64)
        if screen == "fp32":
            bound = 2 * n * 2.0 ** -24 * (np.abs(R64) @ np.abs(A64).T)
        else:
            bound = (bf16_band if screen == "bf16" else fp8_band)(At, Rt)
        assert np.all(np.abs(G - R64 @ A64.T) <= bound), (shape, p)


@pytest.mark.parametrize("with_excl", [True, False])
@pytest.mark.parametrize("k", [1, 10, 20, 33])
def test_select_matches_cpu_sort(k, with_excl):
    """Rows longer than the entries each thread keeps in registers (8192), with a scalar tail."""
    pk = _lib()
    rng = np.random.default_rng(k)
    p, m = 37, 20003
    s = pk.Solver(to_dev(np.eye(m, 64, dtype=np.float32)), 0.1, gram_table=False)
    G = rng.standard_normal((p, m)).astype(np.float32)
    lam = np.quantile(np.abs(G), rng.uniform(0.9, 0.999, p), axis=1).diagonal().astype(np.float64)
    lam[3] = 10.0                                   # a row with no violator
    G[5, :] = -0.5                                  # every entry tied: more candidates than any buffer
    lam[5] = 0.1
    G[6, ::2] = 0.25                                # half the row tied just above lambda
    lam[6] = 0.2
    words = (m + 31) // 32
    excl_bits = (rng.random((p, m)) < 0.3) if with_excl else np.zeros((p, m), dtype=bool)
    excl = np.zeros((p, words), dtype=np.uint32)
    for i in range(p):
        for j in np.nonzero(excl_bits[i])[0]:
            excl[i, j >> 5] |= np.uint32(1 << (j & 31))
    sel, nsel, vmax = s.select(to_dev(G), to_dev(lam), k, excl=to_dev(excl.view(np.int32)) if with_excl else None)
    sel, nsel, vmax = sel.cpu().numpy(), nsel.cpu().numpy(), vmax.cpu().numpy()
    for i in range(p):
        a = np.abs(G[i]).copy()
        a[excl_bits[i]] = -1
        cand = np.nonzero(a.astype(np.float64) > lam[i])[0]
        order = cand[np.lexsort((cand, -a[cand]))][:k]
        assert nsel[i] == len(order)
        np.testing.assert_array_equal(sel[i, :len(order)], order)
        assert np.all(sel[i, len(order):] == -1)
        assert vmax[i] == np.max(np.where(excl_bits[i], 0, np.abs(G[i])))


# ---------------------------------------------------------------------------
# Whole solves
# ---------------------------------------------------------------------------

def _solve_and_check(P, rho=None, rows=None, lam=None, **kw):
    pk = _lib()
    rho = P.rho if rho is None else rho
    lam = lam_rel(P.At, P.Bt, P.lambda_rel) if lam is None else lam
    s = pk.Solver(to_dev(P.At), 0.0, rho=rho, **kw)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    rows = range(P.p) if rows is None else rows
    ref = oracle.solve(P.At, P.Bt[list(rows)], lam[list(rows)], rho, **{k: v for k, v in kw.items() if k in (
        "max_outer", "max_active") and v})
    st = out["status"].cpu().numpy()
    return s, out, ref, lam, st


def test_small_gaussian_full():
    P = bi.small_gaussian()
    s, out, ref, lam, st = _solve_and_check(P)
    pk = _lib()
    assert np.all(st == pk.BMPL_SIG_CONVERGED)
    assert np.all(ref["status"] == oracle.ST_CONVERGED)
    check_batch(P.At, P.Bt, lam, out, ref)
    kkt = out["kkt"].cpu().numpy()
    assert np.all(kkt <= 1e-4)
    # objective and lambda reported by the library
    np.testing.assert_allclose(out["lambda"].cpu().numpy(), lam, rtol=0, atol=0)
    np.testing.assert_allclose(out["objective"].cpu().numpy(), ref["objective"], rtol=1e-9)


@pytest.mark.parametrize("gram_table", [True, False])
@pytest.mark.parametrize("n,m,p,k,rho,c", [(96, 700, 150, 8, 3, 0.05), (64, 4100, 300, 5, 10, 0.05),
                                           (256, 2000, 257, 30, 7, 0.05),
                                           (320, 3000, 100, 50, 10, 0.03)])   # |I| > 64: capacity growth
def test_ragged_tiles(n, m, p, k, rho, c, gram_table):
    P = bi.tiny_gaussian(n=n, m=m, p=p, k=k, sigma=0.01, seed=n + m, lambda_rel=c, rho=rho)
    s, out, ref, lam, st = _solve_and_check(P, gram_table=gram_table)
    pk = _lib()
    assert np.all(st == pk.BMPL_SIG_CONVERGED)
    check_batch(P.At, P.Bt, lam, out, ref)


@pytest.mark.parametrize("block_append", [True, False])
@pytest.mark.parametrize("n,m,p,k,rho,c", [(320, 3000, 100, 50, 10, 0.03), (256, 1500, 64, 60, 25, 0.02)])
def test_block_and_single_appends(n, m, p, k, rho, c, block_append):
    """The inverse factor grown in blocks (default) and one atom at a time: both meet the parity
    rules, including rho above the block width and supports of a few hundred atoms with drops."""
    P = bi.tiny_gaussian(n=n, m=m, p=p, k=k, sigma=0.01, seed=n + k, lambda_rel=c, rho=rho)
    s, out, ref, lam, st = _solve_and_check(P, block_append=block_append)
    pk = _lib()
    assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    check_batch(P.At, P.Bt, lam, out, ref)


def test_timing_counters():
    """Kernel timing and master-problem counters are reported and do not change the results."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=64, k=30, sigma=0.01, seed=5, rho=7)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    plain = pk.Solver(to_dev(P.At), 0.0, rho=P.rho).solve(to_dev(P.Bt), lam=to_dev(lam))
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, timing=True, phases=True)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    t = s.timing()
    assert torch.equal(out["x_idx"], plain["x_idx"]) and torch.equal(out["x_val"], plain["x_val"])
    assert t["solves"] == 1 and t["corr_launches"] >= int(out["iters"].max()) and t["corr_ms"] > 0
    assert t["wall_ms"] >= t["corr_ms"] + t["solve_ms"]
    assert t["corr_flops"] >= 2.0 * P.m * P.n * P.p          # the first pass covers every signal
    assert t["factor_appends"] >= int(out["supp_len"].sum()) and t["sign_fixed_solves"] > 0
    s.reset_timing()
    assert s.timing()["corr_launches"] == 0 and s.timing()["factor_appends"] == 0


def test_relative_lambda_rule():
    pk = _lib()
    P = bi.small_gaussian()
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho)
    out = s.solve(to_dev(P.Bt))
    lam_or = lam_rel(P.At, P.Bt, P.lambda_rel)
    lam_gpu = out["lambda"].cpu().numpy()
    assert np.all(np.abs(lam_gpu - lam_or) <= lam_bound(P.At, P.Bt, P.lambda_rel))
    ref = oracle.solve(P.At, P.Bt, lam_or, P.rho)
    check_batch(P.At, P.Bt, lam_or, out, ref)


@pytest.mark.parametrize("screen", ["fp32", "bf16", "fp8"])
def test_edge_cases(screen):
    pk = _lib()
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    Bt = P.Bt.copy()
    Bt[2, 7] = np.nan           # non-finite signal
    Bt[5] = 0.0                 # zero signal
    lam2 = lam.copy()
    lam2[9] = np.abs(P.At.astype(np.float64) @ P.Bt[9].astype(np.float64)).max() * 1.01   # lambda above max
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, screen=screen)
    out = s.solve(to_dev(Bt), lam=to_dev(lam2))
    st = out["status"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    ln = out["supp_len"].cpu().numpy()
    assert st[2] == pk.BMPL_SIG_NONFINITE and ln[2] == 0
    assert st[5] == pk.BMPL_SIG_CONVERGED and ln[5] == 0 and it[5] == 0
    assert st[9] == pk.BMPL_SIG_CONVERGED and ln[9] == 0 and it[9] == 0
    ok = [i for i in range(P.p) if i not in (2,)]
    ref = oracle.solve(P.At, Bt[ok], lam2[ok], P.rho)
    check_batch(P.At, Bt, lam2[ok], out, ref, rows=range(len(ok)), gpu_rows=ok)
    # a single signal, and an empty batch
    out1 = s.solve(to_dev(P.Bt[:1]), lam=to_dev(lam[:1]))
    ref1 = oracle.solve(P.At, P.Bt[:1], lam[:1], P.rho)
    check_batch(P.At, P.Bt[:1], lam[:1], out1, ref1)
    out0 = s.solve(to_dev(P.Bt[:0]), lam=to_dev(lam[:0]))
    assert out0["status"].numel() == 0


@pytest.mark.parametrize("screen", ["fp32", "bf16", "fp8"])
def test_caps_match_oracle_caps(screen):
    """Iteration and active-set caps; with max_active = 4 the selection is asked for k = 0 atoms once I is
    full (the screening kernels' stop-test-only path)."""
    pk = _lib()
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, max_outer=2, screen=screen)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    st = out["status"].cpu().numpy()
    ref = oracle.solve(P.At, P.Bt, lam, P.rho, max_outer=2)
    assert np.all((st & pk.BMPL_SIG_CAP_ITERS) == (ref["status"] & oracle.ST_CAP_ITERS) * 1)
    np.testing.assert_array_equal(out["iters"].cpu().numpy(), ref["iters"])
    # the capped iterate is the exact master solution on the same active sets
    Xg = dense_from_gpu(out, P.m)
    np.testing.assert_allclose(Xg, ref["X"], atol=1e-5)
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, max_active=4, screen=screen)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    st = out["status"].cpu().numpy()
    ref = oracle.solve(P.At, P.Bt, lam, P.rho, max_active=4)
    assert np.all(((st & pk.BMPL_SIG_CAP_ACTIVE) > 0) == ((ref["status"] & oracle.ST_CAP_ACTIVE) > 0))
    np.testing.assert_allclose(dense_from_gpu(out, P.m), ref["X"], atol=1e-5)


@pytest.mark.parametrize("max_active", [60, 70])
def test_graph_mode_active_cap_inside_a_segment(max_active):
    """Graph segments whose bound on |I| reaches the max_active cap inside the segment (rho = 10, four
    iterations per segment: the cap of 60 or 70 is first reached in the second segment and every later
    segment starts at it).  Each segment's kernels are sized by its own bounds, so results equal the host
    loop's bit for bit, no signal is reported inexact, and the capped results match the oracle's."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=160, k=40, sigma=0.01, seed=91, lambda_rel=0.05, rho=10)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    host = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, max_active=max_active).solve(to_dev(P.Bt), lam=to_dev(lam))
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, max_active=max_active, graph=True)
    for rep in range(2):                            # the second solve replays the cached segments
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        torch.cuda.synchronize()
        for key in ("x_idx", "x_val", "supp_len", "iters", "status"):
            assert torch.equal(out[key], host[key]), (rep, key)
    st = out["status"].cpu().numpy()
    assert not np.any(st & pk.BMPL_SIG_INEXACT)
    assert np.any(st & pk.BMPL_SIG_CAP_ACTIVE) and np.any(st & pk.BMPL_SIG_CONVERGED)
    ref = oracle.solve(P.At, P.Bt, lam, P.rho, max_active=max_active)
    assert np.array_equal((st & pk.BMPL_SIG_CAP_ACTIVE) > 0, (ref["status"] & oracle.ST_CAP_ACTIVE) > 0)
    np.testing.assert_allclose(dense_from_gpu(out, P.m), ref["X"], atol=1e-5)


def test_fp32_stop_certified_within_rounding_band():
    """The natural stop under the float32 product is certified: an atom whose float32 correlation lies
    below lambda while its exact correlation exceeds lambda (1 + 2e-4) is re-scored and admitted.
    The signal is b = a_J + v with v orthogonal to a_J and ||v|| = 3e5, so a_J^T b = 1 is a sum of
    far larger products and its float32 value carries a rounding error of about 1e-3; the other atoms
    live on the coordinates where b is zero (their correlations are exactly 0).  Among seeded v, one
    whose float32 product (the library's own kernel and tile shape, as in the solve's first pass) falls
    at least 3e-4 below the exact value is kept, and lambda is set between the two."""
    pk = _lib()
    n, m, h, J = 2048, 256, 1024, 0
    rng = np.random.default_rng(1302)
    A = np.zeros((m, n))
    A[J, :h] = rng.standard_normal(h)
    A[1:, h:] = rng.standard_normal((m - 1, n - h))
    At = (A / np.linalg.norm(A, axis=1, keepdims=True)).astype(np.float32)
    aJ = At[J].astype(np.float64)
    s = pk.Solver(to_dev(At), 1.0, rho=4)
    for _ in range(200):
        v = np.zeros(n)
        v[:h] = rng.standard_normal(h)
        v -= (v @ aJ) / (aJ @ aJ) * aJ
        v *= 3e5 / np.linalg.norm(v)
        b = (aJ + v).astype(np.float32)
        g = At.astype(np.float64) @ b.astype(np.float64)
        g32 = s.correlate(to_dev(b[None, :]))[0, :m].cpu().numpy()
        if g[J] > 0 and g32[J] < g[J] * (1 - 3e-4):
            break
    else:
        pytest.fail("no seeded signal with a float32 rounding error of 3e-4")
    assert np.all(g[1:] == 0)
    lam = np.array([g[J] / (1 + 2e-4)])
    assert g32[J] <= lam[0] < g[J]
    out = s.solve(to_dev(b[None, :]), lam=to_dev(lam))
    torch.cuda.synchronize()
    assert out["status"].cpu().numpy()[0] == pk.BMPL_SIG_CONVERGED
    assert out["supp_len"].cpu().numpy()[0] == 1 and out["x_idx"].cpu().numpy()[0, 0] == J
    x = dense_from_gpu(out, m)[0]
    r = b.astype(np.float64) - At.astype(np.float64).T @ x
    kkt = np.max(np.maximum(np.abs(At.astype(np.float64) @ r) - lam[0], 0.0)) / lam[0]
    assert kkt <= 1e-4 and out["kkt"].cpu().numpy()[0] <= 1e-4
    ref = oracle.solve(At, b[None, :], lam, 4)
    check_batch(At, b[None, :], lam, out, ref)


def test_warm_start_proposals_keep_parity():
    pk = _lib()
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    rng = np.random.default_rng(5)
    warm = np.full((P.p, 24), -1, dtype=np.int32)
    for i in range(P.p):
        if i % 4 == 0:
            continue                                          # empty proposal
        prop = list(P.supports[i]) + list(rng.integers(0, P.m, 6))   # truth plus junk
        if i % 4 == 1:
            prop = list(rng.integers(0, P.m, 12))                     # all junk
        prop = prop[:24]
        warm[i, :len(prop)] = prop
    warm[3, 0] = P.m + 5                                       # out of range entries are ignored
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam), warm=to_dev(warm))
    st = out["status"].cpu().numpy()
    assert np.all(st & pk.BMPL_SIG_CONVERGED)
    ref = oracle.solve(P.At, P.Bt, lam, P.rho)
    check_batch(P.At, P.Bt, lam, out, ref)
    assert np.all(st[1::4] & pk.BMPL_SIG_FALLBACK)              # junk proposals needed the pursuit


@pytest.mark.parametrize("block_append,graph", [(True, False), (False, True)])
def test_large_warm_proposals(block_append, graph):
    """Proposals of 200 atoms: past 32 new slots in one pass the Gram matrix is kept lazily (entries
    against support members only, a slot's column gathered when it enters S).  Truth plus junk, all junk
    and truth alone, with block and single factor appends."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=48, k=30, sigma=0.01, seed=91, rho=7)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    rng = np.random.default_rng(11)
    warm = np.full((P.p, 200), -1, dtype=np.int32)
    for i in range(P.p):
        truth = list(P.supports[i])
        junk = [int(j) for j in rng.permutation(P.m) if j not in truth]
        prop = {0: truth + junk[:200 - len(truth)], 1: junk[:200], 2: truth}[i % 3]
        warm[i, :len(prop)] = prop
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, block_append=block_append, graph=graph)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam), warm=to_dev(warm))
    st = out["status"].cpu().numpy()
    assert np.all(st & pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    ref = oracle.solve(P.At, P.Bt, lam, P.rho)
    check_batch(P.At, P.Bt, lam, out, ref)
    assert np.all(st[1::3] & pk.BMPL_SIG_FALLBACK)


def test_warm_start_support_outgrows_the_lds_factor():
    """A warm start whose support passes the 64 positions the first master solve keeps in LDS: the
    factor moves to global memory mid-solve and the result keeps parity."""
    pk = _lib()
    P = bi.tiny_gaussian(n=320, m=3000, p=24, k=90, sigma=0.01, seed=93, lambda_rel=0.01, rho=10)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    rng = np.random.default_rng(12)
    warm = np.full((P.p, 160), -1, dtype=np.int32)
    for i in range(P.p):
        truth = list(P.supports[i])
        junk = [int(j) for j in rng.permutation(P.m) if j not in truth]
        prop = truth + junk[:160 - len(truth)]
        warm[i, :len(prop)] = prop
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam), warm=to_dev(warm))
    st = out["status"].cpu().numpy()
    assert np.all(st & pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    assert out["supp_len"].cpu().numpy().max() > 64
    ref = oracle.solve(P.At, P.Bt, lam, P.rho)
    check_batch(P.At, P.Bt, lam, out, ref)


@pytest.mark.parametrize("n", [1024, 3000])
@pytest.mark.parametrize("screen", ["bf16", "fp8"])
def test_screening_with_many_candidates(screen, n):
    """An orthonormal dictionary and flat signals put every atom inside the reduced-precision band of
    the k-th largest correlation (n candidates per signal): the exact re-score runs its second,
    large-LDS pass for them, and the result keeps parity with the oracle.  With 3000 atoms the band
    holds more entries than the single-read screen buffers (2048), so the bfloat16 screen takes its
    sweep fallback and the e4m3 ranking's selection its rounds of argmax."""
    pk = _lib()
    At = np.eye(n, dtype=np.float32)
    rng = np.random.default_rng(21)
    Bt = (np.ones((4, n)) / np.sqrt(n) * (1.0 + 0.01 * rng.standard_normal((4, n)))).astype(np.float32)
    lam = 0.995 * np.abs(Bt.astype(np.float64)).max(axis=1)
    s = pk.Solver(to_dev(At), 0.0, rho=10, screen=screen)
    out = s.solve(to_dev(Bt), lam=to_dev(lam))
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED), st
    ref = oracle.solve(At, Bt, lam, 10)
    check_batch(At, Bt, lam, out, ref)


@pytest.mark.parametrize("screen", ["fp32", "bf16", "fp8"])
def test_odd_shapes(screen):
    """n, m and p that are multiples of nothing the kernels tile by (97 x 1003, 37 signals): padded
    k stages, a ragged atom tile, a ragged signal tile and the scalar tails of the selection."""
    pk = _lib()
    P = bi.tiny_gaussian(n=97, m=1003, p=37, k=9, sigma=0.01, seed=95, rho=3)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, screen=screen)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    ref = oracle.solve(P.At, P.Bt, lam, P.rho)
    check_batch(P.At, P.Bt, lam, out, ref)


@pytest.mark.slow
def test_cs_gaussian_full_size_sampled():
    """2048 x 16384 dictionary, 1024 signals, rho = 10: the benchmark's workload and launch;
    every 43rd signal is checked against the oracle."""
    pk = _lib()
    P = bi.cs_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho)
    out = s.solve(to_dev(P.Bt))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED)
    rows = list(range(0, P.p, 43))
    assert np.all(np.abs(out["lambda"].cpu().numpy() - lam) <= lam_bound(P.At, P.Bt, P.lambda_rel))
    ref = oracle.solve(P.At, P.Bt[rows], lam[rows], P.rho)
    errs = check_batch(P.At, P.Bt, lam[rows], out, ref, rows=range(len(rows)), gpu_rows=rows)
    assert max(e["rel_x"] for e in errs) <= 1e-4


@pytest.mark.parametrize("n,m", [(96, 700), (2048, 300), (64, 129)])
def test_gram_table_matches_float64(n, m):
    pk = _lib()
    rng = np.random.default_rng(n * m)
    At = rng.standard_normal((m, n)).astype(np.float32)
    s = pk.Solver(to_dev(At), 0.1)
    Q = s.gram_table().cpu().numpy()
    A64 = At.astype(np.float64)
    ref = A64 @ A64.T
    # float64 accumulation of exact products: within n ulps of the magnitudes
    bound = n * 2.0 ** -52 * (np.abs(A64) @ np.abs(A64).T) * 2
    assert np.all(np.abs(Q - ref) <= bound)
    assert np.array_equal(Q, Q.T)


def test_graph_mode_matches_host_loop():
    """Captured-graph segments (4 iterations per launch, device-side counts) give the same results."""
    pk = _lib()
    for P in (bi.small_gaussian(), bi.tiny_gaussian(n=256, m=2000, p=257, k=30, sigma=0.01, seed=77, rho=7)):
        lam = lam_rel(P.At, P.Bt, P.lambda_rel)
        host = pk.Solver(to_dev(P.At), 0.0, rho=P.rho).solve(to_dev(P.Bt), lam=to_dev(lam))
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, graph=True)
        for rep in range(3):                       # replays of the cached graphs
            out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
            torch.cuda.synchronize()
            for key in ("x_idx", "supp_len", "iters", "status"):
                assert torch.equal(out[key], host[key]), (rep, key)
            assert torch.equal(out["x_val"], host["x_val"])
        ref = oracle.solve(P.At, P.Bt, lam, P.rho)
        check_batch(P.At, P.Bt, lam, out, ref)


def test_graph_mode_large_batch_buckets():
    """A batch of 700 signals: graph segments that start with 512 or more running signals let the large
    correlation tile serve the middle bucket of counts too, so while signals converge the count passes
    through [64, 512) inside a segment.  Parity with the oracle, and the cached graphs replay exactly."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=700, k=30, sigma=0.01, seed=79, rho=7)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, graph=True)
    outs = [s.solve(to_dev(P.Bt), lam=to_dev(lam)) for _ in range(2)]
    torch.cuda.synchronize()
    for key in ("x_idx", "x_val", "supp_len", "iters", "status"):
        assert torch.equal(outs[0][key], outs[1][key]), key
    it = outs[0]["iters"].cpu().numpy()
    assert it.min() < it.max()                    # the count falls during the solve
    ref = oracle.solve(P.At, P.Bt, lam, P.rho)
    check_batch(P.At, P.Bt, lam, outs[1], ref)


# ---------------------------------------------------------------------------
# Reduced-precision screening (bfloat16 product, exact re-score)
# ---------------------------------------------------------------------------

def bf16_band(At, Rt):
    """Per-entry certified band gamma_n ||a_j|| ||r_i|| of the bfloat16 product."""
    n = At.shape[1]
    gamma = (2.0 ** -7 + 2.0 ** -16 + n * 2.0 ** -24) * 1.01
    an = np.linalg.norm(At.astype(np.float64), axis=1)
    rn = np.linalg.norm(Rt.astype(np.float64), axis=1)
    return gamma * np.outer(rn, an)


@pytest.mark.parametrize("n,m,p", [(128, 700, 33), (2048, 4100, 130)])
def test_bf16_correlate_within_band(n, m, p):
    pk = _lib()
    rng = np.random.default_rng(n + p)
    At = rng.standard_normal((m, n)).astype(np.float32)
    At /= np.linalg.norm(At, axis=1, keepdims=True)
    Rt = rng.standard_normal((p, n)).astype(np.float32)
    s = pk.Solver(to_dev(At), 0.1, screen="bf16")
    G = s.correlate(to_dev(Rt)).cpu().numpy().astype(np.float64)
    ref = Rt.astype(np.float64) @ At.astype(np.float64).T
    band = bf16_band(At, Rt)
    assert np.all(np.abs(G - ref) <= band)
    # and it is a bfloat16 product, not a float32 one: errors well above float32's
    assert np.max(np.abs(G - ref)) > 1e-4 * np.max(np.abs(ref))


def bf16_rne(x):
    """float32 -> nearest bfloat16 (ties to even), as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def bf16_rounding_band(At, Rt):
    """Per-entry band from the operands' own rounding: with a^ = bf16(a), x^ = bf16(r),
    a^ . x^ - a . r = a^ . (x^ - r) + (a^ - a) . r exactly, bounded by Cauchy-Schwarz, plus the
    float32 accumulation's n 2^-24 ||a^|| ||x^||."""
    n = At.shape[1]
    A64, R64 = At.astype(np.float64), Rt.astype(np.float64)
    Ah, Rh = bf16_rne(At).astype(np.float64), bf16_rne(Rt).astype(np.float64)
    nah = np.linalg.norm(Ah, axis=1)
    nda = np.linalg.norm(Ah - A64, axis=1)
    nr = np.linalg.norm(R64, axis=1)
    ndr = np.linalg.norm(Rh - R64, axis=1)
    nrh = np.linalg.norm(Rh, axis=1)
    return np.outer(ndr, nah) + np.outer(nr, nda) + n * 2.0 ** -24 * np.outer(nrh, nah)


@pytest.mark.parametrize("n,m,p", [(128, 700, 33), (2048, 4100, 130)])
def test_bf16_rounding_band_holds_and_is_tighter(n, m, p):
    """The band the screen uses (operand rounding measured, not assumed worst-case) holds entry by entry
    for the MFMA product and is well inside the worst-case band."""
    pk = _lib()
    rng = np.random.default_rng(7 * n + p)
    At = rng.standard_normal((m, n)).astype(np.float32)
    At /= np.linalg.norm(At, axis=1, keepdims=True)
    Rt = rng.standard_normal((p, n)).astype(np.float32)
    s = pk.Solver(to_dev(At), 0.1, screen="bf16")
    G = s.correlate(to_dev(Rt)).cpu().numpy().astype(np.float64)
    ref = Rt.astype(np.float64) @ At.astype(np.float64).T
    tight = bf16_rounding_band(At, Rt)
    assert np.all(np.abs(G - ref) <= tight)
    assert np.max(tight / bf16_band(At, Rt)) < 0.6


@pytest.mark.parametrize("graph", [False, True])
def test_bf16_screening_parity(graph):
    pk = _lib()
    for P in (bi.small_gaussian(), bi.tiny_gaussian(n=256, m=2000, p=257, k=30, sigma=0.01, seed=91, rho=7)):
        lam = lam_rel(P.At, P.Bt, P.lambda_rel)
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, screen="bf16", graph=graph)
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        st = out["status"].cpu().numpy()
        assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st)
        ref = oracle.solve(P.At, P.Bt, lam, P.rho)
        check_batch(P.At, P.Bt, lam, out, ref)
        # same selections as the float32 path up to near-ties: identical supports here
        f32 = pk.Solver(to_dev(P.At), 0.0, rho=P.rho).solve(to_dev(P.Bt), lam=to_dev(lam))
        assert torch.equal(out["supp_len"], f32["supp_len"]) and torch.equal(out["x_idx"], f32["x_idx"])


def test_bf16_relative_lambda_is_exact_maximum():
    pk = _lib()
    P = bi.small_gaussian()
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, screen="bf16")
    out = s.solve(to_dev(P.Bt))
    lam_or = lam_rel(P.At, P.Bt, P.lambda_rel)
    # re-scored in float64 from float32 data: far tighter than the bfloat16 band
    np.testing.assert_allclose(out["lambda"].cpu().numpy(), lam_or, rtol=1e-12)
    ref = oracle.solve(P.At, P.Bt, lam_or, P.rho)
    check_batch(P.At, P.Bt, lam_or, out, ref)


@pytest.mark.slow
def test_cs_gaussian_bf16_full_size_sampled():
    pk = _lib()
    P = bi.cs_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, screen="bf16", graph=True)
    out = s.solve(to_dev(P.Bt))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED)
    np.testing.assert_allclose(out["lambda"].cpu().numpy(), lam, rtol=1e-12)
    rows = list(range(7, P.p, 61))
    ref = oracle.solve(P.At, P.Bt[rows], lam[rows], P.rho)
    check_batch(P.At, P.Bt, lam[rows], out, ref, rows=range(len(rows)), gpu_rows=rows)


# ---------------------------------------------------------------------------
# e4m3 ranking (screen="fp8")
# ---------------------------------------------------------------------------

def fp8_band(At, Rt):
    """Per-entry bound on the e4m3 product with power-of-two row scales s <= 2 max|x| / 448.

    Encoding error per element: 2^-4 |x| in the normal range, s 2^-10 below it (half the subnormal
    spacing 2^-9 times the scale).  Summing |a~ r~ - a r| <= |a~ - a||r~| + |a||r~ - r| over k with
    Cauchy-Schwarz (sum |a| <= sqrt(n) ||a||) gives
      ||a|| ||r|| [2^-3 + 2^-8 + 2 (1 + 2^-4) sqrt(n) 2^-9 / 448 + n (2^-9 / 448)^2],
    plus the accumulation: float32 across instructions, n 2^-24 (1 + 2^-3)^2 ||a|| ||r||, and inside each
    64-term instruction a sum that is not exact in float32 (measured at 1.3e-4 of the sum of |products|
    on gfx950), bounded here by 2^-11 (1 + 2^-3)^2 ||a|| ||r||."""
    n = At.shape[1]
    e = 2.0 ** -9 / 448
    gamma = (2.0 ** -3 + 2.0 ** -8 + 2 * (1 + 2.0 ** -4) * np.sqrt(n) * e + n * e * e
             + (n * 2.0 ** -24 + 2.0 ** -11) * (1 + 2.0 ** -3) ** 2) * 1.01
    an = np.linalg.norm(At.astype(np.float64), axis=1)
    rn = np.linalg.norm(Rt.astype(np.float64), axis=1)
    return gamma * np.outer(rn, an)


def e4m3_decode(codes):
    c = codes.astype(np.int64)
    sgn = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 15
    q = c & 7
    v = np.where(e == 0, q * 2.0 ** -9, (1 + q / 8.0) * 2.0 ** (e - 7))
    return sgn * v


def e4m3_encode_reference(x):
    """Nearest finite e4m3 value (ties to the even code), saturating at 448: brute force."""
    codes = np.arange(127)
    vals = e4m3_decode(codes)
    a = np.abs(x.astype(np.float64))[:, None]
    d = np.abs(a - vals[None, :])
    best = np.argmin(d, axis=1)
    # ties: prefer the even code
    dmin = d[np.arange(len(x)), best]
    tie = (np.abs(d - dmin[:, None]) == 0).sum(axis=1) > 1
    for i in np.nonzero(tie)[0]:
        cand = np.nonzero(d[i] == dmin[i])[0]
        best[i] = cand[(cand & 1) == 0][0]
    return np.where(x < 0, 0x80, 0) | best


@pytest.mark.parametrize("n,m,p", [(128, 700, 33), (1024, 4100, 130)])
def test_fp8_correlate_within_band(n, m, p):
    pk = _lib()
    rng = np.random.default_rng(n + p + 8)
    At = rng.standard_normal((m, n)).astype(np.float32)
    At /= np.linalg.norm(At, axis=1, keepdims=True)
    Rt = (rng.standard_normal((p, n)) * 10.0 ** rng.uniform(-3, 1, (p, 1))).astype(np.float32)
    Rt[0, ::3] *= 1e-3             # entries deep in the subnormal range of the scaled row
    s = pk.Solver(to_dev(At), 0.1, screen="fp8")
    G = s.correlate(to_dev(Rt)).cpu().numpy().astype(np.float64)
    ref = Rt.astype(np.float64) @ At.astype(np.float64).T
    band = fp8_band(At, Rt)
    assert np.all(np.abs(G - ref) <= band), np.max(np.abs(G - ref) / band)
    # an e4m3 product: errors far above a float32 or bfloat16 product's
    assert np.max(np.abs(G - ref)) > 1e-3 * np.max(np.abs(ref))


def test_fp8_encoder_matches_reference():
    """The library's e4m3 rounding, seen through a product with one-hot atoms: G[i, j] = r_i[j]
    rounded to e4m3 at the row's power-of-two scale."""
    pk = _lib()
    n = 128
    rng = np.random.default_rng(3)
    At = np.eye(n, dtype=np.float32)                       # atom j = e_j, scale 1 (max 1 -> 2^-8)
    vals = e4m3_decode(np.arange(127))
    x = np.concatenate([vals[:126], 0.5 * (vals[:125] + vals[1:126]), rng.uniform(-448, 448, 400)])
    rows = []
    for i in range(0, len(x), n):
        r = np.zeros(n, dtype=np.float32)
        chunk = x[i:i + n].astype(np.float32)
        r[:len(chunk)] = chunk
        r[-1] = 448.0          # pins the row's scale to 1
        rows.append(r)
    Rt = np.array(rows)
    s = pk.Solver(to_dev(At), 0.1, screen="fp8")
    G = s.correlate(to_dev(Rt)).cpu().numpy()
    # atom scale: max |e_j| = 1 -> s_a = 2^-8, so a~ = 256 * 2^-8 exactly; the product is r~ exactly
    want = e4m3_decode(e4m3_encode_reference(Rt.ravel().astype(np.float64))).reshape(Rt.shape)
    np.testing.assert_array_equal(G.astype(np.float64), want)


@pytest.mark.parametrize("graph", [False, True])
def test_fp8_ranking_parity(graph):
    pk = _lib()
    for P in (bi.small_gaussian(), bi.tiny_gaussian(n=256, m=2000, p=257, k=30, sigma=0.01, seed=91, rho=7),
              bi.tiny_gaussian(n=320, m=3000, p=100, k=50, sigma=0.01, seed=650, lambda_rel=0.03, rho=10)):
        lam = lam_rel(P.At, P.Bt, P.lambda_rel)
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, screen="fp8", graph=graph)
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        st = out["status"].cpu().numpy()
        assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
        ref = oracle.solve(P.At, P.Bt, lam, P.rho)
        check_batch(P.At, P.Bt, lam, out, ref)


def test_fp8_relative_lambda_rule():
    pk = _lib()
    P = bi.small_gaussian()
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, screen="fp8")
    out = s.solve(to_dev(P.Bt))
    lam_or = lam_rel(P.At, P.Bt, P.lambda_rel)
    np.testing.assert_allclose(out["lambda"].cpu().numpy(), lam_or, rtol=1e-12)
    ref = oracle.solve(P.At, P.Bt, lam_or, P.rho)
    check_batch(P.At, P.Bt, lam_or, out, ref)


@pytest.mark.slow
def test_cs_gaussian_fp8_full_size_sampled():
    pk = _lib()
    P = bi.cs_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, screen="fp8", graph=True)
    out = s.solve(to_dev(P.Bt))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED)
    rows = list(range(11, P.p, 61))
    ref = oracle.solve(P.At, P.Bt[rows], lam[rows], P.rho)
    check_batch(P.At, P.Bt, lam[rows], out, ref, rows=range(len(rows)), gpu_rows=rows)


# ---------------------------------------------------------------------------
# Ragged supports (1024 x 32768, k ~ U{10..400}) and the face-like dictionary
# ---------------------------------------------------------------------------

def _golden_ragged():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ragged1024x32768_oracle.json")
    with open(path) as f:
        raw = json.load(f)
    g = {"rows": np.array(raw["rows"]), "iters": np.array(raw["iters"]),
         "lam": np.array([float.fromhex(v) for v in raw["lam"]])}
    val = [float.fromhex(v) for v in raw["val"]]
    X = np.zeros((len(g["rows"]), 32768))
    off = 0
    for q, ln in enumerate(raw["supp_len"]):
        X[q, raw["idx"][off:off + ln]] = val[off:off + ln]
        off += ln
    return g, X


def test_ragged_supports_against_stored_oracle():
    """Six signals of the ragged workload (supports 10 to 955 atoms, 1 to 152 iterations), solved as
    one batch, against oracle results stored by tests/golden/make_golden.py."""
    pk = _lib()
    g, X = _golden_ragged()
    rows = [int(r) for r in g["rows"]]
    P = bi.ragged_gaussian(indices=rows)
    lam = g["lam"]
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, graph=True)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() == pk.BMPL_SIG_CONVERGED)
    ref = {"X": X}
    check_batch(P.At, P.Bt, lam, out, ref)
    # iteration counts are informational (a near-tie in a selection may change the path, not the
    # result); nearly all agree
    assert np.mean(out["iters"].cpu().numpy() == g["iters"]) >= 0.9


@pytest.mark.slow
@pytest.mark.parametrize("block_append", [False, True])
def test_ragged_full_batch(block_append):
    """All 4096 ragged signals in one solve (graph segments; the active sets of the k >= 200 signals grow
    to ~1600 atoms, so each of their float64 Gram matrices of I reaches ~20 MB, while the k <= 150 signals
    stop with a few hundred slots: every signal's slot block follows its own |I|).  Every signal must
    converge and the stored oracle rows must match, with single appends and with block appends (whose
    kernel streams factors of up to ~980 positions from global memory through the Givens downdate's
    register path, where a missing barrier once corrupted a few signals per run)."""
    pk = _lib()
    g, X = _golden_ragged()
    rows = [int(r) for r in g["rows"]]
    P = bi.ragged_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    np.testing.assert_allclose(lam[rows], g["lam"], rtol=1e-15)
    s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, graph=True, block_append=block_append)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    check_batch(P.At, P.Bt, lam[rows], out, {"X": X}, rows=range(len(rows)), gpu_rows=rows)


@pytest.mark.parametrize("screen", ["fp32", "bf16", "fp8"])
def test_face_like_sampled(screen):
    """Correlated class-structured dictionary (200 classes x 100 atoms, rank-8 class subspaces):
    all 8192 signals solved, 64 sampled signals against the oracle; the l1 mass sits in the true class
    (a few LASSO solutions carry tiny out-of-class coefficients, which the oracle shares)."""
    pk = _lib()
    P = bi.face_like()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, screen=screen, graph=True)
    out = s.solve(to_dev(P.Bt))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
    rows = list(range(3, P.p, 128))
    ref = oracle.solve(P.At, P.Bt[rows], lam[rows], P.rho)
    check_batch(P.At, P.Bt, lam[rows], out, ref, rows=range(len(rows)), gpu_rows=rows)
    cls = P.meta["class_of_atom"]
    Xg = dense_from_gpu(out, P.m)
    for i in rows:
        S = np.nonzero(Xg[i])[0]
        mass = np.bincount(cls[S], weights=np.abs(Xg[i][S]), minlength=int(cls.max()) + 1)
        true_cls = P.supports[i][0] // 100
        assert np.argmax(mass) == true_cls and mass[true_cls] >= 0.99 * mass.sum()


def test_src_classification_face_like():
    """Class-residual classification of the face-like signals from the GPU codes: labels and residuals
    against the float64 reference on the same codes (sampled), and the recognition rate."""
    pk = _lib()
    from oracle import src_oracle
    P = bi.face_like(indices=range(2048))
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, screen="bf16", graph=True)
    Bt = to_dev(P.Bt)
    out = s.solve(Bt)
    cls = P.meta["class_of_atom"].astype(np.int32)
    labels, resid = s.classify(Bt, out, to_dev(cls))
    labels = labels.cpu().numpy()
    resid = resid.cpu().numpy()
    rows = list(range(0, P.p, 16))
    X = dense_from_gpu({k: out[k][rows] for k in ("x_idx", "x_val", "supp_len")}, P.m)
    lab_ref, res_ref = src_oracle.classify(P.At, P.Bt[rows], X, cls)
    np.testing.assert_array_equal(labels[rows], lab_ref)
    np.testing.assert_allclose(resid[rows], res_ref, rtol=1e-9)
    truth = np.array([P.supports[i][0] // 100 for i in range(P.p)])
    acc = float(np.mean(labels == truth))
    print(f"recognition rate {acc:.4f}")
    assert acc >= 0.99


@pytest.mark.parametrize("graph", [False, True])
def test_q_route_parity(graph):
    """Section III's correlation g = beta - Q_{:,S} x_S (float64) in place of the MFMA product."""
    pk = _lib()
    for P in (bi.small_gaussian(), bi.tiny_gaussian(n=256, m=2000, p=257, k=30, sigma=0.01, seed=91, rho=7),
              bi.tiny_gaussian(n=320, m=3000, p=100, k=50, sigma=0.01, seed=650, lambda_rel=0.03, rho=10)):
        lam = lam_rel(P.At, P.Bt, P.lambda_rel)
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, q_route=True, graph=graph)
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        st = out["status"].cpu().numpy()
        assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
        ref = oracle.solve(P.At, P.Bt, lam, P.rho)
        check_batch(P.At, P.Bt, lam, out, ref)


def test_q_route_needs_the_gram_table():
    pk = _lib()
    P = bi.small_gaussian()
    with pytest.raises(pk.BmplError):
        pk.Solver(to_dev(P.At), 0.1, q_route=True, gram_table=False)
    with pytest.raises(pk.BmplError):
        pk.Solver(to_dev(P.At), 0.1, q_route=True, screen="bf16")


@pytest.mark.slow
def test_cs_gaussian_q_route_full_size_sampled():
    pk = _lib()
    P = bi.cs_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), P.lambda_rel, mode="rel", rho=P.rho, q_route=True, graph=True)
    out = s.solve(to_dev(P.Bt))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert np.all(st == pk.BMPL_SIG_CONVERGED)
    rows = list(range(3, P.p, 61))
    ref = oracle.solve(P.At, P.Bt[rows], lam[rows], P.rho)
    check_batch(P.At, P.Bt, lam[rows], out, ref, rows=range(len(rows)), gpu_rows=rows)


@pytest.mark.parametrize("graph,screen", [(False, "fp32"), (True, "fp32"), (True, "bf16")])
def test_smpl_parity(graph, screen):
    """Subspace exploratory matching (Algorithm 2, omega = 3): the LASSO solution at the parity rules,
    and iteration counts close to the SMPL oracle's (the path is the same up to near-ties in |u|)."""
    pk = _lib()
    for P in (bi.small_gaussian(), bi.tiny_gaussian(n=256, m=2000, p=257, k=30, sigma=0.01, seed=91, rho=7),
              bi.tiny_gaussian(n=320, m=3000, p=100, k=50, sigma=0.01, seed=650, lambda_rel=0.03, rho=10)):
        lam = lam_rel(P.At, P.Bt, P.lambda_rel)
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, omega=3, graph=graph, screen=screen)
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        st = out["status"].cpu().numpy()
        assert np.all(st == pk.BMPL_SIG_CONVERGED), np.unique(st, return_counts=True)
        ref = oracle.solve(P.At, P.Bt, lam, P.rho, omega=3)
        check_batch(P.At, P.Bt, lam, out, ref)
        it = out["iters"].cpu().numpy()
        assert np.mean(np.abs(it - ref["iters"])) <= 1.0, (it[:10], ref["iters"][:10])


def test_smpl_needs_the_gram_table_and_a_width_limit():
    pk = _lib()
    P = bi.small_gaussian()
    with pytest.raises(pk.BmplError):
        pk.Solver(to_dev(P.At), 0.1, omega=3, gram_table=False)
    with pytest.raises(pk.BmplError):
        pk.Solver(to_dev(P.At), 0.1, rho=30, omega=3)
