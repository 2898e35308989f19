"""GPU parity of the stopping variants: lambda = 0 (OMP for rho = 1, end of the "Stopping
Conditions" subsection), the early stops of Eq. (10) and the objective-decrease stop of Eq. (13).

These results depend on the path, not only on the problem: the GPU has to take the same atoms at every
outer iteration and stop at the same one as the FP64 oracle.  Both take each decision in their own
arithmetic (the GPU ranks atoms by its float32 correlation product), so a decision whose margin is
within the GPU's rounding can go either way.  Every signal is compared with the oracle (status,
iteration count, and the parity rules of tests/parity.py on x); a signal that differs must have such a
near-tie on the oracle's path at or before the iteration where the two part, and such signals must be
rare.  Margins are measured here from the oracle's own iterates (x after t outer iterations is the
oracle's solve capped at t iterations):
  * selection: the gap between the rho-th and (rho+1)-th largest |g_j| outside I, and between any |g_j|
    and lambda, relative to ||xi|| (the float32 product's error is about 2 n u ||a_j|| ||xi||);
  * Eq. (10): |max_{j not in I} |g_j| - r_inf| relative to ||xi||, | ||xi|| - r_2 | relative to r_2;
  * Eq. (13): |delta^t - eps rho ||b||^2| relative to eps rho ||b||^2.
"""
import numpy as np
import pytest

import bmpl_inputs as bi
import oracle
from tests.parity import check_signal, dense_from_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEL_TIE = 1e-4      # selection margins below this (relative to ||xi||) may flip in float32
STOP_TIE = 1e-6     # stop-rule margins below this (relative) may flip
MAX_TIED = 0.1      # at most this fraction of a batch may part from the oracle


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_5010_amd as pk
    return pk


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lam_rel(At, Bt, c):
    return c * np.abs(At.astype(np.float64) @ Bt.astype(np.float64).T).max(axis=0)


def path_has_near_tie(At, b, lam, rho, T, eps_early=0.0, r_inf_rel=0.0, r2_rel=0.0, omega=1):
    """True if some decision of the oracle's path within its first T + 1 stop tests had a margin
    within the GPU's rounding."""
    A = At.astype(np.float64).T
    b64 = b.astype(np.float64)
    bb = float(b64 @ b64)
    full = oracle.trace(At, b, lam, rho, max_outer=T + 1, omega=omega)
    g0 = np.abs(A.T @ b64)
    r_inf = r_inf_rel * g0.max()
    r_2 = r2_rel * np.sqrt(bb)
    inI = np.zeros(A.shape[1], bool)
    f_prev = None
    for t in range(min(T + 1, full["iters"] + 1)):
        x_t = np.zeros(A.shape[1]) if t == 0 else oracle.trace(At, b, lam, rho, max_outer=t, omega=omega)["x"]
        r = b64 - A @ x_t
        rn = np.linalg.norm(r)
        f = 0.5 * rn * rn + lam * np.abs(x_t).sum()
        v = np.sort(np.abs(A.T @ r)[~inI])[::-1]
        k = rho * omega
        gaps = [abs(v[q] - lam) for q in range(min(len(v), k + 1))]
        if len(v) > k and v[k] > lam:
            gaps.append(v[k - 1] - v[k])
        if min(gaps) <= SEL_TIE * rn:
            return True
        if r_inf_rel > 0 and abs(v[0] - r_inf) <= SEL_TIE * rn:
            return True
        if r2_rel > 0 and abs(rn - r_2) <= STOP_TIE * r_2:
            return True
        if eps_early > 0 and f_prev is not None and abs(abs(f_prev - f) - eps_early * rho * bb) <= STOP_TIE * eps_early * rho * bb:
            return True
        f_prev = f
        if t < len(full["steps"]):
            inI[full["steps"][t][0]] = True
    return False


def compare_path(P, lam, out, rho, expect_status, **stop):
    """Status, iteration count and x of every signal against the oracle, up to near-ties."""
    pk = _lib()
    omega = stop.get("omega", 1)
    ref = oracle.solve(P.At, P.Bt, lam, rho, max_outer=stop.get("max_outer"), omega=omega,
                       eps_early=stop.get("eps_early", 0.0), r_inf_rel=stop.get("r_inf_rel", 0.0),
                       r2_rel=stop.get("r2_rel", 0.0))
    st = out["status"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    Xg = dense_from_gpu(out, P.At.shape[0])
    A64 = P.At.astype(np.float64).T
    oracle_bits = {oracle.ST_EARLY: pk.BMPL_SIG_EARLY, oracle.ST_CAP_ITERS: pk.BMPL_SIG_CAP_ITERS,
                   oracle.ST_CONVERGED: pk.BMPL_SIG_CONVERGED}
    assert np.mean(ref["status"] == expect_status) >= 0.9, np.unique(ref["status"], return_counts=True)
    tied = 0
    for i in range(P.p):
        same = st[i] == oracle_bits.get(int(ref["status"][i]), -1) and it[i] == ref["iters"][i]
        why = "status or iteration count"
        if same:
            try:
                check_signal(A64, P.Bt[i].astype(np.float64), float(lam[i]), Xg[i], ref["X"][i], tag=f"signal {i}")
                continue
            except AssertionError as e:
                why = str(e).splitlines()[0]
        T = int(min(it[i], ref["iters"][i]))
        assert path_has_near_tie(P.At, P.Bt[i], float(lam[i]), rho, T, omega=omega,
                                 **{k: v for k, v in stop.items() if k in ("eps_early", "r_inf_rel", "r2_rel")}), (
            f"signal {i}: GPU status {st[i]} after {it[i]} iterations, oracle {ref['status'][i]} after "
            f"{ref['iters'][i]} ({why}), with no near-tie on the path")
        tied += 1
    assert tied <= MAX_TIED * P.p, f"{tied} of {P.p} signals parted from the oracle at near-ties"
    return ref


@pytest.mark.parametrize("screen,graph", [("fp32", False), ("fp32", True), ("bf16", True)])
def test_omp_lambda0_rho1(screen, graph):
    """lambda = 0, rho = 1: OMP (least squares on I after each greedy pick), 20 iterations."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=64, k=30, sigma=0.01, seed=80, rho=1)
    lam = np.zeros(P.p)
    s = pk.Solver(to_dev(P.At), 0.0, rho=1, max_outer=20, screen=screen, graph=graph)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    compare_path(P, lam, out, 1, oracle.ST_CAP_ITERS, max_outer=20)
    assert np.all(out["supp_len"].cpu().numpy() == 20)


@pytest.mark.parametrize("graph", [False, True])
def test_omp_lambda0_residual_stop(graph):
    """lambda = 0, rho = 1 with Eq. (10)'s residual radius: OMP stopped at ||xi|| <= r_2."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=64, k=30, sigma=0.01, seed=81, rho=1)
    lam = np.zeros(P.p)
    s = pk.Solver(to_dev(P.At), 0.0, rho=1, max_outer=60, r2_rel=0.05, graph=graph)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    compare_path(P, lam, out, 1, oracle.ST_EARLY, max_outer=60, r2_rel=0.05)


def test_batch_omp_lambda0_correlation_stop():
    """lambda = 0, rho = 4 (several atoms per iteration) with Eq. (10)'s correlation radius."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=64, k=30, sigma=0.01, seed=82, rho=4)
    lam = np.zeros(P.p)
    s = pk.Solver(to_dev(P.At), 0.0, rho=4, max_outer=40, r_inf_rel=0.03, graph=True)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    compare_path(P, lam, out, 4, oracle.ST_EARLY, max_outer=40, r_inf_rel=0.03)


@pytest.mark.parametrize("screen,graph,omega", [("fp32", False, 1), ("fp32", True, 1), ("bf16", True, 1),
                                                ("fp32", True, 3)])
def test_early_stop_eq13(screen, graph, omega):
    """The paper's experimental stop, Eq. (13) with eps = 1e-5, at a small lambda (the over-fitting
    regime it is meant for): same stopping iteration and the same x as the oracle."""
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=64, k=30, sigma=0.01, seed=70, lambda_rel=0.002, rho=5)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), 0.0, rho=5, eps_early=1e-5, screen=screen, graph=graph, omega=omega)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    ref = compare_path(P, lam, out, 5, oracle.ST_EARLY, eps_early=1e-5, omega=omega)
    assert ref["iters"].mean() < 20        # far from the 50 iterations of the full solve


@pytest.mark.parametrize("rule", [{"r2_rel": 0.05}, {"r_inf_rel": 0.02}])
def test_early_stop_eq10_lasso(rule):
    pk = _lib()
    P = bi.tiny_gaussian(n=256, m=2000, p=64, k=30, sigma=0.01, seed=71, lambda_rel=0.002, rho=5)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    s = pk.Solver(to_dev(P.At), 0.0, rho=5, graph=True, **rule)
    out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
    torch.cuda.synchronize()
    compare_path(P, lam, out, 5, oracle.ST_EARLY, **rule)


def test_early_stops_off_by_default_and_natural_stop_first():
    """With every early stop off the solve reaches the natural stop; with radii so small that they
    never hold before it, the result is the LASSO solution with status CONVERGED."""
    pk = _lib()
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    ref = oracle.solve(P.At, P.Bt, lam, P.rho)
    for kw in ({}, {"r2_rel": 1e-9, "r_inf_rel": 1e-9, "eps_early": 1e-14}):
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, **kw)
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        assert np.all(out["status"].cpu().numpy() == pk.BMPL_SIG_CONVERGED)
        Xg = dense_from_gpu(out, P.At.shape[0])
        for i in range(P.p):
            check_signal(P.At.astype(np.float64).T, P.Bt[i].astype(np.float64), float(lam[i]), Xg[i], ref["X"][i])


def test_early_stop_radius_one_stops_before_any_atom():
    """r_inf_rel >= 1 (or r2_rel >= 1) holds at the first test: x = 0, no iteration, status EARLY."""
    pk = _lib()
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    for kw in ({"r_inf_rel": 1.0}, {"r2_rel": 1.0}):
        s = pk.Solver(to_dev(P.At), 0.0, rho=P.rho, **kw)
        out = s.solve(to_dev(P.Bt), lam=to_dev(lam))
        assert np.all(out["status"].cpu().numpy() == pk.BMPL_SIG_EARLY)
        assert np.all(out["iters"].cpu().numpy() == 0) and np.all(out["supp_len"].cpu().numpy() == 0)
        ref = oracle.solve(P.At, P.Bt, lam, P.rho, **kw)
        assert np.all(ref["status"] == oracle.ST_EARLY) and np.all(ref["iters"] == 0)
