"""Pins of the FP64 oracle against facts that do not depend on it.

Each test fixes the oracle to something other than itself: brute-force
enumeration of supports and signs, the LASSO optimality conditions (the natural
stopping condition, Eq. (9)), the dual of Eq. (5), closed forms (orthonormal
dictionaries; noiseless sign-consistent recovery), the OMP reduction
(lambda = 0, rho = 1, end of Section II-A), the per-iteration decrease bound of
Lemma 1 with the monotone objective of Section II-B, an independent
full-problem coordinate descent, and exact invariances of the problem.
"""
import itertools

import numpy as np
import pytest

import bmpl_inputs as bi
import oracle


def lam_rel(At, Bt, c):
    return c * np.abs(At.astype(np.float64) @ Bt.astype(np.float64).T).max(axis=0)


def kkt_residuals(At, b, x, lam):
    """(max off-support excess, max on-support deviation) of the LASSO conditions."""
    A = At.astype(np.float64).T
    r = b.astype(np.float64) - A @ x
    g = A.T @ r
    on = x != 0
    off_ex = np.max(np.abs(g[~on]) - lam) if (~on).any() else -np.inf
    on_dev = np.max(np.abs(g[on] - lam * np.sign(x[on]))) if on.any() else 0.0
    return off_ex, on_dev


def brute_force_lasso(At, b, lam):
    """Enumerate every sign vector s in {-1,0,1}^m; keep the ones whose sign-fixed
    normal-equation solution is sign-consistent and dual feasible."""
    A = At.astype(np.float64).T
    b = b.astype(np.float64)
    n, m = A.shape
    sols = []
    for s in itertools.product((-1.0, 0.0, 1.0), repeat=m):
        s = np.array(s)
        S = np.nonzero(s)[0]
        if len(S) > n:
            continue
        x = np.zeros(m)
        if len(S):
            AS = A[:, S]
            xs = np.linalg.solve(AS.T @ AS, AS.T @ b - lam * s[S])
            if np.any(np.sign(xs) != s[S]):
                continue
            x[S] = xs
        g = A.T @ (b - A @ x)
        off = np.setdiff1d(np.arange(m), S)
        if len(off) and np.max(np.abs(g[off])) > lam * (1 + 1e-12):
            continue
        sols.append(x)
    return sols


@pytest.mark.parametrize("seed,lrel", [(1, 0.05), (2, 0.15), (3, 0.01), (4, 0.3)])
def test_brute_force_enumeration(seed, lrel):
    P = bi.tiny_gaussian(n=6, m=10, p=1, k=3, sigma=0.05, seed=seed)
    lam = lam_rel(P.At, P.Bt, lrel)
    sols = brute_force_lasso(P.At, P.Bt[0], lam[0])
    assert len(sols) == 1, "general position gives exactly one LASSO solution"
    r = oracle.solve(P.At, P.Bt, lam, rho=2)
    assert r["status"][0] & oracle.ST_CONVERGED
    np.testing.assert_allclose(r["X"][0], sols[0], rtol=0, atol=1e-10)


def test_kkt_on_every_output():
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    r = oracle.solve(P.At, P.Bt, lam, P.rho)
    assert np.all(r["status"] == oracle.ST_CONVERGED)
    for i in range(P.p):
        off_ex, on_dev = kkt_residuals(P.At, P.Bt[i], r["X"][i], lam[i])
        assert off_ex <= 1e-9 * lam[i]
        assert on_dev <= 1e-9 * lam[i]
        assert r["kkt"][i] <= 1e-9


def test_duality_gap_of_eq5():
    P = bi.small_gaussian()
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    r = oracle.solve(P.At, P.Bt, lam, P.rho)
    A = P.At.astype(np.float64).T
    for i in range(P.p):
        b = P.Bt[i].astype(np.float64)
        x = r["X"][i]
        res = b - A @ x
        F = 0.5 * res @ res + lam[i] * np.abs(x).sum()
        alpha = res * min(1.0, lam[i] / np.abs(A.T @ res).max())
        D = -0.5 * alpha @ alpha + alpha @ b
        assert F - D <= 1e-12 * F
        assert abs(F - r["objective"][i]) <= 1e-12 * F
        assert abs(r["gap"][i] - (F - D)) <= 1e-12 * F


def independent_certificate(At, b, x, lam):
    A = At.astype(np.float64).T
    g = A.T @ (b.astype(np.float64) - A @ x)
    on = x != 0
    off = np.maximum(np.abs(g[~on]) - lam, 0.0).max(initial=0.0)
    onv = np.abs(g[on] - lam * np.sign(x[on])).max(initial=0.0)
    mu = min(np.min(lam - np.abs(g[~on]), initial=np.inf), np.min(np.abs(x[on]), initial=np.inf))
    return max(off, onv) / lam, mu


@pytest.mark.parametrize("max_outer", [1, 2, None])
def test_reported_certificate_and_margin(max_outer):
    # kappa and the margin reported by the oracle equal their definitions, also away from the optimum
    P = bi.small_gaussian(indices=[0, 4, 8])
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    r = oracle.solve(P.At, P.Bt, lam, P.rho, max_outer=max_outer)
    for i in range(P.p):
        kap, mu = independent_certificate(P.At, P.Bt[i], r["X"][i], lam[i])
        assert abs(r["kkt"][i] - kap) <= 1e-9 * max(1.0, kap)
        A = P.At.astype(np.float64).T
        b = P.Bt[i].astype(np.float64)
        res = b - A @ r["X"][i]
        F = 0.5 * res @ res + lam[i] * np.abs(r["X"][i]).sum()
        alpha = res * min(1.0, lam[i] / np.abs(A.T @ res).max())
        assert abs(r["gap"][i] - (F - (-0.5 * alpha @ alpha + alpha @ b))) <= 1e-12 * F
        assert abs(r["margin"][i] - mu) <= 1e-9 * lam[i]
        if max_outer == 1:
            assert kap > 1e-3                        # one iteration is far from optimal here


def test_orthonormal_dictionary_closed_form_and_iteration_count():
    # A with orthonormal columns: x = soft(A^T b, lambda) and MPL needs ceil(|S|/rho) additions,
    # each adding the next rho largest |a_j^T b| (g_j = a_j^T b off I for every iterate).
    rng = np.random.default_rng(7)
    n, m = 64, 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    At = np.ascontiguousarray(Q.T.astype(np.float32))
    b = (Q[:, :25] @ (rng.uniform(0.5, 2.0, 25) * rng.choice([-1, 1], 25))
         + 0.2 * rng.standard_normal(n)).astype(np.float32)
    A64 = At.astype(np.float64).T
    z = A64.T @ b.astype(np.float64)
    order = np.argsort(-np.abs(z), kind="stable")
    # choose lambda in a wide gap of |z| so float32 non-orthogonality cannot reorder anything
    az = np.abs(z)[order]
    gaps = az[:-1] - az[1:]
    q = int(np.argmax(gaps[:30])) if gaps[:30].max() > 1e-3 else 20
    lam = 0.5 * (az[q] + az[q + 1])
    expect = np.sign(z) * np.maximum(np.abs(z) - lam, 0)
    for rho in (1, 3, 4):
        t = oracle.trace(At, b, lam, rho)
        np.testing.assert_allclose(t["x"], expect, atol=2e-5)
        nS = int((expect != 0).sum())
        assert t["iters"] == -(-nS // rho)
        added = np.concatenate([a for a, _ in t["steps"]])
        np.testing.assert_array_equal(added, order[:nS])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_noiseless_sign_consistent_closed_form(seed):
    # b = A x, k-sparse.  If the sign-fixed solution x_S - lambda G_SS^{-1} s is sign consistent
    # and strictly dual feasible off S, it is the LASSO solution (primal-dual witness), and it
    # tends to x as lambda -> 0.
    P = bi.tiny_gaussian(n=128, m=512, p=1, k=5, sigma=0.0, seed=10 + seed)
    S = P.supports[0]
    A = P.At.astype(np.float64).T
    b = P.Bt[0].astype(np.float64)
    AS = A[:, S]
    G = AS.T @ AS
    s = np.sign(P.amplitudes[0])
    errs = []
    for lam in (1e-1, 1e-2, 1e-3):
        xs = np.linalg.solve(G, AS.T @ b - lam * s)
        assert np.all(np.sign(xs) == s)
        xw = np.zeros(512)
        xw[S] = xs
        g = A.T @ (b - A @ xw)
        off = np.setdiff1d(np.arange(512), S)
        assert np.abs(g[off]).max() < lam     # witness certifies uniqueness
        r = oracle.solve(P.At, P.Bt, np.array([lam]), rho=2)
        np.testing.assert_allclose(r["X"][0], xw, rtol=0, atol=1e-10)
        errs.append(np.linalg.norm(r["X"][0][S] - P.amplitudes[0]))
    # exact recovery in the limit: error shrinks linearly with lambda (b is float32-rounded)
    assert errs[2] < 2e-2 * errs[0] + 1e-5


def omp_textbook(A, b, steps):
    r = b.copy()
    I = []
    for _ in range(steps):
        c = np.abs(A.T @ r)
        c[I] = -1
        j = int(np.argmax(c))
        I.append(j)
        xs, *_ = np.linalg.lstsq(A[:, I], b, rcond=None)
        r = b - A[:, I] @ xs
    x = np.zeros(A.shape[1])
    x[I] = xs
    return I, x


@pytest.mark.parametrize("seed", [0, 1])
def test_omp_reduction_lambda0_rho1(seed):
    P = bi.tiny_gaussian(n=64, m=200, p=1, k=8, sigma=0.01, seed=20 + seed)
    steps = 12
    t = oracle.trace(P.At, P.Bt[0], 0.0, 1, max_outer=steps)
    I_or = [int(a[0]) for a, _ in t["steps"]]
    A = P.At.astype(np.float64).T
    I_omp, x_omp = omp_textbook(A, P.Bt[0].astype(np.float64), steps)
    assert I_or == I_omp
    np.testing.assert_allclose(t["x"], x_omp, atol=1e-9)


@pytest.mark.parametrize("rho", [1, 2, 5])
def test_monotone_objective_and_lemma1_bound(rho):
    P = bi.small_gaussian(indices=[0, 3, 7])
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    A = P.At.astype(np.float64).T
    for i in range(P.p):
        t = oracle.trace(P.At, P.Bt[i], lam[i], rho)
        F = t["obj_trace"]
        assert np.all(np.diff(F) <= 1e-12 * F[0])
        I = []
        for step, (added, gsel) in enumerate(t["steps"]):
            I.extend(int(a) for a in added)
            L = np.linalg.eigvalsh(A[:, I].T @ A[:, I]).max()
            bound = ((np.abs(gsel) - lam[i]) ** 2).sum() / (2 * L)
            assert np.all(np.abs(gsel) > lam[i])
            assert F[step] - F[step + 1] >= bound * (1 - 1e-9)


def full_cd(A, b, lam, tol=1e-13, max_rounds=200):
    """Independent full-problem FP64 coordinate descent (covariance updates, active-set inner loops)."""
    n, m = A.shape
    G = A.T @ A
    c = A.T @ b
    x = np.zeros(m)
    grad = c.copy()

    def sweep(idx):
        for j in idx:
            old = x[j]
            z = grad[j] + G[j, j] * old
            nw = np.sign(z) * max(abs(z) - lam, 0.0) / G[j, j]
            if nw != old:
                grad[:] -= G[:, j] * (nw - old)
                x[j] = nw

    for _ in range(max_rounds):
        sweep(range(m))
        for _ in range(100000):
            act = np.nonzero(x)[0]
            before = x.copy()
            sweep(act)
            if np.max(np.abs(x - before)) <= tol:
                break
        g = c - G @ x
        on = x != 0
        viol = max(np.max(np.abs(g[~on]) - lam, initial=0.0),
                   np.max(np.abs(g[on] - lam * np.sign(x[on])), initial=0.0))
        if viol <= 1e-11 * lam:
            break
    return x


def test_cross_solver_full_cd():
    P = bi.small_gaussian(indices=[1, 5, 11])
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    r = oracle.solve(P.At, P.Bt, lam, P.rho)
    A = P.At.astype(np.float64).T
    for i in range(P.p):
        xcd = full_cd(A, P.Bt[i].astype(np.float64), lam[i])
        np.testing.assert_allclose(r["X"][i], xcd, atol=1e-9)


def test_invariances():
    P = bi.small_gaussian(indices=[2, 9])
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    base = oracle.solve(P.At, P.Bt, lam, P.rho)
    rng = np.random.default_rng(3)
    # permuting atoms permutes the solution
    perm = rng.permutation(P.m)
    r = oracle.solve(P.At[perm], P.Bt, lam, P.rho)
    np.testing.assert_allclose(r["X"], base["X"][:, perm], atol=1e-10)
    # permuting signals permutes the results
    r = oracle.solve(P.At, P.Bt[::-1], lam[::-1], P.rho)
    np.testing.assert_allclose(r["X"], base["X"][::-1], atol=1e-12)
    # b -> 2b, lambda -> 2 lambda gives x -> 2x (powers of two keep float32 exact)
    r = oracle.solve(P.At, 2 * P.Bt, 2 * lam, P.rho)
    np.testing.assert_allclose(r["X"], 2 * base["X"], atol=1e-10)
    # flipping atom j flips x_j
    At2 = P.At.copy()
    flip = np.nonzero(base["X"][0])[0][:3]
    At2[flip] *= -1
    r = oracle.solve(At2, P.Bt, lam, P.rho)
    expect = base["X"].copy()
    expect[:, flip] *= -1
    np.testing.assert_allclose(r["X"], expect, atol=1e-10)
    # lambda >= ||A^T b||_inf gives x = 0 after zero iterations
    r = oracle.solve(P.At, P.Bt, lam / P.lambda_rel * 1.0001, P.rho)
    assert np.all(r["X"] == 0) and np.all(r["iters"] == 0) and np.all(r["status"] == oracle.ST_CONVERGED)


def test_caps_and_nonfinite():
    P = bi.small_gaussian(indices=[0, 1])
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    r = oracle.solve(P.At, P.Bt, lam, P.rho, max_outer=1)
    assert np.all(r["status"] & oracle.ST_CAP_ITERS) and np.all(r["iters"] == 1)
    r = oracle.solve(P.At, P.Bt, lam, P.rho, max_active=3)
    assert np.all(r["status"] & oracle.ST_CAP_ACTIVE)
    assert np.all((r["X"] != 0).sum(axis=1) <= 3)
    Bt = P.Bt.copy()
    Bt[1, 5] = np.nan
    r = oracle.solve(P.At, Bt, lam, P.rho)
    assert r["status"][1] == oracle.ST_NONFINITE and r["status"][0] == oracle.ST_CONVERGED


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_smpl_reaches_the_lasso_solution(seed):
    """Subspace exploratory matching (Algorithm 2) changes the path, not the answer: the unique LASSO
    solution, certified by its optimality conditions, and the MPL result to solver precision."""
    P = bi.tiny_gaussian(n=48, m=300, p=6, k=8, sigma=0.01, seed=seed, lambda_rel=0.05, rho=3)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    mpl = oracle.solve(P.At, P.Bt, lam, P.rho)
    smpl = oracle.solve(P.At, P.Bt, lam, P.rho, omega=3)
    assert np.all(smpl["status"] == oracle.ST_CONVERGED)
    for i in range(P.p):
        off, on = kkt_residuals(P.At, P.Bt[i], smpl["X"][i], lam[i])
        assert off <= 1e-9 * lam[i] and on <= 1e-9 * lam[i]
        np.testing.assert_allclose(smpl["X"][i], mpl["X"][i], rtol=0, atol=1e-9 * np.abs(mpl["X"][i]).max())


def test_smpl_brute_force_and_monotone_objective():
    """On m = 10 the SMPL result is the brute-force LASSO minimiser; per outer iteration the objective
    never increases (atoms are never removed from I_t once kept), at most rho atoms are kept."""
    for seed in range(4):
        P = bi.tiny_gaussian(n=6, m=10, p=1, k=3, sigma=0.05, seed=200 + seed, lambda_rel=0.1, rho=2)
        lam = lam_rel(P.At, P.Bt, P.lambda_rel)[0]
        sols = brute_force_lasso(P.At, P.Bt[0], lam)
        assert len(sols) == 1
        tr = oracle.trace(P.At, P.Bt[0], lam, 2, omega=3)
        np.testing.assert_allclose(tr["x"], sols[0], atol=1e-10)
        ob = tr["obj_trace"]
        assert np.all(np.diff(ob) <= 1e-12 * ob[0])
        assert all(len(a) <= 2 for a, _ in tr["steps"])


def test_smpl_keeps_the_atom_with_the_largest_restricted_coefficient():
    """First SMPL iteration with rho = 1, omega = 3, checked by brute force: J_omega = the three largest
    |a_j^T b| (all violating), u = the LASSO minimiser restricted to J_omega (enumeration), and the atom
    kept must be the one with the largest |u_j|."""
    checked = 0
    for seed in range(12):
        P = bi.tiny_gaussian(n=8, m=40, p=1, k=3, sigma=0.05, seed=300 + seed, lambda_rel=0.2, rho=1)
        b = P.Bt[0]
        g = P.At.astype(np.float64) @ b.astype(np.float64)
        lam = 0.2 * np.abs(g).max()
        order = np.lexsort((np.arange(P.m), -np.abs(g)))
        J = order[:3]
        if np.abs(g[J]).min() <= lam:
            continue                      # fewer than three violators: not this case
        u = brute_force_lasso(P.At[J], b, lam)
        assert len(u) == 1
        u = u[0]
        kept = J[np.lexsort((J, -np.abs(u)))[0]]
        tr = oracle.trace(P.At, b, lam, 1, omega=3)
        assert list(tr["steps"][0][0]) == [kept]
        checked += 1
    assert checked >= 4


def test_early_stop_eq13_orthonormal_closed_form():
    """Eq. (13) pinned by a closed form.  With orthonormal atoms, g_j = z_j = a_j^T b for every j outside I,
    the master problem on I is soft thresholding, and the objective after iteration t is
    F_t = ||b||^2 / 2 - sum_{j in I_t} (|z_j| - lambda)^2 / 2, so iteration t lowers it by
    delta_t = sum_{j in J_t} (|z_j| - lambda)^2 / 2, J_t the t-th block of rho atoms in decreasing |z_j|.
    For every t, a tolerance just above delta_t / (rho ||b||^2) must stop the solver right after iteration
    t (status early, x = soft thresholding on the first t blocks) and one just below it one iteration
    later.  This fixes which decrease is tested, the normaliser rho ||b||^2 and the direction of the test."""
    rng = np.random.default_rng(13)
    n, m = 96, 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    At = np.ascontiguousarray(Q.T.astype(np.float32))
    b = (Q[:, :40] @ (rng.uniform(0.5, 3.0, 40) * rng.choice([-1, 1], 40))
         + 0.05 * rng.standard_normal(n)).astype(np.float32)
    b64 = b.astype(np.float64)
    bb = float(b64 @ b64)
    z = At.astype(np.float64) @ b64
    lam = 0.3
    order = np.argsort(-np.abs(z), kind="stable")
    viol = order[np.abs(z[order]) > lam]
    for rho in (3, 5):
        blocks = [viol[i:i + rho] for i in range(0, len(viol), rho)]
        delta = np.array([0.5 * np.sum((np.abs(z[J]) - lam) ** 2) for J in blocks])
        assert np.all(delta[:-1] > delta[1:] * 1.01)     # strictly decreasing: each threshold has one answer
        for t in range(1, len(blocks) - 1):
            for factor, T in ((1 + 1e-3, t), (1 - 1e-3, t + 1)):
                eps = factor * delta[t - 1] / (rho * bb)
                tr = oracle.trace(At, b, lam, rho, eps_early=eps)
                assert tr["status"] & oracle.ST_EARLY, (rho, t, factor)
                assert tr["iters"] == T, (rho, t, factor, tr["iters"])
                keep = np.concatenate(blocks[:T])
                expect = np.zeros(m)
                expect[keep] = np.sign(z[keep]) * (np.abs(z[keep]) - lam)
                np.testing.assert_allclose(tr["x"], expect, atol=2e-5)
                F = 0.5 * bb - np.concatenate([[0.0], np.cumsum(delta[:T])])
                np.testing.assert_allclose(tr["obj_trace"][:T + 1], F, rtol=1e-6)


def test_early_stop_rule_eq13():
    """The objective-decrease stop of Eq. (13): the solver stops at the first outer iteration whose
    decrease is at most eps * rho * ||b||^2, not before; with eps = 0 it runs to the natural stop."""
    P = bi.tiny_gaussian(n=64, m=400, p=4, k=20, sigma=0.02, seed=21, lambda_rel=0.002, rho=2)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    for i in range(P.p):
        b = P.Bt[i]
        bb = float(b.astype(np.float64) @ b.astype(np.float64))
        full = oracle.trace(P.At, b, lam[i], P.rho)
        eps = 1e-4
        tr = oracle.trace(P.At, b, lam[i], P.rho, eps_early=eps)
        ob = tr["obj_trace"]
        T = tr["iters"]
        dec = np.abs(np.diff(ob))
        if tr["status"] & oracle.ST_EARLY:
            assert dec[T - 1] <= eps * P.rho * bb
            assert np.all(dec[:T - 1] > eps * P.rho * bb)
            assert T < full["iters"]
            np.testing.assert_allclose(ob, full["obj_trace"][:T + 1], rtol=1e-12)   # the same path so far
        else:
            assert tr["status"] & oracle.ST_CONVERGED and np.all(dec > eps * P.rho * bb)
        assert full["status"] & oracle.ST_CONVERGED


def omp_residual_stop(A, b, eps_r, eps_g, max_steps):
    """Textbook OMP that stops once ||r|| <= eps_r or max_{j not in I} |a_j^T r| <= eps_g
    (the classical residual-norm and correlation stops)."""
    r = b.copy()
    I = []
    xs = np.zeros(0)
    for _ in range(max_steps):
        c = np.abs(A.T @ r)
        c[I] = -1
        if c.max() <= eps_g or np.linalg.norm(r) <= eps_r:
            break
        I.append(int(np.argmax(c)))
        xs, *_ = np.linalg.lstsq(A[:, I], b, rcond=None)
        r = b - A[:, I] @ xs
    x = np.zeros(A.shape[1])
    x[I] = xs
    return I, x


@pytest.mark.parametrize("seed,r2_rel,rinf_rel", [(0, 0.05, 0.0), (1, 0.2, 0.0), (2, 0.0, 0.1), (3, 0.0, 0.3)])
def test_early_stop_eq10_is_omp_with_its_stop(seed, r2_rel, rinf_rel):
    """Eq. (10) at lambda = 0, rho = 1: OMP with the residual-norm stop ||xi|| <= r_2, or the
    correlation stop ||A^T xi||_inf <= r_inf (radii relative to ||b|| and ||A^T b||_inf)."""
    P = bi.tiny_gaussian(n=64, m=200, p=1, k=12, sigma=0.02, seed=40 + seed)
    A = P.At.astype(np.float64).T
    b = P.Bt[0].astype(np.float64)
    eps_r = r2_rel * np.linalg.norm(b) if r2_rel > 0 else -1.0
    eps_g = rinf_rel * np.abs(A.T @ b).max() if rinf_rel > 0 else -1.0
    I_omp, x_omp = omp_residual_stop(A, b, eps_r, eps_g, 40)
    t = oracle.trace(P.At, P.Bt[0], 0.0, 1, max_outer=40, r2_rel=r2_rel, r_inf_rel=rinf_rel)
    assert t["status"] & oracle.ST_EARLY
    assert 0 < len(I_omp) < 40
    assert [int(a[0]) for a, _ in t["steps"]] == I_omp
    np.testing.assert_allclose(t["x"], x_omp, atol=1e-9)


def test_early_stop_eq10_lasso_rule_along_the_path():
    """Eq. (10) with lambda > 0: the solver stops at the first outer iteration at which the largest
    correlation outside I is at most r_inf (or the residual norm at most r_2), not before, on the same
    path as the full solve."""
    P = bi.tiny_gaussian(n=64, m=400, p=4, k=20, sigma=0.02, seed=22, lambda_rel=0.002, rho=2)
    lam = lam_rel(P.At, P.Bt, P.lambda_rel)
    A = P.At.astype(np.float64).T
    for i in range(P.p):
        b = P.Bt[i]
        b64 = b.astype(np.float64)
        full = oracle.trace(P.At, b, lam[i], P.rho)
        for rinf_rel, r2_rel in ((0.05, 0.0), (0.0, 0.1)):
            tr = oracle.trace(P.At, b, lam[i], P.rho, r_inf_rel=rinf_rel, r2_rel=r2_rel)
            T = tr["iters"]
            assert tr["status"] & oracle.ST_EARLY and 0 < T < full["iters"]
            np.testing.assert_allclose(tr["obj_trace"], full["obj_trace"][:T + 1], rtol=1e-12)
            r_inf = rinf_rel * np.abs(A.T @ b64).max()
            r_2 = r2_rel * np.linalg.norm(b64)
            inI = np.zeros(A.shape[1], bool)
            for t, (added, gsel) in enumerate(tr["steps"]):
                # before step t: neither the correlation rule (largest |g| outside I is the first pick)
                # nor the residual rule held
                x_t = full_x_after(P.At, b, lam[i], P.rho, t)
                if rinf_rel > 0:
                    assert abs(gsel[0]) > r_inf
                if r2_rel > 0:
                    assert np.linalg.norm(b64 - A @ x_t) > r_2
                inI[added] = True
            rT = b64 - A @ tr["x"]
            if rinf_rel > 0:
                assert np.abs(A.T @ rT)[~inI].max() <= r_inf * (1 + 1e-12)
            if r2_rel > 0:
                assert np.linalg.norm(rT) <= r_2 * (1 + 1e-12)


def full_x_after(At, b, lam, rho, t):
    """x after t outer iterations (the iteration cap of the oracle stops it there)."""
    if t == 0:
        return np.zeros(At.shape[0])
    return oracle.trace(At, b, lam, rho, max_outer=t)["x"]
