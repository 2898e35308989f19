"""Parity rules between the GPU library and the FP64 oracle (test infrastructure).

For each signal, with the GPU's sparse result expanded to a dense float64 x
and the objective recomputed here in float64 from it (never taken from the
GPU):
  * relative objective error |F_gpu - F_or| / F_or <= 1e-5 (either side lower fails);
  * relative l2 error ||x_gpu - x_or|| / ||x_or|| <= 1e-4;
  * where the oracle's margin exceeds 1e-3 lambda: identical supports and signs;
  * per atom: every j with lambda - |g_j| > 1e-3 lambda is absent and every j
    with |x_or_j| > 1e-3 lambda is present in the GPU support.
The oracle's g is A^T (b - A x_or) in float64.
"""
from __future__ import annotations

import numpy as np

REL_OBJ = 1e-5
REL_X = 1e-4
MARGIN = 1e-3


def dense_from_gpu(out: dict, m: int) -> np.ndarray:
    idx = out["x_idx"].cpu().numpy()
    val = out["x_val"].cpu().numpy().astype(np.float64)
    ln = out["supp_len"].cpu().numpy()
    p = idx.shape[0]
    X = np.zeros((p, m))
    for i in range(p):
        k = int(ln[i])
        if k:
            assert np.all(np.diff(idx[i, :k]) > 0), "support must be sorted by atom index"
            X[i, idx[i, :k]] = val[i, :k]
    return X


def objective(A64: np.ndarray, b: np.ndarray, x: np.ndarray, lam: float) -> float:
    r = b - A64 @ x
    return 0.5 * float(r @ r) + lam * float(np.abs(x).sum())


def check_signal(A64, b, lam, x_gpu, x_or, tag=""):
    """Assert the parity rules for one signal; returns a dict of the measured errors."""
    F_or = objective(A64, b, x_or, lam)
    F_gpu = objective(A64, b, x_gpu, lam)
    rel_obj = abs(F_gpu - F_or) / F_or if F_or > 0 else abs(F_gpu)
    nx = np.linalg.norm(x_or)
    rel_x = np.linalg.norm(x_gpu - x_or) / nx if nx > 0 else np.linalg.norm(x_gpu)
    g = A64.T @ (b - A64 @ x_or)
    S_or = x_or != 0
    S_gpu = x_gpu != 0
    mu = min(np.min(lam - np.abs(g[~S_or]), initial=np.inf), np.min(np.abs(x_or[S_or]), initial=np.inf))
    assert rel_obj <= REL_OBJ, f"{tag}: relative objective error {rel_obj:.3e}"
    assert rel_x <= REL_X, f"{tag}: relative x error {rel_x:.3e}"
    if mu > MARGIN * lam:
        assert np.array_equal(S_gpu, S_or), f"{tag}: support differs at margin {mu / lam:.3e} lambda"
        assert np.array_equal(np.sign(x_gpu[S_or]), np.sign(x_or[S_or])), f"{tag}: signs differ"
    must_absent = (lam - np.abs(g)) > MARGIN * lam
    must_present = np.abs(x_or) > MARGIN * lam
    assert not np.any(S_gpu & must_absent), f"{tag}: atom with clear dual slack is in the GPU support"
    assert np.all(S_gpu[must_present]), f"{tag}: atom with a clear coefficient is missing"
    return {"rel_obj": rel_obj, "rel_x": rel_x, "margin": mu / lam if lam > 0 else mu}


def check_batch(At, Bt, lam, gpu_out, oracle_res, rows=None, gpu_rows=None):
    """Check every signal; `rows` index the oracle's batch, `gpu_rows` the GPU's (default: same)."""
    A64 = At.astype(np.float64).T
    m = At.shape[0]
    Xg = dense_from_gpu(gpu_out, m)
    rows = range(oracle_res["X"].shape[0]) if rows is None else rows
    errs = []
    for q, i in enumerate(rows):
        gi = i if gpu_rows is None else gpu_rows[q]
        errs.append(check_signal(A64, Bt[gi].astype(np.float64), float(lam[q]), Xg[gi], oracle_res["X"][q],
                                 tag=f"signal {gi}"))
    return errs
