"""Write stored oracle results for workloads whose oracle run is too slow for the test suite.

Calls only the FP64 oracle (oracle/) on seeded inputs from bmpl_inputs; the GPU
tests regenerate the same inputs and compare against these files.

    python tests/golden/make_golden.py            # writes tests/golden/ragged1024x32768_oracle.json
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import bmpl_inputs as bi  # noqa: E402
import oracle  # noqa: E402

def ragged_rows(per_stratum=32, scan=160):
    """The stratified subset of the ragged workload: the first `per_stratum` signals (in index order) with
    k <= 150, whose supports hold about k atoms, and the first `per_stratum` with k >= 200, whose supports
    fill toward n (about a hundred outer iterations each).  Large rows first, so the oracle's dynamic
    schedule starts the long solves early."""
    P = bi.ragged_gaussian(indices=range(scan))
    k = np.array([len(s) for s in P.supports])
    small = [i for i in range(scan) if k[i] <= 150][:per_stratum]
    large = [i for i in range(scan) if k[i] >= 200][:per_stratum]
    assert len(small) == per_stratum and len(large) == per_stratum
    return large + small


def ragged(path, nthreads=0):
    rows = ragged_rows()
    P = bi.ragged_gaussian(indices=rows)
    lam = P.lambda_rel * np.abs(P.At.astype(np.float64) @ P.Bt.astype(np.float64).T).max(axis=0)
    t = time.time()
    r = oracle.solve(P.At, P.Bt, lam, P.rho, nthreads=nthreads)
    el = time.time() - t
    idx = [np.nonzero(r["X"][q])[0].astype(np.int32) for q in range(len(rows))]
    val = [r["X"][q][idx[q]] for q in range(len(rows))]
    rec = {
        "description": ("FP64 oracle results (oracle/mpl_oracle.c) for a stratified subset of the seeded ragged "
                        "workload 1024 x 32768 (bmpl_inputs.ragged_gaussian): 32 signals with k >= 200, then 32 "
                        "with k <= 150; written by tests/golden/make_golden.py; idx/val are the concatenated "
                        "supports (val, lam, objective as float.hex); seconds = the oracle's wall time for the "
                        "64 signals on `threads` host threads (one signal per thread)."),
        "k": [len(s) for s in P.supports],
        "rows": rows, "lam": [float.hex(float(v)) for v in lam], "iters": r["iters"].tolist(),
        "objective": [float.hex(float(v)) for v in r["objective"]], "status": r["status"].tolist(),
        "kkt": r["kkt"].tolist(), "margin": r["margin"].tolist(), "supp_len": [len(i) for i in idx],
        "idx": np.concatenate(idx).tolist(), "val": [float.hex(float(v)) for v in np.concatenate(val)],
        "seconds": el, "threads": nthreads if nthreads > 0 else oracle.max_threads(),
    }
    with open(path, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"wrote {path}: supports {[len(i) for i in idx]}, iterations {list(r['iters'])}, {el:.1f} s", flush=True)


if __name__ == "__main__":
    ragged(os.path.join(HERE, "ragged1024x32768_oracle.json"), nthreads=int(sys.argv[1]) if len(sys.argv) > 1 else 0)
