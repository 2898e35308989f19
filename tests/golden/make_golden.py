"""Write stored oracle results for workloads whose oracle run is too slow for the test suite.

Calls only the FP64 oracle (oracle/) on seeded inputs from bmpl_inputs; the GPU
tests regenerate the same inputs and compare against these files.

    python tests/golden/make_golden.py            # writes tests/golden/ragged1024x32768_oracle.npz
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import bmpl_inputs as bi  # noqa: E402
import oracle  # noqa: E402

# ragged workload: signals with k <= 100 (supports of ~k atoms) and two with k >= 200
# (supports near n, about a hundred outer iterations each)
RAGGED_ROWS = [17, 18, 19, 21, 0, 8]


def ragged(path):
    P = bi.ragged_gaussian(indices=RAGGED_ROWS)
    lam = P.lambda_rel * np.abs(P.At.astype(np.float64) @ P.Bt.astype(np.float64).T).max(axis=0)
    t = time.time()
    r = oracle.solve(P.At, P.Bt, lam, P.rho)
    el = time.time() - t
    idx = [np.nonzero(r["X"][q])[0].astype(np.int32) for q in range(len(RAGGED_ROWS))]
    val = [r["X"][q][idx[q]] for q in range(len(RAGGED_ROWS))]
    np.savez_compressed(
        path, rows=np.array(RAGGED_ROWS), lam=lam, iters=r["iters"], objective=r["objective"],
        status=r["status"], kkt=r["kkt"], margin=r["margin"],
        supp_len=np.array([len(i) for i in idx]), idx=np.concatenate(idx), val=np.concatenate(val),
        seconds=el, threads=oracle.max_threads())
    print(f"wrote {path}: supports {[len(i) for i in idx]}, iterations {list(r['iters'])}, {el:.1f} s", flush=True)


if __name__ == "__main__":
    ragged(os.path.join(HERE, "ragged1024x32768_oracle.npz"))
