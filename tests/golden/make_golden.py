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
    rec = {
        "description": ("FP64 oracle results (oracle/mpl_oracle.c) for rows of the seeded ragged workload "
                        "1024 x 32768 (bmpl_inputs.ragged_gaussian), written by tests/golden/make_golden.py; "
                        "idx/val are the concatenated supports (val, lam, objective as float.hex)."),
        "rows": RAGGED_ROWS, "lam": [float.hex(float(v)) for v in lam], "iters": r["iters"].tolist(),
        "objective": [float.hex(float(v)) for v in r["objective"]], "status": r["status"].tolist(),
        "kkt": r["kkt"].tolist(), "margin": r["margin"].tolist(), "supp_len": [len(i) for i in idx],
        "idx": np.concatenate(idx).tolist(), "val": [float.hex(float(v)) for v in np.concatenate(val)],
        "seconds": el, "threads": oracle.max_threads(),
    }
    with open(path, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"wrote {path}: supports {[len(i) for i in idx]}, iterations {list(r['iters'])}, {el:.1f} s", flush=True)


if __name__ == "__main__":
    ragged(os.path.join(HERE, "ragged1024x32768_oracle.json"))
