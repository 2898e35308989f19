"""FP64 reference of sparse-representation classification (test infrastructure only).

Only the tests and the benchmark's CPU leg use this module; it shares no code with the GPU
library.  The paper's face experiments (Section V, many-face recognition) follow the setting of
sparse-representation-based classification: a test image b is represented over the training
images A by the sparse code x, and its label is the class whose atoms alone reconstruct b best,

    label(b) = argmin_c || b - A delta_c(x) ||_2,

delta_c(x) keeping the coefficients of class c's atoms and zeroing the rest.  Here only classes
with at least one atom in the support compete (reading: a class with no atom in the support
reconstructs nothing), ties go to the lower class index, and an empty support gives -1.
"""
from __future__ import annotations

import numpy as np


def classify(At: np.ndarray, Bt: np.ndarray, X: np.ndarray, class_of_atom: np.ndarray):
    """Labels and winning residual norms for the rows of Bt with dense codes X (rows)."""
    A64 = np.asarray(At, dtype=np.float64)
    cls = np.asarray(class_of_atom)
    labels = np.full(Bt.shape[0], -1, dtype=np.int64)
    resid = np.full(Bt.shape[0], np.nan)
    for i in range(Bt.shape[0]):
        b = np.asarray(Bt[i], dtype=np.float64)
        S = np.nonzero(X[i])[0]
        best, best_r = -1, np.inf
        for c in np.unique(cls[S]):
            Sc = S[cls[S] == c]
            r = np.linalg.norm(b - A64[Sc].T @ X[i, Sc])
            if r < best_r:              # classes visited in increasing order: ties keep the lower one
                best, best_r = int(c), r
        labels[i] = best
        resid[i] = best_r if best >= 0 else np.nan
    return labels, resid
