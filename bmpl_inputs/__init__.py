"""Seeded synthetic problem generators for batch sparse recovery.

This module is shared by the tests, the benchmark and the FP64 oracle harness.
It holds no arithmetic of the solver: it only draws dictionaries A, signals
B = A X + E and the ground-truth X, following the problem model of the paper
(Section I: b = A x + e with a dictionary of unit-norm atoms, Eq. (3) for p
signals at once) and the workloads of its experiments (Gaussian compressive
sensing dictionaries, Section IV; a class-structured face-like dictionary,
Section V).

Conventions
-----------
* Every value is drawn in float64 and rounded once to float32.  The float32
  arrays are the canonical problem; the oracle promotes them exactly to float64.
* ``At`` is the dictionary stored atom-major: an (m, n) C-contiguous float32
  array whose row j is atom a_j.  Read as a column-major n x m matrix with
  leading dimension n, it is A itself.
* ``Bt`` is (p, n) C-contiguous float32: row i is signal b_i (column-major
  n x p B with leading dimension n).
* Seeds: numpy PCG64 streams derived from ``SeedSequence(13025010)`` with the
  spawn key (workload, stream, index), so any single signal can be generated
  on its own (``indices=``) and equals the same signal of the full batch.
* ``lambda_rel`` is the paper's relative regularisation rule
  lambda_i = c * ||A^T b_i||_inf (Section IV-A); computing it is left to the
  caller.
"""
from __future__ import annotations

import dataclasses
import numpy as np

ROOT_SEED = 13025010


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(key))))


@dataclasses.dataclass
class Problem:
    name: str
    At: np.ndarray            # (m, n) float32, atom-major dictionary
    Bt: np.ndarray            # (p, n) float32, one signal per row
    lambda_rel: float         # c in lambda_i = c * ||A^T b_i||_inf
    rho: int                  # atoms added per outer iteration
    supports: list            # ground-truth supports (int64 arrays), one per signal
    amplitudes: list          # ground-truth nonzero values (float64), one per signal
    meta: dict

    @property
    def n(self) -> int:
        return self.At.shape[1]

    @property
    def m(self) -> int:
        return self.At.shape[0]

    @property
    def p(self) -> int:
        return self.Bt.shape[0]


# ---------------------------------------------------------------------------
# Dictionaries
# ---------------------------------------------------------------------------

def gaussian_dictionary(n: int, m: int, wid: int) -> np.ndarray:
    """i.i.d. N(0, 1/n) entries, then every column scaled to unit l2 norm."""
    rng = _rng(wid, 0, 0)
    A = rng.standard_normal((m, n))          # atom-major draw: row j is atom j
    A /= np.sqrt(n)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return np.ascontiguousarray(A.astype(np.float32))


def class_subspace_dictionary(n: int, classes: int, per_class: int, rank: int,
                              noise: float, wid: int):
    """Face-like dictionary: class c spans a random rank-`rank` subspace W_c.

    a_j = normalise(W_c v_j + e_j) with W_c i.i.d. N(0, 1), v_j ~ N(0, I_rank)
    and e_j ~ N(0, noise^2 I).  Returns (At float32, W list float64, class id
    per atom).
    """
    rng = _rng(wid, 0, 0)
    m = classes * per_class
    A = np.empty((m, n))
    W = []
    for c in range(classes):
        Wc = rng.standard_normal((n, rank))
        V = rng.standard_normal((rank, per_class))
        E = noise * rng.standard_normal((n, per_class))
        block = (Wc @ V + E).T
        block /= np.linalg.norm(block, axis=1, keepdims=True)
        A[c * per_class:(c + 1) * per_class] = block
        W.append(Wc)
    cls = np.repeat(np.arange(classes), per_class)
    return np.ascontiguousarray(A.astype(np.float32)), W, cls


# ---------------------------------------------------------------------------
# Signals
# ---------------------------------------------------------------------------

def _sparse_signals(At32: np.ndarray, idx, wid: int, stream: int, k_of, amp_of, sigma: float):
    m, n = At32.shape
    Bt = np.empty((len(idx), n), dtype=np.float32)
    sups, amps = [], []
    for r, i in enumerate(idx):
        rng = _rng(wid, stream, int(i))
        k = int(k_of(rng))
        S = np.sort(rng.choice(m, size=k, replace=False))
        a = amp_of(rng, k)
        b = At32[S].astype(np.float64).T @ a + sigma * rng.standard_normal(n)
        Bt[r] = b.astype(np.float32)
        sups.append(S)
        amps.append(a)
    return Bt, sups, amps


def _signed_uniform(rng, k):
    return rng.choice(np.array([-1.0, 1.0]), size=k) * rng.uniform(1.0, 2.0, size=k)


def _normal(rng, k):
    return rng.standard_normal(k)


def small_gaussian(indices=None) -> Problem:
    """A 128 x 512 Gaussian, p = 16, k = 10 with N(0,1) amplitudes, sigma = 0.01, c = 0.05, rho = 2."""
    n, m, p = 128, 512, 16
    At = gaussian_dictionary(n, m, 0)
    idx = range(p) if indices is None else indices
    Bt, S, a = _sparse_signals(At, idx, 0, 1, lambda r: 10, _normal, 0.01)
    return Problem("gauss128x512", At, Bt, 0.05, 2, S, a, {"k": 10, "sigma": 0.01})


def cs_gaussian(indices=None) -> Problem:
    """A 2048 x 16384 Gaussian, p = 1024, k = 100, amplitudes +-U[1,2], sigma = 0.005, c = 0.02, rho = 10."""
    n, m, p = 2048, 16384, 1024
    At = gaussian_dictionary(n, m, 1)
    idx = range(p) if indices is None else indices
    Bt, S, a = _sparse_signals(At, idx, 1, 1, lambda r: 100, _signed_uniform, 0.005)
    return Problem("cs2048x16384", At, Bt, 0.02, 10, S, a, {"k": 100, "sigma": 0.005})


def ragged_gaussian(indices=None) -> Problem:
    """A 1024 x 32768 Gaussian, p = 4096, k ~ U{10..400}, amplitudes +-U[1,2], sigma = 0.01, c = 0.03, rho = 10."""
    n, m, p = 1024, 32768, 4096
    At = gaussian_dictionary(n, m, 2)
    idx = range(p) if indices is None else indices
    Bt, S, a = _sparse_signals(At, idx, 2, 1, lambda r: r.integers(10, 401), _signed_uniform, 0.01)
    return Problem("ragged1024x32768", At, Bt, 0.03, 10, S, a, {"k": "U{10..400}", "sigma": 0.01})


def face_like(indices=None, p: int = 8192, stream: int = 1) -> Problem:
    """m = 20000 atoms in 200 classes x 100, rank-8 class subspaces in R^1024, c = 0.01, rho = 10.

    Signal i: pick a class c, w ~ N(0, I_8); b = W_c w / ||W_c w|| + e with
    ||e|| = 0.05 (5 % noise), e isotropic.  The ground-truth "support" is the
    class's atom range (the class label), amplitudes are empty.
    """
    n, classes, per = 1024, 200, 100
    At, W, cls = class_subspace_dictionary(n, classes, per, 8, 0.05, 3)
    idx = range(p) if indices is None else indices
    Bt = np.empty((len(idx), n), dtype=np.float32)
    sups, amps = [], []
    for r, i in enumerate(idx):
        rng = _rng(3, stream, int(i))
        c = int(rng.integers(0, classes))
        w = rng.standard_normal(8)
        s = W[c] @ w
        s /= np.linalg.norm(s)
        e = rng.standard_normal(n)
        e *= 0.05 / np.linalg.norm(e)
        Bt[r] = (s + e).astype(np.float32)
        sups.append(np.arange(c * per, (c + 1) * per))
        amps.append(np.empty(0))
    return Problem("face20000", At, Bt, 0.01, 10, sups, amps,
                   {"classes": classes, "per_class": per, "rank": 8, "class_of_atom": cls})


def tiny_gaussian(n: int, m: int, p: int, k: int, sigma: float, seed: int,
                  lambda_rel: float = 0.05, rho: int = 2) -> Problem:
    """Small free-form Gaussian problems for unit tests (seeded by `seed`)."""
    rng = _rng(100, seed, 0)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    At = np.ascontiguousarray(A.astype(np.float32))
    Bt, S, a = _sparse_signals(At, range(p), 100, 1000 + seed, lambda r: k, _normal, sigma)
    return Problem(f"tiny{n}x{m}", At, Bt, lambda_rel, rho, S, a, {"k": k, "sigma": sigma})


def projection(m: int, d: int, seed: int = 0) -> np.ndarray:
    """Fixed random projection of the proposal network's input: m x d, i.i.d. N(0, 1/d), float32."""
    rng = _rng(200, seed, 0)
    return (rng.standard_normal((m, d)) / np.sqrt(d)).astype(np.float32)


def mlp_init(d: int, h: int, m: int, seed: int = 0, prior: float | None = None) -> np.ndarray:
    """Initial flat parameters of the proposal network (layout W1, b1, W2, b2, W3, b3).

    Weights i.i.d. N(0, 1/fan_in); hidden biases zero; output biases at the
    log-odds of `prior` (the expected fraction of atoms in a support), so the
    first scores already sit near the base rate.  float32.
    """
    rng = _rng(201, seed, 0)
    w1 = rng.standard_normal((h, d)) / np.sqrt(d)
    w2 = rng.standard_normal((h, h)) / np.sqrt(h)
    w3 = rng.standard_normal((m, h)) / np.sqrt(h)
    b3 = np.full(m, 0.0 if prior is None else np.log(prior / (1.0 - prior)))
    return np.concatenate([w1.ravel(), np.zeros(h), w2.ravel(), np.zeros(h), w3.ravel(), b3]).astype(np.float32)


WORKLOADS = {
    "gauss128x512": small_gaussian,
    "cs2048x16384": cs_gaussian,
    "ragged1024x32768": ragged_gaussian,
    "face20000": face_like,
}
