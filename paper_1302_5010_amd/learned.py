"""Training and use of the learned support proposal (host-side orchestration only).

Every arithmetic step runs in the library's kernels (bmpl_mlp_* and
bmpl_solve); this module only walks the batches.  Targets are the supports
that BMPL itself returns, so the network learns to predict the method's own
output; at solve time its top-k atoms are the starting active set of every
signal, verified by the natural stopping condition like any other start.
"""
from __future__ import annotations

import torch

from ._binding import BMPL_SIG_CONVERGED, BmplError, ProposalNet, Solver


def label_supports(solver: Solver, Bt: torch.Tensor, chunk: int = 16384) -> dict:
    """Solve every row of ``Bt`` with ``solver``; returns the supports (x_idx, supp_len) and status."""
    idx, lens, status = [], [], []
    for r0 in range(0, Bt.shape[0], chunk):
        out = solver.solve(Bt[r0:r0 + chunk])
        idx.append(out["x_idx"])
        lens.append(out["supp_len"])
        status.append(out["status"])
    return {"x_idx": torch.cat(idx), "supp_len": torch.cat(lens), "status": torch.cat(status)}


def train_proposal(net: ProposalNet, Bt: torch.Tensor, supp: torch.Tensor, supp_len: torch.Tensor, epochs: int,
                   batch: int, lr: float, pos_weight: float, record_every: int = 1) -> list:
    """Adam on the weighted cross-entropy over contiguous batches of the (already shuffled,
    i.i.d.) training signals, ``epochs`` passes.  Returns the recorded losses (device scalars)."""
    if batch > net.max_batch:
        raise BmplError(f"batch {batch} exceeds the network's max_batch {net.max_batch}")
    losses = []
    step = 0
    for _ in range(epochs):
        for r0 in range(0, Bt.shape[0] - batch + 1, batch):
            loss, _ = net.loss_grad(Bt[r0:r0 + batch], supp[r0:r0 + batch], supp_len[r0:r0 + batch], pos_weight,
                                    want_grad=False)
            net.adam_step(lr)
            if step % record_every == 0:
                losses.append(loss)
            step += 1
    return losses


def solve_with_proposal(solver: Solver, net: ProposalNet, Bt: torch.Tensor, k: int = 256) -> dict:
    """Propose the k best-scoring atoms per signal, then solve warm-started from them."""
    prop = net.propose(Bt, k)
    out = solver.solve(Bt, warm=prop)
    out["proposal"] = prop
    return out


def converged(out: dict) -> torch.Tensor:
    return (out["status"] & BMPL_SIG_CONVERGED) > 0
