"""Benchmark: signals solved per second by batched BMPL on one MI355X.

A step is one bmpl_solve over the whole batch: lambda from the relative rule,
then the outer iterations (correlation product, selection, master problem,
residual, certificate) until every signal stops.  Default workload: the
compressive-sensing shape, A 2048 x 16384 Gaussian with unit columns, 1024
signals with 100-sparse +-U[1,2] codes and sigma = 0.005 noise,
lambda_i = 0.02 ||A^T b_i||_inf, rho = 10, KKT tolerance 1e-4, float32
correlation product.  Inputs are seeded and synthetic and resident in HBM
before timing starts.

Printed: one JSON line with the throughput, the correlation kernel's
roofline (HIP-event times of every launch in the timed steps, algorithmic
flops 2 m n p_running per launch), and the FP64 CPU oracle timed on a sample
of the same workload (with its parity against the GPU on that sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}   # MI355X dense matrix peaks
PEAK_HBM_GBS = 8000.0


KERNEL_SOURCES = ("paper_1302_5010_amd/csrc/corr_gemm.hip", "paper_1302_5010_amd/csrc/gemm_tile.h")


def kernel_source_hash() -> str:
    """First 16 hex digits of the sha256 of the correlation kernel's sources, concatenated."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(path: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it was taken on these kernel sources."""
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel_sha256_16") != kernel_source_hash():
            return None
        return rec
    except (OSError, ValueError):
        return None


def screened_measurement(args, pk, torch, At, Bt, P, screen: str) -> dict:
    """Throughput in graph mode and the instrumented kernel breakdown of one screening precision."""
    s = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=True, screen=screen)
    shapes = s.autotune(P.p)["shapes"]
    for _ in range(args.warmup):
        s.solve(Bt)
    torch.cuda.synchronize()
    solved = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solved.append(s.solve(Bt)["status"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    conv = [int(((st & pk.BMPL_SIG_CONVERGED) > 0).sum().item()) for st in solved]
    del s
    st = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, timing=True, screen=screen)
    st.set_tuning(shapes)
    st.solve(Bt)
    torch.cuda.synchronize()
    st.reset_timing()
    for _ in range(args.steps):
        st.solve(Bt)
    torch.cuda.synchronize()
    tb = st.timing()
    ach = tb["corr_flops"] / (tb["corr_ms"] * 1e-3) / 1e12 if tb["corr_ms"] > 0 else 0.0
    peak = PEAK_TFLOPS[screen]
    return {
        "value": sum(conv) / (t1 - t0), "unit": "signals/s", "ms_per_step": (t1 - t0) / args.steps * 1e3,
        "converged_per_step": conv,
        "main_product": {"dtype": screen, "achieved_tflops": ach, "peak_tflops": peak, "frac": ach / peak,
                         "avg_launch_ms": tb["corr_ms"] / max(1, tb["corr_launches"]),
                         "note": "first pass (lambda rule) in bfloat16 for fp8" if screen == "fp8" else ""},
        "kernel_ms_per_step": {k: tb[k] / args.steps for k in ("corr_ms", "select_ms", "solve_ms",
                                                                "other_ms", "wall_ms")},
    }


def q_route_measurement(args, pk, torch, At, Bt, P, tm_mfma) -> dict:
    """Section III's correlation (g = beta - Q_{:,S} x_S, float64, HBM-bound on Q's rows) in place of the
    MFMA product, same workload: throughput and the correlation time per step against the MFMA's."""
    s = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=True, q_route=True)
    for _ in range(args.warmup):
        s.solve(Bt)
    torch.cuda.synchronize()
    solved = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solved.append(s.solve(Bt)["status"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    conv = [int(((st & pk.BMPL_SIG_CONVERGED) > 0).sum().item()) for st in solved]
    del s
    st = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, timing=True, q_route=True)
    st.solve(Bt)
    torch.cuda.synchronize()
    st.reset_timing()
    for _ in range(args.steps):
        st.solve(Bt)
    torch.cuda.synchronize()
    tq = st.timing()
    return {"value": sum(conv) / (t1 - t0), "unit": "signals/s", "ms_per_step": (t1 - t0) / args.steps * 1e3,
            "converged_per_step": conv,
            "correlation_ms_per_step": tq["corr_ms"] / args.steps,
            "mfma_correlation_ms_per_step": tm_mfma["corr_ms"] / args.steps,
            "note": "the first pass (lambda rule) stays the MFMA product in both; the Q-route adds the float64 "
                    "beta = A^T b at set-up (in other_ms)",
            "kernel_ms_per_step": {k: tq[k] / args.steps for k in ("corr_ms", "select_ms", "solve_ms",
                                                                    "other_ms", "wall_ms")}}


def smpl_measurement(args, pk, torch, At, Bt, P, out_mpl) -> dict:
    """Subspace exploratory matching (Algorithm 2, omega = 3) on the same workload: throughput and
    outer iterations against plain MPL's."""
    s = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=True, omega=3)
    s.autotune(P.p)
    for _ in range(args.warmup):
        s.solve(Bt)
    torch.cuda.synchronize()
    solved = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solved.append(s.solve(Bt))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    conv = [int(((o["status"] & pk.BMPL_SIG_CONVERGED) > 0).sum().item()) for o in solved]
    return {"omega": 3, "value": sum(conv) / (t1 - t0), "unit": "signals/s", "ms_per_step": (t1 - t0) / args.steps * 1e3,
            "converged_per_step": conv,
            "iters_mean": float(solved[-1]["iters"].float().mean().item()),
            "mpl_iters_mean": float(out_mpl["iters"].float().mean().item())}


def learned_comparison(args, pk, torch) -> dict:
    """Plain FP32, plain BF16-screened and BF16-screened + learned warm start on the face-like
    dictionary (1024 x 20000, 200 classes of rank-8 subspaces), lambda_i = 0.01 ||A^T b_i||_inf,
    rho = 10.  The proposal network (2048 -> 2048 -> 2048 -> 20000) is trained on supports that
    BMPL returned for signals of a distinct seed stream (not timed); the timed learned step is
    proposal (embedding, network, top-256) + warm-started solve."""
    import bmpl_inputs as bi
    from paper_1302_5010_amd import learned as ln
    dev = torch.device("cuda:0")
    P = bi.face_like(p=args.learned_signals)
    At = torch.from_numpy(P.At).to(dev)
    Bt = torch.from_numpy(P.Bt).to(dev)
    rec = {"workload": f"face20000 (p = {P.p})", "train_signals": args.train_signals, "epochs": args.epochs}

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        outs = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            outs.append(fn())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        conv = int(ln.converged(outs[-1]).sum().item())
        return outs[-1], {"value": conv / dt, "unit": "signals/s", "ms_per_step": dt * 1e3, "converged": conv,
                          "iters_mean": float(outs[-1]["iters"].float().mean().item())}

    plain32 = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=True, screen="fp32")
    plain32.autotune(P.p)
    out32, rec["plain_fp32"] = timed(lambda: plain32.solve(Bt))
    del plain32
    f8 = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=True, screen="fp8")
    f8.autotune(P.p)
    _, rec["plain_fp8"] = timed(lambda: f8.solve(Bt))
    del f8
    bf = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=True, screen="bf16")
    bf.autotune(P.p)
    outbf, rec["plain_bf16"] = timed(lambda: bf.solve(Bt))
    # the face application: class-residual classification of the codes (synthetic classes)
    cls = torch.from_numpy(P.meta["class_of_atom"].astype(np.int32)).to(dev)
    labels, _ = bf.classify(Bt, outbf, cls)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels, _ = bf.classify(Bt, outbf, cls)
    torch.cuda.synchronize()
    truth = np.array([s[0] // P.meta["per_class"] for s in P.supports])
    rec["src_classification"] = {"recognition_rate": float(np.mean(labels.cpu().numpy() == truth)),
                                 "ms": (time.perf_counter() - t0) * 1e3, "classes": P.meta["classes"]}

    # training data: BMPL supports of signals from a distinct seed stream
    t0 = time.perf_counter()
    T = bi.face_like(p=args.train_signals, stream=2)
    Bt_tr = torch.from_numpy(T.Bt).to(dev)
    del T
    t1 = time.perf_counter()
    lab = ln.label_supports(bf, Bt_tr)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    d = h = 2048
    net = pk.ProposalNet(At, torch.from_numpy(bi.projection(P.m, d, seed=0)).to(dev), h, max_batch=4096)
    net.set_params(torch.from_numpy(bi.mlp_init(d, h, P.m, seed=0, prior=10.0 / P.m)).to(dev))
    losses = ln.train_proposal(net, Bt_tr, lab["x_idx"], lab["supp_len"], epochs=args.epochs, batch=1024,
                               lr=1e-3, pos_weight=20.0, record_every=50)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rec["training"] = {"generate_s": t1 - t0, "label_s": t2 - t1, "train_s": t3 - t2,
                       "labelled_converged": int(ln.converged(lab).sum().item()),
                       "loss_every_50_steps": [float(v.item()) for v in losses]}
    del Bt_tr, lab
    outl, rec["bf16_learned"] = timed(lambda: ln.solve_with_proposal(bf, net, Bt, 256))
    xi, sl, pr = outbf["x_idx"].cpu().numpy(), outbf["supp_len"].cpu().numpy(), outl["proposal"].cpu().numpy()
    rec["bf16_learned"]["recall_at_256"] = float(np.mean([np.isin(xi[i, :sl[i]], pr[i]).mean()
                                                          for i in range(P.p) if sl[i] > 0]))
    rec["bf16_learned"]["fallback_fraction"] = float(((outl["status"] & pk.BMPL_SIG_FALLBACK) > 0).float().mean())
    rec["speedup_learned_vs_plain_fp32"] = rec["bf16_learned"]["value"] / rec["plain_fp32"]["value"]
    rec["speedup_learned_vs_plain_bf16"] = rec["bf16_learned"]["value"] / rec["plain_bf16"]["value"]
    # the learned run against the plain FP32 run on a sample of signals
    rows = list(range(0, P.p, max(1, P.p // 32)))
    X32, Xl = sparse_rows(out32, rows, P.m), sparse_rows(outl, rows, P.m)
    rec["max_rel_x_learned_vs_fp32_sample"] = float(max(
        np.linalg.norm(Xl[q] - X32[q]) / max(np.linalg.norm(X32[q]), 1e-300) for q in range(len(rows))))
    del bf, net
    return rec


def sparse_rows(out: dict, rows, m: int) -> np.ndarray:
    """Dense float64 copies of the solutions of the given signals."""
    idx, val, ln = out["x_idx"][rows].cpu().numpy(), out["x_val"][rows].cpu().numpy(), out["supp_len"][rows].cpu().numpy()
    X = np.zeros((len(rows), m))
    for q in range(len(rows)):
        X[q, idx[q, :ln[q]]] = val[q, :ln[q]]
    return X


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cs2048x16384")
    ap.add_argument("--cpu-sample", type=int, default=32, help="signals the oracle solves for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--screen", default="fp32", choices=("fp32", "bf16", "fp8"),
                    help="precision of the correlation product (bf16: certified screening + float32 re-score)")
    ap.add_argument("--no-extra", action="store_true", help="skip the bf16-screened and fp8-ranked measurements")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal comparison on the face-like dictionary")
    ap.add_argument("--learned-signals", type=int, default=16384, help="inference signals of the learned comparison")
    ap.add_argument("--train-signals", type=int, default=200000, help="BMPL-labelled training signals")
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--host-loop", action="store_true",
                    help="drive the outer iterations from the host instead of replaying captured graph segments")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (signals shard with no "
              "per-iteration exchange, so N GPUs run N independent batches)", file=sys.stderr)
        sys.exit(2)

    import torch

    import bmpl_inputs as bi
    import paper_1302_5010_amd as pk

    gen = bi.WORKLOADS[args.workload]
    P = gen()
    dev = torch.device("cuda:0")
    At = torch.from_numpy(P.At).to(dev)
    Bt = torch.from_numpy(P.Bt).to(dev)
    # Throughput: graph-captured segments, no instrumentation.
    solver = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, graph=not args.host_loop,
                       screen=args.screen)
    tune = solver.autotune(P.p)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        out = solver.solve(Bt)
    torch.cuda.synchronize()
    solved = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = solver.solve(Bt)
        solved.append(out["status"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    conv = [int(((s & pk.BMPL_SIG_CONVERGED) > 0).sum().item()) for s in solved]
    kkt = out["kkt"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    supp = out["supp_len"].cpu().numpy()

    # Kernel breakdown and the correlation kernel's roofline: the same steps again with every
    # launch bracketed by HIP events on the solve stream (host-driven loop, same tile shapes).
    timed = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, timing=True, screen=args.screen)
    timed.set_tuning(tune["shapes"])
    for _ in range(args.warmup):
        timed.solve(Bt)
    torch.cuda.synchronize()
    timed.reset_timing()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        timed.solve(Bt)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    tm = timed.timing()
    # master-problem counts (appends, drops, sign-fixed solves, phase ticks): one more instrumented solve
    ph = pk.Solver(At, P.lambda_rel, mode="rel", rho=P.rho, kkt_tol=1e-4, timing=True, phases=True,
                   screen=args.screen)
    ph.set_tuning(tune["shapes"])
    ph.solve(Bt)
    torch.cuda.synchronize()
    tph = ph.timing()
    del ph
    corr_avg_s = tm["corr_ms"] / max(1, tm["corr_launches"]) * 1e-3
    achieved = tm["corr_flops"] / (tm["corr_ms"] * 1e-3) / 1e12 if tm["corr_ms"] > 0 else 0.0
    traffic = None
    rec = load_traffic(os.path.join(ROOT, "profiles", f"corr_gemm_{args.screen}_{args.workload}_pmc.json"))
    if rec is not None:
        traffic = rec.get("hbm_bytes_per_launch")

    result = {
        "metric": "signals solved/sec at KKT tol 1e-4 (" + {"fp32": "plain FP32", "bf16": "BF16-screened",
                                                             "fp8": "FP8-ranked"}[args.screen] + " BMPL)",
        "value": sum(conv) / elapsed,
        "unit": "signals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[args.screen],
        "data": "synthetic (seeded)",
        "config": {"workload": P.name, "n": P.n, "m": P.m, "p": P.p, "rho": P.rho,
                   "lambda_rel": P.lambda_rel, "kkt_tol": 1e-4, "screen": args.screen,
                   "graph": not args.host_loop},
        "roofline": {
            "bound": "mfma",
            "kernel": "corr_gemm_" + args.screen,
            "achieved": achieved,
            "peak": PEAK_TFLOPS[args.screen],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[args.screen],
            "traffic": traffic,
            "avg_launch_ms": corr_avg_s * 1e3,
            "launches": tm["corr_launches"],
            "algorithmic_gflop_per_step": tm["corr_flops"] / args.steps / 1e9,
        },
        "timed_run_ms_per_step": (t3 - t2) / args.steps * 1e3,
        "kernel_ms_per_step": {k: tm[k] / args.steps for k in ("corr_ms", "select_ms", "solve_ms",
                                                                "other_ms", "wall_ms")},
        "master_problem_counts_per_step": {k: tph[k] for k in ("factor_appends", "factor_drops",
                                                                "sign_fixed_solves")},
        "outer_iters_per_step": tm["outer_iters"] / args.steps,
        "solve_phase_us_per_step_summed_over_signals": dict(zip(
            ("load", "gram", "active_set", "certificate", "appends_within_active_set", "writeback"),
            tph["solve_phase_us"])),
        "autotune": tune,
        "signals": {"converged_per_step": conv, "kkt_max": float(np.max(kkt)),
                    "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
                    "support_mean": float(np.mean(supp))},
    }

    if args.screen == "fp32" and not args.no_extra:
        # The same workload with the reduced-precision products: bfloat16 screening (certified band +
        # exact re-score) and e4m3 ranking (exact re-score of the top candidates, bfloat16 certification).
        result["bf16_screened"] = screened_measurement(args, pk, torch, At, Bt, P, "bf16")
        result["fp8_ranked"] = screened_measurement(args, pk, torch, At, Bt, P, "fp8")
        result["q_route"] = q_route_measurement(args, pk, torch, At, Bt, P, tm)
        result["smpl"] = smpl_measurement(args, pk, torch, At, Bt, P, out)

    if not args.no_learned:
        result["learned"] = learned_comparison(args, pk, torch)

    if not args.no_cpu and args.cpu_sample > 0:
        import oracle
        from tests.parity import check_batch
        q = min(args.cpu_sample, P.p)
        rows = list(range(q))
        lam_gpu = out["lambda"].cpu().numpy()
        A64 = P.At.astype(np.float64)
        lam_or = P.lambda_rel * np.abs(A64 @ P.Bt[rows].astype(np.float64).T).max(axis=0)
        threads = min(oracle.max_threads(), q)
        c0 = time.perf_counter()
        ref = oracle.solve(P.At, P.Bt[rows], lam_or, P.rho, nthreads=threads)
        c1 = time.perf_counter()
        errs = check_batch(P.At, P.Bt, lam_or, out, ref, rows=range(q), gpu_rows=rows)
        result["cpu_baseline"] = {
            "value": q / (c1 - c0), "unit": "signals/s", "cores": threads, "kind": "oracle",
            "sample": f"first {q} signals of the same workload, FP64 C oracle, OpenMP one signal per thread",
        }
        result["parity_on_sample"] = {
            "signals": q, "max_rel_obj": float(max(e["rel_obj"] for e in errs)),
            "max_rel_x": float(max(e["rel_x"] for e in errs)),
            "max_rel_lambda": float(np.max(np.abs(lam_gpu[rows] - lam_or) / lam_or)),
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
