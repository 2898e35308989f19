"""GPU: whole solves captured as one graph (BMPL_FLAG_GRAPH with an iteration cap of at most 64).

With the cap known, every pass of the solve is one graph and each signal's slot block is sized for the
largest active set the cap allows, so bmpl_solve enqueues the solve and returns without waiting for the
device.  The results must equal the host loop's (same cap) bit for bit, in every screening mode, with
warm starts, SMPL and caps that stop signals early, and the call must return while the stream is busy.
"""
import time

import numpy as np
import pytest

import bmpl_inputs as bi
import oracle
from tests.parity import check_batch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("x_idx", "x_val", "supp_len", "iters", "status", "kkt", "objective")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_5010_amd as pk
    return pk


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lam_rel(At, Bt, c):
    return c * np.abs(At.astype(np.float64) @ Bt.astype(np.float64).T).max(axis=0)


def _problem():
    return bi.tiny_gaussian(n=256, m=2000, p=300, k=30, sigma=0.01, seed=83, rho=7)


def _assert_same(out, ref, tag):
    torch.cuda.synchronize()
    for key in KEYS:
        assert torch.equal(out[key], ref[key]), (tag, key)


@pytest.mark.parametrize("screen,omega", [("fp32", 1), ("bf16", 1), ("fp8", 1), ("fp32", 3)])
def test_full_depth_graph_matches_host_loop(screen, omega):
    pk = _lib()
    P = _problem()
    lam = to_dev(lam_rel(P.At, P.Bt, P.lambda_rel))
    At, Bt = to_dev(P.At), to_dev(P.Bt)
    need = pk.Solver(At, 0.0, rho=P.rho, screen=screen, omega=omega).solve(Bt, lam=lam)
    it_max = int(need["iters"].max().item())
    assert it_max + 2 <= 64
    # a cap above every signal's need, and one that stops the slowest signals
    converged = None
    for cap in (it_max + 2, max(2, it_max - 2)):
        host = pk.Solver(At, 0.0, rho=P.rho, screen=screen, omega=omega, max_outer=cap).solve(Bt, lam=lam)
        s = pk.Solver(At, 0.0, rho=P.rho, screen=screen, omega=omega, max_outer=cap, graph=True)
        for rep in range(3):                      # the first call captures, the others replay
            _assert_same(s.solve(Bt, lam=lam), host, (screen, omega, cap, rep))
        st = host["status"].cpu().numpy()
        if cap < it_max:
            assert np.any(st & pk.BMPL_SIG_CAP_ITERS)
        else:
            assert np.all(st & pk.BMPL_SIG_CONVERGED)
            converged = host
        s.close()
    if screen == "fp32" and omega == 1:
        ref = oracle.solve(P.At, P.Bt, lam.cpu().numpy(), P.rho)
        check_batch(P.At, P.Bt, lam.cpu().numpy(), converged, ref)


@pytest.mark.parametrize("warm_k", [16, 200])
def test_full_depth_graph_warm_start(warm_k):
    """A warm start (the proposal's master problem first, then the fallback passes) inside the one graph:
    the proposals hold the true support's atoms padded with random ones, some signals miss atoms."""
    pk = _lib()
    P = _problem()
    lam = to_dev(lam_rel(P.At, P.Bt, P.lambda_rel))
    At, Bt = to_dev(P.At), to_dev(P.Bt)
    rng = np.random.default_rng(warm_k)
    prop = np.full((P.p, warm_k), -1, dtype=np.int32)
    for i, s in enumerate(P.supports):
        keep = s[: max(0, len(s) - (i % 3))]      # every third signal misses two atoms
        pad = rng.choice(P.m, size=warm_k, replace=False)
        row = list(dict.fromkeys(list(keep) + list(pad)))[:warm_k]
        prop[i, :len(row)] = row
    warm = to_dev(prop)
    host = pk.Solver(At, 0.0, rho=P.rho, max_outer=30).solve(Bt, lam=lam, warm=warm)
    s = pk.Solver(At, 0.0, rho=P.rho, max_outer=30, graph=True)
    for rep in range(2):
        _assert_same(s.solve(Bt, lam=lam, warm=warm), host, (warm_k, rep))
    assert np.all(host["status"].cpu().numpy() & pk.BMPL_SIG_CONVERGED)


def _spin_cycles(ms_target):
    """Cycles of torch's spin kernel that keep the stream busy for about ms_target milliseconds (grown by
    doubling from a short spin, so no single calibration spin runs much past the target)."""
    c = 1 << 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(40):
        e0.record()
        torch.cuda._sleep(c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        if ms >= ms_target / 4:
            return int(c * ms_target / ms)
        c *= 2
    pytest.skip("the spin kernel does not take measurable time here")


def test_full_depth_solve_does_not_wait_for_the_device():
    """Behind a 400 ms spin on the same stream, the capped graph-mode solve returns at once (the stream
    still busy), while the segmented graph mode (no cap) waits for its first read-back; both then give
    the host loop's results."""
    pk = _lib()
    P = _problem()
    lam = to_dev(lam_rel(P.At, P.Bt, P.lambda_rel))
    At, Bt = to_dev(P.At), to_dev(P.Bt)
    host = pk.Solver(At, 0.0, rho=P.rho, max_outer=40).solve(Bt, lam=lam)
    cyc = _spin_cycles(400.0)
    for cap, waits in ((40, False), (0, True)):
        s = pk.Solver(At, 0.0, rho=P.rho, max_outer=cap, graph=True)
        s.solve(Bt, lam=lam)                      # capture, and the arena and workspace allocations
        torch.cuda.synchronize()
        torch.cuda._sleep(cyc)
        t0 = time.perf_counter()
        out = s.solve(Bt, lam=lam)
        dt = time.perf_counter() - t0
        busy = not torch.cuda.current_stream().query()
        torch.cuda.synchronize()
        if waits:
            assert dt > 0.2, dt
        else:
            assert busy and dt < 0.1, (busy, dt)
        _assert_same(out, host, cap)
        s.close()
