"""The entry point that allocates nothing (bmpl_correlate_noalloc) against bmpl_correlate.

Both run the same kernels, so the products must agree bit for bit: two calls in a row (the second with
fewer residuals, so stale scratch contents from the first would show), in every screening precision,
a size beyond the scratch limit rejected before any work, and the call captured in a HIP graph and
replayed with eager work in between, every replay checked against an eager bmpl_correlate.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_5010_amd as pk
    return pk


def _dictionary(n, m, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    return (A / np.linalg.norm(A, axis=1, keepdims=True)).astype(np.float32), rng


@pytest.mark.parametrize("screen", ["fp32", "bf16", "fp8"])
def test_correlate_noalloc_matches_correlate(screen):
    pk = _lib()
    n, m = 200, 3000
    At, rng = _dictionary(n, m, 7)
    s = pk.Solver(torch.from_numpy(At).cuda(), 0.0, rho=4, screen=screen)
    for p in (300, 37):
        R = torch.from_numpy(rng.standard_normal((p, n)).astype(np.float32)).cuda()
        ref = s.correlate(R)
        G = torch.full((p, m), float("nan"), dtype=torch.float32, device="cuda")
        s.correlate_noalloc(R, G)
        torch.cuda.synchronize()
        print(f"screen={screen} p={p}", flush=True)
        assert torch.equal(G, ref), (screen, p)
    s.close()


def test_correlate_noalloc_rejects_sizes_beyond_the_scratch():
    pk = _lib()
    n, m = 200, 3000
    At, _ = _dictionary(n, m, 8)
    s = pk.Solver(torch.from_numpy(At).cuda(), 0.0, rho=4)
    R = torch.zeros((1, n), dtype=torch.float32, device="cuda")
    G = torch.zeros((1, m), dtype=torch.float32, device="cuda")
    lib = pk._binding._lib
    lib.bmpl_last_error.restype = ctypes.c_char_p
    # (p + 1) * 256 * 4 bytes of staging > 64 MiB: rejected before any memory is touched
    rc = lib.bmpl_correlate_noalloc(s._h, R.data_ptr(), n, 70000, G.data_ptr(), m, None)
    assert rc == -1                        # BMPL_E_INVALID
    assert b"BMPL_NOALLOC_SCRATCH_BYTES" in lib.bmpl_last_error(None)
    s.close()


def test_correlate_noalloc_under_graph_capture():
    pk = _lib()
    n, m, p = 256, 2000, 64
    At, rng = _dictionary(n, m, 9)
    s = pk.Solver(torch.from_numpy(At).cuda(), 0.0, rho=4)
    R = torch.from_numpy(rng.standard_normal((p, n)).astype(np.float32)).cuda()
    G = torch.zeros((p, m), dtype=torch.float32, device="cuda")
    s.correlate_noalloc(R, G)              # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.correlate_noalloc(R, G, stream=torch.cuda.current_stream())
    for rep in range(4):
        R.copy_(torch.from_numpy(rng.standard_normal((p, n)).astype(np.float32)).cuda())   # eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = s.correlate(R)
        torch.cuda.synchronize()
        assert torch.equal(G, ref), rep
    s.close()
