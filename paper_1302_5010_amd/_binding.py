"""ctypes marshalling for libbmpl (argument conversion only)."""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbmpl.so")

BMPL_SIG_CONVERGED = 1
BMPL_SIG_CAP_ITERS = 2
BMPL_SIG_CAP_ACTIVE = 4
BMPL_SIG_NONFINITE = 8
BMPL_SIG_FALLBACK = 16
BMPL_SIG_INEXACT = 32
BMPL_SIG_EARLY = 64

_PREC = {"fp32": 0, "bf16": 1, "fp8": 2}
_MODE = {"abs": 0, "rel": 1}


class BmplError(RuntimeError):
    pass


class _Options(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("kkt_tol", ctypes.c_double), ("screen", ctypes.c_int), ("flags", ctypes.c_int32),
                ("omega", ctypes.c_int32), ("eps_early", ctypes.c_double), ("r_inf_rel", ctypes.c_double),
                ("r2_rel", ctypes.c_double)]


class Timing(ctypes.Structure):
    _fields_ = [("corr_ms", ctypes.c_double), ("corr_launches", ctypes.c_int64), ("corr_flops", ctypes.c_double),
                ("corr_bytes", ctypes.c_double), ("select_ms", ctypes.c_double),
                ("select_launches", ctypes.c_int64), ("solve_ms", ctypes.c_double),
                ("solve_launches", ctypes.c_int64), ("residual_ms", ctypes.c_double), ("other_ms", ctypes.c_double),
                ("wall_ms", ctypes.c_double), ("solves", ctypes.c_int64), ("outer_iters", ctypes.c_int64),
                ("solve_phase_us", ctypes.c_double * 6), ("factor_appends", ctypes.c_int64),
                ("factor_drops", ctypes.c_int64), ("sign_fixed_solves", ctypes.c_int64),
                ("corr_roof_ms", ctypes.c_double), ("solve_step_us", ctypes.c_double * 6)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["solve_phase_us"] = list(self.solve_phase_us)
        d["solve_step_us"] = list(self.solve_step_us)
        return d


BMPL_FLAG_TIMING = 1
BMPL_FLAG_NO_GRAM_TABLE = 2
BMPL_FLAG_GRAPH = 4
BMPL_FLAG_BLOCK_APPEND = 8
BMPL_FLAG_PHASES = 16
BMPL_FLAG_Q_ROUTE = 32
CORR_SHAPES = 15       # BMPL_CORR_SHAPES


class _Result(ctypes.Structure):
    _fields_ = [("x_val_dev", ctypes.c_void_p), ("x_idx_dev", ctypes.c_void_p),
                ("supp_len_dev", ctypes.c_void_p), ("iters_dev", ctypes.c_void_p),
                ("kkt_dev", ctypes.c_void_p), ("lambda_dev", ctypes.c_void_p),
                ("objective_dev", ctypes.c_void_p), ("sig_status_dev", ctypes.c_void_p),
                ("ld_x", ctypes.c_int32)]


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


def library_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libbmpl.so not found at {_LIB_PATH}; run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.bmpl_options_default.argtypes = [ctypes.POINTER(_Options)]
    lib.bmpl_create.argtypes = [vp, i64, i32, i32, ctypes.c_int, dbl, ctypes.POINTER(_Options), vp,
                                ctypes.POINTER(vp)]
    lib.bmpl_solve.argtypes = [vp, vp, i64, i32, vp, vp, i32, ctypes.POINTER(_Result), vp]
    lib.bmpl_destroy.argtypes = [vp]
    lib.bmpl_last_error.restype = ctypes.c_char_p
    lib.bmpl_last_error.argtypes = [ctypes.c_void_p]
    lib.bmpl_correlate.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    lib.bmpl_correlate_noalloc.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    lib.bmpl_select.argtypes = [vp, vp, i64, i32, vp, vp, i32, vp, vp, vp, vp]
    lib.bmpl_get_timing.argtypes = [vp, ctypes.POINTER(Timing)]
    lib.bmpl_gram_table.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.bmpl_autotune.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
    lib.bmpl_set_tuning.argtypes = [vp, ctypes.POINTER(i32)]
    lib.bmpl_reset_timing.argtypes = [vp]
    lib.bmpl_classify.argtypes = [vp, vp, i64, i32, ctypes.POINTER(_Result), vp, vp, vp, vp]
    lib.bmpl_mlp_param_count.argtypes = [i32, i32, i32]
    lib.bmpl_mlp_param_count.restype = i64
    lib.bmpl_mlp_create.argtypes = [vp, i64, i32, i32, vp, i32, i32, i32, vp, ctypes.POINTER(vp)]
    lib.bmpl_mlp_destroy.argtypes = [vp]
    lib.bmpl_mlp_set_params.argtypes = [vp, vp, vp]
    lib.bmpl_mlp_get_params.argtypes = [vp, vp, vp]
    lib.bmpl_mlp_embed.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    lib.bmpl_mlp_forward.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    lib.bmpl_mlp_loss_grad.argtypes = [vp, vp, i64, i32, vp, i32, vp, dbl, vp, vp, vp]
    lib.bmpl_mlp_adam_step.argtypes = [vp, vp, ctypes.POINTER(AdamParams), vp]
    lib.bmpl_mlp_propose.argtypes = [vp, vp, i64, i32, i32, vp, i32, vp]
    lib.bmpl_topk.argtypes = [vp, i64, i32, i32, i32, vp, i32, vp]
    for f in ("bmpl_options_default", "bmpl_create", "bmpl_solve", "bmpl_destroy", "bmpl_correlate",
              "bmpl_correlate_noalloc",
              "bmpl_select", "bmpl_get_timing", "bmpl_reset_timing", "bmpl_gram_table", "bmpl_autotune",
              "bmpl_set_tuning", "bmpl_mlp_create", "bmpl_mlp_destroy", "bmpl_mlp_set_params",
              "bmpl_mlp_get_params", "bmpl_mlp_embed", "bmpl_mlp_forward", "bmpl_mlp_loss_grad",
              "bmpl_mlp_adam_step", "bmpl_mlp_propose", "bmpl_topk", "bmpl_classify"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


_lib = _load()


def _check(rc: int, what: str):
    if rc != 0:
        msg = _lib.bmpl_last_error(None).decode(errors="replace")
        raise BmplError(f"{what} failed ({rc}): {msg}")


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    rc = hip.hipMemcpy(dst, src, nbytes, 3)   # hipMemcpyDeviceToDevice
    if rc != 0:
        raise BmplError(f"hipMemcpy failed ({rc})")


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise BmplError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise BmplError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise BmplError(f"{name} must be contiguous")
    return t


class Solver:
    """A BMPL context: the dictionary on the device plus the lambda rule and options.

    ``At``: (m, n) float32 CUDA tensor, atom j in row j.  ``lam``: lambda
    (``mode='abs'``) or the factor c of lambda_i = c ||A^T b_i||_inf
    (``mode='rel'``).
    """

    def __init__(self, At: torch.Tensor, lam: float, mode: str = "abs", rho: int = 10, max_outer: int = 0,
                 max_active: int = 0, kkt_tol: float = 1e-4, screen: str = "fp32", timing: bool = False,
                 gram_table: bool = True, graph: bool = False, block_append: bool = False, phases: bool = False,
                 q_route: bool = False, omega: int = 1, eps_early: float = 0.0, r_inf_rel: float = 0.0,
                 r2_rel: float = 0.0, stream=None):
        At = _dev(At, torch.float32, "At")
        self.m, self.n = At.shape
        self.device = At.device
        o = _Options()
        _lib.bmpl_options_default(ctypes.byref(o))
        o.rho, o.max_outer, o.max_active, o.kkt_tol, o.omega = rho, max_outer, max_active, kkt_tol, omega
        o.eps_early, o.r_inf_rel, o.r2_rel = eps_early, r_inf_rel, r2_rel
        o.screen = _PREC[screen]
        o.flags = ((BMPL_FLAG_TIMING if timing else 0) | (0 if gram_table else BMPL_FLAG_NO_GRAM_TABLE)
                   | (BMPL_FLAG_GRAPH if graph else 0) | (BMPL_FLAG_BLOCK_APPEND if block_append else 0)
                   | (BMPL_FLAG_PHASES if phases else 0) | (BMPL_FLAG_Q_ROUTE if q_route else 0))
        self.options = o
        self.max_active = max_active if max_active > 0 else min(self.m, 2 * self.n)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_create(At.data_ptr(), self.n, self.n, self.m, _MODE[mode], float(lam), ctypes.byref(o),
                                    _stream_ptr(stream), ctypes.byref(h)), "bmpl_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.bmpl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, Bt: torch.Tensor, lam: torch.Tensor | None = None, warm: torch.Tensor | None = None,
              stream=None, ld_x: int | None = None) -> dict:
        """Solve every row of ``Bt`` ((p, n) float32).  Returns device tensors:
        x_idx/x_val (p, ld_x) sorted by atom, supp_len, iters, kkt, lambda,
        objective, status.  ``lam``: optional (p,) float64 absolute lambdas.
        ``warm``: optional (p, k) int32 proposed atoms (-1 = unused)."""
        Bt = _dev(Bt, torch.float32, "Bt")
        p, n = Bt.shape
        if n != self.n:
            raise BmplError(f"signals have length {n}, dictionary expects {self.n}")
        ld = ld_x if ld_x is not None else min(self.max_active, self.n)
        dev = Bt.device
        out = {
            # the library writes every entry (rows padded with -1 / 0 past supp_len)
            "x_val": torch.empty((p, ld), dtype=torch.float32, device=dev),
            "x_idx": torch.empty((p, ld), dtype=torch.int32, device=dev),
            "supp_len": torch.empty(p, dtype=torch.int32, device=dev),
            "iters": torch.empty(p, dtype=torch.int32, device=dev),
            "kkt": torch.empty(p, dtype=torch.float64, device=dev),
            "lambda": torch.empty(p, dtype=torch.float64, device=dev),
            "objective": torch.empty(p, dtype=torch.float64, device=dev),
            "status": torch.empty(p, dtype=torch.int32, device=dev),
        }
        r = _Result(out["x_val"].data_ptr(), out["x_idx"].data_ptr(), out["supp_len"].data_ptr(),
                    out["iters"].data_ptr(), out["kkt"].data_ptr(), out["lambda"].data_ptr(),
                    out["objective"].data_ptr(), out["status"].data_ptr(), ld)
        lam_ptr = 0
        if lam is not None:
            lam = _dev(lam, torch.float64, "lam")
            if lam.numel() != p:
                raise BmplError("lam must hold one value per signal")
            lam_ptr = lam.data_ptr()
        warm_ptr, warm_k = 0, 0
        if warm is not None:
            warm = _dev(warm, torch.int32, "warm")
            if warm.dim() != 2 or warm.shape[0] != p:
                raise BmplError("warm must be (p, k) int32")
            warm_ptr, warm_k = warm.data_ptr(), warm.shape[1]
        with torch.cuda.device(dev):
            _check(_lib.bmpl_solve(self._h, Bt.data_ptr(), n, p, lam_ptr or None, warm_ptr or None, warm_k,
                                   ctypes.byref(r), _stream_ptr(stream)), "bmpl_solve")
        out["_keep"] = (Bt, lam, warm)
        return out

    def classify(self, Bt: torch.Tensor, out: dict, class_of_atom: torch.Tensor, stream=None):
        """Class-residual labels (p,) int32 and winning residual norms (p,) float64 for the codes in
        ``out`` (a result of :meth:`solve` on the same ``Bt``); ``class_of_atom`` (m,) int32."""
        Bt = _dev(Bt, torch.float32, "Bt")
        cls = _dev(class_of_atom, torch.int32, "class_of_atom")
        if cls.numel() != self.m:
            raise BmplError("class_of_atom must hold one class per atom")
        p = Bt.shape[0]
        labels = torch.empty(p, dtype=torch.int32, device=Bt.device)
        resid = torch.empty(p, dtype=torch.float64, device=Bt.device)
        r = _Result(out["x_val"].data_ptr(), out["x_idx"].data_ptr(), out["supp_len"].data_ptr(), None, None, None,
                    None, None, out["x_idx"].shape[1])
        with torch.cuda.device(Bt.device):
            _check(_lib.bmpl_classify(self._h, Bt.data_ptr(), Bt.shape[1], p, ctypes.byref(r), cls.data_ptr(),
                                      labels.data_ptr(), resid.data_ptr(), _stream_ptr(stream)), "bmpl_classify")
        return labels, resid

    def autotune(self, p: int, stream=None) -> dict:
        """Time every correlation tile shape for this dictionary; the fastest per bucket is kept."""
        shapes = (ctypes.c_int32 * 3)()
        ms = (ctypes.c_double * (3 * CORR_SHAPES))()
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_autotune(self._h, int(p), shapes, ms, _stream_ptr(stream)), "bmpl_autotune")
        return {"shapes": list(shapes), "ms": [list(ms[b * CORR_SHAPES:(b + 1) * CORR_SHAPES]) for b in range(3)]}

    def set_tuning(self, shapes):
        """Correlation tile shape per running-signal bucket (>= 512, 64..511, < 64), each in 0..7."""
        arr = (ctypes.c_int32 * 3)(*[int(v) for v in shapes])
        _check(_lib.bmpl_set_tuning(self._h, arr), "bmpl_set_tuning")

    def gram_table(self) -> torch.Tensor | None:
        """A copy of the float64 Gram table Q = A^T A held by the context, or None."""
        q = ctypes.c_void_p()
        ld = ctypes.c_int64()
        _check(_lib.bmpl_gram_table(self._h, ctypes.byref(q), ctypes.byref(ld)), "bmpl_gram_table")
        if not q.value:
            return None
        out = torch.empty((self.m, self.m), dtype=torch.float64, device=self.device)
        nbytes = self.m * self.m * 8
        torch.cuda.synchronize(self.device)
        _memcpy_d2d(out.data_ptr(), q.value, nbytes)
        return out

    def timing(self) -> dict:
        """Kernel times accumulated since the last reset (needs ``timing=True``)."""
        t = Timing()
        _check(_lib.bmpl_get_timing(self._h, ctypes.byref(t)), "bmpl_get_timing")
        return t.as_dict()

    def reset_timing(self):
        _check(_lib.bmpl_reset_timing(self._h), "bmpl_reset_timing")

    def correlate(self, Rt: torch.Tensor, stream=None) -> torch.Tensor:
        """G (p, m) with G[i, j] = a_j^T r_i for the rows r_i of ``Rt`` ((p, n) float32)."""
        Rt = _dev(Rt, torch.float32, "Rt")
        p = Rt.shape[0]
        G = torch.empty((p, self.m), dtype=torch.float32, device=Rt.device)
        with torch.cuda.device(Rt.device):
            _check(_lib.bmpl_correlate(self._h, Rt.data_ptr(), self.n, p, G.data_ptr(), self.m,
                                       _stream_ptr(stream)), "bmpl_correlate")
        return G

    def correlate_noalloc(self, Rt: torch.Tensor, G: torch.Tensor, stream=None) -> torch.Tensor:
        """bmpl_correlate_noalloc into the caller's G ((p, m) float32): the library allocates nothing and
        does not synchronise, so the call can be captured in a graph."""
        Rt = _dev(Rt, torch.float32, "Rt")
        p = Rt.shape[0]
        if G.dtype != torch.float32 or G.shape != (p, self.m) or not G.is_contiguous() or G.device != Rt.device:
            raise BmplError("G must be a contiguous (p, m) float32 tensor on the residuals' device")
        with torch.cuda.device(Rt.device):
            _check(_lib.bmpl_correlate_noalloc(self._h, Rt.data_ptr(), self.n, p, G.data_ptr(), self.m,
                                               _stream_ptr(stream)), "bmpl_correlate_noalloc")
        return G

    def select(self, G: torch.Tensor, lam: torch.Tensor, k: int, excl: torch.Tensor | None = None, stream=None):
        """Top-k violators per row of G; returns (sel (p, k) int32, nsel (p,), vmax (p,))."""
        G = _dev(G, torch.float32, "G")
        lam = _dev(lam, torch.float64, "lam")
        p = G.shape[0]
        sel = torch.full((p, k), -1, dtype=torch.int32, device=G.device)
        nsel = torch.zeros(p, dtype=torch.int32, device=G.device)
        vmax = torch.zeros(p, dtype=torch.float32, device=G.device)
        ex = 0
        if excl is not None:
            ex = _dev(excl, torch.int32, "excl").data_ptr()
        with torch.cuda.device(G.device):
            _check(_lib.bmpl_select(self._h, G.data_ptr(), G.shape[1], p, lam.data_ptr(), ex or None, k,
                                    sel.data_ptr(), nsel.data_ptr(), vmax.data_ptr(), _stream_ptr(stream)),
                   "bmpl_select")
        return sel, nsel, vmax


def topk(S: torch.Tensor, k: int, L: int | None = None, stream=None) -> torch.Tensor:
    """Per row of ``S`` ((rows, lds) float32), the k largest of the first L columns' indices,
    ascending, ties to the lower index (bmpl_topk)."""
    S = _dev(S, torch.float32, "S")
    rows, lds = S.shape
    L = lds if L is None else L
    out = torch.empty((rows, k), dtype=torch.int32, device=S.device)
    with torch.cuda.device(S.device):
        _check(_lib.bmpl_topk(S.data_ptr(), lds, rows, L, k, out.data_ptr(), k, _stream_ptr(stream)), "bmpl_topk")
    return out


def mlp_param_count(d_in: int, d_hidden: int, m: int) -> int:
    return int(_lib.bmpl_mlp_param_count(d_in, d_hidden, m))


class ProposalNet:
    """The learned support proposal (bmpl_mlp_*): z = unit-RMS (A P)^T b, two GELU layers of
    width ``d_hidden``, m atom scores.  ``At``: (m, n) float32 dictionary, ``P``: (m, d_in)
    float32 projection, both CUDA tensors."""

    def __init__(self, At: torch.Tensor, P: torch.Tensor, d_hidden: int, max_batch: int, stream=None):
        At = _dev(At, torch.float32, "At")
        P = _dev(P, torch.float32, "P")
        self.m, self.n = At.shape
        if P.shape[0] != self.m:
            raise BmplError("P must have one row per atom")
        self.d_in, self.d_hidden, self.max_batch = P.shape[1], d_hidden, max_batch
        self.device = At.device
        self.count = mlp_param_count(self.d_in, d_hidden, self.m)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_create(At.data_ptr(), self.n, self.n, self.m, P.data_ptr(), self.d_in, d_hidden,
                                        max_batch, _stream_ptr(stream), ctypes.byref(h)), "bmpl_mlp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.bmpl_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: torch.Tensor, stream=None):
        params = _dev(params, torch.float32, "params")
        if params.numel() != self.count:
            raise BmplError(f"params must hold {self.count} floats")
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_set_params(self._h, params.data_ptr(), _stream_ptr(stream)), "bmpl_mlp_set_params")

    def get_params(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.count, dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_get_params(self._h, out.data_ptr(), _stream_ptr(stream)), "bmpl_mlp_get_params")
        return out

    def embed(self, Bt: torch.Tensor, stream=None) -> torch.Tensor:
        Bt = _dev(Bt, torch.float32, "Bt")
        Z = torch.empty((Bt.shape[0], self.d_in), dtype=torch.float32, device=Bt.device)
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_embed(self._h, Bt.data_ptr(), Bt.shape[1], Bt.shape[0], Z.data_ptr(), self.d_in,
                                       _stream_ptr(stream)), "bmpl_mlp_embed")
        return Z

    def forward(self, Bt: torch.Tensor, stream=None) -> torch.Tensor:
        Bt = _dev(Bt, torch.float32, "Bt")
        S = torch.empty((Bt.shape[0], self.m), dtype=torch.float32, device=Bt.device)
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_forward(self._h, Bt.data_ptr(), Bt.shape[1], Bt.shape[0], S.data_ptr(), self.m,
                                         _stream_ptr(stream)), "bmpl_mlp_forward")
        return S

    def loss_grad(self, Bt: torch.Tensor, supp: torch.Tensor, supp_len: torch.Tensor, pos_weight: float,
                  want_grad: bool = True, stream=None):
        """Mean loss (device float64 scalar) and, if ``want_grad``, the flat gradient."""
        Bt = _dev(Bt, torch.float32, "Bt")
        supp = _dev(supp, torch.int32, "supp")
        supp_len = _dev(supp_len, torch.int32, "supp_len")
        loss = torch.zeros(1, dtype=torch.float64, device=Bt.device)
        g = torch.empty(self.count, dtype=torch.float32, device=Bt.device) if want_grad else None
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_loss_grad(self._h, Bt.data_ptr(), Bt.shape[1], Bt.shape[0], supp.data_ptr(),
                                           supp.shape[1], supp_len.data_ptr(), float(pos_weight),
                                           g.data_ptr() if g is not None else None, loss.data_ptr(),
                                           _stream_ptr(stream)), "bmpl_mlp_loss_grad")
        return loss, g

    def adam_step(self, lr: float, grad: torch.Tensor | None = None, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, stream=None):
        hp = AdamParams(lr, beta1, beta2, eps)
        gp = _dev(grad, torch.float32, "grad").data_ptr() if grad is not None else None
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_adam_step(self._h, gp, ctypes.byref(hp), _stream_ptr(stream)), "bmpl_mlp_adam_step")

    def propose(self, Bt: torch.Tensor, k: int, stream=None) -> torch.Tensor:
        """(p, k) int32: the k highest-scoring atoms per signal, ascending (bmpl_solve's warm start)."""
        Bt = _dev(Bt, torch.float32, "Bt")
        out = torch.empty((Bt.shape[0], k), dtype=torch.int32, device=Bt.device)
        with torch.cuda.device(self.device):
            _check(_lib.bmpl_mlp_propose(self._h, Bt.data_ptr(), Bt.shape[1], Bt.shape[0], k, out.data_ptr(), k,
                                         _stream_ptr(stream)), "bmpl_mlp_propose")
        return out
