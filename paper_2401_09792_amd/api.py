"""Python front end of libgtucker: a plan object over packed device buffers, and autograd
wrappers.  torch supplies device memory and the stream; every step runs in the library."""

from __future__ import annotations

import ctypes as C
from typing import Dict, Iterable, List, Optional, Sequence

import torch

from . import _binding as B
from ._binding import ChannelDesc, FitOptions, Offsets, TuneResult, check, load


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _buf(t: Optional[torch.Tensor], n: int, dtype: torch.dtype, name: str,
         optional: bool = False) -> Optional[torch.Tensor]:
    """Checks that a buffer handed to the library is a contiguous GPU tensor of the plan's
    element type with exactly the number of elements the plan lays out for it (a smaller
    buffer would let the kernels write past its end)."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Immutable description of a batch of channels plus its device workspace.

    descs: iterable of dicts with keys nr, nt, nsc, group_size, m, n, p, ns.
    Packed buffers (1-D complex64, or complex128 on a "c128" plan): X, A, B, C, G, Ht with
    per-channel blocks at `offsets(c)`; SINR output is float32 (float64 on a "c128" plan)
    [n_snr][total_subcarriers][ns_max].  Every buffer is checked against the plan's sizes and
    element type before the library sees its pointer.
    """

    TTM_PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "split_bf16": 3}
    DTYPES = {"c64": (B.GT_C64, torch.complex64, torch.float32),
              "c128": (B.GT_C128, torch.complex128, torch.float64)}

    def __init__(self, descs: Iterable[dict], iters: int = 20, eig_fp64: bool = False,
                 warm_start: bool = False, ttm_prec: str = "fp32", device="cuda",
                 dtype: str = "c64"):
        """dtype "c128" makes a plan whose SINR calls (forward, full-channel and adjoint) run
        in FP64 on complex128 buffers with float64 outputs; it provides no fit."""
        self.lib = load()
        if dtype not in self.DTYPES:
            raise ValueError(f"dtype must be one of {sorted(self.DTYPES)}")
        code, self.cdtype, self.rdtype = self.DTYPES[dtype]
        self.dtype = dtype
        self.descs: List[dict] = [dict(d) for d in descs]
        arr = (ChannelDesc * len(self.descs))()
        for i, d in enumerate(self.descs):
            arr[i] = ChannelDesc(d["nr"], d["nt"], d["nsc"], d["group_size"], d["m"], d["n"],
                                 d["p"], d["ns"], d.get("a_id", 0), d.get("b_id", 0),
                                 d.get("serving", 0))
        self.sharing = any(d.get("a_id", 0) or d.get("b_id", 0) for d in self.descs)
        opt = FitOptions(int(iters), self.TTM_PREC[ttm_prec], 1 if eig_fp64 else 0,
                         B.GT_FIT_WARM_START if warm_start else 0, code)
        h = C.c_void_p()
        check("gt_plan_create", self.lib.gt_plan_create(arr, len(self.descs), C.byref(opt),
                                                        C.byref(h)))
        self._h = h
        self.iters = int(iters)
        tot = Offsets()
        nsm = C.c_int32()
        check("gt_plan_totals", self.lib.gt_plan_totals(h, C.byref(tot), C.byref(nsm)))
        self.totals = tot
        self.ns_max = nsm.value
        wsb = C.c_size_t()
        check("gt_plan_workspace_bytes", self.lib.gt_plan_workspace_bytes(h, C.byref(wsb)))
        self.ws_bytes = wsb.value
        self.device = torch.device(device)
        self.ws = None
        if self.device.type == "cuda":
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            check("gt_workspace_init", self.lib.gt_workspace_init(h, _ptr(self.ws), self.ws_bytes,
                                                                  _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self.lib.gt_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def n_channels(self) -> int:
        return len(self.descs)

    def offsets(self, c: int) -> Offsets:
        o = Offsets()
        check("gt_plan_offsets", self.lib.gt_plan_offsets(self._h, c, C.byref(o)))
        return o

    # -- buffers ---------------------------------------------------------------------
    def _new(self, n: int, dtype=None) -> torch.Tensor:
        return torch.zeros(n, dtype=dtype or self.cdtype, device=self.device)

    def _cx(self, t, what: str, name: str, optional: bool = False):
        """A packed complex buffer of kind `what` (x, a, b, c, g or ht) at the plan's sizes."""
        return _buf(t, getattr(self.totals, what), self.cdtype, name, optional)

    def _sinr_shape(self, k: int):
        return (k, self.totals.sc, self.ns_max)

    def _real_out(self, t, k: int, name: str, optional: bool = False):
        return _buf(t, k * self.totals.sc * self.ns_max, self.rdtype, name, optional)

    def _status(self, t, optional: bool = True):
        return _buf(t, self.n_channels, torch.int32, "status", optional)

    def empty_factors(self) -> Dict[str, torch.Tensor]:
        t = self.totals
        return dict(A=self._new(t.a), B=self._new(t.b), C=self._new(t.c), G=self._new(t.g))

    # -- calls -----------------------------------------------------------------------
    def fit(self, X: torch.Tensor, factors: Optional[Dict[str, torch.Tensor]] = None,
            trace: Optional[bool] = None) -> Dict[str, torch.Tensor]:
        """Groupwise Tucker compression of every channel in X (packed).  The objective trace is
        returned by default, except for plans that share factors (which provide none)."""
        if trace is None:
            trace = not self.sharing
        self._cx(X, "x", "X")
        f = factors if factors is not None else self.empty_factors()
        for k in ("A", "B", "C", "G"):
            self._cx(f.get(k), k.lower(), f"factors[{k!r}]")
        tr = (torch.zeros(self.n_channels * (1 + 3 * self.iters), dtype=torch.float64,
                          device=self.device) if trace else None)
        st = torch.zeros(self.n_channels, dtype=torch.int32, device=self.device)
        check("gt_tucker_fit", self.lib.gt_tucker_fit(
            self._h, _ptr(X), _ptr(f["A"]), _ptr(f["B"]), _ptr(f["C"]), _ptr(f["G"]), _ptr(tr),
            _ptr(st), _ptr(self.ws), self.ws_bytes, _stream()))
        out = dict(f)
        out["status"] = st
        if tr is not None:
            out["trace"] = tr.view(self.n_channels, 1 + 3 * self.iters)
        return out

    def autotune(self, X: torch.Tensor) -> Dict[str, float]:
        """Times the fit's pass variants on X and keeps the fastest in the plan (synchronises;
        call before capturing fits in a graph)."""
        self._cx(X, "x", "X")
        f = self.empty_factors()
        res = TuneResult()
        check("gt_plan_autotune", self.lib.gt_plan_autotune(
            self._h, _ptr(X), _ptr(f["A"]), _ptr(f["B"]), _ptr(f["C"]), _ptr(f["G"]),
            _ptr(self.ws), self.ws_bytes, _stream(), C.byref(res)))
        return dict(bstep=res.bstep, tpass=res.tpass, split=res.split, probe_ms=res.probe_ms)

    def set_tuning(self, bstep: int = 0, tpass: int = 0, split: int = 2) -> None:
        """Sets the fit's pass variants (the choices autotune makes)."""
        check("gt_plan_set_tuning", self.lib.gt_plan_set_tuning(self._h, bstep, tpass, split))

    def reconstruct(self, A, B_, C_, G, ht: bool = True, xhat: bool = True):
        t = self.totals
        self._cx(A, "a", "A", optional=not xhat)
        self._cx(B_, "b", "B", optional=not xhat)
        self._cx(C_, "c", "C")
        self._cx(G, "g", "G")
        Ht = self._new(t.ht) if ht else None
        Xh = self._new(t.x) if xhat else None
        check("gt_tucker_reconstruct", self.lib.gt_tucker_reconstruct(
            self._h, _ptr(A), _ptr(B_), _ptr(C_), _ptr(G), _ptr(Ht), _ptr(Xh), _ptr(self.ws),
            self.ws_bytes, _stream()))
        return Ht, Xh

    def _sigma2(self, sigma2: Sequence[float]):
        s = [float(v) for v in sigma2]
        return (C.c_float * len(s))(*s), len(s)

    def sinr(self, C_, G, sigma2: Sequence[float], out: Optional[torch.Tensor] = None,
             status: Optional[torch.Tensor] = None) -> torch.Tensor:
        s2, k = self._sigma2(sigma2)
        self._cx(C_, "c", "C")
        self._cx(G, "g", "G")
        self._status(status)
        if out is None:
            out = torch.empty(self._sinr_shape(k), dtype=self.rdtype, device=self.device)
        self._real_out(out, k, "out")
        check("gt_sinr_eval", self.lib.gt_sinr_eval(
            self._h, _ptr(C_), _ptr(G), s2, k, _ptr(out), _ptr(status), _ptr(self.ws),
            self.ws_bytes, _stream()))
        return out

    INTERF = {"none": B.GT_INTERF_NONE, "paper": B.GT_INTERF_PAPER, "all": B.GT_INTERF_ALL}

    def sinr_system(self, C_, G, sigma2: Sequence[float], mode: str = "paper",
                    out: Optional[torch.Tensor] = None,
                    status: Optional[torch.Tensor] = None) -> torch.Tensor:
        """SINR of every UE of a multi-cell system plan (channels labelled by a_id = UE,
        b_id = BS, serving = 1 on each UE's serving link), with the interference of `mode`;
        the UE's values sit at its serving channel's subcarriers."""
        s2, k = self._sigma2(sigma2)
        self._cx(C_, "c", "C")
        self._cx(G, "g", "G")
        self._status(status)
        if out is None:
            out = torch.empty(self._sinr_shape(k), dtype=self.rdtype, device=self.device)
        self._real_out(out, k, "out")
        check("gt_sinr_eval_system", self.lib.gt_sinr_eval_system(
            self._h, _ptr(C_), _ptr(G), s2, k, self.INTERF[mode], _ptr(out), _ptr(status),
            _ptr(self.ws), self.ws_bytes, _stream()))
        return out

    def sinr_full(self, X, sigma2: Sequence[float], out: Optional[torch.Tensor] = None,
                  status: Optional[torch.Tensor] = None) -> torch.Tensor:
        s2, k = self._sigma2(sigma2)
        self._cx(X, "x", "X")
        self._status(status)
        if out is None:
            out = torch.empty(self._sinr_shape(k), dtype=self.rdtype, device=self.device)
        self._real_out(out, k, "out")
        check("gt_sinr_eval_full", self.lib.gt_sinr_eval_full(
            self._h, _ptr(X), s2, k, _ptr(out), _ptr(status), _ptr(self.ws), self.ws_bytes,
            _stream()))
        return out

    # -- channels at general coefficient vectors (mode 3 = path / delay submatrices) ----
    def _weights(self, U, n_pts: int):
        _buf(U, n_pts * self.totals.sc, self.cdtype, "U")

    def combine_full(self, X, U, n_pts: int) -> torch.Tensor:
        """H(t) = sum_s U[t, s] H_s for the n_pts weight rows of every channel (U packed
        [n_pts][nsc] per channel); returns the packed [n_pts][nr][nt] blocks, the X layout of
        `combined_descs(..., compressed=False)`."""
        self._cx(X, "x", "X")
        self._weights(U, n_pts)
        out = self._new(n_pts * sum(d["nr"] * d["nt"] for d in self.descs))
        check("gt_combine_full", self.lib.gt_combine_full(
            self._h, _ptr(X), _ptr(U), int(n_pts), _ptr(out), _ptr(self.ws), self.ws_bytes,
            _stream()))
        return out

    def combine_compressed(self, C_, G, U, n_pts: int) -> torch.Tensor:
        """Ht(t) = G x3 (U[t] C) for the n_pts weight rows of every channel; returns the
        packed [n_pts][m][n] blocks, the X layout of `combined_descs(..., compressed=True)`."""
        self._cx(C_, "c", "C")
        self._cx(G, "g", "G")
        self._weights(U, n_pts)
        out = self._new(n_pts * sum(d["m"] * d["n"] for d in self.descs))
        check("gt_combine_compressed", self.lib.gt_combine_compressed(
            self._h, _ptr(C_), _ptr(G), _ptr(U), int(n_pts), _ptr(out), _ptr(self.ws),
            self.ws_bytes, _stream()))
        return out

    def combined_descs(self, n_pts: int, compressed: bool) -> List[dict]:
        """Descriptors of a plan whose X layout is the output of combine_compressed
        (compressed=True: nr = m, nt = n) or combine_full, with nsc = n_pts and the same ns:
        its sinr_full gives the SINR of every combined channel."""
        out = []
        for d in self.descs:
            r, t = (d["m"], d["n"]) if compressed else (d["nr"], d["nt"])
            out.append(dict(nr=r, nt=t, nsc=int(n_pts), group_size=1, m=d["ns"], n=d["ns"], p=1,
                            ns=d["ns"]))
        return out

    def sinr_backward(self, C_, G, sigma2, grad_sinr, status=None):
        s2, k = self._sigma2(sigma2)
        self._cx(C_, "c", "C")
        self._cx(G, "g", "G")
        self._status(status)
        if not isinstance(grad_sinr, torch.Tensor) or tuple(grad_sinr.shape) != self._sinr_shape(k):
            raise ValueError(f"grad_sinr must have shape {self._sinr_shape(k)}")
        gs = grad_sinr.contiguous().to(self.rdtype)
        gC = torch.empty_like(C_)
        gG = torch.empty_like(G)
        check("gt_sinr_eval_backward", self.lib.gt_sinr_eval_backward(
            self._h, _ptr(C_), _ptr(G), s2, k, _ptr(gs), _ptr(gC), _ptr(gG), _ptr(status),
            _ptr(self.ws), self.ws_bytes, _stream()))
        return gC, gG

    def reconstruct_backward(self, A, B_, C_, G, grad_Ht=None, grad_Xhat=None):
        for t, what in ((A, "a"), (B_, "b"), (C_, "c"), (G, "g")):
            self._cx(t, what, what.upper())
        if grad_Ht is not None:
            grad_Ht = self._cx(grad_Ht.contiguous(), "ht", "grad_Ht")
        if grad_Xhat is not None:
            grad_Xhat = self._cx(grad_Xhat.contiguous(), "x", "grad_Xhat")
        gA, gB, gC, gG = (torch.empty_like(v) for v in (A, B_, C_, G))
        check("gt_tucker_reconstruct_backward", self.lib.gt_tucker_reconstruct_backward(
            self._h, _ptr(A), _ptr(B_), _ptr(C_), _ptr(G),
            _ptr(grad_Ht), _ptr(grad_Xhat),
            _ptr(gA), _ptr(gB), _ptr(gC), _ptr(gG), _ptr(self.ws), self.ws_bytes, _stream()))
        return gA, gB, gC, gG


# -- autograd ----------------------------------------------------------------------------

class SinrFn(torch.autograd.Function):
    """SINR of the compressed form as a differentiable function of (C, G)."""

    @staticmethod
    def forward(ctx, plan: Plan, C_, G, sigma2):
        ctx.plan = plan
        ctx.sigma2 = list(sigma2)
        ctx.save_for_backward(C_, G)
        return plan.sinr(C_.detach(), G.detach(), sigma2)

    @staticmethod
    def backward(ctx, grad):
        C_, G = ctx.saved_tensors
        gC, gG = ctx.plan.sinr_backward(C_.detach(), G.detach(), ctx.sigma2, grad)
        return None, gC, gG, None


class ReconstructFn(torch.autograd.Function):
    """(Ht, Xhat) as a differentiable function of (A, B, C, G)."""

    @staticmethod
    def forward(ctx, plan: Plan, A, B_, C_, G):
        ctx.plan = plan
        ctx.save_for_backward(A, B_, C_, G)
        Ht, Xh = plan.reconstruct(A.detach(), B_.detach(), C_.detach(), G.detach())
        return Ht, Xh

    @staticmethod
    def backward(ctx, gHt, gX):
        A, B_, C_, G = ctx.saved_tensors
        gA, gB, gC, gG = ctx.plan.reconstruct_backward(A.detach(), B_.detach(), C_.detach(),
                                                       G.detach(), gHt, gX)
        return None, gA, gB, gC, gG


# -- helpers -----------------------------------------------------------------------------

def profile_enable(on: bool = True) -> None:
    check("gt_profile_enable", load().gt_profile_enable(1 if on else 0))


def profile_reset() -> None:
    check("gt_profile_reset", load().gt_profile_reset())


def profile_query(name: str):
    ms = C.c_double()
    cnt = C.c_int64()
    check("gt_profile_query", load().gt_profile_query(name.encode(), C.byref(ms), C.byref(cnt)))
    return ms.value, cnt.value


def desc_from_config(cfg) -> dict:
    return dict(nr=cfg.nr, nt=cfg.nt, nsc=cfg.nsc, group_size=cfg.group_size, m=cfg.m, n=cfg.n,
                p=cfg.p, ns=cfg.ns)
