"""Python binding of the serving engine (include/wsserve.h): argument marshalling only.

    eng = Engine(precision="fp32", streams=4, max_batch=16, arena_bytes=8 << 30)
    t = eng.submit_apply(dict(family="log"), density)          # CPU float64 [n, n]
    t2 = eng.submit_ls(kappa=20.0, contrast=m, u_inc=f)          # CPU float64 / complex128
    out, res = eng.wait(t)
    eng.close()

Host arrays are CPU torch tensors (page-locked ones let the engine copy
asynchronously); outputs are allocated here unless given.  The engine keeps
references to a request's arrays until its result has been collected.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .api import _FAMILIES as FAMILIES, _dev_ptr

PRECISIONS = {"fp64": L.WS_FP64, "fp32": L.WS_FP32}


def _kernel(spec: dict) -> L.WsKernel:
    fam = FAMILIES[spec["family"]]
    return L.WsKernel(fam, float(spec.get("scale", 1.0)), float(spec.get("gamma", 0.0)),
                      float(spec.get("kappa", 0.0)), float(spec.get("beta", 0.0)))


def _host(t: torch.Tensor, dtype: torch.dtype, n: int, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cpu" or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous CPU {dtype} tensor")
    if tuple(t.shape) != (n, n):
        raise ValueError(f"{what} must have shape ({n}, {n})")
    return t


class Engine:
    def __init__(self, precision: str = "fp64", streams: int = 1, max_batch: int = 1, max_plans: int = 32,
                 max_skips: int = 8, arena_bytes: int = 4 << 30, device="cuda:0", pin_outputs: bool = True,
                 mix_plans: bool = False):
        self.lib = L.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.cfg = L.WsServeConfig(PRECISIONS[precision], streams, max_batch, max_plans, max_skips,
                                   1 if mix_plans else 0)
        self.precision = precision
        self.pin_outputs = pin_outputs
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            torch.cuda.synchronize()
            L.check(self.lib.serve_create(ctypes.byref(self.cfg), _dev_ptr(self.arena), arena_bytes, ctypes.byref(h)))
        self.handle = h
        self._held = {}

    def _new_out(self, n, dtype):
        return torch.empty((n, n), dtype=dtype, pin_memory=self.pin_outputs)

    def _submit(self, req: L.WsRequest, held) -> int:
        t = ctypes.c_ulonglong()
        L.check(self.lib.serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._held[t.value] = held
        return t.value

    def request_apply(self, kernel: dict, density: torch.Tensor, out: torch.Tensor | None = None):
        n = density.shape[-1]
        cplx = kernel["family"] == "helmholtz"
        dt = torch.complex128 if cplx else torch.float64
        _host(density, dt, n, "density")
        out = self._new_out(n, dt) if out is None else _host(out, dt, n, "out")
        req = L.WsRequest(L.WS_REQ_APPLY, _kernel(kernel), n, density.data_ptr(), None, out.data_ptr(), 0.0, 0, 0)
        return req, (density, out)

    def request_ls(self, kappa: float, contrast: torch.Tensor, u_inc: torch.Tensor, tol: float = 1e-8,
                   restart: int = 50, max_matvecs: int = 4000, out: torch.Tensor | None = None):
        n = u_inc.shape[-1]
        _host(u_inc, torch.complex128, n, "u_inc")
        _host(contrast, torch.float64, n, "contrast")
        out = self._new_out(n, torch.complex128) if out is None else _host(out, torch.complex128, n, "out")
        req = L.WsRequest(L.WS_REQ_LS, L.WsKernel(L.WS_HELMHOLTZ, 1.0, 0.0, float(kappa)), n, u_inc.data_ptr(),
                          contrast.data_ptr(), out.data_ptr(), float(tol), int(restart), int(max_matvecs))
        return req, (u_inc, contrast, out)

    def submit_request(self, req: L.WsRequest, held) -> int:
        """Submit a request built by request_apply or request_ls (its buffers held until it completes)."""
        return self._submit(req, held)

    def submit_apply(self, kernel: dict, density: torch.Tensor, out: torch.Tensor | None = None) -> int:
        req, held = self.request_apply(kernel, density, out)
        return self._submit(req, held)

    def submit_ls(self, kappa: float, contrast: torch.Tensor, u_inc: torch.Tensor, **kw) -> int:
        req, held = self.request_ls(kappa, contrast, u_inc, **kw)
        return self._submit(req, held)

    def footprint(self, req: L.WsRequest) -> int:
        b = ctypes.c_size_t()
        L.check(self.lib.serve_footprint(ctypes.byref(self.cfg), ctypes.byref(req), ctypes.byref(b)))
        return b.value

    def wait(self, ticket: int, timeout: float | None = None):
        """(output tensor, result dict) once the request is done; None on time-out."""
        res = L.WsResult()
        rc = self.lib.serve_wait(self.handle, ticket, -1.0 if timeout is None else float(timeout), ctypes.byref(res))
        L.check(rc)
        if rc == 0:
            return None
        held = self._held.pop(ticket)
        info = dict(status=res.status, batch=res.batch, t_submit=res.t_submit, t_start=res.t_start,
                    t_done=res.t_done)
        if len(held) == 3:
            info.update(iterations=res.ls.iterations, matvecs=res.ls.matvecs, refinements=res.ls.refinements,
                        rel_residual=res.ls.rel_residual)
        if res.status < 0:
            raise L.WsError(res.status, self.lib.conv_last_error().decode(errors="replace"))
        return held[-1], info

    def now(self) -> float:
        return self.lib.serve_now(self.handle)

    def stats(self) -> dict:
        st = L.WsServeStats()
        L.check(self.lib.serve_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in L.WsServeStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.serve_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
