"""Python binding of libwsconv: argument marshalling around the C-ABI.

PyTorch supplies device memory and the stream; every step of the method runs
in the HIP kernels of libwsconv.so.

    plan = ConvPlan("log", n=256, scale=1.0)          # moments built on the GPU
    out = plan.apply(u)                               # u: [batch, n, n] float64 on cuda
    u, info = ConvPlan("helmholtz", n=256, kappa=20).ls_solve(m, u_inc, tol=1e-8)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

_FAMILIES = {"log": L.WS_LOG, "power": L.WS_POWER, "helmholtz": L.WS_HELMHOLTZ, "yukawa": L.WS_YUKAWA}
_PRECISIONS = {"fp64": L.WS_FP64, "fp32": L.WS_FP32}


@dataclass
class FsDesc:
    """Fourier smoothing of one density (Section 2.4): shape 'disc' or 'square'."""
    shape: str
    c1: float
    c2: float
    size: float
    psi_r1: float
    psi_r2: float

    def to_c(self) -> L.WsFsDesc:
        code = {"none": L.WS_FS_NONE, "disc": L.WS_FS_DISC, "square": L.WS_FS_SQUARE}[self.shape]
        return L.WsFsDesc(code, self.c1, self.c2, self.size, self.psi_r1, self.psi_r2)


@dataclass
class LsInfo:
    status: int
    iterations: int
    matvecs: int
    refinements: int
    rel_residual: float


def _stream_ptr(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def default_support_radius(b: int) -> float:
    """Support radius a plan declares when the caller names none.

    b = 2: 0.39 about (1/2, 1/2), where every period-2 density here lives (the
    C-infinity cutoff of radius 0.4 is below 1e-23 beyond r = 0.3964, and the
    smoothing windows end at 0.39); the default a then lies in its window
    [0.39 + sqrt(2)/2, 1.5 - 0.39] (Section 2.1).  b = 3: anywhere in D (0).
    """
    return 0.39 if b == 2 else 0.0


class ConvPlan:
    """A plan for A_n with one kernel, grid and precision (conv_plan).

    support_radius: radius about (1/2, 1/2) outside which the densities vanish
    (None: default_support_radius(b)); a and the support are checked against
    the validity window of Section 2.1 unless force_a is set.
    """

    def __init__(self, family: str, n: int, b: int = 2, a: float = 0.0, scale: float = 1.0,
                 gamma: float = 0.0, kappa: float = 0.0, precision: str = "fp64",
                 support_radius: float | None = None, force_a: bool = False, device="cuda", stream=None,
                 beta: float = 0.0):
        self.lib = L.load()
        self.family = family
        self.n = n
        self.b = b
        self.precision = precision
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.kernel = L.WsKernel(_FAMILIES[family], scale, gamma, kappa, beta)
        if support_radius is None:
            support_radius = default_support_radius(b)
        self.support_radius = support_radius
        self.grid = L.WsGrid(n, b, a, support_radius, 1 if force_a else 0)
        prec = _PRECISIONS[precision]
        pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        L.check(self.lib.conv_plan_query(ctypes.byref(self.kernel), ctypes.byref(self.grid), prec,
                                         ctypes.byref(pb), ctypes.byref(wb)))
        self.plan_bytes = pb.value
        self.work_bytes = wb.value
        self.buf = torch.empty(self.plan_bytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.conv_plan(ctypes.byref(self.kernel), ctypes.byref(self.grid), prec,
                                       _dev_ptr(self.buf), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.a = self.lib.conv_plan_radius(h)
        self.chunk = L.check(self.lib.conv_apply_chunk(h))
        self._work = None

    # ------------------------------------------------------------------
    @property
    def real_dtype(self):
        return torch.float64 if self.precision == "fp64" else torch.float32

    @property
    def dtype(self):
        if self.family == "helmholtz":
            return torch.complex128 if self.precision == "fp64" else torch.complex64
        return self.real_dtype

    def workspace(self, batch: int) -> torch.Tensor:
        need = max(1, batch) * self.work_bytes
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._work

    def apply(self, density: torch.Tensor, out: torch.Tensor | None = None, fs=None, work=None,
              stream=None) -> torch.Tensor:
        """(A_n u)(x_j) for a [batch, n, n] (or [n, n]) tensor of samples (conv_apply)."""
        squeeze = density.dim() == 2
        u = density.unsqueeze(0) if squeeze else density
        if u.dtype != self.dtype or u.device != self.device or not u.is_contiguous():
            raise ValueError(f"density must be a contiguous {self.dtype} tensor on {self.device}")
        if u.shape[-2:] != (self.n, self.n):
            raise ValueError(f"density must have trailing shape ({self.n}, {self.n})")
        batch = u.shape[0]
        if out is None:
            out = torch.empty_like(u)
        elif squeeze:
            out = out.unsqueeze(0)
        w = work if work is not None else self.workspace(batch)
        fs_arr = None
        if fs is not None:
            if len(fs) != batch:
                raise ValueError("one smoothing descriptor per density")
            fs_arr = (L.WsFsDesc * batch)(*[(f.to_c() if f is not None else L.WsFsDesc(0, 0, 0, 0, 0, 0))
                                            for f in fs])
        with torch.cuda.device(self.device):
            L.check(self.lib.conv_apply(self.handle, batch, _dev_ptr(u), _dev_ptr(out), _dev_ptr(w),
                                        fs_arr, _stream_ptr(stream)))
        return out[0] if squeeze else out

    def apply_noalloc(self, density: torch.Tensor, out: torch.Tensor | None = None, fs=None,
                      stream=None) -> torch.Tensor:
        """conv_apply_noalloc: as apply, with the intermediate in the library's fixed device array
        (no workspace; allocates nothing beyond `out` when out is None)."""
        squeeze = density.dim() == 2
        u = density.unsqueeze(0) if squeeze else density
        if u.dtype != self.dtype or u.device != self.device or not u.is_contiguous():
            raise ValueError(f"density must be a contiguous {self.dtype} tensor on {self.device}")
        if u.shape[-2:] != (self.n, self.n):
            raise ValueError(f"density must have trailing shape ({self.n}, {self.n})")
        batch = u.shape[0]
        if out is None:
            out = torch.empty_like(u)
        elif squeeze:
            out = out.unsqueeze(0)
        fs_arr = None
        if fs is not None:
            if len(fs) != batch:
                raise ValueError("one smoothing descriptor per density")
            fs_arr = (L.WsFsDesc * batch)(*[(f.to_c() if f is not None else L.WsFsDesc(0, 0, 0, 0, 0, 0))
                                            for f in fs])
        with torch.cuda.device(self.device):
            L.check(self.lib.conv_apply_noalloc(self.handle, batch, _dev_ptr(u), _dev_ptr(out), fs_arr,
                                                _stream_ptr(stream)))
        return out[0] if squeeze else out

    def apply_pass(self, pass_index: int, density: torch.Tensor, out: torch.Tensor, work: torch.Tensor,
                   stream=None) -> None:
        """Enqueue one pass of the apply (conv_apply_pass); no argument copies, no checks beyond the C side."""
        with torch.cuda.device(self.device):
            L.check(self.lib.conv_apply_pass(self.handle, pass_index, density.shape[0], _dev_ptr(density),
                                             _dev_ptr(out), _dev_ptr(work), _stream_ptr(stream)))

    def eval(self, density: torch.Tensor, targets: torch.Tensor, out: torch.Tensor | None = None,
             work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """(A_n u)(x) at arbitrary points (conv_eval): targets is a [count, 2] float64 tensor of
        (x1, x2); returns a complex128 [count] tensor."""
        if density.dtype != self.dtype or density.device != self.device or not density.is_contiguous() \
                or density.shape != (self.n, self.n):
            raise ValueError(f"density must be a contiguous ({self.n}, {self.n}) {self.dtype} tensor on {self.device}")
        if targets.dtype != torch.float64 or targets.device != self.device or not targets.is_contiguous() \
                or targets.dim() != 2 or targets.shape[1] != 2:
            raise ValueError("targets must be a contiguous [count, 2] float64 tensor on the plan's device")
        count = targets.shape[0]
        res = out if out is not None else torch.empty(count, dtype=torch.complex128, device=self.device)
        if work is None:
            nbytes = ctypes.c_size_t()
            L.check(self.lib.conv_eval_query(self.handle, ctypes.byref(nbytes)))
            work = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            L.check(self.lib.conv_eval(self.handle, _dev_ptr(density), count, _dev_ptr(targets), _dev_ptr(res),
                                       _dev_ptr(work), _stream_ptr(stream)))
        return res

    def ls_workspace(self, restart: int, mixed: bool, fs: "FsDesc | None" = None) -> torch.Tensor:
        nbytes = ctypes.c_size_t()
        if fs is None:
            L.check(self.lib.ls_solve_query(self.handle, restart, int(mixed), ctypes.byref(nbytes)))
        else:
            d = fs.to_c()
            L.check(self.lib.ls_solve_fs_query(self.handle, ctypes.byref(d), restart, int(mixed),
                                               ctypes.byref(nbytes)))
        return torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)

    def ls_solve(self, contrast: torch.Tensor, u_inc: torch.Tensor, tol: float = 1e-8, restart: int = 50,
                 max_matvecs: int = 5000, mixed: bool = False, out: torch.Tensor | None = None,
                 work: torch.Tensor | None = None, stream=None, fs: "FsDesc | None" = None):
        """Solve u + kappa^2 A_n(m u) = u_inc (ls_solve); returns (u, LsInfo).

        With fs (a disc or square Omega and the window psi), `contrast` is a
        smooth extension m_tilde of a contrast that jumps across the boundary of
        Omega, and the operator uses m_tilde chi^n psi (ls_solve_fs)."""
        if contrast.dtype != torch.float64 or u_inc.dtype != torch.complex128:
            raise ValueError("contrast must be float64 and u_inc complex128")
        for t in (contrast, u_inc):
            if t.device != self.device or not t.is_contiguous() or t.shape != (self.n, self.n):
                raise ValueError(f"inputs must be contiguous ({self.n}, {self.n}) tensors on {self.device}")
        u = out if out is not None else torch.empty_like(u_inc)
        w = work if work is not None else self.ls_workspace(restart, mixed, fs)
        info = L.WsLsInfo()
        with torch.cuda.device(self.device):
            if fs is None:
                L.check(self.lib.ls_solve(self.handle, _dev_ptr(contrast), _dev_ptr(u_inc), tol, restart,
                                          max_matvecs, int(mixed), _dev_ptr(u), _dev_ptr(w), ctypes.byref(info),
                                          _stream_ptr(stream)))
            else:
                d = fs.to_c()
                L.check(self.lib.ls_solve_fs(self.handle, _dev_ptr(contrast), ctypes.byref(d), _dev_ptr(u_inc),
                                             tol, restart, max_matvecs, int(mixed), _dev_ptr(u), _dev_ptr(w),
                                             ctypes.byref(info), _stream_ptr(stream)))
        return u, LsInfo(info.status, info.iterations, info.matvecs, info.refinements, info.rel_residual)

    def ls_batch_workspace(self, count: int, restart: int = 50, mixed: bool = False) -> torch.Tensor:
        nb = ctypes.c_size_t()
        L.check(self.lib.ls_solve_batch_query(self.handle, count, restart, int(mixed), ctypes.byref(nb)))
        return torch.empty(nb.value, dtype=torch.uint8, device=self.device)

    def ls_solve_batch(self, contrast: torch.Tensor, u_inc: torch.Tensor, tol: float = 1e-8, restart: int = 50,
                       max_matvecs: int = 5000, mixed: bool = False, out: torch.Tensor | None = None,
                       work: torch.Tensor | None = None, stream=None):
        """Several solves with this plan at once (ls_solve_batch): contrast [count, n, n] float64,
        u_inc [count, n, n] complex128; returns (u [count, n, n], [LsInfo] * count)."""
        if contrast.dtype != torch.float64 or u_inc.dtype != torch.complex128:
            raise ValueError("contrast must be float64 and u_inc complex128")
        count = u_inc.shape[0]
        for t in (contrast, u_inc):
            if t.device != self.device or not t.is_contiguous() or t.shape != (count, self.n, self.n):
                raise ValueError(f"inputs must be contiguous ({count}, {self.n}, {self.n}) tensors on {self.device}")
        u = out if out is not None else torch.empty_like(u_inc)
        w = work if work is not None else self.ls_batch_workspace(count, restart, mixed)
        infos = (L.WsLsInfo * count)()
        with torch.cuda.device(self.device):
            L.check(self.lib.ls_solve_batch(self.handle, count, _dev_ptr(contrast), _dev_ptr(u_inc), tol, restart,
                                            max_matvecs, int(mixed), _dev_ptr(u), _dev_ptr(w), infos,
                                            _stream_ptr(stream)))
        return u, [LsInfo(i.status, i.iterations, i.matvecs, i.refinements, i.rel_residual) for i in infos]

    def moments(self, k1, k2):
        """Moments ghat(k) at integer frequencies (conv_plan_moments); complex numpy array."""
        import numpy as np
        k1 = np.asarray(k1, dtype=np.int32).ravel()
        k2 = np.asarray(k2, dtype=np.int32).ravel()
        out = np.zeros(2 * len(k1), dtype=np.float64)
        L.check(self.lib.conv_plan_moments(
            self.handle, len(k1), k1.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            k2.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(None)))
        return out[0::2] + 1j * out[1::2]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.conv_destroy(h)
            self.handle = None


def apply_multi(plans, densities, outs=None, stream=None):
    """conv_apply_multi: item i applies plans[i] to densities[i] ([batch_i, n_i, n_i] on the device).

    Densities of different sizes and kernels share each pass's launch.  Returns the outputs
    (allocated here unless given)."""
    if len(plans) != len(densities):
        raise ValueError("one density tensor per plan")
    count = len(plans)
    if count == 0:
        return []
    lib = plans[0].lib
    dev = plans[0].device
    us, os_, ws = [], [], []
    for i, (p, d) in enumerate(zip(plans, densities)):
        u = d.unsqueeze(0) if d.dim() == 2 else d
        if u.dtype != p.dtype or u.device != p.device or not u.is_contiguous() or u.shape[-2:] != (p.n, p.n):
            raise ValueError(f"density {i} must be a contiguous {p.dtype} [batch, {p.n}, {p.n}] tensor on {p.device}")
        o = torch.empty_like(u) if outs is None else (outs[i].unsqueeze(0) if outs[i].dim() == 2 else outs[i])
        us.append(u)
        os_.append(o)
        # one work buffer per item (items must not share scratch)
        ws.append(torch.empty(max(1, min(u.shape[0], p.chunk)) * p.work_bytes, dtype=torch.uint8, device=dev))
    arr = lambda xs: (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
    handles = (ctypes.c_void_p * count)(*[p.handle.value for p in plans])
    batches = (ctypes.c_int * count)(*[u.shape[0] for u in us])
    with torch.cuda.device(dev):
        L.check(lib.conv_apply_multi(count, handles, batches, arr(us), arr(os_), arr(ws), _stream_ptr(stream)))
    return [o[0] if d.dim() == 2 else o for o, d in zip(os_, densities)]
