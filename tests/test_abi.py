"""The C-ABI library loads, exports every declared entry point, and rejects bad
arguments on the host (no GPU needed: none of these calls reaches the device)."""
import ctypes
import os
import re

import pytest

from paper_2107_03958_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2107_03958_amd import build
        build.build(jobs=8)
    return L.load()


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:int|void|double|const char\*)\s+(\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"conv_plan", "conv_apply", "ls_solve", "conv_destroy", "conv_last_error"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS), "binding and header disagree"


def _query(lib, family=L.WS_LOG, n=64, b=2, a=0.0, gamma=0.0, kappa=0.0, prec=L.WS_FP64, rho=None, force=0):
    k = L.WsKernel(family, 1.0, gamma, kappa)
    g = L.WsGrid(n, b, a, (0.39 if b == 2 else 0.0) if rho is None else rho, force)
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib.conv_plan_query(ctypes.byref(k), ctypes.byref(g), prec, ctypes.byref(pb), ctypes.byref(wb))
    return rc, pb.value, wb.value


def test_plan_query_sizes(lib):
    rc, pb, wb = _query(lib, n=2048)
    assert rc == L.WS_OK
    assert wb == 2048 * 2048 * 16                    # half spectrum, complex128
    assert pb >= 2048 * 2049 * 8                     # FP64 moment table
    rc, pb32, wb32 = _query(lib, n=2048, prec=L.WS_FP32)
    assert rc == 0 and wb32 == wb // 2 and pb32 > pb
    rc, pbh, wbh = _query(lib, family=L.WS_HELMHOLTZ, kappa=20.0, n=1024)
    assert rc == 0 and wbh == 1024 * 2048 * 16


def test_plan_query_sizes_period3(lib):
    # b = 3: nb = 3n; real half spectrum n x 3n/2, complex n x 3n; moment
    # tables of (3n/2 + 1) folded rows per intermediate column
    rc, pb, wb = _query(lib, n=1024, b=3)
    assert rc == L.WS_OK and wb == 1024 * 1536 * 16
    assert pb >= 1537 * 1536 * 8 + 1537 * 8 + 3072 * 16
    rc, pbh, wbh = _query(lib, family=L.WS_HELMHOLTZ, kappa=20.0, n=512, b=3)
    assert rc == L.WS_OK and wbh == 512 * 1536 * 16
    assert pbh >= 769 * 1536 * 16
    rc, pb, wb = _query(lib, n=2048, b=3)
    assert rc == L.WS_OK and wb == 2048 * 3072 * 16


@pytest.mark.parametrize("kw,code", [
    (dict(n=100), L.WS_EUNSUPPORTED),
    (dict(n=8), L.WS_EUNSUPPORTED),
    (dict(n=4096), L.WS_EUNSUPPORTED),
    (dict(b=4), L.WS_EUNSUPPORTED),
    (dict(b=0), L.WS_EINVAL),
    (dict(a=2.5), L.WS_EINVAL),
    (dict(family=L.WS_POWER, gamma=0.5), L.WS_EINVAL),
    (dict(family=L.WS_POWER, gamma=-2.0), L.WS_EINVAL),
    (dict(family=L.WS_HELMHOLTZ, kappa=0.0), L.WS_EINVAL),
    (dict(family=7), L.WS_EINVAL),
    (dict(prec=5), L.WS_EINVAL),
])
def test_plan_query_rejects(lib, kw, code):
    rc, _, _ = _query(lib, **kw)
    assert rc == code
    assert lib.conv_last_error().decode()


def test_null_handles_rejected(lib):
    assert lib.conv_apply(None, 1, None, None, None, None, None) == L.WS_EINVAL
    assert b"plan" in lib.conv_last_error()
    nb = ctypes.c_size_t()
    assert lib.ls_solve_query(None, 50, 0, ctypes.byref(nb)) == L.WS_EINVAL
    info = L.WsLsInfo()
    assert lib.ls_solve(None, None, None, 1e-8, 50, 100, 0, None, None, ctypes.byref(info), None) == L.WS_EINVAL
    h = ctypes.c_void_p()
    k = L.WsKernel(L.WS_LOG, 1.0, 0.0, 0.0)
    g = L.WsGrid(64, 2, 0.0, 0.39, 0)
    assert lib.conv_plan(ctypes.byref(k), ctypes.byref(g), L.WS_FP64, None, None, ctypes.byref(h)) == L.WS_EINVAL
    assert lib.conv_plan_radius(None) == 0.0
    lib.conv_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(ImportError):
        L._lib_backup = L._lib
        try:
            L._lib = None
            L.load(str(tmp_path / "missing.so"))
        finally:
            L._lib = L._lib_backup


@pytest.mark.parametrize("precision", [L.WS_FP64, L.WS_FP32])
def test_serve_footprint_covers_ls_workspace(lib, precision):
    # serve_footprint is host-only.  An LS request's device footprint must hold
    # its Krylov basis (restart + 1 vectors), the residual and work vectors and
    # the apply intermediate of its matvec (n x 2n complex at period 2).
    n, restart = 256, 50
    cfg = L.WsServeConfig(precision, 1, 1, 4, 4, 0)
    buf = ctypes.c_int(0)   # any non-NULL host address: only the pointers' presence is checked
    req = L.WsRequest(L.WS_REQ_LS, L.WsKernel(L.WS_HELMHOLTZ, 1.0, 0.0, 20.0), n,
                      ctypes.addressof(buf), ctypes.addressof(buf), ctypes.addressof(buf), 1e-8, restart, 1000)
    fp = ctypes.c_size_t()
    assert lib.serve_footprint(ctypes.byref(cfg), ctypes.byref(req), ctypes.byref(fp)) == L.WS_OK
    rc, plan_bytes, _ = _query(lib, family=L.WS_HELMHOLTZ, kappa=20.0, n=n, prec=precision)
    assert rc == L.WS_OK
    esz = 16 if precision == L.WS_FP64 else 8
    N = n * n
    own = N * 8 + 2 * N * 16                         # contrast, incident field, solution (staged)
    krylov = (restart + 3) * N * esz                 # V (restart + 1), r, t
    apply_work = n * 2 * n * esz                     # the matvec's intermediate
    assert fp.value - plan_bytes - own >= krylov + apply_work


def test_truncation_radius_window(lib):
    # Section 2.1: a must cover every target-to-support distance and stay short of the
    # periodic images.  Disc support rho about the centre: [rho + sqrt(2)/2, b - 1/2 - rho];
    # support anywhere in D: [sqrt(2), b - 1].
    import math
    ok, bad = L.WS_OK, L.WS_EINVAL
    assert _query(lib, b=2, rho=0.39)[0] == ok                       # default a = 1.1036 in [1.0971, 1.11]
    assert _query(lib, b=2, rho=0.4)[0] == bad                       # [1.1071, 1.1] is empty
    assert _query(lib, b=2, rho=0.0)[0] == bad                       # [sqrt 2, 1] is empty at b = 2
    assert _query(lib, b=2, rho=0.0, force=1)[0] == ok               # forced
    assert _query(lib, b=2, rho=0.2, a=0.3)[0] == bad                # a below rho + sqrt(2)/2
    assert _query(lib, b=2, rho=0.2, a=0.3, force=1)[0] == ok
    assert _query(lib, b=2, rho=0.2, a=0.2 + math.sqrt(2) / 2)[0] == ok   # window ends are valid
    assert _query(lib, b=2, rho=0.2, a=1.3)[0] == ok
    assert _query(lib, b=2, rho=0.2, a=1.31)[0] == bad               # beyond b - 1/2 - rho
    assert _query(lib, b=3, rho=0.0)[0] == ok                        # default 1.6036 in [sqrt 2, 2]
    assert _query(lib, b=3, rho=0.0, a=1.4)[0] == bad
    assert _query(lib, b=3, rho=0.0, a=2.05)[0] == bad
    assert _query(lib, b=3, rho=0.0, a=2.0)[0] == ok
    assert _query(lib, b=2, rho=0.8)[0] == bad                       # rho >= sqrt(2)/2: not a disc in D
    assert _query(lib, b=2, a=2.5, force=1)[0] == bad                # 0 < a < b always
    rc = _query(lib, b=2, rho=0.2, a=0.3)[0]
    assert "validity window" in lib.conv_last_error().decode()
