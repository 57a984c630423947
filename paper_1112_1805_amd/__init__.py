"""Python binding of the MI355X shearlet-segmentation library (libshearseg.so).

Argument marshalling only: every function forwards to the C entry point of the same
name declared in include/shearseg.h.  Device arrays are torch tensors on the plan's GPU
(their data_ptr() is passed); the stream is torch's current stream.  No computation of
the method happens in Python, and there is no CPU fallback: if the HIP library is not
built, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SHEARSEG_LIB") or os.path.join(_HERE, "libshearseg.so")

SHS_OK, SHS_E_INVALID, SHS_E_UNSUPPORTED, SHS_E_NOMEM, SHS_E_DEVICE, SHS_E_NUMERIC, SHS_E_WORKSPACE = \
    0, -1, -2, -3, -4, -5, -6
SHS_STORE_F32, SHS_STORE_BF16, SHS_STORE_F16 = 0, 1, 2
SHS_NOALLOC_MAX_BYTES = 64 << 20   # include/shearseg.h
STORE_CODES = {"f32": SHS_STORE_F32, "bf16": SHS_STORE_BF16, "f16": SHS_STORE_F16}


class ShsShape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("channels", ctypes.c_int32), ("q", ctypes.c_int32),
                ("J", ctypes.c_int32), ("store", ctypes.c_int32)]


class ShsParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.POINTER(ctypes.c_float)), ("lambda_len", ctypes.c_int32),
                ("gamma", ctypes.c_float), ("iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("resume", ctypes.c_int32)]


class ShsPdParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.POINTER(ctypes.c_float)), ("lambda_len", ctypes.c_int32),
                ("tau", ctypes.c_float), ("sigma", ctypes.c_float), ("iters", ctypes.c_int32)]


class ShsNlGraphParams(ctypes.Structure):
    _fields_ = [("patch", ctypes.c_int32), ("window", ctypes.c_int32), ("a", ctypes.c_float),
                ("m", ctypes.c_int32)]


class ShsNlParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_float), ("tau", ctypes.c_float), ("sigma", ctypes.c_float),
                ("iters", ctypes.c_int32), ("blocks", ctypes.c_int32), ("max_degree", ctypes.c_int32)]


class ShsStats(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int32), ("energy", ctypes.c_double),
                ("energy_surrogate", ctypes.c_double), ("r_primal", ctypes.c_double),
                ("r_dual", ctypes.c_double), ("r_combined", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ShsKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class ShsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None
_VP, _SZ, _I32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
_SIGS = {
    "shs_plan_create": (_I32, [ctypes.POINTER(ShsShape), ctypes.c_int, ctypes.POINTER(_VP)]),
    "shs_plan_destroy": (_I32, [_VP]),
    "shs_workspace_bytes": (_SZ, [_VP]),
    "shs_state_bytes": (_SZ, [_VP]),
    "shs_plan_describe": (ctypes.c_char_p, [_VP]),
    "shs_num_filters": (_I32, [_I32]),
    "shs_filters": (_I32, [_VP, _VP, _VP]),
    "shs_datacost": (_I32, [_VP, _VP, ctypes.POINTER(ctypes.c_float), ctypes.c_float, _VP, _VP]),
    "shs_shearlet_forward": (_I32, [_VP, _I32, _VP, _VP, _VP, _SZ, _VP]),
    "shs_shearlet_adjoint": (_I32, [_VP, _I32, _VP, _VP, _VP, _SZ, _VP]),
    "shs_shearlet_denoise": (_I32, [_VP, _I32, ctypes.POINTER(ctypes.c_float), _I32, _VP, _VP, _VP, _SZ, _VP]),
    "shs_solve": (_I32, [_VP, ctypes.POINTER(ShsParams), _VP, _VP, _SZ, _VP, _VP, _VP,
                         ctypes.POINTER(ShsStats), _VP]),
    "shs_solve_noalloc": (_I32, [_VP, ctypes.POINTER(ShsParams), _VP, _VP, _VP, _VP,
                                 ctypes.POINTER(ShsStats), _VP]),
    "shs_solve_pd": (_I32, [_VP, ctypes.POINTER(ShsPdParams), _VP, _VP, _SZ, _VP, _VP, _VP,
                            ctypes.POINTER(ShsStats), _VP]),
    "shs_solve_tv": (_I32, [_VP, ctypes.POINTER(ShsParams), _VP, _VP, _SZ, _VP, _VP, _VP,
                            ctypes.POINTER(ShsStats), _VP]),
    "shs_nl_graph": (_I32, [_I32, _I32, _VP, ctypes.POINTER(ShsNlGraphParams), _VP, _VP,
                            ctypes.POINTER(ctypes.c_int32)]),
    "shs_solve_nl": (_I32, [_VP, ctypes.POINTER(ShsNlParams), _VP, _VP, _VP, _VP, _SZ, _VP, _VP, _VP,
                            ctypes.POINTER(ShsStats), _VP]),
    "shs_energy": (_I32, [_VP, ctypes.POINTER(ShsParams), _VP, _VP, _VP, _SZ,
                          ctypes.POINTER(ctypes.c_double), _VP]),
    "shs_batch_create": (_I32, [_I32, ctypes.POINTER(ShsShape), ctypes.c_int, ctypes.POINTER(_VP)]),
    "shs_batch_destroy": (_I32, [_VP]),
    "shs_batch_workspace_bytes": (_SZ, [_VP]),
    "shs_solve_batch": (_I32, [_VP, ctypes.POINTER(ShsParams), ctypes.POINTER(_VP), _VP, _SZ,
                               ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP, _VP]),
    "shs_profile_begin": (_I32, []),
    "shs_profile_begin_classes": (_I32, [ctypes.c_char_p]),
    "shs_profile_end": (_I32, [ctypes.POINTER(ShsKernelTime), _I32]),
    "shs_status_str": (ctypes.c_char_p, [_I32]),
    "shs_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libshearseg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1112_1805_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != SHS_OK:
        raise ShsError(status, where, lib().shs_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _expect(t, shape, dtype_name, what):
    import torch
    dt = {"f32": torch.float32, "f64": torch.float64, "i32": torch.int32}[dtype_name]
    if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: need a contiguous {dtype_name} CUDA tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)} cuda={t.is_cuda} contiguous={t.is_contiguous()}")


def _params(lam, gamma, iters, tol=0.0, check_every=1, resume=False):
    arr = np.ascontiguousarray(np.asarray(lam, dtype=np.float32).ravel())
    p = ShsParams()
    p.lambda_ = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    p.lambda_len = arr.size
    p.gamma = float(gamma)
    p.iters = int(iters)
    p.tol = float(tol)
    p.check_every = int(check_every)
    p.resume = 1 if resume else 0
    return p, arr   # keep `arr` alive while p is used


# --------------------------------------------------------------------------- C names
def nl_graph(img, patch: int = 5, window: int = 15, a: float = 2.0, m: int = 5):
    """shs_nl_graph on a host image [C][N][N]: (nbr, rev) int32 [2m][N][N] and the largest degree."""
    img = np.ascontiguousarray(np.asarray(img, dtype=np.float32))
    if img.ndim == 2:
        img = img[None]
    C, n, _ = img.shape
    nbr = np.empty((2 * m, n, n), dtype=np.int32)
    rev = np.empty((2 * m, n, n), dtype=np.int32)
    md = ctypes.c_int32(0)
    prm = ShsNlGraphParams(patch, window, a, m)
    _check(lib().shs_nl_graph(n, C, img.ctypes.data, ctypes.byref(prm), nbr.ctypes.data, rev.ctypes.data,
                              ctypes.byref(md)), "shs_nl_graph")
    return nbr, rev, int(md.value)


def shs_num_filters(J: int) -> int:
    return lib().shs_num_filters(J)


def shs_profile_begin(classes=None) -> None:
    """Time every library kernel launch (classes=None) or only the named kernel classes
    (an iterable of names such as "row_solve", or one comma-separated string)."""
    if classes is None:
        _check(lib().shs_profile_begin(), "shs_profile_begin")
    else:
        csv = classes if isinstance(classes, str) else ",".join(classes)
        _check(lib().shs_profile_begin_classes(csv.encode()), "shs_profile_begin_classes")


def shs_profile_end() -> dict:
    """{kernel class: (launches, total event-measured ms)} since shs_profile_begin()."""
    buf = (ShsKernelTime * 32)()
    k = lib().shs_profile_end(buf, 32)
    if k < 0:
        raise ShsError(-4, "shs_profile_end", lib().shs_last_error().decode())
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(k)}


def shs_plan_create(n: int, channels: int, q: int, J: int, store: str = "f32", device: int = 0) -> "Plan":
    return Plan(n, channels, q, J, store, device)


class Plan:
    """Owns an shs_plan* (filter bank and twiddles on the device)."""

    def __init__(self, n, channels, q, J, store="f32", device=0):
        shape = ShsShape(n, channels, q, J, STORE_CODES[store] if isinstance(store, str) else int(store))
        h = _VP()
        _check(lib().shs_plan_create(ctypes.byref(shape), device, ctypes.byref(h)), "shs_plan_create")
        self.handle = h
        self.n, self.channels, self.q, self.J, self.store, self.device = n, channels, q, J, store, device
        self.eta = lib().shs_num_filters(J)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.shs_plan_destroy(h)
            self.handle = None

    # -- sizes
    def workspace_bytes(self) -> int:
        return int(lib().shs_workspace_bytes(self.handle))

    def state_bytes(self) -> int:
        return int(lib().shs_state_bytes(self.handle))

    def describe(self) -> str:
        """shs_plan_describe: the plan's launch schedule."""
        return lib().shs_plan_describe(self.handle).decode()

    def new_workspace(self):
        import torch
        nb = self.workspace_bytes()
        return torch.empty((nb + 255) // 256 * 256, dtype=torch.uint8, device=f"cuda:{self.device}")

    # -- entry points (same names as the C ABI, without the shs_ prefix)
    def filters(self, out, stream=None):
        _expect(out, (self.eta, self.n, self.n // 2 + 1), "f32", "d_psi")
        _check(lib().shs_filters(self.handle, _ptr(out), _stream(stream)), "shs_filters")
        return out

    def datacost(self, img, codebook, out, p: float = 2.0, stream=None):
        _expect(img, (self.channels, self.n, self.n), "f32", "d_img")
        _expect(out, (self.q, self.n, self.n), "f32", "d_s")
        cb = np.ascontiguousarray(np.asarray(codebook, dtype=np.float32).reshape(self.q, self.channels))
        _check(lib().shs_datacost(self.handle, _ptr(img), cb.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  float(p), _ptr(out), _stream(stream)), "shs_datacost")
        return out

    def shearlet_forward(self, f, c, ws, stream=None):
        count = f.shape[0]
        _expect(f, (count, self.n, self.n), "f32", "d_f")
        _expect(c, (count, self.eta, self.n, self.n), "f32", "d_c")
        _check(lib().shs_shearlet_forward(self.handle, count, _ptr(f), _ptr(c), _ptr(ws), ws.numel(),
                                          _stream(stream)), "shs_shearlet_forward")
        return c

    def shearlet_adjoint(self, c, f, ws, stream=None):
        count = c.shape[0]
        _expect(c, (count, self.eta, self.n, self.n), "f32", "d_c")
        _expect(f, (count, self.n, self.n), "f32", "d_f")
        _check(lib().shs_shearlet_adjoint(self.handle, count, _ptr(c), _ptr(f), _ptr(ws), ws.numel(),
                                          _stream(stream)), "shs_shearlet_adjoint")
        return f

    def shearlet_denoise(self, f, lam, ws, out=None, stream=None):
        """S^T S_lambda S f (shs_shearlet_denoise); `lam` per scale (J+1) or per filter (eta)."""
        count = f.shape[0]
        _expect(f, (count, self.n, self.n), "f32", "d_f")
        if out is None:
            import torch
            out = torch.empty_like(f)
        _expect(out, (count, self.n, self.n), "f32", "d_out")
        arr = np.ascontiguousarray(np.asarray(lam, dtype=np.float32).ravel())
        _check(lib().shs_shearlet_denoise(self.handle, count, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          arr.size, _ptr(f), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
               "shs_shearlet_denoise")
        return out

    def solve(self, s, ws, lam, gamma, iters, u=None, labels=None, hist=None, want_stats=True,
              tol=0.0, check_every=1, resume=False, stream=None):
        _expect(s, (self.q, self.n, self.n), "f32", "d_s")
        if u is not None:
            _expect(u, (self.q, self.n, self.n), "f32", "d_u")
        if labels is not None:
            _expect(labels, (self.n, self.n), "i32", "d_labels")
        if hist is not None:
            _expect(hist, (iters, 4), "f64", "d_hist")
        prm, keep = _params(lam, gamma, iters, tol, check_every, resume)
        st = ShsStats()
        _check(lib().shs_solve(self.handle, ctypes.byref(prm), _ptr(s), _ptr(ws), ws.numel(), _ptr(u),
                               _ptr(labels), _ptr(hist), ctypes.byref(st) if want_stats else None,
                               _stream(stream)), "shs_solve")
        del keep
        return st.as_dict() if want_stats else None

    def solve_noalloc(self, s, lam, gamma, iters, u=None, labels=None, hist=None, want_stats=True,
                      tol=0.0, check_every=1, resume=False, stream=None):
        """shs_solve_noalloc: solve() with the library's per-GPU device array as workspace."""
        _expect(s, (self.q, self.n, self.n), "f32", "d_s")
        if u is not None:
            _expect(u, (self.q, self.n, self.n), "f32", "d_u")
        if labels is not None:
            _expect(labels, (self.n, self.n), "i32", "d_labels")
        if hist is not None:
            _expect(hist, (iters, 4), "f64", "d_hist")
        prm, keep = _params(lam, gamma, iters, tol, check_every, resume)
        st = ShsStats()
        _check(lib().shs_solve_noalloc(self.handle, ctypes.byref(prm), _ptr(s), _ptr(u), _ptr(labels), _ptr(hist),
                                       ctypes.byref(st) if want_stats else None, _stream(stream)),
               "shs_solve_noalloc")
        del keep
        return st.as_dict() if want_stats else None

    def solve_pd(self, s, ws, lam, tau, sigma, iters, u=None, labels=None, hist=None, want_stats=True,
                 stream=None):
        """Primal-dual solver (shs_solve_pd); same outputs as solve()."""
        _expect(s, (self.q, self.n, self.n), "f32", "d_s")
        if u is not None:
            _expect(u, (self.q, self.n, self.n), "f32", "d_u")
        if labels is not None:
            _expect(labels, (self.n, self.n), "i32", "d_labels")
        if hist is not None:
            _expect(hist, (iters, 4), "f64", "d_hist")
        arr = np.ascontiguousarray(np.asarray(lam, dtype=np.float32).ravel())
        prm = ShsPdParams()
        prm.lambda_ = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        prm.lambda_len = arr.size
        prm.tau = float(tau)
        prm.sigma = float(sigma)
        prm.iters = int(iters)
        st = ShsStats()
        _check(lib().shs_solve_pd(self.handle, ctypes.byref(prm), _ptr(s), _ptr(ws), ws.numel(), _ptr(u),
                                  _ptr(labels), _ptr(hist), ctypes.byref(st) if want_stats else None,
                                  _stream(stream)), "shs_solve_pd")
        del arr
        return st.as_dict() if want_stats else None

    def solve_tv(self, s, ws, lam, gamma, iters, u=None, labels=None, hist=None, want_stats=True, tol=0.0,
                 check_every=1, stream=None):
        """TV comparison model (shs_solve_tv): `lam` is the single TV weight."""
        _expect(s, (self.q, self.n, self.n), "f32", "d_s")
        if u is not None:
            _expect(u, (self.q, self.n, self.n), "f32", "d_u")
        if labels is not None:
            _expect(labels, (self.n, self.n), "i32", "d_labels")
        if hist is not None:
            _expect(hist, (iters, 4), "f64", "d_hist")
        prm, keep = _params([lam], gamma, iters, tol, check_every, False)
        st = ShsStats()
        _check(lib().shs_solve_tv(self.handle, ctypes.byref(prm), _ptr(s), _ptr(ws), ws.numel(), _ptr(u),
                                  _ptr(labels), _ptr(hist), ctypes.byref(st) if want_stats else None,
                                  _stream(stream)), "shs_solve_tv")
        del keep
        return st.as_dict() if want_stats else None

    def solve_nl(self, s, nbr, rev, ws, lam, tau, sigma, iters, max_degree, u=None, labels=None, hist=None,
                 want_stats=True, stream=None):
        """NL model (shs_solve_nl); nbr, rev: device int32 [blocks][N][N] from nl_graph()."""
        _expect(s, (self.q, self.n, self.n), "f32", "d_s")
        blocks = nbr.shape[0]
        _expect(nbr, (blocks, self.n, self.n), "i32", "d_nbr")
        _expect(rev, (blocks, self.n, self.n), "i32", "d_rev")
        if u is not None:
            _expect(u, (self.q, self.n, self.n), "f32", "d_u")
        if labels is not None:
            _expect(labels, (self.n, self.n), "i32", "d_labels")
        if hist is not None:
            _expect(hist, (iters, 4), "f64", "d_hist")
        prm = ShsNlParams(float(lam), float(tau), float(sigma), int(iters), int(blocks), int(max_degree))
        st = ShsStats()
        _check(lib().shs_solve_nl(self.handle, ctypes.byref(prm), _ptr(s), _ptr(nbr), _ptr(rev), _ptr(ws),
                                  ws.numel(), _ptr(u), _ptr(labels), _ptr(hist),
                                  ctypes.byref(st) if want_stats else None, _stream(stream)), "shs_solve_nl")
        return st.as_dict() if want_stats else None

    def energy(self, s, u, ws, lam, stream=None) -> float:
        _expect(s, (self.q, self.n, self.n), "f32", "d_s")
        _expect(u, (self.q, self.n, self.n), "f32", "d_u")
        prm, keep = _params(lam, 1.0, 0)
        e = ctypes.c_double()
        _check(lib().shs_energy(self.handle, ctypes.byref(prm), _ptr(s), _ptr(u), _ptr(ws), ws.numel(),
                                ctypes.byref(e), _stream(stream)), "shs_energy")
        del keep
        return float(e.value)


class Batch:
    """Owns an shs_batch* : `count` images of different sizes / label counts solved together."""

    def __init__(self, shapes, device=0):
        """shapes: sequence of (n, channels, q, J, store)."""
        arr = (ShsShape * len(shapes))(*[ShsShape(n, C, q, J, STORE_CODES[st] if isinstance(st, str) else int(st))
                                          for n, C, q, J, st in shapes])
        h = _VP()
        _check(lib().shs_batch_create(len(shapes), arr, device, ctypes.byref(h)), "shs_batch_create")
        self.handle = h
        self.shapes = [tuple(x) for x in shapes]
        self.count = len(shapes)
        self.device = device

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.shs_batch_destroy(h)
            self.handle = None

    def workspace_bytes(self) -> int:
        return int(lib().shs_batch_workspace_bytes(self.handle))

    def new_workspace(self):
        import torch
        nb = self.workspace_bytes()
        return torch.empty((nb + 255) // 256 * 256, dtype=torch.uint8, device=f"cuda:{self.device}")

    def solve(self, s_list, ws, lams, gammas, iters, u_list=None, labels_list=None, stats=None, stream=None):
        """shs_solve_batch.  s_list/u_list/labels_list: one device tensor per image; stats: None or
        a float64 device tensor [count][5]."""
        n = self.count
        for i, (nn, C, q, J, st) in enumerate(self.shapes):
            _expect(s_list[i], (q, nn, nn), "f32", f"d_s[{i}]")
            if u_list is not None:
                _expect(u_list[i], (q, nn, nn), "f32", f"d_u[{i}]")
            if labels_list is not None:
                _expect(labels_list[i], (nn, nn), "i32", f"d_labels[{i}]")
        if stats is not None:
            _expect(stats, (n, 5), "f64", "d_stats")
        prm = (ShsParams * n)()
        keep = []
        for i in range(n):
            p_i, arr = _params(lams[i], gammas[i], iters)
            prm[i] = p_i
            keep.append(arr)
        ptrs = lambda ts: (_VP * n)(*[t.data_ptr() for t in ts]) if ts is not None else None
        _check(lib().shs_solve_batch(self.handle, prm, ptrs(s_list), _ptr(ws), ws.numel(), ptrs(u_list),
                                     ptrs(labels_list), _ptr(stats), _stream(stream)), "shs_solve_batch")
        del keep


def segment(img, codebook, J, lam, gamma, iters, store="f32", p=2.0, device=0, hist=False):
    """Convenience: data term + ADMM solve for one image (torch tensor [C][N][N] on the GPU).
    Returns (u [q][N][N], labels [N][N], stats dict, hist or None)."""
    import torch
    C, n, _ = img.shape
    cb = np.asarray(codebook, dtype=np.float32)
    q = cb.shape[0]
    plan = Plan(n, C, q, J, store, device)
    dev = img.device
    s = torch.empty((q, n, n), dtype=torch.float32, device=dev)
    plan.datacost(img, cb, s, p)
    ws = plan.new_workspace()
    u = torch.empty((q, n, n), dtype=torch.float32, device=dev)
    labels = torch.empty((n, n), dtype=torch.int32, device=dev)
    h = torch.empty((iters, 4), dtype=torch.float64, device=dev) if hist else None
    stats = plan.solve(s, ws, lam, gamma, iters, u=u, labels=labels, hist=h)
    return u, labels, stats, h
