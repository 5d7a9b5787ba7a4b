"""Python binding of libobk (ctypes): argument marshalling only.

Every step of the plan and the sweep runs inside ``libobk.so`` (HIP kernels
for gfx950 plus the host graph passes).  There is no fallback: if the library
is not built, importing works but the first call raises ``ObkError``.

Inputs are numpy arrays (host memory) or torch CUDA tensors (device memory,
``on_device``); torch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Any

import numpy as np

__all__ = ["ObkError", "Plan", "plan", "plan_system", "rcm_host", "first_fit_host", "solve_batch",
           "batch_tune", "Batch", "lib", "LIB_PATH", "STATUS", "FP64", "FP32_IR"]

HERE = os.path.dirname(os.path.abspath(__file__))
# OBK_LIB names another build of the same sources (the sanitizer test loads
# a host-sanitized build this way)
LIB_PATH = os.environ.get("OBK_LIB") or os.path.join(HERE, "libobk.so")

FP64, FP32_IR = 0, 1
STATUS = {0: "converged", 1: "maxit", 2: "diverged", 3: "nonfinite"}
ERRORS = {-1: "OBK_E_ARG", -2: "OBK_E_CSR", -3: "OBK_E_NOT_SQUARE", -4: "OBK_E_NONFINITE",
          -5: "OBK_E_NOMEM", -6: "OBK_E_HIP", -7: "OBK_E_BUSY", -8: "OBK_E_INCONSISTENT"}


class ObkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("on_device", ctypes.c_int)]


class _Opts(ctypes.Structure):
    _fields_ = [("use_rcm", ctypes.c_int), ("precision", ctypes.c_int), ("inner_sweeps", ctypes.c_int),
                ("check_every", ctypes.c_int), ("reject_inconsistent", ctypes.c_int),
                ("hbm_budget", ctypes.c_size_t), ("block_k", ctypes.c_int), ("block_wgs", ctypes.c_int),
                ("block_maxit", ctypes.c_int), ("block_tol", ctypes.c_double), ("block_solver", ctypes.c_int),
                ("sweep_kernel", ctypes.c_int), ("omega", ctypes.c_double), ("max_group", ctypes.c_int),
                ("deterministic", ctypes.c_int), ("alloc", ctypes.c_void_p), ("dealloc", ctypes.c_void_p),
                ("ctx", ctypes.c_void_p)]


# obk_opts.alloc / dealloc: the caller's device allocator
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEALLOC_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _BatchOpts(ctypes.Structure):
    _fields_ = [("wgs_per_cu", ctypes.c_int), ("team_work", ctypes.c_int64), ("max_team", ctypes.c_int),
                ("tiles_per_wg", ctypes.c_int)]


class _KernelProfile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("outer_steps", ctypes.c_int64), ("relres0", ctypes.c_double),
                ("relres", ctypes.c_double), ("seconds", ctypes.c_double), ("status", ctypes.c_int)]


@dataclasses.dataclass
class Info:
    sweeps: int
    outer_steps: int
    relres0: float
    relres: float
    seconds: float
    status: str


_lib = None
_P = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ObkError(-6, f"{LIB_PATH} is not built (run __graft_entry__.build() or "
                               "python paper_2401_00672_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        L.obk_opts_default.argtypes = [ctypes.POINTER(_Opts)]
        L.obk_plan_engine.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.obk_plan_lambda_bound.argtypes = [_P, ctypes.POINTER(ctypes.c_double), _P]
        L.obk_validate_layout_host.argtypes = [ctypes.c_int64, ctypes.c_int32] + [_P] * 11 + [ctypes.c_int32,
                                                                                           ctypes.c_double]
        L.obk_banded_emulate_host.argtypes = [ctypes.c_int64, _P, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int64, ctypes.c_double, _P, _P]
        L.obk_plan.argtypes = [ctypes.POINTER(_Csr), _P, ctypes.c_double, ctypes.POINTER(_Opts), _P,
                               ctypes.POINTER(_P)]
        L.obk_solve.argtypes = [_P, _P, ctypes.c_double, ctypes.c_int64, _P, ctypes.POINTER(_Info), _P]
        L.obk_solve_noalloc.argtypes = [_P, _P, ctypes.c_double, ctypes.c_int64, _P, ctypes.POINTER(_Info), _P]
        L.obk_free.argtypes = [_P]
        L.obk_free.restype = None
        L.obk_free_async.argtypes = [_P, _P]
        L.obk_free_async.restype = ctypes.c_int
        L.obk_plan_perm.argtypes = [_P, _P]
        L.obk_plan_groups.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int32)]
        L.obk_plan_bytes.argtypes = [_P, ctypes.POINTER(ctypes.c_size_t)]
        L.obk_plan_stats.argtypes = [_P] + [ctypes.POINTER(ctypes.c_int64)] * 2 + \
            [ctypes.POINTER(ctypes.c_int32)] + [ctypes.POINTER(ctypes.c_int64)] * 2
        L.obk_sweep_device.argtypes = [_P, _P, ctypes.c_int64, _P]
        L.obk_sweep_profile.argtypes = [_P, _P, ctypes.c_int64, _P, ctypes.POINTER(_KernelProfile),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.obk_plan_blocks.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _P]
        L.obk_plan_block_solvers.argtypes = [_P, _P, _P]
        L.obk_plan_complex.argtypes = [ctypes.POINTER(_Csr), _P, ctypes.c_double, ctypes.POINTER(_Opts), _P,
                                       ctypes.POINTER(_P)]
        L.obk_block_zn_nn.argtypes = [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.obk_block_select_k.argtypes = [ctypes.POINTER(_Csr), _P, ctypes.c_double, _P, ctypes.c_int32,
                                         ctypes.POINTER(_Opts), _P, ctypes.POINTER(ctypes.c_int32), _P, _P]
        L.obk_select_delta.argtypes = [ctypes.POINTER(_Csr), _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                       ctypes.POINTER(_Opts), _P, ctypes.POINTER(ctypes.c_double), _P, _P, _P]
        L.obk_plan_set_opts.argtypes = [_P, ctypes.POINTER(_Opts)]
        L.obk_plan_set_opts.restype = ctypes.c_int
        L.obk_last_error.restype = ctypes.c_char_p
        L.obk_rcm_host.argtypes = [ctypes.c_int64, _P, _P, _P]
        L.obk_first_fit_host.argtypes = [ctypes.c_int64, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int32)]
        L.obk_batch_create.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_BatchOpts), ctypes.POINTER(_P)]
        L.obk_batch_begin.argtypes = [_P, _P, _P]
        L.obk_batch_reset.argtypes = [_P, _P, ctypes.c_int, _P]
        L.obk_batch_step.argtypes = [_P, ctypes.c_double, _P, _P, _P]
        L.obk_batch_enable.argtypes = [_P, _P, _P]
        L.obk_batch_start.argtypes = [_P, ctypes.c_int, _P, _P]
        L.obk_batch_result.argtypes = [_P, ctypes.c_int, _P, _P]
        L.obk_batch_free.argtypes = [_P]
        L.obk_batch_free.restype = None
        L.obk_solve_batch.argtypes = [_P, ctypes.c_int, _P, ctypes.c_double, ctypes.c_int64, _P, _P,
                                      ctypes.POINTER(_BatchOpts), _P]
        L.obk_batch_tune.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_BatchOpts), ctypes.POINTER(ctypes.c_double)]
        for name in ("obk_opts_default", "obk_plan", "obk_solve", "obk_plan_perm", "obk_plan_groups",
                     "obk_plan_bytes", "obk_plan_stats", "obk_sweep_device", "obk_sweep_profile", "obk_rcm_host",
                     "obk_first_fit_host", "obk_batch_create", "obk_batch_reset", "obk_batch_begin", "obk_batch_step",
                     "obk_batch_enable", "obk_batch_start", "obk_batch_result", "obk_solve_batch", "obk_batch_tune",
                     "obk_plan_blocks", "obk_plan_block_solvers", "obk_block_zn_nn", "obk_block_select_k",
                     "obk_plan_complex",
                     "obk_select_delta"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code: int) -> None:
    if code != 0:
        raise ObkError(code, lib().obk_last_error().decode(errors="replace"))


def _is_torch(a: Any) -> bool:
    return type(a).__module__.startswith("torch")


def _dev_ptr(t, dtype_name: str) -> int:
    import torch
    want = {"int64": torch.int64, "int32": torch.int32, "float64": torch.float64,
            "complex128": torch.complex128}[dtype_name]
    if not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise ObkError(-1, f"expected a contiguous CUDA tensor of {dtype_name}")
    return t.data_ptr()


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _stream(stream) -> int | None:
    if stream is not None:
        return int(stream)
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Plan:
    """A device-resident OBK-RCM plan (reordered, grouped system + workspace)."""

    def __init__(self, handle: int, n: int, nnz: int, on_device: bool, opts: dict | None = None,
                 n_ext: int | None = None, cplx: bool = False):
        self._opts = dict(opts or {})
        self.cplx = cplx                            # complex system: x0, x, x~ are complex128
        self._h = handle
        self.n = n                                  # unknowns of the caller's system
        self.n_ext = n if n_ext is None else n_ext  # size of the (extended) square system
        self.nnz = nnz
        self.on_device = on_device

    # -- lifetime
    def free(self, stream=None) -> None:
        """obk_free; with a stream, obk_free_async: waits only for that stream
        (all work using the plan must be done or queued there), and the
        library keeps the plan's memory for later plans."""
        if self._h:
            if stream is None:
                lib().obk_free(self._h)
            else:
                _check(lib().obk_free_async(self._h, _stream(stream)))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    @property
    def handle(self) -> int:
        if not self._h:
            raise ObkError(-1, "plan has been freed")
        return self._h

    # -- solve
    def solve(self, x0=None, tol: float = 0.0, maxit: int = 100, out=None, stream=None):
        """Sweeps from x0 (None = 0); returns (x, Info).  x is a numpy array for a
        host plan and a torch CUDA tensor for a device plan."""
        info = _Info()
        if self.on_device:
            import torch
            tname = "complex128" if self.cplx else "float64"
            x = out if out is not None else torch.empty(self.n, dtype=getattr(torch, tname), device="cuda")
            px = _dev_ptr(x, tname)
            p0 = None if x0 is None else _dev_ptr(x0, tname)
            st = _stream(stream) or torch.cuda.current_stream().cuda_stream
        else:
            dt = np.complex128 if self.cplx else np.float64
            x = out if out is not None else np.empty(self.n, dtype=dt)
            px = x.ctypes.data
            x0h = None if x0 is None else _host(x0, dt)
            p0 = None if x0h is None else x0h.ctypes.data
            st = _stream(stream)
        _check(lib().obk_solve(self.handle, p0, float(tol), int(maxit), px, ctypes.byref(info), st))
        return x, Info(info.sweeps, info.outer_steps, info.relres0, info.relres, info.seconds,
                       STATUS.get(info.status, str(info.status)))

    def solve_noalloc(self, x0=None, tol: float = 0.0, maxit: int = 100, out=None, stream=None):
        """obk_solve_noalloc: obk_solve on device tensors (x0 None = 0; out, if
        given, receives x) without any device allocation; real one-row-block
        plans.  Returns (x, Info)."""
        import torch
        info = _Info()
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        px = _dev_ptr(x, "float64")
        p0 = None if x0 is None else _dev_ptr(x0, "float64")
        st = _stream(stream) or torch.cuda.current_stream().cuda_stream
        _check(lib().obk_solve_noalloc(self.handle, p0, float(tol), int(maxit), px, ctypes.byref(info), st))
        return x, Info(info.sweeps, info.outer_steps, info.relres0, info.relres, info.seconds,
                       STATUS.get(info.status, str(info.status)))

    def sweep_device(self, x_tilde, sweeps: int, stream=None) -> None:
        """Enqueue `sweeps` sweeps on a device iterate in reordered coordinates."""
        import torch
        st = _stream(stream) or torch.cuda.current_stream().cuda_stream
        _check(lib().obk_sweep_device(self.handle, _dev_ptr(x_tilde, "complex128" if self.cplx else "float64"),
                                      int(sweeps), st))

    def sweep_profile(self, x_tilde, sweeps: int, stream=None) -> list[dict]:
        """obk_sweep_profile: eager FP64 sweeps with HIP events around every
        launch; per kernel the launches, event seconds and algorithmic bytes."""
        import torch
        st = _stream(stream) or torch.cuda.current_stream().cuda_stream
        out = (_KernelProfile * 8)()
        n = ctypes.c_int32()
        _check(lib().obk_sweep_profile(self.handle, _dev_ptr(x_tilde, "complex128" if self.cplx else "float64"),
                                       int(sweeps), st, out, 8, ctypes.byref(n)))
        return [{"name": out[i].name.decode(), "launches": out[i].launches, "seconds": out[i].seconds,
                 "bytes": out[i].bytes} for i in range(n.value)]

    def set_opts(self, precision: int | None = None, inner_sweeps: int | None = None,
                 check_every: int | None = None, block_wgs: int | None = None, block_maxit: int | None = None,
                 block_tol: float | None = None) -> None:
        """obk_plan_set_opts: change solve options without replanning."""
        o = _Opts()
        lib().obk_opts_default(ctypes.byref(o))
        new = {"precision": precision, "inner_sweeps": inner_sweeps, "check_every": check_every,
               "block_wgs": block_wgs, "block_maxit": block_maxit, "block_tol": block_tol}
        for key, val in new.items():
            v = self._opts.get(key, getattr(o, key)) if val is None else val
            setattr(o, key, type(getattr(o, key))(v))
        _check(lib().obk_plan_set_opts(self.handle, ctypes.byref(o)))
        self._opts.update({key: getattr(o, key) for key in new})

    def blocks(self) -> dict:
        """obk_plan_blocks (block form): block row ranges, the |cos| table of
        the centroids, the Oclass pairs in the order formed, Nclass, and the CG
        iterations spent per block so far."""
        k = ctypes.c_int32(0)
        _check(lib().obk_plan_blocks(self.handle, ctypes.byref(k), None, None, None, None))
        kk = int(k.value)
        bptr = np.empty(kk + 1, dtype=np.int64)
        partner = np.empty(kk, dtype=np.int32)
        cos = np.empty((kk, kk), dtype=np.float64)
        iters = np.empty(kk, dtype=np.int64)
        _check(lib().obk_plan_blocks(self.handle, ctypes.byref(k), bptr.ctypes.data, partner.ctypes.data,
                                     cos.ctypes.data, iters.ctypes.data))
        pairs = [(a, int(partner[a])) for a in range(kk) if partner[a] > a]
        nclass = [a for a in range(kk) if partner[a] < 0]
        direct = np.empty(kk, dtype=np.int32)
        bw = np.empty(kk, dtype=np.int64)
        _check(lib().obk_plan_block_solvers(self.handle, direct.ctypes.data, bw.ctypes.data))
        return {"k": kk, "bptr": bptr, "partner": partner, "cos": cos, "pairs": pairs, "nclass": nclass,
                "cg_iters": iters, "direct": direct.astype(bool), "factor_bandwidth": bw}

    # -- introspection
    def perm(self) -> np.ndarray:
        p = np.empty(self.n_ext, dtype=np.int32)
        _check(lib().obk_plan_perm(self.handle, p.ctypes.data))
        return p

    def groups(self):
        g = np.empty(self.n_ext, dtype=np.int32)
        ng = ctypes.c_int32(0)
        _check(lib().obk_plan_groups(self.handle, g.ctypes.data, ctypes.byref(ng)))
        return g, int(ng.value)

    def block_zn_nn(self) -> tuple[float, float]:
        """obk_block_zn_nn: Definitions 1-2 on the plan's centroid cosine table."""
        zn, nn = ctypes.c_double(), ctypes.c_double()
        _check(lib().obk_block_zn_nn(self.handle, ctypes.byref(zn), ctypes.byref(nn)))
        return zn.value, nn.value

    def device_bytes(self) -> int:
        b = ctypes.c_size_t(0)
        _check(lib().obk_plan_bytes(self.handle, ctypes.byref(b)))
        return int(b.value)

    def engine(self) -> dict:
        """obk_plan_engine: which kernels run the FP64 sweeps ("banded" with its
        slab count, or "phases")."""
        e, sl = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().obk_plan_engine(self.handle, ctypes.byref(e), ctypes.byref(sl)))
        return {"engine": "banded" if e.value == 2 else "phases", "slabs": sl.value}

    def lambda_bound(self):
        """obk_plan_lambda_bound: (plan bound, per-group bounds) on
        lambda_max(B_g B_g^H), B_g the unit-norm rows of group g."""
        _, ng = self.groups()
        per = np.zeros(max(ng, 1), dtype=np.float64)
        b = ctypes.c_double()
        _check(lib().obk_plan_lambda_bound(self.handle, ctypes.byref(b), per.ctypes.data))
        return b.value, per[:ng]

    def stats(self) -> dict:
        n, nnz, bw, nc = (ctypes.c_int64() for _ in range(4))
        ng = ctypes.c_int32()
        _check(lib().obk_plan_stats(self.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(ng),
                                    ctypes.byref(bw), ctypes.byref(nc)))
        return {"n": n.value, "nnz": nnz.value, "groups": ng.value, "bandwidth": bw.value,
                "conflicts": nc.value}


def plan_complex(row_ptr, col, val, f, delta: float, **kw) -> Plan:
    """obk_plan_complex on a complex CSR system (host numpy or device torch
    arrays; val and f complex128)."""
    return plan(row_ptr, col, val, f, delta, _complex=True, **kw)


def plan(row_ptr, col, val, f, delta: float, *, n: int | None = None, n_cols: int | None = None,
         use_rcm: bool = True, rcm_engine: str = "auto", precision: int = FP64, inner_sweeps: int = 8,
         check_every: int = 1, reject_inconsistent: bool = False, hbm_budget: int = 0, block_k: int = 0,
         block_wgs: int = 0, block_maxit: int = 0, block_tol: float = 1e-14, block_solver: str = "direct",
         sweep_kernel: str = "auto", omega: float = 1.0, max_group: int = 0, deterministic: bool = True,
         allocator=None, stream=None, _complex: bool = False) -> Plan:
    """obk_plan on a CSR system: numpy arrays (host) or torch CUDA tensors (device).
    block_k > 0 selects the block form of Algorithm 4 (k uniform blocks, exact
    block projections); delta is then the centroid cosine threshold.
    rcm_engine ("auto", "device" or "host") picks how the reverse Cuthill-McKee
    order is formed; the order is the same.  allocator: an object with
    alloc(nbytes) -> device pointer (int, 0 on failure) and dealloc(ptr), used
    for the plan's device memory (obk_opts.alloc / dealloc)."""
    on_device = _is_torch(row_ptr)
    if on_device:
        nrows = int(row_ptr.numel()) - 1 if n is None else int(n)
        nnz = int(col.numel())
        keep = (row_ptr, col, val, f)
        vt = "complex128" if _complex else "float64"
        ptrs = (_dev_ptr(row_ptr, "int64"), _dev_ptr(col, "int32"), _dev_ptr(val, vt), _dev_ptr(f, vt))
        import torch
        st = _stream(stream) or torch.cuda.current_stream().cuda_stream
    else:
        vt = np.complex128 if _complex else np.float64
        rp, ci, v, ff = _host(row_ptr, np.int64), _host(col, np.int32), _host(val, vt), _host(f, vt)
        nrows = len(rp) - 1 if n is None else int(n)
        nnz = len(ci)
        keep = (rp, ci, v, ff)
        ptrs = (rp.ctypes.data, ci.ctypes.data if nnz else None, v.ctypes.data if nnz else None,
                ff.ctypes.data)
        st = _stream(stream)
    ncols = nrows if n_cols is None else int(n_cols)
    csr = _Csr(nrows, ncols, nnz, ptrs[0], ptrs[1], ptrs[2], 1 if on_device else 0)
    opts = _Opts()
    lib().obk_opts_default(ctypes.byref(opts))
    engines = {"auto": 1, "device": 2, "host": 3}
    if rcm_engine not in engines:
        raise ValueError(f"rcm_engine must be one of {sorted(engines)}")
    opts.use_rcm = engines[rcm_engine] if use_rcm else 0
    opts.precision = int(precision)
    opts.inner_sweeps = int(inner_sweeps)
    opts.check_every = int(check_every)
    opts.reject_inconsistent = 1 if reject_inconsistent else 0
    opts.hbm_budget = int(hbm_budget)
    opts.block_k = int(block_k)
    opts.block_wgs = int(block_wgs)
    opts.block_maxit = int(block_maxit)
    opts.block_tol = float(block_tol)
    solvers = {"direct": 0, "cg": 1}
    if block_solver not in solvers:
        raise ValueError(f"block_solver must be one of {sorted(solvers)}")
    opts.block_solver = solvers[block_solver]
    kernels = {"auto": 0, "phases": 1, "banded": 2}
    if sweep_kernel not in kernels:
        raise ValueError(f"sweep_kernel must be one of {sorted(kernels)}")
    opts.sweep_kernel = kernels[sweep_kernel]
    opts.omega = float(omega)
    opts.max_group = int(max_group)
    opts.deterministic = 1 if deterministic else 0
    callbacks = None
    if allocator is not None:
        callbacks = (ALLOC_FN(lambda nbytes, ctx: allocator.alloc(int(nbytes)) or None),
                     DEALLOC_FN(lambda ptr, ctx: allocator.dealloc(ptr)))
        opts.alloc = ctypes.cast(callbacks[0], ctypes.c_void_p)
        opts.dealloc = ctypes.cast(callbacks[1], ctypes.c_void_p)
    h = _P()
    entry = lib().obk_plan_complex if _complex else lib().obk_plan
    _check(entry(ctypes.byref(csr), ptrs[3], float(delta), ctypes.byref(opts), st, ctypes.byref(h)))
    del keep
    plan_obj = Plan(h.value, ncols, nnz, on_device,
                {"precision": int(precision), "inner_sweeps": int(inner_sweeps), "check_every": int(check_every),
                 "block_wgs": int(block_wgs), "block_maxit": int(block_maxit), "block_tol": float(block_tol)},
                n_ext=max(nrows, ncols), cplx=bool(_complex))
    plan_obj._callbacks = callbacks     # the allocator callbacks live as long as the plan
    return plan_obj


def select_block_k(s, thr: float, candidates, stream=None):
    """obk_block_select_k on a ``synth.System`` (host arrays): the block count
    of largest zn, then least nn, among `candidates` (Section 3.6).  Returns
    (best_k, [(k, zn, nn), ...])."""
    rp, ci, v, ff = _host(s.row_ptr, np.int64), _host(s.col, np.int32), _host(s.val, np.float64), \
        _host(s.f, np.float64)
    nrows = s.m if hasattr(s, "m") else len(rp) - 1
    ncols = s.n
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    csr = _Csr(nrows, ncols, len(ci), rp.ctypes.data, ci.ctypes.data if len(ci) else None,
               v.ctypes.data if len(ci) else None, 0)
    opts = _Opts()
    lib().obk_opts_default(ctypes.byref(opts))
    zn = np.zeros(len(cand))
    nn = np.zeros(len(cand))
    best = ctypes.c_int32(0)
    _check(lib().obk_block_select_k(ctypes.byref(csr), ff.ctypes.data, float(thr), cand.ctypes.data, len(cand),
                                    ctypes.byref(opts), _stream(stream), ctypes.byref(best), zn.ctypes.data,
                                    nn.ctypes.data))
    return int(best.value), [(int(k), float(a), float(b)) for k, a, b in zip(cand, zn, nn)]


def select_delta(s, candidates=(0.5, 0.2, 0.1, 0.05, 0.02, 0.01), tol: float = 1e-8, maxit: int = 1000,
                 stream=None, **opt_kw):
    """obk_select_delta on a real ``synth.System`` (host arrays): plan and
    solve to `tol` for each candidate threshold (default: the six values of
    Table 5) and return (best_delta, [(delta, seconds, sweeps, relres), ...]).
    opt_kw sets obk_opts fields (e.g. block_k=8 for the block form)."""
    rp, ci, v, ff = _host(s.row_ptr, np.int64), _host(s.col, np.int32), _host(s.val, np.float64), \
        _host(s.f, np.float64)
    nrows = s.m if hasattr(s, "m") else len(rp) - 1
    csr = _Csr(nrows, s.n, len(ci), rp.ctypes.data, ci.ctypes.data if len(ci) else None,
               v.ctypes.data if len(ci) else None, 0)
    opts = _Opts()
    lib().obk_opts_default(ctypes.byref(opts))
    for key, val in opt_kw.items():
        setattr(opts, key, type(getattr(opts, key))(val))
    cand = np.ascontiguousarray(candidates, dtype=np.float64)
    sec = np.zeros(len(cand))
    swp = np.zeros(len(cand), dtype=np.int64)
    rel = np.zeros(len(cand))
    best = ctypes.c_double(0.0)
    _check(lib().obk_select_delta(ctypes.byref(csr), ff.ctypes.data, cand.ctypes.data, len(cand), float(tol),
                                  int(maxit), ctypes.byref(opts), _stream(stream), ctypes.byref(best),
                                  sec.ctypes.data, swp.ctypes.data, rel.ctypes.data))
    return float(best.value), [(float(d), float(t), int(k), float(r)) for d, t, k, r in zip(cand, sec, swp, rel)]


def rcm_host(gptr, gadj) -> np.ndarray:
    """obk_rcm_host: RCM order of a symmetric adjacency structure (no GPU needed)."""
    gptr = _host(gptr, np.int64)
    gadj = _host(gadj, np.int32)
    n = len(gptr) - 1
    perm = np.empty(max(n, 0), dtype=np.int32)
    _check(lib().obk_rcm_host(n, gptr.ctypes.data, gadj.ctypes.data if gadj.size else None,
                              perm.ctypes.data if n else None))
    return perm


def banded_emulate_host(rp, ci, v, f, inv, group, ngroups: int, slabs: int, sweeps: int, x,
                        omega: float = 1.0) -> tuple[np.ndarray, dict]:
    """obk_banded_emulate_host: the banded engine's layout for `slabs` slabs and
    its sweeps run on the host; returns (x after the sweeps, layout stats)."""
    rp, ci, v = _host(rp, np.int64), _host(ci, np.int32), _host(v, np.float64)
    f, inv, group = _host(f, np.float64), _host(inv, np.float64), _host(group, np.int32)
    xo = np.array(x, dtype=np.float64, copy=True)
    st = np.zeros(4, np.int64)
    n = len(rp) - 1
    _check(lib().obk_banded_emulate_host(n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, f.ctypes.data,
                                         inv.ctypes.data, group.ctypes.data, int(ngroups), int(slabs), int(sweeps),
                                         float(omega), xo.ctypes.data, st.ctypes.data))
    return xo, {"slabs": int(st[0]), "cached": int(st[1]), "streamed": int(st[2]), "lds_bytes": int(st[3])}


def validate_layout_host(n, gptr, grow, group_of_row, rptr, rcol, rval, tptr, tcol, sptr, srow, sval, delta,
                         cplx: bool = False) -> None:
    """obk_validate_layout_host: the plan validator on a layout given as host
    arrays (raises ObkError OBK_E_ARG naming the first violation)."""
    arrs = [_host(gptr, np.int64), _host(grow, np.int32), _host(group_of_row, np.int32), _host(rptr, np.int64),
            _host(rcol, np.int32), _host(rval, np.float64), _host(tptr, np.int64), _host(tcol, np.int32),
            _host(sptr, np.int64), _host(srow, np.int32), _host(sval, np.float64)]
    ptrs = [a.ctypes.data if a.size else None for a in arrs]
    _check(lib().obk_validate_layout_host(int(n), len(arrs[0]) - 1, *ptrs, int(bool(cplx)), float(delta)))


def first_fit_host(cptr, cidx, active):
    """obk_first_fit_host: first-fit grouping from conflict lists (no GPU needed)."""
    cptr = _host(cptr, np.int64)
    cidx = _host(cidx, np.int32)
    active = _host(active, np.uint8)
    n = len(cptr) - 1
    g = np.empty(max(n, 0), dtype=np.int32)
    ng = ctypes.c_int32(0)
    _check(lib().obk_first_fit_host(n, cptr.ctypes.data, cidx.ctypes.data if cidx.size else None,
                                    active.ctypes.data, g.ctypes.data if n else None, ctypes.byref(ng)))
    return g, int(ng.value)


def plan_system(s, delta: float, **kw) -> Plan:
    """obk_plan on a ``synth.System`` or ``synth.RectSystem`` (host arrays)."""
    if hasattr(s, "m"):
        return plan(s.row_ptr, s.col, s.val, s.f, delta, n=s.m, n_cols=s.n, **kw)
    if np.iscomplexobj(s.val):
        return plan_complex(s.row_ptr, s.col, s.val, s.f, delta, **kw)
    return plan(s.row_ptr, s.col, s.val, s.f, delta, **kw)


# ------------------------------------------------------------------ batches
def _handles(plans):
    arr = (_P * len(plans))(*[p.handle for p in plans])
    return arr


def _batch_opts(opts):
    if opts is None:
        return None
    if isinstance(opts, _BatchOpts):
        return opts
    return _BatchOpts(int(opts.get("wgs_per_cu", 0)), int(opts.get("team_work", 0)), int(opts.get("max_team", 0)),
                      int(opts.get("tiles_per_wg", 0)))


def _ptr_array(arrays, on_device, dtype_name="float64"):
    if arrays is None:
        return None, []
    keep, ptrs = [], []
    for a in arrays:
        if a is None:
            ptrs.append(None)
        elif on_device:
            ptrs.append(_dev_ptr(a, dtype_name))
        else:
            h = _host(a, np.float64)
            keep.append(h)
            ptrs.append(h.ctypes.data)
    return (_P * len(ptrs))(*ptrs), keep


def solve_batch(plans, x0=None, tol: float = 1e-10, maxit: int = 100, opts=None, stream=None):
    """obk_solve_batch: solve all plans together; returns (list of x, list of Info)."""
    plans = list(plans)
    on_dev = bool(plans) and plans[0].on_device
    if on_dev:
        import torch
        xs = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p in plans]
        st = _stream(stream) or torch.cuda.current_stream().cuda_stream
    else:
        xs = [np.empty(p.n, dtype=np.float64) for p in plans]
        st = _stream(stream)
    x0arr, keep0 = _ptr_array(x0, on_dev)
    xarr, keep1 = _ptr_array(xs, on_dev) if not on_dev else ((_P * len(xs))(*[x.data_ptr() for x in xs]), [])
    if not on_dev:
        xarr = (_P * len(xs))(*[x.ctypes.data for x in xs])
    infos = (_Info * max(len(plans), 1))()
    o = _batch_opts(opts)
    _check(lib().obk_solve_batch(_handles(plans), len(plans), x0arr, float(tol), int(maxit), xarr, infos,
                                 ctypes.byref(o) if o is not None else None, st))
    out = [Info(i.sweeps, i.outer_steps, i.relres0, i.relres, i.seconds, STATUS.get(i.status, str(i.status)))
           for i in list(infos)[:len(plans)]]
    return xs, out


def batch_tune(plans):
    """obk_batch_tune: returns (dict of the fastest tunables, seconds per step)."""
    plans = list(plans)
    best = _BatchOpts()
    sec = ctypes.c_double(0)
    _check(lib().obk_batch_tune(_handles(plans), len(plans), ctypes.byref(best), ctypes.byref(sec)))
    return ({"wgs_per_cu": best.wgs_per_cu, "team_work": best.team_work, "max_team": best.max_team,
             "tiles_per_wg": best.tiles_per_wg}, sec.value)


class Batch:
    """A batch of plans advanced in shared launches (obk_batch_*)."""

    def __init__(self, plans, opts=None):
        self.plans = list(plans)
        self._keep = _handles(self.plans)
        h = _P()
        o = _batch_opts(opts)
        _check(lib().obk_batch_create(self._keep, len(self.plans), ctypes.byref(o) if o is not None else None,
                                      ctypes.byref(h)))
        self._h = h.value

    def reset(self, plans, stream=None):
        """obk_batch_reset: the same batch object over a new member list;
        members keep their iterates, new ones need start()."""
        plans = list(plans)
        keep = _handles(plans)
        code = lib().obk_batch_reset(self._h, keep, len(plans), _stream(stream))
        if code not in (0, -1, -7):
            self.plans, self._keep = [], _handles([])   # the library left the batch empty
        _check(code)
        self.plans, self._keep = plans, keep

    def begin(self, x0=None, stream=None):
        on_dev = bool(self.plans) and self.plans[0].on_device
        arr, keep = _ptr_array(x0, on_dev)
        _check(lib().obk_batch_begin(self._h, arr, _stream(stream)))

    def start(self, i: int, x0=None, stream=None):
        """obk_batch_start: initialise system i alone (x0 None: zeros)."""
        ptr = None
        keep = None
        if x0 is not None:
            if self.plans[i].on_device:
                ptr = _dev_ptr(x0, "float64")
            else:
                keep = np.ascontiguousarray(x0, dtype=np.float64)
                ptr = keep.ctypes.data
        _check(lib().obk_batch_start(self._h, int(i), ptr, _stream(stream)))

    def step(self, tol: float, stream=None):
        n = len(self.plans)
        rr = np.empty(max(n, 1), np.float64)
        act = np.empty(max(n, 1), np.int32)
        _check(lib().obk_batch_step(self._h, float(tol), rr.ctypes.data, act.ctypes.data, _stream(stream)))
        return rr[:n], act[:n].astype(bool)

    def enable(self, enabled, stream=None):
        e = np.ascontiguousarray(enabled, dtype=np.int32)
        _check(lib().obk_batch_enable(self._h, e.ctypes.data, _stream(stream)))

    def result(self, i: int, stream=None):
        p = self.plans[i]
        if p.on_device:
            import torch
            x = torch.empty(p.n, dtype=torch.float64, device="cuda")
            _check(lib().obk_batch_result(self._h, int(i), x.data_ptr(), _stream(stream)))
        else:
            x = np.empty(p.n, np.float64)
            _check(lib().obk_batch_result(self._h, int(i), x.ctypes.data, _stream(stream)))
        return x

    def free(self):
        if self._h:
            lib().obk_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
