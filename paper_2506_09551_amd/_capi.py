"""ctypes binding of the C ABI in ``include/msb.h``.

Argument marshalling only: every function forwards to the HIP library
``libmsb.so`` built in this directory; device buffers are torch tensors on a
ROCm device (their ``data_ptr()`` is passed), streams are torch streams.  There
is no fallback: if the library is missing or the device is not a gfx950 GPU
the calls raise.
"""
from __future__ import annotations

import ctypes
import math
from ctypes import POINTER, c_double, c_int, c_int64, c_void_p
from pathlib import Path

MSB_MAX_BOND_TYPES = 8
STATUS = {0: "MSB_OK", 1: "MSB_EINVAL", 2: "MSB_ENOMEM", 3: "MSB_EHIP",
          4: "MSB_BREAKDOWN", 5: "MSB_NOT_CONVERGED", 6: "MSB_FLOOR"}
MSB_OK, MSB_EINVAL, MSB_ENOMEM, MSB_EHIP, MSB_BREAKDOWN, MSB_NOT_CONVERGED, MSB_FLOOR = range(7)
MSB_C128, MSB_C64 = 0, 1

LIB_PATH = Path(__file__).resolve().parent / "libmsb.so"


class MsbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class msb_model(ctypes.Structure):
    _fields_ = [("n_sites", c_int), ("n_up", c_int), ("n_dn", c_int), ("n_bonds", c_int),
                ("bond_i", POINTER(c_int)), ("bond_j", POINTER(c_int)),
                ("bond_t", POINTER(c_double)), ("U", c_double), ("bond_t_rev", POINTER(c_double))]


class msb_system(ctypes.Structure):
    _fields_ = [("core_site", c_int), ("Uc", c_double), ("E_G", c_double), ("Gamma", c_double),
                ("U", c_double), ("n_amp", c_int), ("t_amp", c_double * MSB_MAX_BOND_TYPES)]


class msb_info(ctypes.Structure):
    _fields_ = [("iters", c_int), ("mvms", c_int), ("breakdown_iter", c_int), ("flushes", c_int),
                ("sys_iters", POINTER(c_int)), ("shift_iters", POINTER(c_int)),
                ("resid_rec", POINTER(c_double)), ("resid_true", POINTER(c_double)),
                ("t_iter_ms", c_double), ("t_flush_ms", c_double), ("t_true_ms", c_double),
                ("t_gemm_ms", c_double), ("n_gemm", c_int), ("gemm_flops", c_double),
                ("gemm_bytes", c_double), ("replacements", c_int),
                ("seed_hist", POINTER(c_double)), ("hist_len", c_int),
                ("apply_threads", c_int), ("apply_ept", c_int), ("apply_nv", c_int), ("apply_passes", c_int),
                ("apply_order", c_int), ("t_setup_ms", c_double), ("t_alloc_ms", c_double), ("t_wall_ms", c_double),
                ("apply_panel_width", c_int), ("group", c_int), ("bank_slots", c_int)]


class msb_shape(ctypes.Structure):
    _fields_ = [("threads", c_int), ("elems_per_thread", c_int), ("vectors", c_int), ("passes", c_int),
                ("row_order", c_int), ("panel_width", c_int), ("ms", c_double)]


class msb_opts(ctypes.Structure):
    _fields_ = [("chunk", c_int), ("bank_slots", c_int), ("batch", c_int),
                ("replace_every", c_int), ("use_graph", c_int), ("mem_fraction", c_double),
                ("assembly_engine", c_int), ("autotune", c_int), ("dual", c_int), ("direct_ap", c_int),
                ("interleave", c_int)]


_lib = None


def lib():
    """Load ``libmsb.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise OSError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()     # torch's HIP runtime must claim the device before the library's
        L = ctypes.CDLL(str(LIB_PATH))
        L.msb_last_error.restype = ctypes.c_char_p
        L.msb_device_ok.restype = c_int
        L.msb_stream_create.argtypes = [POINTER(c_void_p)]
        L.msb_stream_create.restype = c_int
        L.msb_stream_destroy.argtypes = [c_void_p]
        L.msb_stream_destroy.restype = c_int
        L.msb_create.argtypes = [POINTER(msb_model), POINTER(c_void_p)]
        L.msb_create.restype = c_int
        L.msb_destroy.argtypes = [c_void_p]
        L.msb_destroy.restype = None
        L.msb_release_workspace.argtypes = [c_void_p]
        L.msb_release_workspace.restype = c_int
        L.msb_dim.argtypes = [c_void_p]
        L.msb_dim.restype = c_int64
        L.msb_sector_info.argtypes = [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int)]
        L.msb_sector_info.restype = c_int
        L.msb_apply.argtypes = [c_void_p, POINTER(msb_system), c_int, c_double, c_int, c_void_p,
                                c_void_p, c_void_p]
        L.msb_apply.restype = c_int
        L.msb_apply_block.argtypes = [c_void_p, POINTER(msb_system), c_int, c_double, c_int, c_int, c_void_p,
                                      c_void_p, c_int, POINTER(c_double), c_void_p]
        L.msb_apply_block.restype = c_int
        L.msb_apply_noalloc.argtypes = [c_void_p, POINTER(msb_system), c_int, c_double, c_int, c_void_p,
                                        c_void_p, c_void_p]
        L.msb_apply_noalloc.restype = c_int
        L.msb_apply_timed.argtypes = [c_void_p, POINTER(msb_system), c_int, c_double, c_int,
                                      c_void_p, c_void_p, c_int, POINTER(c_double), c_void_p]
        L.msb_apply_timed.restype = c_int
        L.msb_number_op.argtypes = [c_void_p, c_int, c_double, c_double, c_int, c_int, c_void_p,
                                    c_void_p, c_void_p]
        L.msb_number_op.restype = c_int
        L.msb_ground_state.argtypes = [c_void_p, POINTER(msb_system), c_void_p, c_double, c_int,
                                       POINTER(c_double), c_void_p, POINTER(c_int), c_void_p]
        L.msb_ground_state.restype = c_int
        L.msb_solve.argtypes = [c_void_p, POINTER(msb_system), c_int, c_void_p, POINTER(c_double),
                                c_int, c_double, c_double, c_int, c_int, c_void_p,
                                POINTER(msb_info), POINTER(msb_opts), c_void_p]
        L.msb_solve.restype = c_int
        L.msb_solve_reseed.argtypes = [c_void_p, POINTER(msb_system), c_int, c_void_p, POINTER(c_double),
                                       c_int, c_double, c_double, c_int, c_int, c_double, c_int, c_void_p,
                                       POINTER(c_double), POINTER(c_double), POINTER(c_int),
                                       POINTER(msb_opts), c_void_p]
        L.msb_solve_reseed.restype = c_int
        L.msb_dipole.argtypes = [c_void_p, c_void_p, c_int, c_int, POINTER(c_double), c_int, c_int,
                                 c_void_p, c_void_p, c_void_p]
        L.msb_dipole.restype = c_int
        L.msb_combine.argtypes = [c_void_p, c_int, c_int, c_int, c_void_p, POINTER(c_double),
                                  POINTER(c_double), POINTER(c_int), POINTER(c_double),
                                  POINTER(c_double), c_void_p, c_void_p]
        L.msb_combine.restype = c_int
        L.msb_spectrum.argtypes = [c_void_p, POINTER(msb_system), c_void_p, c_int, POINTER(c_double),
                                   c_int, c_double, c_int, c_double, POINTER(c_double),
                                   POINTER(c_int), c_void_p]
        L.msb_spectrum.restype = c_int
        L.msb_spectrum_cf.argtypes = [c_void_p, POINTER(msb_system), c_void_p, c_int, POINTER(c_double),
                                      c_int, c_double, c_int, c_double, POINTER(c_double),
                                      POINTER(c_int), POINTER(c_double), POINTER(c_double), c_int, c_void_p]
        L.msb_spectrum_cf.restype = c_int
        L.msb_autotune.argtypes = [c_void_p, c_int, c_int, POINTER(msb_shape), c_int, POINTER(c_int),
                                   c_void_p]
        L.msb_autotune.restype = c_int
        L.msb_set_shape.argtypes = [c_void_p, c_int, c_int, POINTER(msb_shape)]
        L.msb_set_shape.restype = c_int
        L.msb_mlp_num_params.restype = c_int64
        L.msb_mlp_create.argtypes = [c_int, POINTER(c_double), POINTER(c_double), c_double, POINTER(c_void_p)]
        L.msb_mlp_create.restype = c_int
        L.msb_mlp_destroy.argtypes = [c_void_p]
        L.msb_mlp_destroy.restype = None
        L.msb_mlp_set_params.argtypes = [c_void_p, c_int, c_void_p]
        L.msb_mlp_set_params.restype = c_int
        L.msb_mlp_get_params.argtypes = [c_void_p, c_int, c_void_p]
        L.msb_mlp_get_params.restype = c_int
        L.msb_mlp_grad.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_int, POINTER(c_double), c_void_p]
        L.msb_mlp_grad.restype = c_int
        L.msb_mlp_train.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int, c_int, c_double,
                                    c_void_p, c_void_p]
        L.msb_mlp_train.restype = c_int
        L.msb_mlp_predict.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
        L.msb_mlp_predict.restype = c_int
        L.msb_mlp_fallback.argtypes = [c_void_p, c_void_p, c_int, c_int, c_double, c_void_p]
        L.msb_mlp_fallback.restype = c_int
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C entry points the binding expects the library to export."""
    return ["msb_create", "msb_destroy", "msb_release_workspace", "msb_dim", "msb_sector_info", "msb_last_error",
            "msb_device_ok", "msb_stream_create", "msb_stream_destroy", "msb_apply", "msb_apply_block", "msb_apply_noalloc", "msb_apply_timed", "msb_number_op", "msb_ground_state", "msb_solve",
            "msb_solve_reseed", "msb_dipole",
            "msb_combine", "msb_spectrum", "msb_spectrum_cf", "msb_autotune", "msb_set_shape",
            "msb_mlp_num_params", "msb_mlp_create", "msb_mlp_destroy", "msb_mlp_set_params",
            "msb_mlp_get_params", "msb_mlp_grad", "msb_mlp_train", "msb_mlp_predict", "msb_mlp_fallback"]


def _check(status: int):
    if status != MSB_OK:
        raise MsbError(status, lib().msb_last_error().decode())


class LibStream:
    """A stream of the library's own HIP runtime (msb_stream_create).

    Its handle goes to the C ABI as it is; the call is ordered after the work
    already queued on it.  Release it with ``close()``."""

    def __init__(self):
        h = c_void_p()
        _check(lib().msb_stream_create(ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle is not None and self.handle.value:
            _check(lib().msb_stream_destroy(self.handle))
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _stream_ptr(stream):
    """Stream argument of a C call.

    A ``LibStream`` is passed through: it belongs to the library's runtime.
    A torch stream (or None: torch's current stream) is synchronised and NULL
    is passed: torch ships its own HIP runtime, separate from the one the
    library links, so a torch stream handle means nothing to the library
    (device pointers are shared: both runtimes map into the same process
    address space).  Every library call is blocking, so its outputs are
    complete on return.
    """
    if isinstance(stream, LibStream):
        return stream.handle
    import torch
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    return c_void_p(0)


def _ptr(t, dtype=None, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


def _prec_dtype(prec: int):
    import torch
    return torch.complex128 if prec == MSB_C128 else torch.complex64


def make_system(core_site=-1, Uc=0.0, E_G=0.0, Gamma=0.0, U=None, t_amp=None) -> msb_system:
    s = msb_system()
    s.core_site = int(core_site)
    s.Uc = float(Uc)
    s.E_G = float(E_G)
    s.Gamma = float(Gamma)
    s.U = math.nan if U is None else float(U)
    amps = list(t_amp) if t_amp is not None else []
    if len(amps) > MSB_MAX_BOND_TYPES:
        raise ValueError("too many bond amplitudes")
    s.n_amp = len(amps)
    for i, a in enumerate(amps):
        s.t_amp[i] = float(a)
    return s


def _systems(systems):
    if isinstance(systems, msb_system):
        systems = [systems]
    arr = (msb_system * len(systems))(*systems)
    return arr, len(systems)


# ---- C entry points ---------------------------------------------------------

def msb_device_ok() -> bool:
    return bool(lib().msb_device_ok())


def msb_create(n_sites: int, n_up: int, n_dn: int, bonds, U: float) -> c_void_p:
    """Context for H on the (n_up, n_dn) sector; bonds = [(i, j, t), ...], or
    directed [(i, j, t, t_rev), ...] (t moves an electron i -> j, t_rev back)."""
    nb = len(bonds)
    bi = (c_int * max(nb, 1))(*[int(b[0]) for b in bonds])
    bj = (c_int * max(nb, 1))(*[int(b[1]) for b in bonds])
    bt = (c_double * max(nb, 1))(*[float(b[2]) for b in bonds])
    directed = any(len(b) > 3 for b in bonds)
    btr = (c_double * max(nb, 1))(*[float(b[3] if len(b) > 3 else b[2]) for b in bonds]) if directed else None
    m = msb_model(int(n_sites), int(n_up), int(n_dn), nb, bi, bj, bt, float(U),
                  ctypes.cast(btr, POINTER(c_double)) if directed else None)
    ctx = c_void_p()
    _check(lib().msb_create(ctypes.byref(m), ctypes.byref(ctx)))
    return ctx


def msb_destroy(ctx):
    lib().msb_destroy(ctx)


def msb_release_workspace(ctx):
    """Free the context's solve / spectrum workspace (reallocated on next use)."""
    _check(lib().msb_release_workspace(ctx))


def msb_dim(ctx) -> int:
    return int(lib().msb_dim(ctx))


def msb_sector_info(ctx):
    nu, nd, nt = c_int(), c_int(), c_int()
    _check(lib().msb_sector_info(ctx, ctypes.byref(nu), ctypes.byref(nd), ctypes.byref(nt)))
    return nu.value, nd.value, nt.value


def msb_apply(ctx, systems, shift: float, prec: int, x, y, stream=None):
    arr, n = _systems(systems)
    D = msb_dim(ctx)
    dt = _prec_dtype(prec)
    _check(lib().msb_apply(ctx, arr, n, float(shift), int(prec), _ptr(x, dt, n * D, "x"),
                           _ptr(y, dt, n * D, "y"), _stream_ptr(stream)))


def msb_apply_block(ctx, systems, shift: float, prec: int, group: int, x, y, reps: int = 0, stream=None):
    """Block apply on interleaved groups: x, y [ceil(nsys/group)][D][group] (any
    contiguous tensor of that many elements); returns the mean time (ms) of
    `reps` timed applies, or None when reps == 0."""
    arr, n = _systems(systems)
    D = msb_dim(ctx)
    dt = _prec_dtype(prec)
    ng = (n + group - 1) // group
    ms = c_double()
    _check(lib().msb_apply_block(ctx, arr, n, float(shift), int(prec), int(group), _ptr(x, dt, ng * group * D, "x"),
                                 _ptr(y, dt, ng * group * D, "y"), int(reps),
                                 ctypes.byref(ms) if reps > 0 else None, _stream_ptr(stream)))
    return ms.value if reps > 0 else None


def msb_apply_noalloc(ctx, systems, shift: float, prec: int, x, y, stream=None):
    """msb_apply without any allocation (systems staged in the library's fixed array)."""
    arr, n = _systems(systems)
    D = msb_dim(ctx)
    dt = _prec_dtype(prec)
    _check(lib().msb_apply_noalloc(ctx, arr, n, float(shift), int(prec), _ptr(x, dt, n * D, "x"),
                                   _ptr(y, dt, n * D, "y"), _stream_ptr(stream)))


def msb_apply_timed(ctx, systems, shift: float, prec: int, x, y, reps: int, stream=None) -> float:
    """Mean duration (ms) of `reps` back-to-back applies, timed with HIP events on `stream`."""
    arr, n = _systems(systems)
    D = msb_dim(ctx)
    dt = _prec_dtype(prec)
    ms = c_double()
    _check(lib().msb_apply_timed(ctx, arr, n, float(shift), int(prec), _ptr(x, dt, n * D, "x"),
                                 _ptr(y, dt, n * D, "y"), int(reps), ctypes.byref(ms),
                                 _stream_ptr(stream)))
    return ms.value


def msb_number_op(ctx, site: int, w_up: float, w_dn: float, x, y, stream=None):
    import torch
    D = msb_dim(ctx)
    x_real = 1 if x.dtype == torch.float64 else 0
    if not x_real and x.dtype != torch.complex128:
        raise TypeError("x must be float64 or complex128")
    count = x.numel() // D
    _check(lib().msb_number_op(ctx, int(site), float(w_up), float(w_dn), count, x_real,
                               _ptr(x, None, count * D, "x"), _ptr(y, torch.complex128, count * D, "y"),
                               _stream_ptr(stream)))


def msb_ground_state(ctx, system, x0, tol: float, maxit: int, G, stream=None):
    """Returns (E_G, iters); G (float64 [D]) receives the ground state."""
    import torch
    D = msb_dim(ctx)
    e = c_double()
    it = c_int()
    st = lib().msb_ground_state(ctx, ctypes.byref(system), _ptr(x0, torch.float64, D, "x0"),
                                float(tol), int(maxit), ctypes.byref(e),
                                _ptr(G, torch.float64, D, "G"), ctypes.byref(it), _stream_ptr(stream))
    _check(st)
    return e.value, it.value


def msb_solve(ctx, systems, E, w_in, seed_shift: float, tol: float, maxit: int, prec: int, psi,
              want_true: bool = False, opts: dict | None = None, stream=None, raise_on_fail=True,
              hist_len: int = 0):
    """Multi-shift solve; returns (status, info dict)."""
    import numpy as np
    import torch
    arr, n = _systems(systems)
    D = msb_dim(ctx)
    w = np.ascontiguousarray(np.asarray(w_in, dtype=np.float64))
    ns = len(w)
    sys_iters = (c_int * n)()
    shift_iters = (c_int * (n * ns))()
    resid_rec = (c_double * (n * ns))()
    resid_true = (c_double * (n * ns))() if want_true else None
    info = msb_info()
    info.sys_iters = sys_iters
    info.shift_iters = shift_iters
    info.resid_rec = resid_rec
    info.resid_true = ctypes.cast(resid_true, POINTER(c_double)) if want_true else None
    seed_hist = (c_double * (n * hist_len))() if hist_len > 0 else None
    if hist_len > 0:
        info.seed_hist = ctypes.cast(seed_hist, POINTER(c_double))
        info.hist_len = int(hist_len)
    o = msb_opts()
    for k, v in (opts or {}).items():
        setattr(o, k, v)
    st = lib().msb_solve(ctx, arr, n, _ptr(E, torch.complex128, n * D, "E"),
                         w.ctypes.data_as(POINTER(c_double)), ns, float(seed_shift), float(tol),
                         int(maxit), int(prec), _ptr(psi, _prec_dtype(prec), n * ns * D, "psi"),
                         ctypes.byref(info), ctypes.byref(o), _stream_ptr(stream))
    out = {
        "status": st, "iters": info.iters, "mvms": info.mvms, "breakdown_iter": info.breakdown_iter,
        "flushes": info.flushes,
        "sys_iters": np.frombuffer(sys_iters, dtype=np.int32).copy(),
        "shift_iters": np.frombuffer(shift_iters, dtype=np.int32).reshape(n, ns).copy(),
        "resid_rec": np.frombuffer(resid_rec, dtype=np.float64).reshape(n, ns).copy(),
        "resid_true": (np.frombuffer(resid_true, dtype=np.float64).reshape(n, ns).copy()
                       if want_true else None),
        "t_iter_ms": info.t_iter_ms, "t_flush_ms": info.t_flush_ms, "t_true_ms": info.t_true_ms,
        "t_gemm_ms": info.t_gemm_ms, "n_gemm": info.n_gemm, "gemm_flops": info.gemm_flops,
        "gemm_bytes": info.gemm_bytes, "replacements": info.replacements,
        "seed_hist": (np.frombuffer(seed_hist, dtype=np.float64).reshape(n, hist_len).copy()
                      if hist_len > 0 else None),
        "apply_shape": (info.apply_threads, info.apply_ept, info.apply_nv, info.apply_passes,
                        info.apply_order, info.apply_panel_width),
        "t_setup_ms": info.t_setup_ms, "t_alloc_ms": info.t_alloc_ms, "t_wall_ms": info.t_wall_ms,
        "group": info.group, "bank_slots": info.bank_slots,
    }
    if raise_on_fail and st != MSB_OK:
        raise MsbError(st, lib().msb_last_error().decode())
    return st, out


def msb_solve_reseed(ctx, systems, E, w_in, seed_shift: float, tol: float, maxit: int, prec: int, psi,
                     reseed_tol: float, max_rounds: int = 8, opts: dict | None = None, stream=None,
                     raise_on_fail=True):
    """Multi-shift solve with adaptive reseeding; returns (status, info dict with
    seed_of [nsys][n_shift], resid_true [nsys][n_shift], rounds [nsys])."""
    import numpy as np
    import torch
    arr, n = _systems(systems)
    D = msb_dim(ctx)
    w = np.ascontiguousarray(np.asarray(w_in, dtype=np.float64))
    ns = len(w)
    seed_of = np.empty((n, ns), dtype=np.float64)
    rt = np.empty((n, ns), dtype=np.float64)
    rounds = np.empty(n, dtype=np.int32)
    o = msb_opts()
    for k, v in (opts or {}).items():
        setattr(o, k, v)
    st = lib().msb_solve_reseed(ctx, arr, n, _ptr(E, torch.complex128, n * D, "E"),
                                w.ctypes.data_as(POINTER(c_double)), ns, float(seed_shift), float(tol),
                                int(maxit), int(prec), float(reseed_tol), int(max_rounds),
                                _ptr(psi, _prec_dtype(prec), n * ns * D, "psi"),
                                seed_of.ctypes.data_as(POINTER(c_double)), rt.ctypes.data_as(POINTER(c_double)),
                                rounds.ctypes.data_as(POINTER(c_int)), ctypes.byref(o), _stream_ptr(stream))
    if raise_on_fail and st != MSB_OK:
        raise MsbError(st, lib().msb_last_error().decode())
    return st, {"status": st, "seed_of": seed_of, "resid_true": rt, "rounds": rounds}


def msb_dipole(src_ctx, dst_ctx, spin: int, create: bool, coef, x, y, accumulate=False, stream=None):
    """y[v] (+)= sum_j coef[j] c+_{j spin} x[v] (create) or c_{j spin}; x, y complex128 [nvec][D]."""
    import numpy as np
    import torch
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128))
    if c.ndim != 1:
        raise ValueError("coef must be one complex number per site")
    cc = np.ascontiguousarray(np.stack([c.real, c.imag], axis=1).ravel())
    nvec = x.shape[0] if x.dim() == 2 else 1
    _check(lib().msb_dipole(src_ctx, dst_ctx, int(spin), int(bool(create)), cc.ctypes.data_as(POINTER(c_double)),
                            nvec, int(bool(accumulate)), _ptr(x, torch.complex128, nvec * msb_dim(src_ctx), "x"),
                            _ptr(y, torch.complex128, nvec * msb_dim(dst_ctx), "y"), _stream_ptr(stream)))


def msb_combine(ctx, psi, nsys: int, n_shift: int, prec: int, phases, phi, o1=None, stream=None):
    """phi[k] = sum_s phases[s] * O1_s psi[s][k]; o1 = [(site, w_up, w_dn), ...] or None."""
    import torch
    D = msb_dim(ctx)
    pre = (c_double * nsys)(*[complex(p).real for p in phases])
    pim = (c_double * nsys)(*[complex(p).imag for p in phases])
    if o1 is not None:
        site = (c_int * nsys)(*[int(o[0]) for o in o1])
        wu = (c_double * nsys)(*[float(o[1]) for o in o1])
        wd = (c_double * nsys)(*[float(o[2]) for o in o1])
    else:
        site, wu, wd = None, None, None
    _check(lib().msb_combine(ctx, nsys, n_shift, int(prec),
                             _ptr(psi, _prec_dtype(prec), nsys * n_shift * D, "psi"), pre, pim,
                             site, wu, wd, _ptr(phi, torch.complex128, n_shift * D, "phi"),
                             _stream_ptr(stream)))


def msb_spectrum(ctx, system, phi, w, eta: float, lanczos_max: int, cf_tol: float, stream=None):
    """Returns (I [n, n_w] numpy, depth [n] numpy)."""
    import numpy as np
    import torch
    D = msb_dim(ctx)
    n = phi.numel() // D
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    I = np.zeros((n, len(wv)), dtype=np.float64)
    depth = np.zeros(n, dtype=np.int32)
    _check(lib().msb_spectrum(ctx, ctypes.byref(system), _ptr(phi, torch.complex128, n * D, "phi"),
                              n, wv.ctypes.data_as(POINTER(c_double)), len(wv), float(eta),
                              int(lanczos_max), float(cf_tol), I.ctypes.data_as(POINTER(c_double)),
                              depth.ctypes.data_as(POINTER(c_int)), _stream_ptr(stream)))
    return I, depth


def msb_spectrum_cf(ctx, system, phi, w, eta: float, lanczos_max: int, cf_tol: float, ld: int, stream=None):
    """msb_spectrum plus its continued fraction: returns (I [n, n_w], depth [n],
    a [n, ld], b [n, ld]) with b[:, 0] = |phi| (numpy)."""
    import numpy as np
    import torch
    D = msb_dim(ctx)
    n = phi.numel() // D
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    I = np.zeros((n, len(wv)), dtype=np.float64)
    depth = np.zeros(n, dtype=np.int32)
    a = np.zeros((n, ld), dtype=np.float64)
    b = np.zeros((n, ld), dtype=np.float64)
    _check(lib().msb_spectrum_cf(ctx, ctypes.byref(system), _ptr(phi, torch.complex128, n * D, "phi"),
                                 n, wv.ctypes.data_as(POINTER(c_double)), len(wv), float(eta),
                                 int(lanczos_max), float(cf_tol), I.ctypes.data_as(POINTER(c_double)),
                                 depth.ctypes.data_as(POINTER(c_int)), a.ctypes.data_as(POINTER(c_double)),
                                 b.ctypes.data_as(POINTER(c_double)), int(ld), _stream_ptr(stream)))
    return I, depth, a, b


def msb_autotune(ctx, nsys: int, prec: int, stream=None):
    """Time every usable apply shape; returns
    [(threads, elems_per_thread, vectors, passes, row_order, ms, panel_width), ...]."""
    tab = (msb_shape * 256)()
    n = c_int(0)
    _check(lib().msb_autotune(ctx, int(nsys), int(prec), tab, 256, ctypes.byref(n), _stream_ptr(stream)))
    return [(t.threads, t.elems_per_thread, t.vectors, t.passes, t.row_order, t.ms, t.panel_width)
            for t in tab[:min(n.value, 256)]]


def msb_set_shape(ctx, nsys: int, prec: int, shape):
    """Pin the apply shape (threads, elems_per_thread, vectors[, passes[, row_order[, ms[,
    panel_width]]]]) -- an entry of msb_autotune's table; None returns to the default."""
    sh = msb_shape()
    if shape is not None:
        sh.threads, sh.elems_per_thread, sh.vectors = (int(v) for v in shape[:3])
        sh.passes = int(shape[3]) if len(shape) >= 4 else 1
        sh.row_order = int(shape[4]) if len(shape) >= 5 else 0
        sh.panel_width = int(shape[6]) if len(shape) >= 7 else 0
    _check(lib().msb_set_shape(ctx, int(nsys), int(prec), ctypes.byref(sh)))


# ---- learned form: ensemble surrogate --------------------------------------

def msb_mlp_num_params() -> int:
    return int(lib().msb_mlp_num_params())


def msb_mlp_create(members: int, in_shift, in_scale, out_scale: float) -> c_void_p:
    sh = (c_double * 6)(*[float(v) for v in in_shift])
    sc = (c_double * 6)(*[float(v) for v in in_scale])
    h = c_void_p()
    _check(lib().msb_mlp_create(int(members), sh, sc, float(out_scale), ctypes.byref(h)))
    return h


def msb_mlp_destroy(mlp):
    lib().msb_mlp_destroy(mlp)


def msb_mlp_set_params(mlp, member: int, params):
    """params: host float32 array of msb_mlp_num_params() values."""
    import numpy as np
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    if p.size != msb_mlp_num_params():
        raise ValueError("wrong parameter count")
    _check(lib().msb_mlp_set_params(mlp, int(member), p.ctypes.data_as(c_void_p)))


def msb_mlp_get_params(mlp, member: int):
    import numpy as np
    p = np.empty(msb_mlp_num_params(), dtype=np.float32)
    _check(lib().msb_mlp_get_params(mlp, int(member), p.ctypes.data_as(c_void_p)))
    return p


def msb_mlp_grad(mlp, member: int, X, T):
    """(loss, grad) of one member on device float32 X [n][6], T [n]."""
    import numpy as np
    import torch
    n = T.numel()
    _stream_ptr(None)
    g = np.empty(msb_mlp_num_params(), dtype=np.float32)
    loss = c_double()
    _check(lib().msb_mlp_grad(mlp, int(member), _ptr(X, torch.float32, n * 6, "X"), _ptr(T, torch.float32, n, "T"),
                              int(n), ctypes.byref(loss), g.ctypes.data_as(c_void_p)))
    return loss.value, g


def msb_mlp_train(mlp, X, T, perm, batch: int, steps: int, lr: float, members: int):
    """Adam steps on device X [n][6], T [n] with device int32 perm [members][steps*batch];
    returns the loss history [members][steps]."""
    import numpy as np
    import torch
    n = T.numel()
    hist = np.empty((members, steps), dtype=np.float64)
    _check(lib().msb_mlp_train(mlp, _ptr(X, torch.float32, n * 6, "X"), _ptr(T, torch.float32, n, "T"), int(n),
                               _ptr(perm, torch.int32, members * steps * batch, "perm"), int(batch), int(steps),
                               float(lr), hist.ctypes.data_as(c_void_p), _stream_ptr(None)))
    return hist


def msb_mlp_predict(mlp, X, mean, sd):
    """Ensemble mean / standard deviation at device X [n][6] into device float32 [n] tensors."""
    import torch
    n = mean.numel()
    _check(lib().msb_mlp_predict(mlp, _ptr(X, torch.float32, n * 6, "X"), int(n), _ptr(mean, torch.float32, n, "mean"),
                                 _ptr(sd, torch.float32, n, "sd"), _stream_ptr(None)))


def msb_mlp_fallback(mean, sd, frac: float):
    """Row mask of a host [n_rows][n_cols] prediction grid (numpy float32)."""
    import numpy as np
    mu = np.ascontiguousarray(np.asarray(mean, dtype=np.float32))
    s = np.ascontiguousarray(np.asarray(sd, dtype=np.float32))
    if mu.ndim != 2 or mu.shape != s.shape:
        raise ValueError("mean and sd must be matching 2-D grids")
    mask = np.empty(mu.shape[0], dtype=np.int32)
    _check(lib().msb_mlp_fallback(mu.ctypes.data_as(c_void_p), s.ctypes.data_as(c_void_p), mu.shape[0], mu.shape[1],
                                  float(frac), mask.ctypes.data_as(c_void_p)))
    return mask.astype(bool)
