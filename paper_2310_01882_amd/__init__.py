"""Python binding of libmistencil (MI355X stencil sweeps).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libmistencil.so. PyTorch supplies device memory and the current
stream. Fields are 3D tensors of shape (nz + 2, ny + 2, nx + 2) with a unit
x stride (row and plane pitch may be padded), base element = halo cell
(-1, -1, -1).

The names mirror the C ABI in include/mistencil.h: stencil_apply,
residual_norm, jacobi_sweeps, jacobi_solve, advect_source.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
# MS_LIB_PATH selects another build of the same library (the host-sanitizer
# build of sanitize.py); the default is the in-tree library.
LIB_PATH = os.environ.get("MS_LIB_PATH") or os.path.join(_HERE, "libmistencil.so")

MS_OK = 0
MS_NOT_CONVERGED = 1
MS_EINVAL = -1
MS_EUNSUPPORTED = -2
MS_EHIP = -3
MS_EWORKSPACE = -4
MS_ENONFINITE = -5

MS_F64 = 0
MS_F32 = 1
MS_SOLVE_F64 = 0
MS_SOLVE_F32_REFINED = 1
MS_METHOD_JACOBI = 0
MS_METHOD_RBGS = 1
MS_JIT_FIELD, MS_JIT_PARAM, MS_JIT_PROFILE, MS_JIT_OUTPUT = 0, 1, 2, 3
MS_START_RESIDUAL, MS_START_SLOW_MODES, MS_START_FORCE = 0, 1, 2


class MsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("sy", ctypes.c_int64), ("sz", ctypes.c_int64)]


class Tap(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_int8), ("dy", ctypes.c_int8), ("dz", ctypes.c_int8),
                ("reserved", ctypes.c_int8 * 5), ("w", ctypes.c_double)]


class Stencil(ctypes.Structure):
    _fields_ = [("ntaps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("taps", ctypes.POINTER(Tap)), ("rhs_coef", ctypes.c_double),
                ("scale", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_sweeps", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("inner_eta", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("max_inner", ctypes.c_int32), ("stall_window", ctypes.c_int32),
                ("temporal_block", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("method", ctypes.c_int32)]


class SolveResult(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("outer_iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("rel_final", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("vec_ok", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("wx", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("target_blocks", ctypes.c_int64), ("us_per_sweep", ctypes.c_double)]


class Instance(ctypes.Structure):
    _fields_ = [("grid", Grid), ("x", ctypes.c_void_p), ("f", ctypes.c_void_p)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("team", ctypes.c_int32), ("tx", ctypes.c_int32),
                ("zsplit", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("us_per_sweep", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes); every symbol include/mistencil.h declares.
SIGNATURES = {
    "ms_last_error": (ctypes.c_char_p, []),
    "ms_version": (ctypes.c_char_p, []),
    "stencil_apply": (_I, [ctypes.POINTER(Stencil), ctypes.POINTER(Grid), _I, _P, _P, _P, _P]),
    "residual_workspace_bytes": (_SZ, [ctypes.POINTER(Grid)]),
    "residual_norm": (_I, [ctypes.POINTER(Grid), _I, _P, _P, ctypes.POINTER(_D), _I, _P, _SZ, _P]),
    "jacobi_sweeps_workspace_bytes": (_SZ, [ctypes.POINTER(Grid)]),
    "jacobi_sweeps": (_I, [ctypes.POINTER(Grid), _I, _P, _P, _P, _I64, _P, _P, _SZ, _P]),
    "jacobi_sweeps_tb": (_I, [ctypes.POINTER(Grid), _I, _P, _P, _P, _I64, _I, _P, _P, _SZ, _P]),
    "jacobi_sweeps_noalloc_scratch_bytes": (_SZ, []),
    "jacobi_sweeps_noalloc": (_I, [ctypes.POINTER(Grid), _I, _P, _P, _P, _I64, _I, _P, _P]),
    "rbgs_sweeps": (_I, [ctypes.POINTER(Grid), _I, _P, _P, _P, _I64, _P, _P, _SZ, _P]),
    "jacobi_sweeps_streamed_workspace_bytes": (_SZ, [ctypes.POINTER(Grid), _I, _I, _I]),
    "jacobi_sweeps_streamed": (_I, [ctypes.POINTER(Grid), _I, _P, _P, _P, _I64, _I, _I, _P, _SZ,
                                    _P]),
    "ms_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "jacobi_workspace_bytes": (_SZ, [ctypes.POINTER(Grid), ctypes.POINTER(SolveOpts)]),
    "jacobi_solve": (_I, [ctypes.POINTER(Grid), ctypes.POINTER(SolveOpts), _P, _P, _P, _SZ,
                          ctypes.POINTER(_D), ctypes.POINTER(SolveResult), _P]),
    "advect_source": (_I, [ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _D, _D, _P, _P, _P, _P]),
    "jacobi_batched_workspace_bytes": (_SZ, [_I, ctypes.POINTER(Instance),
                                             ctypes.POINTER(SolveOpts)]),
    "jacobi_solve_batched": (_I, [_I, ctypes.POINTER(Instance), ctypes.POINTER(SolveOpts), _P,
                                  _SZ, ctypes.POINTER(SolveResult), _P]),
    "jacobi_batched_plan_workspace_bytes": (_SZ, [_I]),
    "jacobi_batched_streams_workspace_bytes": (_SZ, [_I, ctypes.POINTER(Instance),
                                                     ctypes.POINTER(SolveOpts), _I]),
    "jacobi_solve_batched_streams": (_I, [_I, ctypes.POINTER(Instance), ctypes.POINTER(SolveOpts),
                                          _I, _P, _SZ, ctypes.POINTER(SolveResult), _P]),
    "jacobi_batched_plan_from_estimates": (_I, [_I, ctypes.POINTER(Grid), ctypes.POINTER(_D),
                                                _I, _I, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]),
    "jacobi_batched_plan": (_I, [_I, ctypes.POINTER(Instance), ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_D), _P, _SZ,
                                 _P]),
    "ms_autotune_sweeps": (_I, [ctypes.POINTER(Grid), _I, _P, _P, _P, _I, _P, _SZ,
                                ctypes.POINTER(Tuning), _P]),
    "ms_sweep_shape": (_I, [ctypes.POINTER(Grid), _I, ctypes.POINTER(ctypes.c_void_p), _I,
                            ctypes.POINTER(Tuning)]),
    "ms_tuning_get": (_I, [ctypes.POINTER(Tuning), _I]),
    "ms_tuning_set": (_I, [ctypes.POINTER(Tuning), _I]),
    "ms_tuning_clear": (None, []),
    "jacobi_batched_autotune_workspace_bytes": (_SZ, [_I, ctypes.POINTER(Instance),
                                                      ctypes.POINTER(SolveOpts)]),
    "jacobi_batched_autotune": (_I, [_I, ctypes.POINTER(Instance), ctypes.POINTER(SolveOpts), _I,
                                     _P, _SZ, ctypes.POINTER(BatchTuning), _P]),
    "ms_batch_tuning_get": (_I, [ctypes.POINTER(BatchTuning), _I]),
    "ms_batch_tuning_set": (_I, [ctypes.POINTER(BatchTuning), _I]),
    "ms_batch_tuning_clear": (None, []),
    "conv3d_bf16_fwd": (_I, [_I, _I, _I, _I, _P, _P, _P, _P, _P, _I, _P]),
    "conv3d_bf16_dgrad": (_I, [_I, _I, _I, _I, _P, _P, _P, _P, _P]),
    "conv3d_bf16_wgrad_workspace_bytes": (_SZ, [_I]),
    "conv3d_bf16_wgrad": (_I, [_I, _I, _I, _I, _P, _P, _P, _P, _P, _SZ, _P]),
    "cnn_mse_grad": (_I, [_I, _I, _I, _P, _P, _P, _P, _I, _P]),
    "cnn_adam": (_I, [_I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_float, _I, _P]),
    "cnn_pack_weights": (_I, [_I, _P, _P, _P, _P]),
    "cnn_features_workspace_bytes": (_SZ, [ctypes.POINTER(Grid)]),
    "cnn_features": (_I, [ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _SZ, _P]),
    "cnn_guess": (_I, [ctypes.POINTER(Grid), _P, _P, _D, _P, _P]),
    "cnn_target": (_I, [ctypes.POINTER(Grid), _P, _P, _D, _P, _P]),
    "ms_stream_probe": (_I, [_P, _P, _P, _I64, _I, _I, _P]),
    "warmstart_params_floats": (_SZ, []),
    "warmstart_params_bytes": (_SZ, []),
    "warmstart_layer_offset": (_SZ, [_I]),
    "warmstart_workspace_bytes": (_SZ, [ctypes.POINTER(Grid), _I]),
    "warmstart_forward": (_I, [ctypes.POINTER(Grid), _P, _P, _P, _D, _I, _I, _P, _P, _SZ, _P, _P,
                               _P]),
    "warmstart_train_step": (_I, [ctypes.POINTER(Grid), _P, _P, _P, _P, _D, ctypes.c_float, _I,
                                  _P, _SZ, _P, _P]),
    "ms_jit_compile": (_I, [ctypes.c_char_p, _I, ctypes.POINTER(_P)]),
    "ms_jit_apply": (_I, [_P, ctypes.POINTER(Grid), ctypes.POINTER(_P), _I, ctypes.POINTER(_D),
                          _I, ctypes.POINTER(_P), _I, ctypes.POINTER(_P), _I, _P]),
    "ms_jit_signature": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                              ctypes.POINTER(_I)]),
    "ms_jit_name": (ctypes.c_char_p, [_P, _I, _I]),
    "ms_jit_source": (ctypes.c_char_p, [_P]),
    "ms_jit_free": (None, [_P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python paper_2310_01882_amd/build.py). "
            "There is no fallback implementation.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return (lib.ms_last_error() or b"").decode()


def _check(rc: int, allow=(MS_OK,)):
    if rc not in allow:
        raise MsError(rc, last_error())
    return rc


# ------------------------------------------------------------------ helpers

def _field_check(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dim() != 3:
        raise ValueError(f"{name} must be 3D (nz+2, ny+2, nx+2)")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.stride(2) != 1:
        raise ValueError(f"{name} must have unit x stride")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


def grid_of(t: torch.Tensor) -> Grid:
    nz2, ny2, nx2 = t.shape
    return Grid(nx2 - 2, ny2 - 2, nz2 - 2, 0, t.stride(1), t.stride(0))


def _same_layout(a: torch.Tensor, b: torch.Tensor, names: str):
    if a.shape != b.shape or a.stride() != b.stride():
        raise ValueError(f"{names} must share shape and strides")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return MS_F64
    if t.dtype == torch.float32:
        return MS_F32
    raise TypeError("fields must be float64 or float32")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def alloc_field(nx: int, ny: int, nz: int, dtype=torch.float64, device="cuda",
                fill=0.0) -> torch.Tensor:
    """Allocate a halo-padded field whose interior rows start on 128-byte
    boundaries: the row and plane pitch are rounded up to 128 bytes and the
    base (halo cell (-1, -1, -1)) sits one element before a boundary, so
    every 64-lane row access of a sweep covers whole cache lines."""
    esz = torch.tensor([], dtype=dtype).element_size()
    a = 128 // esz
    sy = -(-(nx + 2) // a) * a
    sz = sy * (ny + 2)
    sz = -(-sz // a) * a
    span = (nz + 1) * sz + (ny + 1) * sy + nx + 2
    store = torch.empty(a - 1 + span, dtype=dtype, device=device)
    t = store.as_strided((nz + 2, ny + 2, nx + 2), (sz, sy, 1), a - 1)
    if fill is not None:
        t.fill_(fill)
    return t


def field_from(arr, dtype=None, device="cuda") -> torch.Tensor:
    """Copy a (nz+2, ny+2, nx+2) host array into an aligned device field."""
    src = torch.as_tensor(arr)
    if dtype is not None:
        src = src.to(dtype)
    nz2, ny2, nx2 = src.shape
    t = alloc_field(nx2 - 2, ny2 - 2, nz2 - 2, src.dtype, device, fill=None)
    t.copy_(src)
    return t


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# --------------------------------------------------------------- entry points

def stencil_apply(taps, inp, out, rhs=None, rhs_coef=0.0, scale=1.0, stream=None):
    """out[p] = scale * (sum_t w_t in[p + o_t] (in tap order) + rhs_coef * rhs[p]).

    ``taps`` is a sequence of (dx, dy, dz, w)."""
    _field_check(inp, "inp")
    _field_check(out, "out", inp.dtype)
    _same_layout(inp, out, "inp/out")
    if rhs is not None:
        _field_check(rhs, "rhs", inp.dtype)
        _same_layout(inp, rhs, "inp/rhs")
    arr = (Tap * max(len(taps), 1))()
    for n, (dx, dy, dz, w) in enumerate(taps):
        arr[n].dx, arr[n].dy, arr[n].dz, arr[n].w = int(dx), int(dy), int(dz), float(w)
    st = Stencil(len(taps), 0, arr, float(rhs_coef), float(scale))
    g = grid_of(inp)
    _check(lib.stencil_apply(ctypes.byref(st), ctypes.byref(g), _dtype_code(inp), _ptr(inp),
                             _ptr(rhs), _ptr(out), _stream(stream)))
    return out


def residual_norm(u, f=None, out=None, stream=None) -> float:
    """||f - L(u)||_2 over the interior (FP64 accumulation). With ``out`` (a
    1-element float64 device tensor) the result stays on the device."""
    _field_check(u, "u")
    if f is not None:
        _field_check(f, "f", u.dtype)
        _same_layout(u, f, "u/f")
    g = grid_of(u)
    ws = _workspace(lib.residual_workspace_bytes(ctypes.byref(g)), u.device)
    if out is not None:
        _check(lib.residual_norm(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(f),
                                 ctypes.cast(ctypes.c_void_p(out.data_ptr()), ctypes.POINTER(_D)),
                                 1, _ptr(ws), ws.numel(), _stream(stream)))
        return out
    val = ctypes.c_double(0.0)
    _check(lib.residual_norm(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(f),
                             ctypes.byref(val), 0, _ptr(ws), ws.numel(), _stream(stream)))
    return val.value


def jacobi_sweeps_workspace(u) -> torch.Tensor:
    g = grid_of(u)
    return _workspace(lib.jacobi_sweeps_workspace_bytes(ctypes.byref(g)), u.device)


def jacobi_sweeps(u, u_tmp, n, f=None, res=None, work=None, stream=None, temporal_block=1):
    """Exactly ``n`` Jacobi sweeps with ping-pong buffers; returns the buffer
    holding u_n (``u`` if the number of passes is even, else ``u_tmp``).
    ``res`` (float64 device tensor of n + 1 entries, optional) receives
    ||r(u_k)||, k = 0..n. ``temporal_block`` = 2 fuses two sweeps per pass."""
    _field_check(u, "u")
    _field_check(u_tmp, "u_tmp", u.dtype)
    _same_layout(u, u_tmp, "u/u_tmp")
    if f is not None:
        _field_check(f, "f", u.dtype)
        _same_layout(u, f, "u/f")
    if res is not None and (res.dtype != torch.float64 or res.numel() < n + 1):
        raise ValueError("res must be float64 with n + 1 entries")
    g = grid_of(u)
    if work is None:
        work = jacobi_sweeps_workspace(u)
    tb = int(temporal_block)
    if tb == 1:
        _check(lib.jacobi_sweeps(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(u_tmp), _ptr(f),
                                 int(n), _ptr(res), _ptr(work), work.numel(), _stream(stream)))
        passes = n
    else:
        _check(lib.jacobi_sweeps_tb(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(u_tmp),
                                    _ptr(f), int(n), tb, _ptr(res), _ptr(work), work.numel(),
                                    _stream(stream)))
        passes = n // 2 + n % 2
    return u if passes % 2 == 0 else u_tmp


def stream_probe(a, out, b=None, blocks=2048, form=0, stream=None):
    """ms_stream_probe: out = a (+ b) over float64 device tensors."""
    for t, name in ((a, "a"), (out, "out"), (b, "b")):
        if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if out.numel() != a.numel() or (b is not None and b.numel() != a.numel()):
        raise ValueError("a, b and out must have the same size")
    _check(lib.ms_stream_probe(_ptr(a), _ptr(b), _ptr(out), a.numel(), int(blocks), int(form),
                               _stream(stream)))
    return out


def jacobi_sweeps_noalloc(u, u_tmp, n, f=None, res=None, stream=None, temporal_block=1):
    """``jacobi_sweeps`` through the entry point that allocates nothing: the
    residual partials live in the library's fixed per-device array, so calls
    that overlap in time on one GPU race. Same arguments (no ``work``), same
    results, same returned buffer."""
    _field_check(u, "u")
    _field_check(u_tmp, "u_tmp", u.dtype)
    _same_layout(u, u_tmp, "u/u_tmp")
    if f is not None:
        _field_check(f, "f", u.dtype)
        _same_layout(u, f, "u/f")
    if res is not None and (res.dtype != torch.float64 or res.numel() < n + 1):
        raise ValueError("res must be float64 with n + 1 entries")
    g = grid_of(u)
    tb = int(temporal_block)
    _check(lib.jacobi_sweeps_noalloc(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(u_tmp),
                                     _ptr(f), int(n), tb, _ptr(res), _stream(stream)))
    passes = n if tb == 1 else n // 2 + n % 2
    return u if passes % 2 == 0 else u_tmp


def rbgs_sweeps(u, u_tmp, n, f=None, res=None, work=None, stream=None):
    """Exactly ``n`` red-black Gauss-Seidel sweeps with ping-pong buffers;
    returns the buffer holding u_n (``u`` if n is even, else ``u_tmp``).
    ``res`` (float64 device tensor of n + 1 entries, optional) receives
    ||r(u_k)||, k = 0..n."""
    _field_check(u, "u")
    _field_check(u_tmp, "u_tmp", u.dtype)
    _same_layout(u, u_tmp, "u/u_tmp")
    if f is not None:
        _field_check(f, "f", u.dtype)
        _same_layout(u, f, "u/f")
    if res is not None and (res.dtype != torch.float64 or res.numel() < n + 1):
        raise ValueError("res must be float64 with n + 1 entries")
    g = grid_of(u)
    if work is None:
        work = jacobi_sweeps_workspace(u)
    _check(lib.rbgs_sweeps(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(u_tmp), _ptr(f), int(n),
                           _ptr(res), _ptr(work), work.numel(), _stream(stream)))
    return u if n % 2 == 0 else u_tmp


def jacobi_sweeps_streamed(u, u_tmp, n, f=None, sweeps_per_pass=16, slab_planes=64,
                           work=None, stream=None):
    """Exactly ``n`` Jacobi sweeps of a field held in host memory (``u``,
    ``u_tmp``, ``f``: CPU tensors of one layout, pinned for overlap), in z
    slabs of ``slab_planes`` planes with ``sweeps_per_pass`` sweeps per trip
    through the device; returns the tensor holding u_n."""
    for name, t in (("u", u), ("u_tmp", u_tmp)) + ((("f", f),) if f is not None else ()):
        if t.device.type != "cpu" or t.dim() != 3 or t.stride(2) != 1:
            raise ValueError(f"{name} must be a 3-D host tensor with unit x stride")
        if t.dtype != u.dtype or t.shape != u.shape or t.stride() != u.stride():
            raise ValueError(f"{name} must share u's dtype, shape and strides")
    g = grid_of(u)
    code = MS_F64 if u.dtype == torch.float64 else MS_F32
    if work is None:
        nbytes = lib.jacobi_sweeps_streamed_workspace_bytes(ctypes.byref(g), code,
                                                            int(sweeps_per_pass), int(slab_planes))
        if nbytes == 0:
            raise MsError(MS_EINVAL, last_error())
        work = _workspace(nbytes, torch.device("cuda"))
    _check(lib.jacobi_sweeps_streamed(ctypes.byref(g), code, _ptr(u), _ptr(u_tmp), _ptr(f), int(n),
                                      int(sweeps_per_pass), int(slab_planes), _ptr(work),
                                      work.numel(), _stream(stream)))
    passes = -(-int(n) // min(int(sweeps_per_pass), u.shape[0] - 2)) if n > 0 else 0
    return u if passes % 2 == 0 else u_tmp


@dataclass
class SolveInfo:
    status: int
    sweeps: int
    outer_iters: int
    res0: float
    res_final: float
    rel_final: float
    hist: list
    seconds: float = 0.0


def solve_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib.ms_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, v)
    return o


def jacobi_workspace(u, opts: SolveOpts) -> torch.Tensor:
    g = grid_of(u)
    n = lib.jacobi_workspace_bytes(ctypes.byref(g), ctypes.byref(opts))
    if n == 0:
        raise MsError(MS_EINVAL, last_error())
    return _workspace(n, u.device)


def jacobi_solve(u, f=None, work=None, want_hist=False, stream=None, **opts) -> SolveInfo:
    """Convergence-controlled solve of L(u) = f; ``u`` (float64) holds the
    initial guess and Dirichlet halo on entry and the answer on return.
    Keyword options map onto ms_solve_opts (rel_tol, max_sweeps, precision,
    check_every, inner_eta, max_outer, max_inner, stall_window,
    temporal_block, use_graph, method)."""
    _field_check(u, "u", torch.float64)
    if f is not None:
        _field_check(f, "f", torch.float64)
        _same_layout(u, f, "u/f")
    o = solve_opts(**opts)
    g = grid_of(u)
    if work is None:
        work = jacobi_workspace(u, o)
    hist = None
    if want_hist:
        n = (o.max_sweeps + 1) if o.precision == MS_SOLVE_F64 else (o.max_outer + 1)
        hist = (ctypes.c_double * int(n))()
    r = SolveResult()
    rc = lib.jacobi_solve(ctypes.byref(g), ctypes.byref(o), _ptr(u), _ptr(f), _ptr(work),
                          work.numel(), hist, ctypes.byref(r), _stream(stream))
    _check(rc, allow=(MS_OK, MS_NOT_CONVERGED))
    h = []
    if want_hist:
        cnt = (r.sweeps + 1) if o.precision == MS_SOLVE_F64 else (r.outer_iters + 1)
        h = list(hist[:cnt])
    return SolveInfo(rc, r.sweeps, r.outer_iters, r.res0, r.res_final, r.rel_final, h, r.seconds)


def advect_source(u, v, w, tzc1, tzc2, tcx, tcy, su, sv, sw, stream=None):
    """Fused three-field advection source term (FP64); outputs su, sv, sw."""
    for name, t in (("u", u), ("v", v), ("w", w), ("su", su), ("sv", sv), ("sw", sw)):
        _field_check(t, name, torch.float64)
        _same_layout(u, t, f"u/{name}")
    nz = u.shape[0] - 2
    for name, t in (("tzc1", tzc1), ("tzc2", tzc2)):
        if t.dtype != torch.float64 or t.numel() != nz or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name} must be a contiguous float64 device vector of length nz")
    g = grid_of(u)
    _check(lib.advect_source(ctypes.byref(g), _ptr(u), _ptr(v), _ptr(w), _ptr(tzc1), _ptr(tzc2),
                             float(tcx), float(tcy), _ptr(su), _ptr(sv), _ptr(sw), _stream(stream)))
    return su, sv, sw


def _instances(xs, fs):
    if len(xs) != len(fs):
        raise ValueError("xs and fs must have the same length")
    arr = (Instance * len(xs))()
    for n, (x, f) in enumerate(zip(xs, fs)):
        _field_check(x, f"xs[{n}]", torch.float64)
        if f is not None:
            _field_check(f, f"fs[{n}]", torch.float64)
            _same_layout(x, f, f"xs[{n}]/fs[{n}]")
        arr[n].grid = grid_of(x)
        arr[n].x = x.data_ptr()
        arr[n].f = f.data_ptr() if f is not None else None
    return arr


def jacobi_solve_batched_streams(xs, fs, workers=4, work=None, stream=None, **opts):
    """Solve every instance as jacobi_solve would, on ``workers`` concurrent
    streams (largest estimated work first). Returns a SolveInfo per
    instance; raises MsError on errors other than non-convergence."""
    arr = _instances(xs, fs)
    o = solve_opts(**opts)
    if work is None:
        nbytes = lib.jacobi_batched_streams_workspace_bytes(len(xs), arr, ctypes.byref(o),
                                                            int(workers))
        if nbytes == 0:
            raise MsError(MS_EINVAL, last_error())
        work = _workspace(nbytes, xs[0].device)
    res = (SolveResult * len(xs))()
    rc = lib.jacobi_solve_batched_streams(len(xs), arr, ctypes.byref(o), int(workers), _ptr(work),
                                          work.numel(), res, _stream(stream))
    _check(rc, allow=(MS_OK, MS_NOT_CONVERGED))
    return [SolveInfo(r.status, r.sweeps, r.outer_iters, r.res0, r.res_final, r.rel_final, [],
                      r.seconds) for r in res]


def batched_plan_from_estimates(dims, est_sweeps, blocks, precision=MS_SOLVE_F32_REFINED):
    """The batched planner alone, on the host: (team sizes, groups, grid
    blocks) for instances of interior extents ``dims`` ((nx, ny, nz) each)
    with the given sweep estimates on ``blocks`` resident blocks."""
    n = len(dims)
    grids = (Grid * n)(*[Grid(nx, ny, nz, 0, nx + 2, (nx + 2) * (ny + 2)) for nx, ny, nz in dims])
    est = (_D * n)(*[float(e) for e in est_sweeps])
    teams = (ctypes.c_int * n)()
    groups = (ctypes.c_int * n)()
    g = ctypes.c_int(0)
    _check(lib.jacobi_batched_plan_from_estimates(n, grids, est, int(blocks), int(precision),
                                                  teams, groups, ctypes.byref(g)))
    return list(teams), list(groups), g.value


def batched_plan(xs, fs, stream=None, with_estimates=False, with_groups=False, **opts):
    """(team sizes, grid blocks) the batched solve would use; with
    ``with_estimates`` also the per-instance sweep estimates it plans with
    (from one device pass over the instances), and with ``with_groups`` the
    index of the team that runs each instance (a team runs its instances one
    after the other)."""
    arr = _instances(xs, fs)
    o = solve_opts(**opts)
    teams = (ctypes.c_int * len(xs))()
    groups = (ctypes.c_int * len(xs))()
    est = (_D * len(xs))()
    g = ctypes.c_int(0)
    work = _workspace(lib.jacobi_batched_plan_workspace_bytes(len(xs)), xs[0].device)
    _check(lib.jacobi_batched_plan(len(xs), arr, ctypes.byref(o), teams, groups,
                                   ctypes.byref(g), est, _ptr(work), work.numel(),
                                   _stream(stream)))
    out = [list(teams), g.value]
    if with_estimates:
        out.append(list(est))
    if with_groups:
        out.append(list(groups))
    return tuple(out)


def jacobi_solve_batched(xs, fs, work=None, stream=None, **opts):
    """Solve every instance (xs[i]: float64 field, initial guess + halo; fs[i]:
    right-hand side or None) in one persistent launch. Returns a SolveInfo per
    instance; raises MsError on errors other than non-convergence."""
    arr = _instances(xs, fs)
    o = solve_opts(**opts)
    if work is None:
        nbytes = lib.jacobi_batched_workspace_bytes(len(xs), arr, ctypes.byref(o))
        if nbytes == 0:
            raise MsError(MS_EINVAL, last_error())
        work = _workspace(nbytes, xs[0].device)
    res = (SolveResult * len(xs))()
    rc = lib.jacobi_solve_batched(len(xs), arr, ctypes.byref(o), _ptr(work), work.numel(), res,
                                  _stream(stream))
    _check(rc, allow=(MS_OK, MS_NOT_CONVERGED))
    return [SolveInfo(r.status, r.sweeps, r.outer_iters, r.res0, r.res_final, r.rel_final, [],
                      r.seconds) for r in res]


# ------------------------------------------------------------------ tuning

_TUNING_FIELDS = [name for name, _ in Tuning._fields_]


def autotune_sweeps(u, u_tmp, f=None, sweeps_per_trial=10, stream=None) -> dict:
    """Time every sweep tile shape on (scratch) fields laid out like the real
    ones, keep the fastest for this grid, dtype and alignment, return it."""
    _field_check(u, "u")
    _field_check(u_tmp, "u_tmp", u.dtype)
    _same_layout(u, u_tmp, "u/u_tmp")
    if f is not None:
        _field_check(f, "f", u.dtype)
        _same_layout(u, f, "u/f")
    g = grid_of(u)
    work = jacobi_sweeps_workspace(u)
    best = Tuning()
    _check(lib.ms_autotune_sweeps(ctypes.byref(g), _dtype_code(u), _ptr(u), _ptr(u_tmp), _ptr(f),
                                  int(sweeps_per_trial), _ptr(work), work.numel(),
                                  ctypes.byref(best), _stream(stream)))
    return {k: getattr(best, k) for k in _TUNING_FIELDS}


def sweep_shape(*fields) -> dict:
    """The tile shape a sweep over these fields (same grid and dtype) would
    launch with: the tuned entry for their grid and alignment if there is
    one, else the default (vec_ok is the widest lane the alignment allows)."""
    for i, t in enumerate(fields):
        _field_check(t, f"fields[{i}]", fields[0].dtype)
        _same_layout(fields[0], t, "fields")
    arr = (ctypes.c_void_p * len(fields))(*[t.data_ptr() for t in fields])
    out = Tuning()
    g = grid_of(fields[0])
    _check(lib.ms_sweep_shape(ctypes.byref(g), _dtype_code(fields[0]), arr, len(fields),
                              ctypes.byref(out)))
    return {k: getattr(out, k) for k in _TUNING_FIELDS}


def tuning_table() -> list:
    n = lib.ms_tuning_get(None, 0)
    arr = (Tuning * max(n, 1))()
    lib.ms_tuning_get(arr, n)
    return [{k: getattr(arr[i], k) for k in _TUNING_FIELDS} for i in range(n)]


def tuning_load(entries) -> None:
    arr = (Tuning * max(len(entries), 1))()
    for i, e in enumerate(entries):
        for k in _TUNING_FIELDS:
            setattr(arr[i], k, e[k])
    _check(lib.ms_tuning_set(arr, len(entries)))


def tuning_save_json(path) -> None:
    import json
    with open(path, "w") as fh:
        json.dump(tuning_table(), fh, indent=1)


def tuning_load_json(path) -> None:
    import json
    with open(path) as fh:
        tuning_load(json.load(fh))


def tuning_clear() -> None:
    lib.ms_tuning_clear()


_BATCH_TUNING_FIELDS = [name for name, _ in BatchTuning._fields_ if name != "reserved"]


def batched_autotune(xs, fs, sweeps_per_trial=20, work=None, stream=None, **opts) -> list:
    """Time every batched tile shape on this batch (the xs are not touched),
    keep each instance's fastest for later batched solves with the same
    options, and return them (one dict per instance)."""
    arr = _instances(xs, fs)
    o = solve_opts(**opts)
    if work is None:
        nbytes = lib.jacobi_batched_autotune_workspace_bytes(len(xs), arr, ctypes.byref(o))
        if nbytes == 0:
            raise MsError(MS_EINVAL, last_error())
        work = _workspace(nbytes, xs[0].device)
    best = (BatchTuning * len(xs))()
    _check(lib.jacobi_batched_autotune(len(xs), arr, ctypes.byref(o), int(sweeps_per_trial),
                                       _ptr(work), work.numel(), best, _stream(stream)))
    return [{k: getattr(b, k) for k in _BATCH_TUNING_FIELDS} for b in best]


def batch_tuning_table() -> list:
    n = lib.ms_batch_tuning_get(None, 0)
    arr = (BatchTuning * max(n, 1))()
    lib.ms_batch_tuning_get(arr, n)
    return [{k: getattr(arr[i], k) for k in _BATCH_TUNING_FIELDS} for i in range(n)]


def batch_tuning_load(entries) -> None:
    arr = (BatchTuning * max(len(entries), 1))()
    for i, e in enumerate(entries):
        for k in _BATCH_TUNING_FIELDS:
            setattr(arr[i], k, e.get(k, 0.0) if k == "us_per_sweep" else e[k])
    _check(lib.ms_batch_tuning_set(arr, len(entries)))


def batch_tuning_clear() -> None:
    lib.ms_batch_tuning_clear()


# ------------------------------------------------- runtime-compiled stencils

class JitStencil:
    """A stencil program compiled for the device (ms_jit_compile); the
    language is described in include/mistencil.h. ``fields``, ``params``,
    ``profiles`` and ``outputs`` list the declared names in argument order;
    ``source`` is the generated HIP source."""

    def __init__(self, program: str, dtype=torch.float64):
        if dtype not in (torch.float64, torch.float32):
            raise ValueError("dtype must be float64 or float32")
        self.dtype = dtype
        self._lib = lib
        h = _P()
        _check(lib.ms_jit_compile(program.encode(), MS_F64 if dtype == torch.float64 else MS_F32,
                                  ctypes.byref(h)))
        self._h = h
        n = [_I() for _ in range(4)]
        _check(lib.ms_jit_signature(h, *[ctypes.byref(x) for x in n]))
        self.fields, self.params, self.profiles, self.outputs = (
            [lib.ms_jit_name(h, kind, i).decode() for i in range(c.value)]
            for kind, c in zip((MS_JIT_FIELD, MS_JIT_PARAM, MS_JIT_PROFILE, MS_JIT_OUTPUT), n))
        self.source = lib.ms_jit_source(h).decode()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ms_jit_free(h)
            self._h = None

    def apply(self, fields, outputs, params=(), profiles=(), stream=None):
        """Run the program: ``fields`` and ``outputs`` are device fields of
        one layout (the program's dtype), ``params`` floats, ``profiles``
        contiguous device vectors of nz values; each in declaration order."""
        fields, outputs = list(fields), list(outputs)
        if not outputs:
            raise ValueError("no outputs")
        ref = outputs[0]
        for n, t in enumerate(fields):
            _field_check(t, f"fields[{n}]", self.dtype)
            _same_layout(ref, t, f"outputs[0]/fields[{n}]")
        for n, t in enumerate(outputs):
            _field_check(t, f"outputs[{n}]", self.dtype)
            _same_layout(ref, t, f"outputs[0]/outputs[{n}]")
        nz = ref.shape[0] - 2
        for n, t in enumerate(profiles):
            if (t.dtype != self.dtype or t.numel() != nz or not t.is_contiguous()
                    or t.device.type != "cuda"):
                raise ValueError(f"profiles[{n}] must be a contiguous device vector of nz values "
                                 "in the program's dtype")
        g = grid_of(ref)
        fa = (_P * max(len(fields), 1))(*[t.data_ptr() for t in fields])
        pa = (_D * max(len(params), 1))(*[float(x) for x in params])
        qa = (_P * max(len(profiles), 1))(*[t.data_ptr() for t in profiles])
        oa = (_P * len(outputs))(*[t.data_ptr() for t in outputs])
        _check(lib.ms_jit_apply(self._h, ctypes.byref(g), fa, len(fields), pa, len(params), qa,
                                len(profiles), oa, len(outputs), _stream(stream)))
        return outputs
