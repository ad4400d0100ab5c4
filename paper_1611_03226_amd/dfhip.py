"""Thin Python binding of libdfhip.so: one function per C entry point, same
names, argument marshalling only (numpy arrays for host buffers, torch
tensors for device buffers, torch streams for HIP streams).  Every call
raises DFError on a non-zero status.  All computation happens in the HIP
library; if it is not built, importing this module fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfhip.so")

DF_OK, DF_EINVAL, DF_EAGAIN, DF_ENOMEM, DF_ESTATE, DF_EDEVICE, DF_ECONTROL, DF_EINDEX = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "DF_OK", -1: "DF_EINVAL", -2: "DF_EAGAIN", -3: "DF_ENOMEM", -4: "DF_ESTATE",
                -5: "DF_EDEVICE", -6: "DF_ECONTROL", -7: "DF_EINDEX"}
DF_C64, DF_U8, DF_I32, DF_I64 = 1, 2, 3, 4
DF_ACTOR_DPD, DF_ACTOR_MOTION, DF_ACTOR_GAUSS5, DF_ACTOR_THRES, DF_ACTOR_MED5 = 1, 2, 3, 4, 5
DF_DPD_CTRL, DF_DPD_IN, DF_DPD_OUT = 0, 1, 2
DF_MD_CUR, DF_MD_PREV, DF_MD_MASK, DF_MD_INDEX = 0, 1, 2, 3
DF_GAUSS_IN, DF_GAUSS_OUT, DF_GAUSS_OUT2 = 0, 1, 2
DF_THRES_CUR, DF_THRES_PREV, DF_THRES_OUT = 0, 1, 2
DF_MED_IN, DF_MED_OUT = 0, 1
DF_HIST_BRANCH, DF_HIST_SHARED = 0, 1
DF_FIRE_PARTIAL = 1
DF_FIRE_PERSISTENT, DF_FIRE_GRAPH = 1, 2
DF_PIPE_SEPARATE = 2
DF_CTRL_COUNT, DF_CTRL_MASK = 0, 1

_NP_DTYPE = {DF_C64: np.complex64, DF_U8: np.uint8, DF_I32: np.int32, DF_I64: np.int64}


class DFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class DpdParams(C.Structure):
    _fields_ = [("n_branches_max", C.c_int32), ("n_taps", C.c_int32), ("firing_size", C.c_int64),
                ("coeffs", C.c_void_p), ("coeffs_on_device", C.c_int32), ("history_mode", C.c_int32),
                ("control_mode", C.c_int32), ("reserved", C.c_int32)]


class MotionParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("diff_threshold", C.c_int32),
                ("min_changed_permille", C.c_int32), ("self_delay", C.c_int32)]


class FrameParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("rate", C.c_int32), ("threshold", C.c_int32)]


_P = C.c_void_p
_I32, _I64 = C.c_int32, C.c_int64
_SIGS = {
    "df_graph_create": ([C.POINTER(_P), C.c_int, _P], _I32),
    "df_graph_destroy": ([_P], _I32),
    "df_sync": ([_P], _I32),
    "df_last_error": ([_P], C.c_char_p),
    "df_version": ([], C.c_char_p),
    "df_fifo_create": ([_P, C.c_int, _I64, _I64, _I64, _P, C.POINTER(_I32)], _I32),
    "df_fifo_status": ([_P, _I32, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)], _I32),
    "df_fifo_create_paper": ([_P, C.c_int, _I64, _I64, _I64, _P, C.POINTER(_I32)], _I32),
    "df_fifo_bytes": ([_P, _I32], _I64),
    "df_debug_read_slots": ([_P, _I32, _P, _I64], _I32),
    "df_fifo_info": ([_P, _I32, C.POINTER(_I32), C.POINTER(_I64), C.POINTER(_I64)], _I32),
    "df_port_rate": ([_P, _I32, _I32, C.POINTER(_I64)], _I32),
    "df_actor_create": ([_P, C.c_int, _P, C.c_size_t, C.POINTER(_I32)], _I32),
    "df_connect": ([_P, _I32, _I32, _I32], _I32),
    "df_push": ([_P, _I32, _P, _I64, C.c_int], _I32),
    "df_pop": ([_P, _I32, _P, _I64, C.c_int, C.POINTER(_I64)], _I32),
    "df_fire": ([_P, _I32, _I64, C.c_int, C.POINTER(_I64)], _I32),
    "df_fire_many": ([_P, _I32, _P, _P, C.c_int], _I32),
    "df_fire_pipeline": ([_P, _I32, _I32, _I32, _I64, C.c_int, C.POINTER(_I64)], _I32),
    "df_stream_dpd": ([_P, _I32, _P, _P, _P, _I64, _I64], _I32),
    "df_set_tile": ([_P, _I32, _I32, _I32], _I32),
    "df_profile_enable": ([_P, _I32], _I32),
    "df_profile_read": ([_P, C.POINTER(C.c_double), C.POINTER(_I64)], _I32),
    "df_profile_read_actor": ([_P, _I32, C.POINTER(C.c_double), C.POINTER(_I64)], _I32),
    "df_debug_last_batch": ([_P, _I32, _P, _P, _P, _I64, C.POINTER(_I64)], _I32),
    "df_debug_set_counters": ([_P, _I32, _I64, _I64], _I32),
    "df_dpd_forward": ([_P, _P, _P, _P, _P, _I64, _I64, _I64, _I32, _I32, _I32], _I32),
    "df_dpd_forward_noalloc": ([_P, _P, _P, _P, _P, _I64, _I64, _I64, _I32, _I32, _I32], _I32),
    "df_dpd_forward_noalloc_max_bytes": ([], _I64),
    "df_dpd_forward_network": ([_P, _P, _P, _P, _P, _I64, _I64, _I64, _I32, _I32, _I32], _I32),
    "df_dpd_coeff_adjoint": ([_P, _P, _P, _P, _P, _I64, _I64, _I64, _I32, _I32, _I32, _P, _I64], _I32),
    "df_dpd_coeff_adjoint_work_bytes": ([_I64, _I64, _I64, _I32, _I32], _I64),
    "df_mp_input_adjoint": ([_P, _P, _P, _P, _P, _I64, _I64, _I32, _I32], _I32),
    "df_stream_copy": ([_P, _P, _P, _I64], _I32),
    "df_hbm_ref": ([_P, _I32, _P, _P, _I64], _I32),
    "df_paper_channel_bytes": ([_I64, _I64, _I32], _I64),
}
EXPORTED = tuple(_SIGS)


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1611_03226_amd.build` "
                          "(the HIP library is required, there is no fallback)")
    lib = C.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = load_library()


def _check(status: int, g=None) -> None:
    if status != DF_OK:
        msg = _lib.df_last_error(g)
        raise DFError(status, msg.decode() if msg else "")


# ------------------------------------------------------------------ marshalling

def _is_tensor(a) -> bool:
    return type(a).__module__.startswith("torch")


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _host_ptr(a: np.ndarray):
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("host buffers must be C-contiguous")
    return a.ctypes.data


def _dev_ptr(t):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return t.data_ptr()


_TORCH_DTYPE_NAME = {DF_C64: "complex64", DF_U8: "uint8", DF_I32: "int32", DF_I64: "int64"}


def _tensor_dtype_ok(t, dt: int) -> bool:
    return str(t.dtype) == "torch." + _TORCH_DTYPE_NAME[dt]


def host_tokens(data, dt: int, elems_per_token: int, n_tokens: int | None = None):
    """Host source buffer for n_tokens tokens of dtype dt: returns (array,
    n).  Integer data is converted only when every value is representable,
    complex data only to complex64; anything else raises ValueError.  n
    defaults to the whole tokens the buffer holds, which must then be a
    whole number."""
    want = np.dtype(_NP_DTYPE[dt])
    a = np.asarray(data)
    if a.dtype != want:
        if a.dtype.kind in "iub" and want.kind in "iu":
            b = a.astype(want)
            if not np.array_equal(b.astype(a.dtype), a):
                raise ValueError(f"values do not fit the channel's {want} tokens")
            a = b
        elif a.dtype.kind == "c" and want.kind == "c":
            a = a.astype(want)
        else:
            raise ValueError(f"buffer dtype {a.dtype} does not match the channel's {want} tokens")
    a = np.ascontiguousarray(a)
    if n_tokens is None:
        if a.size % elems_per_token:
            raise ValueError(f"buffer of {a.size} elements is not a whole number of "
                             f"{elems_per_token}-element tokens")
        n_tokens = a.size // elems_per_token
    if n_tokens < 0:
        raise ValueError("negative token count")
    if a.size < n_tokens * elems_per_token:
        raise ValueError(f"buffer of {a.size} elements holds fewer than {n_tokens} tokens "
                         f"of {elems_per_token} elements")
    return a, n_tokens


def host_dest(dst, dt: int, elems_per_token: int, max_tokens: int | None = None) -> int:
    """Check a host destination for up to max_tokens tokens; returns the
    token count (default: as many whole tokens as dst holds)."""
    want = np.dtype(_NP_DTYPE[dt])
    if not isinstance(dst, np.ndarray):
        raise ValueError("host destinations must be numpy arrays")
    if dst.dtype != want:
        raise ValueError(f"destination dtype {dst.dtype} does not match the channel's {want} tokens")
    if not dst.flags["C_CONTIGUOUS"] or not dst.flags["WRITEABLE"]:
        raise ValueError("host destinations must be C-contiguous and writeable")
    room = dst.size // elems_per_token
    if max_tokens is None:
        return room
    if max_tokens < 0:
        raise ValueError("negative token count")
    if max_tokens > room:
        raise ValueError(f"destination of {dst.size} elements has room for {room} tokens, "
                         f"not {max_tokens}")
    return max_tokens


def device_tokens(t, dt: int, elems_per_token: int, n_tokens: int | None = None) -> int:
    """Check a device tensor for n_tokens tokens (source or destination);
    returns the token count (default: the whole tokens it holds)."""
    if not _tensor_dtype_ok(t, dt):
        raise ValueError(f"tensor dtype {t.dtype} does not match the channel's "
                         f"{_TORCH_DTYPE_NAME[dt]} tokens")
    room = t.numel() // elems_per_token
    if n_tokens is None:
        return room
    if n_tokens < 0:
        raise ValueError("negative token count")
    if n_tokens > room:
        raise ValueError(f"tensor of {t.numel()} elements holds {room} tokens, not {n_tokens}")
    return n_tokens


# ------------------------------------------------------------------ graph

def df_version() -> str:
    return _lib.df_version().decode()


def df_paper_channel_bytes(token_bytes: int, rate: int, has_delay: bool) -> int:
    """Channel bytes by the paper's sizing rule (host arithmetic, -1 if invalid)."""
    return int(_lib.df_paper_channel_bytes(token_bytes, rate, 1 if has_delay else 0))


def df_graph_create(device: int = 0, stream=None) -> int:
    g = C.c_void_p()
    _check(_lib.df_graph_create(C.byref(g), device, _stream_ptr(stream)))
    return g.value


def df_graph_destroy(g) -> None:
    _check(_lib.df_graph_destroy(g))


def df_sync(g) -> None:
    _check(_lib.df_sync(g), g)


def df_last_error(g=None) -> str:
    return _lib.df_last_error(g).decode()


def df_fifo_create(g, dtype: int, elems_per_token: int = 1, capacity: int = 0, n_initial: int = 0,
                   initial: np.ndarray | None = None) -> int:
    out = C.c_int32()
    ptr = None
    if initial is not None:
        initial = np.ascontiguousarray(initial, dtype=_NP_DTYPE[dtype])
        if initial.size != n_initial * elems_per_token:
            raise ValueError("initial has the wrong number of elements")
        ptr = _host_ptr(initial)
    _check(_lib.df_fifo_create(g, dtype, elems_per_token, capacity, n_initial, ptr, C.byref(out)), g)
    return out.value


def df_fifo_create_paper(g, dtype: int, elems_per_token: int, rate: int, n_initial: int = 0,
                         initial: np.ndarray | None = None) -> int:
    """A channel in the paper's layout: 2*rate slots, or 3*rate + 1 with one delay token."""
    out = C.c_int32()
    ptr = None
    if initial is not None:
        initial = np.ascontiguousarray(initial, dtype=_NP_DTYPE[dtype])
        if initial.size != n_initial * elems_per_token:
            raise ValueError("initial has the wrong number of elements")
        ptr = _host_ptr(initial)
    _check(_lib.df_fifo_create_paper(g, dtype, elems_per_token, rate, n_initial, ptr, C.byref(out)), g)
    return out.value


def df_fifo_bytes(g, fifo: int) -> int:
    return int(_lib.df_fifo_bytes(g, fifo))


def df_debug_read_slots(g, fifo: int) -> np.ndarray:
    """Raw slot storage of a channel as a [slots, elems_per_token] array."""
    dt, ept, tb = df_fifo_info(g, fifo)
    nbytes = df_fifo_bytes(g, fifo)
    out = np.zeros(nbytes // tb * ept, _NP_DTYPE[dt])
    _check(_lib.df_debug_read_slots(g, fifo, _host_ptr(out), out.nbytes), g)
    return out.reshape(-1, ept)


def df_fifo_status(g, fifo: int):
    r, w, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(_lib.df_fifo_status(g, fifo, C.byref(r), C.byref(w), C.byref(c)), g)
    return r.value, w.value, c.value


def df_actor_create(g, kind: int, params) -> int:
    out = C.c_int32()
    _check(_lib.df_actor_create(g, kind, C.byref(params), C.sizeof(params), C.byref(out)), g)
    return out.value


def df_connect(g, actor: int, port: int, fifo: int) -> None:
    _check(_lib.df_connect(g, actor, port, fifo), g)


def df_fifo_info(g, fifo: int):
    """(dtype, elems_per_token, token_bytes) of a channel."""
    dt, e, b = C.c_int32(), C.c_int64(), C.c_int64()
    _check(_lib.df_fifo_info(g, fifo, C.byref(dt), C.byref(e), C.byref(b)), g)
    return dt.value, e.value, b.value


def df_port_rate(g, actor: int, port: int) -> int:
    out = C.c_int64()
    _check(_lib.df_port_rate(g, actor, port, C.byref(out)), g)
    return out.value


def df_push(g, fifo: int, data, n_tokens: int | None = None) -> None:
    """Push host (numpy) or device (torch) data; n_tokens defaults to the
    whole tokens data holds.  dtype and size are checked against the channel."""
    dt, ept, _ = df_fifo_info(g, fifo)
    if _is_tensor(data):
        n = device_tokens(data, dt, ept, n_tokens)
        _check(_lib.df_push(g, fifo, _dev_ptr(data), n, 1), g)
    else:
        a, n = host_tokens(data, dt, ept, n_tokens)
        _check(_lib.df_push(g, fifo, _host_ptr(a), n, 0), g)


def df_pop(g, fifo: int, dst, max_tokens: int | None = None) -> int:
    """Pop into host (numpy) or device (torch) dst; returns tokens moved.
    max_tokens defaults to the whole tokens dst has room for."""
    dt, ept, _ = df_fifo_info(g, fifo)
    out = C.c_int64()
    if _is_tensor(dst):
        n = device_tokens(dst, dt, ept, max_tokens)
        _check(_lib.df_pop(g, fifo, _dev_ptr(dst), n, 1, C.byref(out)), g)
    else:
        n = host_dest(dst, dt, ept, max_tokens)
        _check(_lib.df_pop(g, fifo, _host_ptr(dst), n, 0, C.byref(out)), g)
    return out.value


def df_fire(g, actor: int, n_firings: int, flags: int = 0) -> int:
    out = C.c_int64()
    _check(_lib.df_fire(g, actor, n_firings, flags, C.byref(out)), g)
    return out.value


def df_fire_many(g, actors, n_firings, flags: int = 0) -> None:
    a = np.ascontiguousarray(actors, dtype=np.int32)
    n = np.ascontiguousarray(n_firings, dtype=np.int64)
    if a.shape != n.shape:
        raise ValueError("actors and n_firings differ in length")
    _check(_lib.df_fire_many(g, len(a), _host_ptr(a), _host_ptr(n), flags), g)


def df_fire_pipeline(g, gauss: int, thres: int, med: int, n_firings: int, flags: int = 0) -> int:
    out = C.c_int64()
    _check(_lib.df_fire_pipeline(g, gauss, thres, med, n_firings, flags, C.byref(out)), g)
    return out.value


def df_stream_dpd(g, actor: int, x: np.ndarray, ctrl: np.ndarray, y: np.ndarray, n_batches: int,
                  firings_per_batch: int) -> None:
    """Host arrays in, host array out, with transfers and firings overlapped."""
    r = df_port_rate(g, actor, DF_DPD_IN)
    nf = n_batches * firings_per_batch
    if n_batches < 0 or firings_per_batch < 1:
        raise ValueError("bad batch counts")
    for name, a, want, n in (("x", x, np.complex64, nf * r), ("ctrl", ctrl, np.int32, nf),
                             ("y", y, np.complex64, nf * r)):
        if not isinstance(a, np.ndarray) or a.dtype != want:
            raise ValueError(f"{name} must be a {np.dtype(want)} numpy array")
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("host buffers must be C-contiguous")
        if a.size < n:
            raise ValueError(f"{name} holds {a.size} elements, {n} needed")
    if not y.flags["WRITEABLE"]:
        raise ValueError("y must be writeable")
    _check(_lib.df_stream_dpd(g, actor, _host_ptr(x), _host_ptr(ctrl), _host_ptr(y), n_batches,
                              firings_per_batch), g)


def df_set_tile(g, tile_outputs: int = 0, outputs_per_thread: int = 0, blocks_per_cu: int = 0) -> None:
    _check(_lib.df_set_tile(g, tile_outputs, outputs_per_thread, blocks_per_cu), g)


def df_profile_enable(g, enable: bool = True) -> None:
    _check(_lib.df_profile_enable(g, 1 if enable else 0), g)


def df_profile_read(g):
    """(summed body-kernel milliseconds, launches) since the last read."""
    t, n = C.c_double(), C.c_int64()
    _check(_lib.df_profile_read(g, C.byref(t), C.byref(n)), g)
    return t.value, n.value


def df_profile_read_actor(g, actor: int):
    """(summed body-kernel milliseconds, launches) of one actor since the last read."""
    t, n = C.c_double(), C.c_int64()
    _check(_lib.df_profile_read_actor(g, actor, C.byref(t), C.byref(n)), g)
    return t.value, n.value


def df_debug_set_counters(g, fifo: int, read_idx: int, write_idx: int) -> None:
    """Test hook: overwrite a channel's device counters (host bookkeeping unchanged)."""
    _check(_lib.df_debug_set_counters(g, fifo, read_idx, write_idx), g)


def df_debug_last_batch(g, actor: int, n_branches_max: int, cap: int):
    rates = np.zeros((n_branches_max, cap), np.int32)
    offs = np.zeros((n_branches_max, cap), np.int64)
    prev = np.zeros((n_branches_max, cap), np.int64)
    n = C.c_int64()
    _check(_lib.df_debug_last_batch(g, actor, _host_ptr(rates), _host_ptr(offs), _host_ptr(prev), cap,
                                    C.byref(n)), g)
    k = n.value
    return rates[:, :k], offs[:, :k], prev[:, :k]


# ------------------------------------------------------------------ stateless

def check_dpd_tensors(x, ctrl, h, y, r: int, coeff_name: str = "h") -> None:
    """Shapes and dtypes of the stateless predistortion calls: x, y complex64
    [S, L] of equal shape, L a multiple of r, h complex64 [B, M], ctrl None
    or int32 [S, L/r]."""
    if x.dim() != 2 or tuple(y.shape) != tuple(x.shape):
        raise ValueError(f"x and {'y' if y is not None else 'G'} must be [S, L] of equal shape")
    for name, t in (("x", x), ("y", y)):
        if not _tensor_dtype_ok(t, DF_C64):
            raise ValueError(f"{name} must be complex64, got {t.dtype}")
    if h.dim() != 2 or not _tensor_dtype_ok(h, DF_C64):
        raise ValueError(f"{coeff_name} must be a complex64 [B, M] tensor")
    S, L = x.shape
    if r < 1 or L % r:
        raise ValueError(f"L = {L} is not a multiple of r = {r}")
    if ctrl is not None:
        if not _tensor_dtype_ok(ctrl, DF_I32) or tuple(ctrl.shape) != (S, L // r):
            raise ValueError(f"ctrl must be int32 of shape ({S}, {L // r})")


def df_dpd_forward(x, ctrl, h, y, r: int, hist: int = DF_HIST_BRANCH, stream=None) -> None:
    """x, y: complex64 device tensors [S, L]; ctrl int32 [S, L/r] or None; h complex64 [B, M]."""
    check_dpd_tensors(x, ctrl, h, y, r)
    S, L = x.shape
    B, M = h.shape
    _check(_lib.df_dpd_forward(_stream_ptr(stream), _dev_ptr(x), None if ctrl is None else _dev_ptr(ctrl),
                               _dev_ptr(h), _dev_ptr(y), S, L, r, B, M, hist))


def df_dpd_forward_noalloc(x, ctrl, h, y, r: int, hist: int = DF_HIST_BRANCH, stream=None) -> None:
    """df_dpd_forward without any allocation (fixed per-GPU scratch; calls
    overlapping on one GPU race)."""
    check_dpd_tensors(x, ctrl, h, y, r)
    S, L = x.shape
    B, M = h.shape
    _check(_lib.df_dpd_forward_noalloc(_stream_ptr(stream), _dev_ptr(x), None if ctrl is None else _dev_ptr(ctrl),
                                       _dev_ptr(h), _dev_ptr(y), S, L, r, B, M, hist))


def df_dpd_forward_noalloc_max_bytes() -> int:
    return int(_lib.df_dpd_forward_noalloc_max_bytes())


def df_dpd_forward_network(x, ctrl, h, y, r: int, mask: bool = False, stream=None) -> None:
    """Same as df_dpd_forward (branch history), through materialised branch
    channels; mask=True reads the control tokens as bit masks of active branches."""
    if ctrl is None:
        raise ValueError("the network form needs control tokens")
    check_dpd_tensors(x, ctrl, h, y, r)
    S, L = x.shape
    B, M = h.shape
    _check(_lib.df_dpd_forward_network(_stream_ptr(stream), _dev_ptr(x), _dev_ptr(ctrl), _dev_ptr(h), _dev_ptr(y),
                                       S, L, r, B, M, DF_CTRL_MASK if mask else DF_CTRL_COUNT))


def df_dpd_coeff_adjoint_work_bytes(S: int, L: int, r: int, B: int, M: int) -> int:
    return int(_lib.df_dpd_coeff_adjoint_work_bytes(S, L, r, B, M))


def df_dpd_coeff_adjoint(x, ctrl, G, grad_h, r: int, work, hist: int = DF_HIST_BRANCH, stream=None) -> None:
    check_dpd_tensors(x, ctrl, grad_h, G, r, coeff_name="grad_h")
    S, L = x.shape
    B, M = grad_h.shape
    need = df_dpd_coeff_adjoint_work_bytes(S, L, r, B, M)
    if work.numel() * work.element_size() < need:
        raise ValueError(f"work buffer holds {work.numel() * work.element_size()} bytes, {need} needed")
    _check(_lib.df_dpd_coeff_adjoint(_stream_ptr(stream), _dev_ptr(x), None if ctrl is None else _dev_ptr(ctrl),
                                     _dev_ptr(G), _dev_ptr(grad_h), S, L, r, B, M, hist, _dev_ptr(work),
                                     work.numel() * work.element_size()))


def df_mp_input_adjoint(u, a, g, Gu, stream=None) -> None:
    if u.dim() != 2 or tuple(g.shape) != tuple(u.shape) or tuple(Gu.shape) != tuple(u.shape):
        raise ValueError("u, g and Gu must be [S, L] of equal shape")
    for name, t in (("u", u), ("a", a), ("g", g), ("Gu", Gu)):
        if not _tensor_dtype_ok(t, DF_C64):
            raise ValueError(f"{name} must be complex64, got {t.dtype}")
    if a.dim() != 2:
        raise ValueError("a must be a [K, Q] tensor")
    S, L = u.shape
    K, Q = a.shape
    _check(_lib.df_mp_input_adjoint(_stream_ptr(stream), _dev_ptr(u), _dev_ptr(a), _dev_ptr(g), _dev_ptr(Gu),
                                    S, L, K, Q))


def df_stream_copy(src, dst, nbytes: int, stream=None) -> None:
    """Plain device copy of nbytes (bandwidth / traffic-counter reference)."""
    _check(_lib.df_stream_copy(_stream_ptr(stream), _dev_ptr(src), _dev_ptr(dst), nbytes))


HBM_REF_COPY, HBM_REF_READ, HBM_REF_WRITE, HBM_REF_2R1W = 0, 1, 2, 3


def df_hbm_ref(mode: int, src, dst, nbytes: int, stream=None) -> None:
    """One bandwidth-reference access mix over nbytes (see the header)."""
    need_src = 2 * nbytes if mode == HBM_REF_2R1W else (0 if mode == HBM_REF_WRITE else nbytes)
    need_dst = 16 if mode == HBM_REF_READ else nbytes
    if src is not None and src.numel() * src.element_size() < need_src:
        raise ValueError(f"src holds fewer than {need_src} bytes")
    if dst.numel() * dst.element_size() < need_dst:
        raise ValueError(f"dst holds fewer than {need_dst} bytes")
    _check(_lib.df_hbm_ref(_stream_ptr(stream), mode, None if src is None else _dev_ptr(src), _dev_ptr(dst), nbytes))
