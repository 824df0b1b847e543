"""Python binding of libhtn (include/htn.h): same names, argument marshalling
only.  Every computation runs in the HIP library; there is no fallback.

Tensors may be numpy arrays or torch tensors (host or device).  Device
tensors are borrowed by the library, so the returned :class:`Net` keeps a
reference to them.  Streams are torch streams or raw hipStream_t integers.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhtn.so")

HTN_F64, HTN_F32, HTN_BF16 = 0, 1, 2
HTN_SUM_PLAIN, HTN_SUM_FP64, HTN_SUM_COMPENSATED = 0, 1, 2
HTN_EXEC_AUTO, HTN_EXEC_STEPS, HTN_EXEC_FUSED = 0, 1, 2
HTN_PATH_GREEDY, HTN_PATH_LEARNED, HTN_PATH_SAMPLED = -1, -2, -3
HTN_OPT_EXEC, HTN_OPT_MAX_INTERMEDIATE, HTN_OPT_FUSED_LDS_BYTES, HTN_OPT_MFMA = 0, 1, 2, 3
HTN_OPT_PATH_SAMPLES, HTN_OPT_PATH_SEED, HTN_OPT_FUSED_THREADS, HTN_OPT_SLICE, HTN_OPT_QUEUE = 4, 5, 6, 7, 8
HTN_MODEL_FEATURES, HTN_MODEL_HIDDEN = 26, 64

STATUS = ["HTN_OK", "HTN_E_ARG", "HTN_E_LABEL", "HTN_E_SHAPE", "HTN_E_PATH", "HTN_E_OOM",
          "HTN_E_DEVICE", "HTN_E_UNSUPPORTED", "HTN_E_STATE"]


class HtnError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{self.name}: {message}")


class htn_info(ctypes.Structure):
    _fields_ = [("out_elements", ctypes.c_int64), ("out_dtype", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_kernel_steps", ctypes.c_int32),
                ("n_absorbed", ctypes.c_int32), ("fused_ok", ctypes.c_int32),
                ("fused_lds_bytes", ctypes.c_int32), ("mults", ctypes.c_double),
                ("peak_elements", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
                ("input_bytes", ctypes.c_int64), ("n_slices", ctypes.c_int64)]


HTN_TRUNC_MAX_RANK = 16


class htn_truncation(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("rank", ctypes.c_int32),
                ("dims", ctypes.c_int64 * HTN_TRUNC_MAX_RANK),
                ("kept", ctypes.POINTER(ctypes.c_int32) * HTN_TRUNC_MAX_RANK),
                ("n_kept", ctypes.c_int32 * HTN_TRUNC_MAX_RANK)]


class htn_gather(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("rank", ctypes.c_int32),
                ("dims", ctypes.c_int64 * HTN_TRUNC_MAX_RANK), ("out_rank", ctypes.c_int32),
                ("n_axes", ctypes.c_int32 * HTN_TRUNC_MAX_RANK), ("axes", ctypes.c_int32 * HTN_TRUNC_MAX_RANK),
                ("kept", ctypes.POINTER(ctypes.c_int32) * HTN_TRUNC_MAX_RANK),
                ("n_kept", ctypes.c_int32 * HTN_TRUNC_MAX_RANK)]


HTN_SV_U1, HTN_SV_CZ, HTN_SV_CX, HTN_SV_RZZ, HTN_SV_PROJ = 0, 1, 2, 3, 4


class htn_sv_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("m", ctypes.c_double * 8)]


class htn_sv_instance(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("init", ctypes.POINTER(ctypes.c_double)), ("n_ops", ctypes.c_int32),
                ("ops", ctypes.POINTER(htn_sv_op)), ("observable", ctypes.c_char_p), ("n_kept", ctypes.c_int32),
                ("kept", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def load_library():
    """Load libhtn.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2410_15080_amd/build.py")
    try:
        # torch carries its own HIP runtime (same soname); loading it first
        # makes the library bind to that one, so torch and the library share
        # one runtime whichever of them touches the GPU first
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64 = ctypes.c_int32, ctypes.c_int64
    i32p = ctypes.POINTER(I32)
    i64p = ctypes.POINTER(I64)
    f32p = ctypes.POINTER(ctypes.c_float)
    sigs = {
        "htn_create": (I32, [ctypes.POINTER(P), I32, i32p, i32p, I32, i64p, ctypes.POINTER(P), I32, I32,
                             i32p, I32, I32, I32]),
        "htn_set_path": (I32, [P, I32, i32p]),
        "htn_get_path": (I32, [P, i32p, i32p, I32, ctypes.POINTER(ctypes.c_double)]),
        "htn_set_option": (I32, [P, I32, I64]),
        "htn_get_info": (I32, [P, ctypes.POINTER(htn_info)]),
        "htn_get_slicing": (I32, [P, i32p, i32p, I32, i64p]),
        "htn_contract": (I32, [P, P, P]),
        "htn_contract_noalloc": (I32, [P, P, P]),
        "htn_contract_batch": (I32, [I32, ctypes.POINTER(P), ctypes.POINTER(P), P]),
        "htn_batch_create": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(P)]),
        "htn_batch_set_graph": (I32, [P, I32]),
        "htn_batch_graph_state": (I32, [P, i32p]),
        "htn_set_allocator": (I32, [P, P, P]),
        "htn_batch_run": (I32, [P, ctypes.POINTER(P), P]),
        "htn_batch_timestamps": (I32, [P, i64p]),
        "htn_batch_destroy": (None, [P]),
        "htn_batch_set_phase_timing": (I32, [P, I32]),
        "htn_batch_phase_times": (I32, [P, i64p]),
        "htn_update_data": (I32, [P, ctypes.POINTER(P), I32]),
        "htn_destroy": (None, [P]),
        "htn_status_string": (ctypes.c_char_p, [I32]),
        "htn_last_error": (ctypes.c_char_p, []),
        "htn_plan_json": (I32, [P, ctypes.c_char_p, I64, i64p]),
        "htn_plan_tables": (I32, [P, i32p, I64, i64p]),
        "htn_batch_step_times": (I32, [P, f32p, I32]),
        "htn_model_param_count": (I64, []),
        "htn_model_create": (I32, [ctypes.POINTER(P), ctypes.c_uint64]),
        "htn_model_set_params": (I32, [P, f32p]),
        "htn_model_get_params": (I32, [P, f32p]),
        "htn_model_forward": (I32, [P, I32, P, P, P]),
        "htn_model_gradients": (I32, [P, I32, P, P, P, P, P]),
        "htn_model_adam_step": (I32, [P, P, ctypes.c_float, P]),
        "htn_model_train": (I32, [P, I32, P, P, I32, I32, ctypes.c_float, ctypes.c_uint64, f32p, P]),
        "htn_model_destroy": (None, [P]),
        "htn_set_model": (I32, [P, P]),
        "htn_step_features": (I32, [P, f32p, I32, i32p]),
        "htn_autotune": (I32, [I32, ctypes.POINTER(P), ctypes.POINTER(P), P, i32p, i32p, f32p]),
        "htn_batch_set_event_timing": (I32, [P, I32]),
        "htn_batch_launch_ms": (I32, [P, f32p, f32p, i32p]),
        "htn_batch_queue_info": (I32, [P, i32p, i32p, i32p]),
        "htn_qpd_sample": (I32, [I32, ctypes.POINTER(ctypes.c_double), I64, ctypes.POINTER(ctypes.c_double),
                                 i64p, ctypes.POINTER(ctypes.c_double)]),
        "htn_truncate_create": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(htn_truncation), I32]),
        "htn_truncate_run": (I32, [P, P]),
        "htn_truncate_destroy": (None, [P]),
        "htn_qpd_fuse": (I32, [I32, i32p, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                               ctypes.POINTER(ctypes.c_double)]),
        "htn_gather_create": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(htn_gather), I32]),
        "htn_qt_eval_create": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(htn_sv_instance), I64, i64p, i64p,
                                     ctypes.POINTER(ctypes.c_double)]),
        "htn_qt_eval_run": (I32, [P, P, P, P]),
        "htn_qt_eval_info": (I32, [P, i64p, i64p]),
        "htn_qt_eval_destroy": (None, [P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols(header: str | None = None):
    """Function names declared in include/htn.h."""
    header = header or os.path.join(os.path.dirname(_HERE), "include", "htn.h")
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(htn_\w+)\s*\(", text, re.M)))


def _check(st: int):
    if st != 0:
        lib = load_library()
        raise HtnError(st, lib.htn_last_error().decode())


def _arr(x, dtype):
    a = np.ascontiguousarray(np.asarray(x, dtype=dtype))
    return a, a.ctypes.data_as(ctypes.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t) -> int:
    name = str(getattr(t, "dtype", t))
    if "float64" in name:
        return HTN_F64
    if "float32" in name:
        return HTN_F32
    if "bfloat16" in name:
        return HTN_BF16
    raise TypeError(f"unsupported tensor dtype {name}")


def _is_device(t) -> bool:
    return hasattr(t, "is_cuda") and bool(t.is_cuda)


def _data_ptr(t) -> int:
    if hasattr(t, "data_ptr"):
        return int(t.data_ptr())
    return int(t.ctypes.data)


class Net:
    """Handle of an htn_net_t plus the Python objects it borrows."""

    def __init__(self, handle, keep, n_tensors):
        self.handle = handle
        self._keep = keep
        self.n_tensors = n_tensors

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                htn_destroy(self)
            except Exception:
                pass


class Model:
    """Handle of an htn_model_t (cost model on the device)."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                htn_model_destroy(self)
            except Exception:
                pass


class Batch:
    def __init__(self, handle, nets):
        self.handle = handle
        self.nets = nets

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                htn_batch_destroy(self)
            except Exception:
                pass


def _marshal_data(tensors, storage):
    keep = []
    ptrs = []
    on_dev = None
    for t in tensors:
        if not hasattr(t, "data_ptr"):
            t = np.ascontiguousarray(t)
        elif not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        d = _is_device(t)
        if on_dev is None:
            on_dev = d
        elif on_dev != d:
            raise ValueError("all tensors must be on the host or all on the device")
        if _dtype_code(t) != storage:
            raise ValueError("every tensor must have the storage dtype")
        keep.append(t)
        ptrs.append(_data_ptr(t))
    arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
    return keep, arr, int(bool(on_dev))


def htn_create(tensors, labels, dims, out_labels=(), compute=HTN_F64, final_sum=HTN_SUM_PLAIN,
               storage=None) -> Net:
    lib = load_library()
    if storage is None:
        storage = _dtype_code(tensors[0])
    for t, ls in zip(tensors, labels):
        shape = tuple(t.shape)
        if len(shape) != len(ls) or any(0 <= l < len(dims) and shape[k] != dims[l] for k, l in enumerate(ls)):
            raise ValueError(f"tensor shape {shape} does not match labels {ls}")
    keep, ptrs, on_dev = _marshal_data(tensors, storage)
    ranks, rp = _arr([len(l) for l in labels], np.int32)
    flat, fp = _arr([x for l in labels for x in l] or [0], np.int32)
    d, dp = _arr(dims, np.int64)
    o, op = _arr(list(out_labels) or [0], np.int32)
    h = ctypes.c_void_p()
    _check(lib.htn_create(ctypes.byref(h), len(tensors), rp, fp, len(dims), dp, ptrs, on_dev,
                          len(out_labels), op, storage, compute, final_sum))
    return Net(h, keep if on_dev else [], len(tensors))


def htn_set_path(net: Net, path) -> None:
    lib = load_library()
    if isinstance(path, int):
        _check(lib.htn_set_path(net.handle, path, None))
        return
    a, p = _arr(np.asarray(path, dtype=np.int32).reshape(-1) if len(path) else [0], np.int32)
    _check(lib.htn_set_path(net.handle, len(path), p))


def htn_get_path(net: Net):
    """Returns (list of (i, j) pairs, multiplication count)."""
    lib = load_library()
    n = ctypes.c_int32()
    m = ctypes.c_double()
    _check(lib.htn_get_path(net.handle, ctypes.byref(n), None, 0, ctypes.byref(m)))
    buf = np.zeros(max(1, 2 * n.value), dtype=np.int32)
    _check(lib.htn_get_path(net.handle, ctypes.byref(n), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            n.value, ctypes.byref(m)))
    return [(int(buf[2 * t]), int(buf[2 * t + 1])) for t in range(n.value)], float(m.value)


def htn_set_option(net: Net, opt: int, value: int) -> None:
    _check(load_library().htn_set_option(net.handle, opt, int(value)))


def htn_get_info(net: Net) -> htn_info:
    info = htn_info()
    _check(load_library().htn_get_info(net.handle, ctypes.byref(info)))
    return info


def htn_get_slicing(net: Net):
    """(sliced labels, number of slices) of the current plan."""
    lib = load_library()
    n = ctypes.c_int32()
    s = ctypes.c_int64()
    buf = np.zeros(64, dtype=np.int32)
    _check(lib.htn_get_slicing(net.handle, ctypes.byref(n), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 64,
                               ctypes.byref(s)))
    return [int(x) for x in buf[: n.value]], int(s.value)


def htn_contract(net: Net, out, stream=None) -> None:
    _check(load_library().htn_contract(net.handle, ctypes.c_void_p(_data_ptr(out)), _stream_ptr(stream)))


HTN_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def htn_contract_noalloc(net: Net, out, stream=None) -> None:
    _check(load_library().htn_contract_noalloc(net.handle, ctypes.c_void_p(_data_ptr(out)), _stream_ptr(stream)))


def pointer_array(outs):
    """Device addresses of `outs` as a C array, reusable across calls."""
    if isinstance(outs, ctypes.Array):
        return outs
    return (ctypes.c_void_p * len(outs))(*[_data_ptr(o) for o in outs])


def htn_contract_batch(nets, outs, stream=None) -> None:
    lib = load_library()
    hs = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
    _check(lib.htn_contract_batch(len(nets), hs, pointer_array(outs), _stream_ptr(stream)))


def htn_autotune(nets, outs, stream=None):
    """Returns (threads, lds_bytes, median ms) of the configuration applied."""
    handles = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
    optrs = pointer_array(outs)
    t, l = ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_float()
    _check(load_library().htn_autotune(len(nets), handles, optrs, _stream_ptr(stream), ctypes.byref(t),
                                       ctypes.byref(l), ctypes.byref(ms)))
    return int(t.value), int(l.value), float(ms.value)


def htn_batch_create(nets) -> Batch:
    lib = load_library()
    hs = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
    h = ctypes.c_void_p()
    _check(lib.htn_batch_create(ctypes.byref(h), len(nets), hs))
    return Batch(h, list(nets))


def htn_batch_set_graph(batch: Batch, use_graph) -> None:
    """use_graph: False/0, True/1, or HTN_GRAPH_FORCE_FAILURE."""
    _check(load_library().htn_batch_set_graph(batch.handle, int(use_graph)))


HTN_GRAPH_FORCE_FAILURE = 2


def htn_batch_graph_state(batch: Batch) -> int:
    """0 eager, 1 replaying a captured graph, 2 capture failed (eager)."""
    st = ctypes.c_int32()
    _check(load_library().htn_batch_graph_state(batch.handle, ctypes.byref(st)))
    return int(st.value)


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None  # keeps the installed callbacks alive


def htn_set_allocator(alloc, free) -> None:
    """Install Python callables alloc(nbytes) -> int address (0 on failure)
    and free(address) as the library's device allocator; (None, None)
    restores hipMalloc / hipFree."""
    global _allocator_refs
    lib = load_library()
    if alloc is None and free is None:
        _check(lib.htn_set_allocator(None, None, None))
        _allocator_refs = None
        return

    def _a(nbytes, ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:
            return None

    def _f(ptr, ctx):
        free(int(ptr))

    refs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(lib.htn_set_allocator(ctypes.cast(refs[0], ctypes.c_void_p), ctypes.cast(refs[1], ctypes.c_void_p),
                                 None))
    _allocator_refs = refs


def use_torch_allocator() -> None:
    """Route the library's device memory through PyTorch's caching allocator
    (on the current device and stream)."""
    import torch

    def alloc(n):
        return torch.cuda.caching_allocator_alloc(n)

    def free(p):
        torch.cuda.caching_allocator_delete(p)

    htn_set_allocator(alloc, free)


def htn_batch_run(batch: Batch, outs, stream=None) -> None:
    """outs: output tensors, or a pointer_array() built once for them."""
    _check(load_library().htn_batch_run(batch.handle, pointer_array(outs), _stream_ptr(stream)))


def htn_batch_timestamps(batch: Batch) -> np.ndarray:
    t = np.zeros(2 * len(batch.nets), dtype=np.int64)
    _check(load_library().htn_batch_timestamps(batch.handle, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return t.reshape(-1, 2)


def htn_batch_set_phase_timing(batch: Batch, max_phases: int) -> None:
    _check(load_library().htn_batch_set_phase_timing(batch.handle, int(max_phases)))
    batch.max_phases = int(max_phases)


def htn_batch_phase_times(batch: Batch) -> np.ndarray:
    """[n_nets, max_phases] clock ticks (100 MHz) at the end of each phase."""
    t = np.zeros(len(batch.nets) * batch.max_phases, dtype=np.int64)
    _check(load_library().htn_batch_phase_times(batch.handle, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return t.reshape(len(batch.nets), batch.max_phases)


def htn_batch_set_event_timing(batch: Batch, on: bool) -> None:
    _check(load_library().htn_batch_set_event_timing(batch.handle, 1 if on else 0))


def htn_batch_launch_ms(batch: Batch):
    """(mean prep-launch ms, mean fused-launch ms, runs) since the last read."""
    a, b = ctypes.c_float(), ctypes.c_float()
    k = ctypes.c_int32()
    _check(load_library().htn_batch_launch_ms(batch.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(k)))
    return float(a.value), float(b.value), int(k.value)


def htn_batch_queue_info(batch: Batch):
    """(networks in the batch's work queue, tasks, error flag); waits for
    the device and clears the flag."""
    a, t, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().htn_batch_queue_info(batch.handle, ctypes.byref(a), ctypes.byref(t), ctypes.byref(e)))
    return int(a.value), int(t.value), int(e.value)


def htn_batch_destroy(batch: Batch) -> None:
    if batch.handle:
        load_library().htn_batch_destroy(batch.handle)
        batch.handle = None


def htn_update_data(net: Net, tensors, storage=None) -> None:
    if storage is None:
        storage = _dtype_code(tensors[0])
    keep, ptrs, on_dev = _marshal_data(tensors, storage)
    _check(load_library().htn_update_data(net.handle, ptrs, on_dev))
    net._keep = keep if on_dev else []


def htn_destroy(net: Net) -> None:
    if net.handle:
        load_library().htn_destroy(net.handle)
        net.handle = None


def htn_status_string(status: int) -> str:
    return load_library().htn_status_string(status).decode()


def htn_last_error() -> str:
    return load_library().htn_last_error().decode()


def htn_plan_json(net: Net) -> str:
    lib = load_library()
    need = ctypes.c_int64()
    _check(lib.htn_plan_json(net.handle, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib.htn_plan_json(net.handle, buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def htn_plan_tables(net: Net) -> np.ndarray:
    lib = load_library()
    need = ctypes.c_int64()
    _check(lib.htn_plan_tables(net.handle, None, 0, ctypes.byref(need)))
    buf = np.zeros(max(1, need.value), dtype=np.int32)
    _check(lib.htn_plan_tables(net.handle, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), need.value,
                               ctypes.byref(need)))
    return buf[: need.value]


def output_dtype_name(net: Net) -> str:
    return {HTN_F64: "float64", HTN_F32: "float32", HTN_BF16: "bfloat16"}[htn_get_info(net).out_dtype]


def new_output(net: Net, device="cuda"):
    """Allocate a torch tensor of the net's output shape (flat) and dtype."""
    import torch
    info = htn_get_info(net)
    dt = {HTN_F64: torch.float64, HTN_F32: torch.float32}[info.out_dtype]
    return torch.empty(max(1, info.out_elements), dtype=dt, device=device)


# ------------------------------------------------------------ cost model

def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _device_f32(t, name):
    if not (_is_device(t) and str(t.dtype) == "torch.float32" and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    return ctypes.c_void_p(_data_ptr(t))


def htn_model_param_count() -> int:
    return int(load_library().htn_model_param_count())


def htn_model_create(seed: int = 0) -> Model:
    h = ctypes.c_void_p()
    _check(load_library().htn_model_create(ctypes.byref(h), ctypes.c_uint64(seed)))
    return Model(h)


def htn_model_set_params(model: Model, params) -> None:
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != htn_model_param_count():
        raise ValueError("wrong parameter count")
    _check(load_library().htn_model_set_params(model.handle, _f32p(a)))


def htn_model_get_params(model: Model) -> np.ndarray:
    a = np.zeros(htn_model_param_count(), dtype=np.float32)
    _check(load_library().htn_model_get_params(model.handle, _f32p(a)))
    return a


def htn_model_forward(model: Model, x, y, stream=None) -> None:
    """x: [n, HTN_MODEL_FEATURES] float32 device tensor; y: [n] float32 device tensor."""
    n = int(x.shape[0])
    if tuple(x.shape) != (n, HTN_MODEL_FEATURES) or y.numel() != n:
        raise ValueError("shape mismatch")
    _check(load_library().htn_model_forward(model.handle, n, _device_f32(x, "x"), _device_f32(y, "y"),
                                            _stream_ptr(stream)))


def htn_model_gradients(model: Model, x, t, grad, loss=None, stream=None) -> None:
    n = int(x.shape[0])
    if tuple(x.shape) != (n, HTN_MODEL_FEATURES) or t.numel() != n or grad.numel() != htn_model_param_count():
        raise ValueError("shape mismatch")
    lp = _device_f32(loss, "loss") if loss is not None else None
    _check(load_library().htn_model_gradients(model.handle, n, _device_f32(x, "x"), _device_f32(t, "t"),
                                              _device_f32(grad, "grad"), lp, _stream_ptr(stream)))


def htn_model_adam_step(model: Model, grad, lr: float, stream=None) -> None:
    _check(load_library().htn_model_adam_step(model.handle, _device_f32(grad, "grad"), float(lr),
                                              _stream_ptr(stream)))


def htn_model_train(model: Model, x, t, epochs: int, batch: int, lr: float, seed: int = 0,
                    stream=None) -> np.ndarray:
    """Returns the mean minibatch loss of each epoch."""
    n = int(x.shape[0])
    if tuple(x.shape) != (n, HTN_MODEL_FEATURES) or t.numel() != n:
        raise ValueError("shape mismatch")
    losses = np.zeros(max(1, epochs), dtype=np.float32)
    _check(load_library().htn_model_train(model.handle, n, _device_f32(x, "x"), _device_f32(t, "t"), int(epochs),
                                          int(batch), float(lr), ctypes.c_uint64(seed), _f32p(losses),
                                          _stream_ptr(stream)))
    return losses[:epochs]


def htn_model_destroy(model: Model) -> None:
    if model.handle:
        load_library().htn_model_destroy(model.handle)
        model.handle = None


def htn_set_model(net: Net, model) -> None:
    """Attach a cost model to a net (None detaches); the net keeps a reference."""
    net._model = model
    _check(load_library().htn_set_model(net.handle, model.handle if model is not None else None))


def htn_step_features(net: Net) -> np.ndarray:
    """[kernel steps, HTN_MODEL_FEATURES] features of the current plan."""
    lib = load_library()
    k = ctypes.c_int32()
    _check(lib.htn_step_features(net.handle, None, 0, ctypes.byref(k)))
    a = np.zeros((max(1, k.value), HTN_MODEL_FEATURES), dtype=np.float32)
    _check(lib.htn_step_features(net.handle, _f32p(a), k.value, ctypes.byref(k)))
    return a[: k.value]


def htn_batch_step_times(batch: Batch, capacity: int) -> np.ndarray:
    """[nets, capacity] kernel-step durations (microseconds, NaN if not recorded)."""
    a = np.zeros((len(batch.nets), max(1, capacity)), dtype=np.float32)
    _check(load_library().htn_batch_step_times(batch.handle, _f32p(a), int(capacity)))
    return a[:, :capacity]


# ---------------------------------------------------------------------------
# QPD sampling and truncation (Sec. 4.3)
# ---------------------------------------------------------------------------

def htn_qpd_sample(coeffs, s_qpd: int, uniforms):
    """(counts int64[n], weights float64[n]) of one CT's s_qpd draws."""
    lib = load_library()
    c, cp = _arr(coeffs, np.float64)
    u, up = _arr(uniforms, np.float64)
    if u.shape != (int(s_qpd),):
        raise HtnError(1, "uniforms must hold s_qpd values")
    counts = np.zeros(c.size, dtype=np.int64)
    weights = np.zeros(c.size, dtype=np.float64)
    _check(lib.htn_qpd_sample(int(c.size), cp, int(s_qpd), up,
                              counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return counts, weights


class Trunc:
    """Handle of htn_truncate_create; keeps the borrowed buffers alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.htn_truncate_destroy(self.handle)
            self.handle = None


def htn_truncate_create(items, dtype=HTN_F64) -> Trunc:
    """items: (src, dst, dims, kept) per tensor; src/dst device tensors (or
    pointers), kept[a] a list of indices or None (whole axis)."""
    lib = load_library()
    arr = (htn_truncation * len(items))()
    keep = []
    for i, (src, dst, dims, kept) in enumerate(items):
        it = arr[i]
        it.src = _data_ptr(src) if not isinstance(src, int) else src
        it.dst = _data_ptr(dst) if not isinstance(dst, int) else dst
        it.rank = len(dims)
        for a, d in enumerate(dims):
            it.dims[a] = int(d)
            if kept is not None and kept[a] is not None:
                k, kp = _arr(kept[a], np.int32)
                keep.append(k)
                it.kept[a] = kp
                it.n_kept[a] = int(k.size)
        keep += [src, dst]
    h = ctypes.c_void_p()
    _check(lib.htn_truncate_create(ctypes.byref(h), len(items), arr, int(dtype)))
    return Trunc(h, keep)


def htn_truncate_run(t: Trunc, stream=None) -> None:
    _check(load_library().htn_truncate_run(t.handle, _stream_ptr(stream)))


def htn_truncate_destroy(t: Trunc) -> None:
    if t.handle:
        load_library().htn_truncate_destroy(t.handle)
        t.handle = None


def htn_qpd_fuse(coeffs):
    """Tensor product of the CTs `coeffs` (row-major, first slowest)."""
    lib = load_library()
    arrs = [np.ascontiguousarray(c, dtype=np.float64).reshape(-1) for c in coeffs]
    d, dp = _arr([a.size for a in arrs], np.int32)
    dpp = ctypes.POINTER(ctypes.c_double)
    ptrs = (dpp * len(arrs))(*[a.ctypes.data_as(dpp) for a in arrs])
    out = np.zeros(int(np.prod([a.size for a in arrs])), dtype=np.float64)
    _check(lib.htn_qpd_fuse(len(arrs), dp, ptrs, out.ctypes.data_as(dpp)))
    return out


def htn_gather_create(items, dtype=HTN_F64) -> Trunc:
    """items: (src, dst, dims, groups, kept) per tensor: groups[o] lists the
    input axes merged into output axis o (first slowest), kept[o] its kept
    indices or None (all)."""
    lib = load_library()
    arr = (htn_gather * len(items))()
    keep = []
    for i, (src, dst, dims, groups, kept) in enumerate(items):
        it = arr[i]
        it.src = _data_ptr(src) if not isinstance(src, int) else src
        it.dst = _data_ptr(dst) if not isinstance(dst, int) else dst
        it.rank = len(dims)
        for a, d in enumerate(dims):
            it.dims[a] = int(d)
        it.out_rank = len(groups)
        flat = [a for g in groups for a in g]
        for k, a in enumerate(flat):
            it.axes[k] = int(a)
        for o, g in enumerate(groups):
            it.n_axes[o] = len(g)
            if kept is not None and kept[o] is not None:
                k, kp = _arr(kept[o], np.int32)
                keep.append(k)
                it.kept[o] = kp
                it.n_kept[o] = int(k.size)
        keep += [src, dst]
    h = ctypes.c_void_p()
    _check(lib.htn_gather_create(ctypes.byref(h), len(items), arr, int(dtype)))
    return Trunc(h, keep)


class QtEval:
    """Handle of htn_qt_eval_create."""

    def __init__(self, handle, n_outputs, n_entries):
        self.handle, self.n_outputs, self.n_entries = handle, n_outputs, n_entries

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.htn_qt_eval_destroy(self.handle)
            self.handle = None


def htn_qt_eval_create(instances, entry_start, term_output, term_coef) -> QtEval:
    """instances: (n_qubits, init [n][4] float64, ops [(kind, q0, q1, m8)],
    observable str, kept list) tuples; entry CSR as numpy arrays."""
    lib = load_library()
    arr = (htn_sv_instance * len(instances))()
    keep = []
    for i, (n, init, ops, obs, kept) in enumerate(instances):
        it = arr[i]
        it.n_qubits = int(n)
        a, ap = _arr(np.asarray(init, dtype=np.float64).reshape(-1), np.float64)
        keep.append(a)
        it.init = ap
        oa = (htn_sv_op * max(1, len(ops)))()
        for j, (kind, q0, q1, m) in enumerate(ops):
            oa[j].kind, oa[j].q0, oa[j].q1 = int(kind), int(q0), int(q1)
            for c in range(8):
                oa[j].m[c] = float(m[c])
        keep.append(oa)
        it.n_ops = len(ops)
        it.ops = oa
        ob = obs.encode()
        keep.append(ob)
        it.observable = ob
        k, kp = _arr(list(kept) or [0], np.int32)
        keep.append(k)
        it.n_kept = len(kept)
        it.kept = kp
    st, sp = _arr(entry_start, np.int64)
    to, tp = _arr(term_output if len(term_output) else [0], np.int64)
    tc, cp = _arr(term_coef if len(term_coef) else [0.0], np.float64)
    h = ctypes.c_void_p()
    _check(lib.htn_qt_eval_create(ctypes.byref(h), len(instances), arr, len(entry_start) - 1, sp, tp, cp))
    n_out, n_ent = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.htn_qt_eval_info(h, ctypes.byref(n_out), ctypes.byref(n_ent)))
    return QtEval(h, int(n_out.value), int(n_ent.value))


def htn_qt_eval_run(q: QtEval, entries, outputs=None, stream=None) -> None:
    _check(load_library().htn_qt_eval_run(q.handle, ctypes.c_void_p(_data_ptr(entries)),
                                          ctypes.c_void_p(_data_ptr(outputs)) if outputs is not None else None,
                                          _stream_ptr(stream)))
