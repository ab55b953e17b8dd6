"""ctypes binding of ``include/tr_stream.h`` (argument marshalling only).

Every computation runs in ``libtrstream.so``; this module converts NumPy
arrays and torch tensors to the pointers, sizes and memory orders that the C
ABI expects and turns status codes into exceptions.  Loading fails loudly if
the library has not been built.
"""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtrstream.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "tr_stream.h")

TR_F64, TR_F32, TR_BF16 = 0, 1, 2
DTYPES = {"f64": TR_F64, "f32": TR_F32, "bf16": TR_BF16}
SKETCHES = {None: 0, "none": 0, "uniform": 1, "leverage": 2, "ksrft": 3}
STATUS = {0: "TR_OK", 1: "TR_ERR_ARG", 2: "TR_ERR_SHAPE", 3: "TR_ERR_NOMEM",
          4: "TR_ERR_DEVICE", 5: "TR_ERR_NONFINITE", 6: "TR_ERR_STATE",
          7: "TR_ERR_SINGULAR", 8: "TR_ERR_UNSUPPORTED"}


class TRError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        self.status = STATUS.get(code, str(code))
        super().__init__(f"{self.status}: {msg}")


class tr_config(ctypes.Structure):
    _fields_ = [
        ("order", c_int32),
        ("dims", POINTER(c_int64)),
        ("ranks", POINTER(c_int32)),
        ("compute_dtype", c_int32),
        ("sketch", c_int32),
        ("sketch_size", c_int64),
        ("rescale", c_int32),
        ("temporal_normal_eq", c_int32),
        ("seed", c_uint64),
        ("max_slices", c_int64),
        ("check_finite", c_int32),
        ("device", c_int32),
        ("hip_stream", c_void_p),
        ("sweeps", c_int32),
        ("init_max_sweeps", c_int32),
        ("init_tol", c_double),
    ]


class tr_stats(ctypes.Structure):
    _fields_ = [
        ("pinv_fallbacks", c_int64),
        ("init_sweeps", c_int32),
        ("init_rel_err", c_double),
    ]


_lib = None


def load():
    """Load libtrstream.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2307_00719_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "tr_stream_init": ([POINTER(tr_config), P, c_int64, c_int32, POINTER(c_void_p), c_int32,
                            POINTER(c_void_p)], c_int32),
        "tr_stream_update": ([P, P, c_int32, c_int64, c_int32], c_int32),
        "tr_reconstruct_error": ([P, P, c_int64, c_int32, POINTER(c_double)], c_int32),
        "tr_stream_get_cores": ([P, POINTER(c_void_p)], c_int32),
        "tr_stream_get_PQ": ([P, c_int32, P, P], c_int32),
        "tr_stream_sync": ([P], c_int32),
        "tr_stream_get_samples": ([P, P], c_int32),
        "tr_stream_set_samples": ([P, P, P, c_int64], c_int32),
        "tr_stream_get_stats": ([P, POINTER(tr_stats)], c_int32),
        "tr_batch_als": ([POINTER(tr_config), P, c_int64, c_int32, P, c_int32, c_int32, c_double,
                          POINTER(c_void_p), P, P], c_int32),
        "tr_stream_save": ([P, c_char_p], c_int32),
        "tr_stream_load": ([c_char_p, POINTER(tr_config), POINTER(c_void_p)], c_int32),
        "tr_stream_num_slices": ([P], c_int64),
        "tr_stream_profile": ([P, c_int32], c_int32),
        "tr_stream_profile_read": ([P, c_int32, POINTER(c_double), POINTER(c_int64)], c_int32),
        "tr_last_error": ([P], c_char_p),
        "tr_stream_destroy": ([P], None),
        "tr_workspace_bytes": ([c_int32, P, P, c_int32], c_size_t),
        "tr_mttkrp": ([c_int32, P, P, c_int32, c_int32, P, POINTER(c_void_p), P, c_int32, P,
                       c_size_t, P], c_int32),
        "tr_mttkrp_noalloc": ([c_int32, P, P, c_int32, c_int32, P, POINTER(c_void_p), P, c_int32,
                               P], c_int32),
        "tr_mttkrp_noalloc_max_bytes": ([], c_size_t),
        "tr_gram_chain": ([c_int32, P, P, c_int32, POINTER(c_void_p), P, c_int32, P, c_size_t,
                           P], c_int32),
        "tr_fit_loss_fwd": ([c_int32, P, P, c_int32, P, POINTER(c_void_p), P, P, c_size_t, P],
                            c_int32),
        "tr_fit_loss_bwd": ([c_int32, P, P, c_int32, P, POINTER(c_void_p), c_double,
                             POINTER(c_void_p), P, c_size_t, P], c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def declared_functions():
    """Names of the functions declared in include/tr_stream.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tr_[A-Za-z_]+)\s*\(", text)))


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _colmajor_torch(x):
    """A torch tensor whose memory is first-index-fastest."""
    nd = x.dim()
    want = []
    acc = 1
    for s in x.shape:
        want.append(acc)
        acc *= s
    if list(x.stride()) == want:
        return x
    perm = list(range(nd - 1, -1, -1))
    return x.permute(perm).contiguous().permute(perm)


def as_buffer(x, dtype=None):
    """(pointer, keepalive, is_device, dtype code) for an array or tensor."""
    if _is_torch(x):
        import torch
        t = _colmajor_torch(x)
        code = {torch.float64: TR_F64, torch.float32: TR_F32, torch.bfloat16: TR_BF16}[t.dtype]
        return c_void_p(t.data_ptr()), t, int(t.is_cuda), code
    a = np.asarray(x)
    if dtype is not None:
        a = a.astype(dtype, copy=False)
    a = np.asfortranarray(a)
    code = {np.dtype(np.float64): TR_F64, np.dtype(np.float32): TR_F32}[a.dtype]
    return c_void_p(a.ctypes.data), a, 0, code


def _check(code, handle=None):
    if code != 0:
        msg = ""
        if handle is not None:
            m = load().tr_last_error(handle)
            msg = m.decode() if m else ""
        raise TRError(code, msg)


def _ptr_array(ptrs):
    arr = (c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p.value if isinstance(p, c_void_p) else p
    return arr


# ---------------------------------------------------------------------------
# functions with the C ABI's names
# ---------------------------------------------------------------------------

def make_config(shape, ranks, compute_dtype="f64", sketch=None, sketch_size=0, rescale=True,
                temporal_literal=True, seed=0, max_slices=0, check_finite=False, device=0,
                hip_stream=None, sweeps=1, init_max_sweeps=0, init_tol=0.0):
    """(tr_config, keepalive) for a tensor of `shape` (I_1..I_{N-1}, t)."""
    N = len(shape)
    dims = (c_int64 * (N - 1))(*shape[:-1])
    rk = (c_int32 * N)(*[int(r) for r in ranks])
    cfg = tr_config(order=N, dims=dims, ranks=rk, compute_dtype=DTYPES[compute_dtype],
                    sketch=SKETCHES[sketch], sketch_size=int(sketch_size),
                    rescale=int(bool(rescale)), temporal_normal_eq=int(not temporal_literal),
                    seed=int(seed), max_slices=int(max_slices),
                    check_finite=int(bool(check_finite)), device=int(device),
                    hip_stream=hip_stream, sweeps=int(sweeps),
                    init_max_sweeps=int(init_max_sweeps), init_tol=float(init_tol))
    return cfg, (dims, rk)


def tr_stream_init(X_init, cores_init, ranks, compute_dtype="f64", sketch=None, sketch_size=0,
                   rescale=True, temporal_literal=True, seed=0, max_slices=0,
                   check_finite=False, device=0, hip_stream=None, sweeps=1, init_max_sweeps=0,
                   init_tol=0.0):
    """Returns an opaque handle (c_void_p).  X_init: (I_1..I_{N-1}, t_init).
    cores_init None: the library initialises the cores by batch TR-ALS on
    X_init from its counter-based random start (seed)."""
    lib = load()
    shape = tuple(X_init.shape)
    cfg, ckeep = make_config(shape, ranks, compute_dtype, sketch, sketch_size, rescale,
                             temporal_literal, seed, max_slices, check_finite, device, hip_stream,
                             sweeps, init_max_sweeps, init_tol)
    xp, xkeep, xdev, _ = as_buffer(X_init, np.float64)
    if cores_init is None:
        cptr, cdev, cbufs = None, 0, []
    else:
        cbufs = [as_buffer(G, np.float64) for G in cores_init]
        cdev = cbufs[0][2]
        cptr = _ptr_array([b[0] for b in cbufs])
    handle = c_void_p()
    code = lib.tr_stream_init(ctypes.byref(cfg), xp, shape[-1], xdev, cptr, cdev,
                              ctypes.byref(handle))
    if code != 0:
        msg = ""
        if handle:
            m = lib.tr_last_error(handle)
            msg = m.decode() if m else ""
            lib.tr_stream_destroy(handle)
        raise TRError(code, msg)
    return handle


def tr_stream_update(handle, X_new):
    lib = load()
    xp, keep, xdev, code_dt = as_buffer(X_new)
    _check(lib.tr_stream_update(handle, xp, code_dt, X_new.shape[-1], xdev), handle)
    return keep


def tr_reconstruct_error(handle, X_all):
    lib = load()
    xp, keep, xdev, _ = as_buffer(X_all, np.float64)
    out = c_double()
    _check(lib.tr_reconstruct_error(handle, xp, X_all.shape[-1], xdev, ctypes.byref(out)), handle)
    return out.value


def tr_stream_get_cores(handle, dims, ranks):
    """dims: I_1..I_{N-1}; returns host cores (R_n, I_n, R_{n+1}) float64."""
    lib = load()
    N = len(ranks)
    T = lib.tr_stream_num_slices(handle)
    full = list(dims) + [T]
    outs = [np.zeros((ranks[k], full[k], ranks[(k + 1) % N]), order="F") for k in range(N)]
    _check(lib.tr_stream_get_cores(handle, _ptr_array([o.ctypes.data for o in outs])), handle)
    return outs


def tr_stream_get_PQ(handle, n, In, d):
    lib = load()
    P = np.zeros((In, d))
    Q = np.zeros((d, d))
    _check(lib.tr_stream_get_PQ(handle, n, P.ctypes.data, Q.ctypes.data), handle)
    return P, Q


def tr_stream_get_samples(handle, N, m):
    out = np.zeros((N, m), dtype=np.int32)
    _check(load().tr_stream_get_samples(handle, out.ctypes.data), handle)
    return out


def tr_stream_set_samples(handle, idxs=None, signs=None):
    """idxs: N x m integer array (row q = indices into core q) or None;
    signs: N vectors of +-1 (the D_k of the next KSRFT step, the last as long
    as the next batch) or None."""
    a = None if idxs is None else np.ascontiguousarray(idxs, dtype=np.int32)
    sg, t = None, 0
    if signs is not None:
        sg = np.ascontiguousarray(np.concatenate([np.asarray(v).ravel() for v in signs]),
                                  dtype=np.int8)
        t = int(np.asarray(signs[-1]).size)
    _check(load().tr_stream_set_samples(handle, None if a is None else a.ctypes.data,
                                        None if sg is None else sg.ctypes.data, t), handle)


def tr_stream_get_stats(handle):
    """dict of the handle's counters (tr_stats)."""
    st = tr_stats()
    _check(load().tr_stream_get_stats(handle, ctypes.byref(st)), handle)
    return {"pinv_fallbacks": st.pinv_fallbacks, "init_sweeps": st.init_sweeps,
            "init_rel_err": st.init_rel_err}


def tr_batch_als(X, ranks, cores_in=None, max_sweeps=100, tol=1e-8, compute_dtype="f64", seed=0,
                 device=0, hip_stream=None):
    """Batch TR-ALS-NE (Alg. 2) on the device over the whole tensor X
    (I_1..I_{N-1}, T).  Returns (cores, rel_errs) with host cores
    (R_n, I_n, R_{n+1}) and the error of the start and after every sweep."""
    lib = load()
    shape = tuple(X.shape)
    N = len(shape)
    cfg, ckeep = make_config(shape, ranks, compute_dtype, seed=seed, device=device,
                             hip_stream=hip_stream)
    xp, xkeep, xdev, _ = as_buffer(X, np.float64)
    if cores_in is None:
        cptr, cdev, cbufs = None, 0, []
    else:
        cbufs = [as_buffer(G, np.float64) for G in cores_in]
        cdev = cbufs[0][2]
        cptr = _ptr_array([b[0] for b in cbufs])
    outs = [np.zeros((ranks[k], shape[k], ranks[(k + 1) % N]), order="F") for k in range(N)]
    errs = np.zeros(int(max_sweeps) + 1)
    done = c_int32()
    _check(lib.tr_batch_als(ctypes.byref(cfg), xp, shape[-1], xdev, cptr, cdev, int(max_sweeps),
                            float(tol), _ptr_array([o.ctypes.data for o in outs]),
                            errs.ctypes.data, ctypes.byref(done)))
    return outs, errs[:done.value + 1].copy()


def tr_stream_save(handle, path):
    _check(load().tr_stream_save(handle, os.fsencode(path)), handle)


def tr_stream_load(path, dims=None, ranks=None, compute_dtype="f64", sketch=None,
                   sketch_size=0, device=0, hip_stream=None, max_slices=0):
    """Returns a handle resumed from a file written by tr_stream_save.  With
    dims (I_1..I_{N-1}) and ranks given, the library checks them, the dtype
    and the sketch against the saved state."""
    lib = load()
    keep = []
    cfg = tr_config(order=0, max_slices=int(max_slices), device=int(device),
                    hip_stream=hip_stream)
    if dims is not None:
        N = len(ranks)
        d = (c_int64 * (N - 1))(*[int(i) for i in dims])
        r = (c_int32 * N)(*[int(x) for x in ranks])
        keep += [d, r]
        cfg.order, cfg.dims, cfg.ranks = N, d, r
        cfg.compute_dtype, cfg.sketch = DTYPES[compute_dtype], SKETCHES[sketch]
        cfg.sketch_size = int(sketch_size)
    handle = c_void_p()
    code = lib.tr_stream_load(os.fsencode(path), ctypes.byref(cfg), ctypes.byref(handle))
    if code != 0:
        msg = ""
        if handle:
            m = lib.tr_last_error(handle)
            msg = m.decode() if m else ""
            lib.tr_stream_destroy(handle)
        raise TRError(code, msg)
    return handle


def tr_stream_sync(handle):
    _check(load().tr_stream_sync(handle), handle)


def tr_stream_profile(handle, enable):
    _check(load().tr_stream_profile(handle, int(enable)), handle)


def tr_stream_profile_read(handle, kind):
    """(total milliseconds, launches) of one kernel kind since profiling began."""
    ms, n = c_double(), c_int64()
    _check(load().tr_stream_profile_read(handle, int(kind), ctypes.byref(ms), ctypes.byref(n)),
           handle)
    return ms.value, n.value


def tr_stream_num_slices(handle):
    return load().tr_stream_num_slices(handle)


def tr_last_error(handle):
    m = load().tr_last_error(handle)
    return m.decode() if m else ""


def tr_stream_destroy(handle):
    load().tr_stream_destroy(handle)


def tr_workspace_bytes(dims, ranks, dt):
    N = len(dims)
    d = (c_int64 * N)(*dims)
    r = (c_int32 * N)(*ranks)
    return load().tr_workspace_bytes(N, d, r, DTYPES[dt] if isinstance(dt, str) else dt)


def _shape_args(dims, ranks):
    N = len(dims)
    return N, (c_int64 * N)(*[int(x) for x in dims]), (c_int32 * N)(*[int(x) for x in ranks])


def tr_mttkrp(dims, ranks, dt, n, X_ptr, core_ptrs, P_ptr, accumulate, ws_ptr, ws_bytes, stream):
    N, d, r = _shape_args(dims, ranks)
    _check(load().tr_mttkrp(N, d, r, dt, n, X_ptr, _ptr_array(core_ptrs), P_ptr, int(accumulate),
                            ws_ptr, ws_bytes, stream))


def tr_mttkrp_noalloc(dims, ranks, dt, n, X_ptr, core_ptrs, P_ptr, accumulate, stream):
    N, d, r = _shape_args(dims, ranks)
    _check(load().tr_mttkrp_noalloc(N, d, r, dt, n, X_ptr, _ptr_array(core_ptrs), P_ptr,
                                    int(accumulate), stream))


def tr_mttkrp_noalloc_max_bytes():
    return load().tr_mttkrp_noalloc_max_bytes()


def tr_gram_chain(dims, ranks, n, Z_ptrs, Q_ptr, accumulate, ws_ptr, ws_bytes, stream):
    N, d, r = _shape_args(dims, ranks)
    _check(load().tr_gram_chain(N, d, r, n, _ptr_array(Z_ptrs), Q_ptr, int(accumulate), ws_ptr,
                                ws_bytes, stream))


def tr_fit_loss_fwd(dims, ranks, dt, X_ptr, core_ptrs, loss_ptr, ws_ptr, ws_bytes, stream):
    N, d, r = _shape_args(dims, ranks)
    _check(load().tr_fit_loss_fwd(N, d, r, dt, X_ptr, _ptr_array(core_ptrs), loss_ptr, ws_ptr,
                                  ws_bytes, stream))


def tr_fit_loss_bwd(dims, ranks, dt, X_ptr, core_ptrs, grad_scale, grad_ptrs, ws_ptr, ws_bytes,
                    stream):
    N, d, r = _shape_args(dims, ranks)
    _check(load().tr_fit_loss_bwd(N, d, r, dt, X_ptr, _ptr_array(core_ptrs), float(grad_scale),
                                  _ptr_array(grad_ptrs), ws_ptr, ws_bytes, stream))
