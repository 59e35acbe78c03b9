"""Python binding of libmrg355.so (MI355X / gfx950 multi-stream MRG32k3a).

Argument marshalling only: every step runs in the HIP library.  Functions
carry the C-ABI names (include/mrg355.h); tensors are torch CUDA tensors
(device memory) or numpy arrays (host memory), passed by pointer.  The HIP
stream is torch's current stream unless one is given.

Stream records are 18 uint32 words (cur, start, sub); on the torch side they
are held as int32 tensors of shape (n, 18) and never used for arithmetic.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libmrg355.so")

MRG_GEN_MRG32K3A, MRG_GEN_MRG31K3P = 1, 2
MRG_UNIFORM, MRG_NORMAL, MRG_EXPONENTIAL, MRG_RAW = 0, 1, 2, 3
MRG_F64, MRG_F32, MRG_U32 = 0, 1, 2
MRG_RESET_STREAM, MRG_RESET_SUBSTREAM, MRG_NEXT_SUBSTREAM = 0, 1, 2
MRG_OK = 0
MRG_E_BUSY = -7
STATUS = {0: "MRG_OK", -1: "MRG_E_INVALID_ARG", -2: "MRG_E_INVALID_SEED", -3: "MRG_E_UNSUPPORTED",
          -4: "MRG_E_HIP", -5: "MRG_E_NOMEM", -6: "MRG_E_CORRUPT_STATE", -7: "MRG_E_BUSY"}
MRG_CHECK_LOG, MRG_CHECK_SQRT, MRG_CHECK_SINPI, MRG_CHECK_COSPI = 0, 1, 2, 3
MRG_CHECK_LOG_F32OUT, MRG_CHECK_SQRT_F32OUT, MRG_CHECK_SINPI_F32OUT, MRG_CHECK_COSPI_F32OUT = 4, 5, 6, 7
REC_WORDS = 18
MRG_BATCH_STATIC_WORKSPACE_BYTES = 16 << 20  # mrg_batch_launch_static's device array, per GPU


class MrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class mrg_creator(ctypes.Structure):
    _fields_ = [("s", ctypes.c_uint32 * 6)]


class mrg_launch_cfg(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("nontemporal", ctypes.c_uint32), ("arith", ctypes.c_uint32),
                ("streams_per_lane", ctypes.c_uint32), ("xcd_remap", ctypes.c_uint32),
                ("lockstep", ctypes.c_uint32)]


CFG_KEYS = ("block", "chunk", "nontemporal", "arith", "streams_per_lane", "xcd_remap", "lockstep")


def launch_cfg(cfg):
    """dict -> mrg_launch_cfg (missing keys are 0 = automatic)."""
    unknown = set(cfg) - set(CFG_KEYS)
    if unknown:
        raise ValueError(f"unknown launch keys {sorted(unknown)}")
    return mrg_launch_cfg(*[int(cfg.get(k, 0)) for k in CFG_KEYS])


class mrg_request(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_void_p), ("n_streams", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("dist", ctypes.c_int), ("dtype", ctypes.c_int), ("param", ctypes.c_double),
                ("out", ctypes.c_void_p)]


class mrg_batch_cfg(ctypes.Structure):
    _fields_ = [("tile_units", ctypes.c_uint32), ("waves_per_simd", ctypes.c_uint32),
                ("wide_stores", ctypes.c_uint32), ("gang_waves", ctypes.c_uint32)]


class mrg_server_cfg(ctypes.Structure):
    _fields_ = [("n_sessions", ctypes.c_uint32), ("streams_per_session", ctypes.c_uint32),
                ("seed", ctypes.c_uint32 * 6), ("pool", ctypes.c_void_p), ("pool_bytes", ctypes.c_size_t),
                ("lanes", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("tile_units", ctypes.c_uint32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class mrg_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "released", "rejected",
                                                "samples_completed", "launches", "pool_in_use",
                                                "pool_peak", "max_in_flight", "max_lanes_busy")]


_lib = None


def lib():
    """Load libmrg355.so.  Raises when it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing; build it with "
                              "`python -m paper_2201_06604_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        vp, sz, u64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
        u32p = ctypes.POINTER(ctypes.c_uint32)
        crp = ctypes.POINTER(mrg_creator)
        sig = {
            "mrg_abi_version": (i32, []),
            "mrg_status_string": (ctypes.c_char_p, [i32]),
            "mrg_last_error": (ctypes.c_char_p, []),
            "mrg_seed_check": (i32, [i32, u32p]),
            "mrg_creator_init": (i32, [i32, crp, u32p]),
            "mrg_streams_create_host": (i32, [i32, crp, sz, vp]),
            "mrg_streams_create_device": (i32, [i32, crp, sz, vp, vp]),
            "mrg_streams_reset": (i32, [i32, vp, sz, i32, vp]),
            "mrg_streams_advance": (i32, [i32, vp, sz, u64, vp]),
            "mrg_generate": (i32, [i32, vp, sz, u64, i32, i32, ctypes.c_double, vp, vp]),
            "mrg_generate_ex": (i32, [i32, vp, sz, u64, i32, i32, ctypes.c_double, vp,
                                      ctypes.POINTER(mrg_launch_cfg), vp]),
            "mrg_generate_plan": (i32, [i32, sz, u64, i32, i32, ctypes.c_double,
                                        ctypes.POINTER(mrg_launch_cfg), ctypes.POINTER(mrg_launch_cfg)]),
            "mrg_streams_export_size": (i32, [sz, i32, ctypes.POINTER(sz)]),
            "mrg_streams_export": (i32, [i32, vp, sz, crp, vp, sz, ctypes.POINTER(sz), vp]),
            "mrg_streams_import": (i32, [i32, vp, sz, vp, sz, ctypes.POINTER(sz), crp, vp]),
            "mrg_batch_plan_create": (i32, [i32, ctypes.POINTER(mrg_request), sz,
                                            ctypes.POINTER(mrg_batch_cfg), ctypes.POINTER(vp)]),
            "mrg_batch_plan_destroy": (None, [vp]),
            "mrg_batch_workspace_size": (i32, [vp, ctypes.POINTER(sz)]),
            "mrg_batch_tile_count": (i32, [vp, ctypes.POINTER(sz)]),
            "mrg_batch_upload": (i32, [vp, vp, vp]),
            "mrg_batch_launch": (i32, [vp, vp, vp]),
            "mrg_batch_launch_static": (i32, [vp, vp]),
            "mrg_batch_request_times": (i32, [vp, vp, ctypes.POINTER(ctypes.c_uint64), vp]),
            "mrg_batch_autotune": (i32, [vp, vp, sz, vp, ctypes.POINTER(mrg_batch_cfg),
                                         ctypes.POINTER(ctypes.c_double)]),
            "mrg_batch_autotune_workspace_size": (i32, [vp, ctypes.POINTER(sz)]),
            "mrg_generate_paper": (i32, [i32, vp, sz, u64, u64, u64, ctypes.c_uint32, ctypes.c_uint32, i32, i32,
                                         ctypes.c_double, vp, vp]),
            "mrg_tables_sample": (i32, [i32, vp, sz, vp, vp, vp, vp, vp, vp, vp]),
            "mrg_fisher_sim": (i32, [i32, vp, u64, i32, i32, ctypes.POINTER(ctypes.c_int32), vp, vp,
                                     ctypes.POINTER(ctypes.c_double), vp]),
            "mrg_fisher_pvalue": (ctypes.c_double, [u64, u64]),
            "mrg_transform_accuracy": (i32, [i32, i32, u64, u64, vp, vp]),
            "mrg_store_ceiling": (i32, [sz, u64, i32, vp, vp]),
            "mrg_now_ns": (u64, []),
            "mrg_server_workspace_size": (i32, [ctypes.POINTER(mrg_server_cfg), ctypes.POINTER(sz)]),
            "mrg_server_create": (i32, [ctypes.POINTER(mrg_server_cfg), ctypes.POINTER(vp)]),
            "mrg_server_destroy": (None, [vp]),
            "mrg_server_submit": (i32, [vp, ctypes.c_uint32, u64, i32, i32, ctypes.c_double, u64,
                                        ctypes.POINTER(u64), ctypes.POINTER(u64)]),
            "mrg_server_poll": (i32, [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(u64)]),
            "mrg_server_release": (i32, [vp, u64]),
            "mrg_server_stats_get": (i32, [vp, ctypes.POINTER(mrg_server_stats)]),
            "mrg_server_drive": (i32, [vp, sz, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(u64), i32, i32, ctypes.c_double,
                                       ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


EXPORTED = ["mrg_abi_version", "mrg_status_string", "mrg_last_error", "mrg_seed_check",
            "mrg_creator_init", "mrg_streams_create_host", "mrg_streams_create_device",
            "mrg_streams_reset", "mrg_streams_advance", "mrg_generate", "mrg_generate_ex", "mrg_generate_plan",
            "mrg_streams_export_size", "mrg_streams_export", "mrg_streams_import",
            "mrg_generate_paper", "mrg_tables_sample", "mrg_fisher_sim", "mrg_fisher_pvalue",
            "mrg_batch_plan_create", "mrg_batch_plan_destroy", "mrg_batch_workspace_size",
            "mrg_batch_tile_count", "mrg_batch_upload", "mrg_batch_launch", "mrg_batch_launch_static",
            "mrg_batch_request_times", "mrg_batch_autotune", "mrg_batch_autotune_workspace_size",
            "mrg_transform_accuracy", "mrg_store_ceiling",
            "mrg_now_ns", "mrg_server_workspace_size", "mrg_server_create",
            "mrg_server_destroy", "mrg_server_submit", "mrg_server_poll", "mrg_server_release",
            "mrg_server_stats_get", "mrg_server_drive"]


def _check(st):
    if st != MRG_OK:
        raise MrgError(st, lib().mrg_last_error().decode())
    return st


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    """Device pointer of a torch CUDA tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    if not t.is_cuda:
        raise ValueError("expected a device (CUDA) tensor")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, n_bytes, what, esz=None):
    """A device tensor `t` must hold n_bytes contiguous bytes (and, when esz
    is given, elements of that size): the library cannot see buffer sizes,
    so a short buffer would be written past its end."""
    if t is None or isinstance(t, int):
        return
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a device (CUDA) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if esz is not None and t.element_size() != esz:
        raise ValueError(f"{what}: expected {esz}-byte elements, got {t.element_size()}")
    if t.numel() * t.element_size() < n_bytes:
        raise ValueError(f"{what}: needs {n_bytes} bytes, has {t.numel() * t.element_size()}")


def _seed_arr(seed):
    a = np.ascontiguousarray(np.asarray(seed, dtype=np.uint64).astype(np.uint32))
    if a.shape != (6,) or not np.array_equal(a.astype(np.uint64), np.asarray(seed, dtype=np.uint64)):
        raise ValueError("seed must be 6 integers below 2^32")
    return a


# ------------------------------------------------------------------ C names
def mrg_abi_version():
    return lib().mrg_abi_version()


def mrg_seed_check(seed, gen=MRG_GEN_MRG32K3A):
    """Returns the status code (0 = valid) without raising."""
    a = _seed_arr(seed)
    return lib().mrg_seed_check(gen, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))


def mrg_creator_init(seed, gen=MRG_GEN_MRG32K3A):
    c = mrg_creator()
    a = _seed_arr(seed)
    _check(lib().mrg_creator_init(gen, ctypes.byref(c), a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return c


def creator_words(c):
    return np.array(list(c.s), dtype=np.uint32)


def mrg_streams_create_host(creator, n, gen=MRG_GEN_MRG32K3A):
    """n stream records as a host numpy array (n, 18) uint32; `creator` advances."""
    out = np.zeros((n, REC_WORDS), dtype=np.uint32)
    _check(lib().mrg_streams_create_host(gen, ctypes.byref(creator), n,
                                         out.ctypes.data_as(ctypes.c_void_p) if n else None))
    return out


def new_streams_tensor(n, device="cuda"):
    import torch
    return torch.empty((n, REC_WORDS), dtype=torch.int32, device=device)


def mrg_streams_create_device(creator, n, out=None, gen=MRG_GEN_MRG32K3A, stream=None):
    """n stream records written by a kernel into `out` (torch int32 (n,18) on
    the device; allocated when None); `creator` advances."""
    if out is None:
        out = new_streams_tensor(max(n, 1))
    _need(out, n * REC_WORDS * 4, "stream records")
    _check(lib().mrg_streams_create_device(gen, ctypes.byref(creator), n, _dptr(out), _stream(stream)))
    return out


def mrg_streams_reset(streams, kind, n=None, gen=MRG_GEN_MRG32K3A, stream=None):
    n = streams.shape[0] if n is None else n
    _need(streams, n * REC_WORDS * 4, "stream records")
    _check(lib().mrg_streams_reset(gen, _dptr(streams), n, kind, _stream(stream)))


def mrg_streams_advance(streams, steps, n=None, gen=MRG_GEN_MRG32K3A, stream=None):
    n = streams.shape[0] if n is None else n
    _need(streams, n * REC_WORDS * 4, "stream records")
    _check(lib().mrg_streams_advance(gen, _dptr(streams), n, steps, _stream(stream)))


_TORCH_DT = {MRG_F64: "float64", MRG_F32: "float32", MRG_U32: "int32"}


def new_output(n, dtype, device="cuda"):
    import torch
    return torch.empty(max(n, 1), dtype=getattr(torch, _TORCH_DT[dtype]), device=device)


def mrg_generate(streams, n, dist=MRG_UNIFORM, dtype=MRG_F64, param=1.0, out=None,
                 n_streams=None, cfg=None, gen=MRG_GEN_MRG32K3A, stream=None):
    """n numbers from the device stream records `streams` into `out`
    (element k*S + s = draw k of stream s).  U32 results come back in an
    int32 tensor holding the raw 32-bit words.  `cfg` = dict with keys of
    CFG_KEYS selects a launch shape (results do not change)."""
    S = streams.shape[0] if n_streams is None else n_streams
    if out is None:
        out = new_output(n, dtype)
    _need(streams, S * REC_WORDS * 4, "stream records")
    _need(out, n * (8 if dtype == MRG_F64 else 4), "output", 8 if dtype == MRG_F64 else 4)
    if cfg is None:
        st = lib().mrg_generate(gen, _dptr(streams), S, n, dist, dtype, param, _dptr(out),
                                _stream(stream))
    else:
        c = launch_cfg(cfg)
        st = lib().mrg_generate_ex(gen, _dptr(streams), S, n, dist, dtype, param, _dptr(out),
                                   ctypes.byref(c), _stream(stream))
    _check(st)
    return out


def mrg_generate_plan(n_streams, n, dist=MRG_UNIFORM, dtype=MRG_F64, param=1.0, cfg=None,
                      gen=MRG_GEN_MRG32K3A):
    """The launch shape mrg_generate would use (host only, nothing runs), as
    a dict with the keys of CFG_KEYS."""
    res = mrg_launch_cfg()
    c = None if cfg is None else ctypes.byref(launch_cfg(cfg))
    _check(lib().mrg_generate_plan(gen, n_streams, n, dist, dtype, param, c, ctypes.byref(res)))
    return {k: int(getattr(res, k)) for k in CFG_KEYS}


def mrg_generate_status(streams_ptr, n_streams, n, dist, dtype, param, out_ptr,
                        gen=MRG_GEN_MRG32K3A, stream=0):
    """Raw call returning the status code (for error-path tests)."""
    return lib().mrg_generate(gen, ctypes.c_void_p(streams_ptr), n_streams, n, dist, dtype, param,
                              ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream))


def mrg_streams_export(streams, n=None, creator=None, gen=MRG_GEN_MRG32K3A, stream=None):
    """Save n device records (+ creator) into a bytes object."""
    n = streams.shape[0] if n is None else n
    _need(streams, n * REC_WORDS * 4, "stream records")
    need = ctypes.c_size_t()
    _check(lib().mrg_streams_export_size(n, 1 if creator is not None else 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    ln = ctypes.c_size_t()
    _check(lib().mrg_streams_export(gen, _dptr(streams) if n else None, n,
                                    ctypes.byref(creator) if creator is not None else None,
                                    buf, need.value, ctypes.byref(ln), _stream(stream)))
    return buf.raw[:ln.value]


def mrg_streams_import(data, out, creator=None, gen=MRG_GEN_MRG32K3A, stream=None):
    """Restore records from `data` into device tensor `out` (and `creator`).
    Returns the number of records."""
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    cnt = ctypes.c_size_t()
    _check(lib().mrg_streams_import(gen, buf, len(data), _dptr(out) if out is not None else None,
                                    out.shape[0] if out is not None else 0, ctypes.byref(cnt),
                                    ctypes.byref(creator) if creator is not None else None,
                                    _stream(stream)))
    return cnt.value


def mrg_generate_paper(streams, nrow, ncol, G0, G1, dist=MRG_UNIFORM, dtype=MRG_F64, param=1.0, out=None,
                       npad=None, gen=MRG_GEN_MRG32K3A, stream=None):
    """clrng's placement (Listing 1 / Listing 2): an nrow x ncol block of an
    nrow x npad buffer from a G0 x G1 lattice of work-items (Nglobal).
    Returns the nrow x npad tensor (columns past ncol untouched)."""
    import torch
    npad = ncol if npad is None else npad
    if out is None:
        out = torch.empty((max(nrow, 1), max(npad, 1)), dtype=getattr(torch, _TORCH_DT[dtype]),
                          device=streams.device)
    esz = 8 if dtype == MRG_F64 else 4
    _need(out, nrow * npad * esz, "output", esz)
    _check(lib().mrg_generate_paper(gen, _dptr(streams), streams.shape[0], nrow, ncol, npad, G0, G1, dist, dtype,
                                    param, _dptr(out), _stream(stream)))
    return out


def mrg_tables_sample(streams, I, J, rows, cols, tables=None, stats=None, n=None,
                      gen=MRG_GEN_MRG32K3A, stream=None):
    """Random contingency tables with fixed margins (Section 4): table t of
    shape I[t] x J[t] (<= 5 x 5) with margins rows[t, :5], cols[t, :5] (device
    int32) from stream t.  Returns (tables [n, 5, 5] int32, stats [n] f64 or
    None); pass stats=True to have the statistics allocated."""
    import torch
    n = I.shape[0] if n is None else n
    if n > streams.shape[0] or n > I.shape[0] or n > J.shape[0]:
        raise ValueError("n exceeds the streams or shapes given")
    if rows.numel() < 5 * n or cols.numel() < 5 * n:
        raise ValueError("rows and cols need 5 entries per table")
    for t in (I, J, rows, cols):
        if t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("shapes and margins must be contiguous int32 tensors")
    if tables is not None and tables.numel() < 25 * n:
        raise ValueError("tables needs 25 entries per table")
    if tables is None:
        tables = torch.empty((max(n, 1), 5, 5), dtype=torch.int32, device=streams.device)
    if stats is True:
        stats = torch.empty(max(n, 1), dtype=torch.float64, device=streams.device)
    _check(lib().mrg_tables_sample(gen, _dptr(streams), n, _dptr(I), _dptr(J), _dptr(rows), _dptr(cols),
                                   _dptr(tables), _dptr(stats) if stats is not None else None,
                                   _stream(stream)))
    return tables, stats


def mrg_fisher_sim(streams, observed, B=None, stats=None, count=None, gen=MRG_GEN_MRG32K3A, stream=None):
    """Monte-Carlo Fisher test (Section 4) of the host table `observed` with B
    replicates, replicate b from stream b.  Returns (count device tensor
    [1] int64, observed statistic, stats tensor or None).  Pass stats=True to
    keep the replicates' statistics."""
    import torch
    obs = np.ascontiguousarray(np.asarray(observed, dtype=np.int32))
    if obs.ndim != 2:
        raise ValueError("observed must be a 2-D table")
    B = streams.shape[0] if B is None else B
    if B > streams.shape[0]:
        raise ValueError("B exceeds the number of streams")
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=streams.device)
    if stats is True:
        stats = torch.empty(max(B, 1), dtype=torch.float64, device=streams.device)
    ostat = ctypes.c_double()
    _check(lib().mrg_fisher_sim(gen, _dptr(streams), B, obs.shape[0], obs.shape[1],
                                obs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(count),
                                _dptr(stats) if stats is not None else None, ctypes.byref(ostat),
                                _stream(stream)))
    return count, ostat.value, stats


def mrg_fisher_pvalue(count, B):
    return lib().mrg_fisher_pvalue(int(count), int(B))


def mrg_transform_accuracy(fn, z_begin=1, z_end=None, gen=MRG_GEN_MRG32K3A, result=None, stream=None):
    """Distance in ulp between the library's own log / sqrt / sin(pi t) /
    cos(pi t) and the HIP device math library over every generator output z
    in [z_begin, z_end) (default: all of [1, m1]).  Returns a dict with the
    histogram (0, 1, 2, 3, >= 4 ulp), the largest distance and the z where it
    occurs.  Synchronises the stream."""
    import torch
    if z_end is None:
        z_end = (4294967087 if gen == MRG_GEN_MRG32K3A else 2147483647) + 1
    if result is None:
        result = torch.empty(8, dtype=torch.int64, device="cuda")
    _need(result, 64, "result", 8)
    _check(lib().mrg_transform_accuracy(gen, fn, z_begin, z_end, _dptr(result), _stream(stream)))
    r = result.cpu().numpy().view(np.uint64)
    return {"hist": [int(v) for v in r[:5]], "max_ulp": int(r[5] >> np.uint64(32)),
            "z_at_max": int(r[5] & np.uint64(0xffffffff))}


def mrg_store_ceiling(n_streams, n, dtype=MRG_F64, out=None, stream=None):
    """Write 0.5 into n elements of `out` with mrg_generate's store pattern
    for uniforms of this dtype over n_streams streams (nothing computed)."""
    esz = 8 if dtype == MRG_F64 else 4
    if out is None:
        out = new_output(n, dtype)
    _need(out, n * esz, "output", esz)
    _check(lib().mrg_store_ceiling(n_streams, n, dtype, _dptr(out), _stream(stream)))
    return out


def as_u32(t):
    """Device int32 tensor -> host numpy uint32 (bit reinterpretation)."""
    return t.detach().cpu().numpy().view(np.uint32)


# ------------------------------------------------------------------ batching
def make_request(streams, n, dist, dtype, param=1.0, out=None, n_streams=None):
    """mrg_request for device tensors `streams` ((S,18) int32) and `out`."""
    S = streams.shape[0] if n_streams is None else n_streams
    _need(streams, S * REC_WORDS * 4, "stream records")
    _need(out, n * (8 if dtype == MRG_F64 else 4), "output", 8 if dtype == MRG_F64 else 4)
    return mrg_request(streams.data_ptr() if streams is not None else None, S, n, dist, dtype, param,
                       out.data_ptr() if out is not None else None)


class BatchPlan:
    """Owns an mrg_batch_plan; the device workspace is a torch uint8 tensor."""

    def __init__(self, requests, cfg=None, gen=MRG_GEN_MRG32K3A):
        arr = (mrg_request * max(len(requests), 1))(*requests)
        c = None if cfg is None else ctypes.byref(mrg_batch_cfg(cfg.get("tile_units", 0),
                                                                cfg.get("waves_per_simd", 0),
                                                                cfg.get("wide_stores", 0),
                                                                cfg.get("gang_waves", 0)))
        self._p = ctypes.c_void_p()
        _check(lib().mrg_batch_plan_create(gen, arr, len(requests), c, ctypes.byref(self._p)))
        self.n_req = len(requests)
        self.workspace = None

    def __del__(self):
        if getattr(self, "_p", None) and self._p.value and _lib is not None:
            _lib.mrg_batch_plan_destroy(self._p)
            self._p = None

    def workspace_size(self):
        b = ctypes.c_size_t()
        _check(lib().mrg_batch_workspace_size(self._p, ctypes.byref(b)))
        return b.value

    def tile_count(self):
        b = ctypes.c_size_t()
        _check(lib().mrg_batch_tile_count(self._p, ctypes.byref(b)))
        return b.value

    def alloc_workspace(self, nbytes=None, device="cuda"):
        import torch
        nbytes = self.workspace_size() if nbytes is None else nbytes
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self._ws_bytes = nbytes
        return self._ws_ptr

    def upload(self, stream=None):
        if self.workspace is None:
            self.alloc_workspace()
        _check(lib().mrg_batch_upload(self._p, ctypes.c_void_p(self._ws_ptr), _stream(stream)))

    def launch(self, stream=None):
        _check(lib().mrg_batch_launch(self._p, ctypes.c_void_p(self._ws_ptr), _stream(stream)))

    def launch_static(self, stream=None):
        """Upload and launch with the library's static device workspace (no
        allocation anywhere; the plan must outlive the launch)."""
        _check(lib().mrg_batch_launch_static(self._p, _stream(stream)))

    def request_times(self, stream=None):
        """Device real-time clock ticks (100 MHz): [start, done_0, ..., done_{n-1}]."""
        t = (ctypes.c_uint64 * (self.n_req + 1))()
        _check(lib().mrg_batch_request_times(self._p, ctypes.c_void_p(self._ws_ptr), t, _stream(stream)))
        return np.array(list(t), dtype=np.uint64)

    def autotune_workspace_size(self):
        b = ctypes.c_size_t()
        _check(lib().mrg_batch_autotune_workspace_size(self._p, ctypes.byref(b)))
        return b.value

    def autotune(self, stream=None):
        """Time the candidate shapes and keep the fastest; the workspace is
        grown first so that every candidate fits (then uploaded again).  A
        graph captured with the previous workspace must be captured again
        after this call, and the plan's tables are re-cut for the chosen shape."""
        need = self.autotune_workspace_size()
        if self.workspace is None or self._ws_bytes < need:
            self.alloc_workspace(need)
        best = mrg_batch_cfg()
        ms = ctypes.c_double()
        _check(lib().mrg_batch_autotune(self._p, ctypes.c_void_p(self._ws_ptr), self._ws_bytes,
                                        _stream(stream), ctypes.byref(best), ctypes.byref(ms)))
        return dict(tile_units=best.tile_units, waves_per_simd=best.waves_per_simd,
                    wide_stores=best.wide_stores, gang_waves=best.gang_waves), ms.value


# ------------------------------------------------------------------ serving
def mrg_now_ns():
    return lib().mrg_now_ns()


class Server:
    """Owns an mrg_server.  `pool` is a device tensor the outputs live in."""

    def __init__(self, n_sessions, seed, pool, streams_per_session=0, lanes=0, max_batch=0, mode=0,
                 tile_units=0):
        cfg = mrg_server_cfg()
        cfg.n_sessions = n_sessions
        cfg.streams_per_session = streams_per_session
        for i, v in enumerate(_seed_arr(seed)):
            cfg.seed[i] = int(v)
        self.pool = pool
        cfg.pool = pool.data_ptr()
        cfg.pool_bytes = pool.numel() * pool.element_size()
        cfg.lanes, cfg.max_batch, cfg.mode, cfg.tile_units = lanes, max_batch, mode, tile_units
        need = ctypes.c_size_t()
        _check(lib().mrg_server_workspace_size(ctypes.byref(cfg), ctypes.byref(need)))
        import torch
        self.workspace = torch.empty(need.value + 256, dtype=torch.uint8, device=pool.device)
        cfg.workspace = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        cfg.workspace_bytes = need.value
        self._s = ctypes.c_void_p()
        _check(lib().mrg_server_create(ctypes.byref(cfg), ctypes.byref(self._s)))
        self.S = streams_per_session or 64

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            lib().mrg_server_destroy(self._s)
            self._s = None
        self.workspace = None

    def __del__(self):
        if _lib is not None:
            self.close()

    def submit(self, session, n, dist=MRG_NORMAL, dtype=MRG_F64, param=1.0, t_arrival_ns=None):
        t = ctypes.c_uint64()
        off = ctypes.c_uint64()
        arr = mrg_now_ns() if t_arrival_ns is None else t_arrival_ns
        _check(lib().mrg_server_submit(self._s, session, n, dist, dtype, param, arr, ctypes.byref(t),
                                       ctypes.byref(off)))
        return t.value, off.value

    def submit_status(self, session, n, dist=MRG_NORMAL, dtype=MRG_F64, param=1.0):
        t = ctypes.c_uint64()
        return lib().mrg_server_submit(self._s, session, n, dist, dtype, param, mrg_now_ns(), ctypes.byref(t),
                                       None)

    def poll(self, ticket):
        """(done, device address of the output, completion time ns)."""
        d = ctypes.c_int()
        p = ctypes.c_void_p()
        t = ctypes.c_uint64()
        st = lib().mrg_server_poll(self._s, ticket, ctypes.byref(d), ctypes.byref(p), ctypes.byref(t))
        if st == MRG_E_BUSY:
            return False, None, 0
        _check(st)
        return bool(d.value), p.value, t.value

    def release(self, ticket):
        _check(lib().mrg_server_release(self._s, ticket))

    def stats(self):
        st = mrg_server_stats()
        _check(lib().mrg_server_stats_get(self._s, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def drive(self, t_arrival_ns, sessions, n_draws, dist=MRG_NORMAL, dtype=MRG_F64, param=1.0):
        """Open-loop replay; returns (latency_ns array, span_ns)."""
        n = len(t_arrival_ns)
        ta = np.ascontiguousarray(t_arrival_ns, dtype=np.uint64)
        se = np.ascontiguousarray(sessions, dtype=np.uint32)
        nd = np.ascontiguousarray(n_draws, dtype=np.uint64)
        lat = np.zeros(n, dtype=np.uint64)
        span = ctypes.c_uint64()
        u64p = ctypes.POINTER(ctypes.c_uint64)
        _check(lib().mrg_server_drive(self._s, n, ta.ctypes.data_as(u64p),
                                      se.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                      nd.ctypes.data_as(u64p), dist, dtype, param, lat.ctypes.data_as(u64p),
                                      ctypes.byref(span)))
        return lat, span.value
