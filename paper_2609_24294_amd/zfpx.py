"""Thin ctypes binding of libzfpx.so (declared in include/zfpx.h).

Argument marshalling only: every step of the coding runs in the HIP
kernels of the library.  PyTorch supplies device memory (tensors) and
streams; the functions take CUDA/HIP tensors and pass their device pointers
and the current HIP stream through the C ABI.  There is no fallback: if the
library is not built, importing this module raises.

Compressed streams are held in int64 tensors (one element per 64-bit word).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzfpx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python -m paper_2609_24294_amd.build)")

_lib = ctypes.CDLL(LIB_PATH)

_c = ctypes
_P = _c.c_void_p
_I64 = _c.c_int64
_I32 = _c.c_int32
_INT = _c.c_int
_SZ = _c.c_size_t
_PI64 = _c.POINTER(_c.c_int64)
_PI32 = _c.POINTER(_c.c_int32)

_SIGS = {
    "zfpx_status_string": (_c.c_char_p, [_INT]),
    "zfpx_version": (_INT, []),
    "zfpx_device_cus": (_INT, []),
    "zfpx_fixed_rate_bytes": (_I64, [_I64, _I64, _I64, _INT]),
    "zfpx_encode_fixed_rate": (_INT, [_P, _I64, _I64, _I64, _I64, _I64, _I64, _INT, _P, _SZ, _P]),
    "zfpx_decode_fixed_rate": (_INT, [_P, _SZ, _I64, _I64, _I64, _I64, _I64, _I64, _INT, _P, _P]),
    "zfpx_plan_create": (_INT, [_I32, _PI64, _PI64, _PI32, _PI32, _PI64, _PI32, _c.POINTER(_P)]),
    "zfpx_plan_destroy": (_INT, [_P]),
    "zfpx_plan_info": (_INT, [_P, _PI64, _PI64, _PI64]),
    "zfpx_plan_sizes": (_INT, [_P, _INT, _PI64, _PI64, _PI64]),
    "zfpx_pack_encode": (_INT, [_P, _P, _I64, _INT, _P, _SZ, _P]),
    "zfpx_decode_unpack": (_INT, [_P, _P, _SZ, _INT, _P, _I64, _P]),
    "zfpx_pack_encode_chunks": (_INT, [_P, _I32, _I32, _P, _I64, _INT, _P, _SZ, _P]),
    "zfpx_decode_unpack_chunks": (_INT, [_P, _I32, _I32, _P, _SZ, _INT, _P, _I64, _P]),
    "zfpx_plan_set_config": (_INT, [_P, _INT, _INT, _INT, _INT]),
    "zfpx_plan_get_config": (_INT, [_P, _INT, _INT, _c.POINTER(_INT), _c.POINTER(_INT)]),
    "zfpx_autotune": (_INT, [_P, _INT, _INT, _P, _I64, _P, _SZ, _P, _I64, _c.c_char_p, _P,
                             _c.POINTER(_c.c_double)]),
    "zfpx_graph_create": (_INT, [_P, _INT, _P, _I64, _P, _SZ, _P, _I64, _c.POINTER(_P)]),
    "zfpx_graph_launch": (_INT, [_P, _P]),
    "zfpx_graph_destroy": (_INT, [_P]),
    "zfpx_server_create": (_INT, [_SZ, _I32, _I32, _c.POINTER(_P)]),
    "zfpx_server_submit": (_INT, [_P, _P, _c.POINTER(_c.c_uint64)]),
    "zfpx_server_progress": (_INT, [_P]),
    "zfpx_server_poll": (_INT, [_P, _c.c_uint64, _c.POINTER(_INT), _c.POINTER(_c.c_double)]),
    "zfpx_server_drain": (_INT, [_P, _c.c_double]),
    "zfpx_server_stats": (_INT, [_P, _c.POINTER(_c.c_uint64), _c.POINTER(_SZ),
                                 _c.POINTER(_c.c_uint64)]),
    "zfpx_server_set_max_queue": (_INT, [_P, _SZ]),
    "zfpx_server_set_idle_us": (_INT, [_P, _c.c_uint64]),
    "zfpx_server_destroy": (_INT, [_P]),
    "zfpx_server_replay": (_INT, [_P, _P, _P, _I64, _c.c_double, _P]),
    "zfpx_plain_replay": (_INT, [_P, _P, _I64, _c.c_double, _P, _P]),
    "zfpx_pipeline_create": (_INT, [_P, _INT, _I32, _c.POINTER(_P)]),
    "zfpx_pipeline_send": (_INT, [_P, _P, _I64, _P, _SZ, _P, _SZ, _P, _P]),
    "zfpx_pipeline_recv": (_INT, [_P, _P, _SZ, _P, _SZ, _P, _I64, _P, _P]),
    "zfpx_pipeline_destroy": (_INT, [_P]),
    "zfpx_accuracy_minexp": (_INT, [_c.c_double]),
    "zfpx_plan_var_sizes": (_INT, [_P, _INT, _PI64, _PI64, _c.POINTER(_SZ)]),
    "zfpx_plan_encode_var": (_INT, [_P, _P, _I64, _INT, _INT, _INT, _P, _SZ, _P, _P, _P, _SZ,
                                    _P]),
    "zfpx_plan_encode_var_noalloc": (_INT, [_P, _P, _I64, _INT, _INT, _INT, _P, _SZ, _P, _P,
                                            _P]),
    "zfpx_noalloc_scratch_bytes": (_SZ, []),
    "zfpx_plan_decode_var": (_INT, [_P, _P, _SZ, _P, _P, _INT, _INT, _INT, _P, _I64, _P]),
    "zfpx_plan_var_chunk_offsets": (_INT, [_P, _P, _P, _P, _P]),
    "f16_truncate": (_INT, [_P, _SZ, _P, _P]),
    "f16_restore": (_INT, [_P, _SZ, _P, _P]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

OK, EINVAL, ENOSPC, EHIP, ENOMEM, EAGAIN, ESTATE = 0, -1, -2, -3, -4, -5, -6
OP_ENCODE, OP_DECODE = 0, 1


class ZfpxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {zfpx_status_string(status)} ({status})")


def zfpx_status_string(status: int) -> str:
    return _lib.zfpx_status_string(int(status)).decode()


def _check(st: int, where: str) -> None:
    if st != OK:
        raise ZfpxError(st, where)


def library():
    """The loaded ctypes library (for calls with raw pointers)."""
    return _lib


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def _dev(t: torch.Tensor, dtype=None) -> int:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def zfpx_version() -> int:
    return _lib.zfpx_version()


def zfpx_device_cus() -> int:
    return _lib.zfpx_device_cus()


# ---------------------------------------------------------------------------
# Regular arrays
# ---------------------------------------------------------------------------

def zfpx_fixed_rate_bytes(nx: int, ny: int, nz: int, rate: int) -> int:
    n = _lib.zfpx_fixed_rate_bytes(nx, ny, nz, rate)
    _check(n if n < 0 else 0, "zfpx_fixed_rate_bytes")
    return n


def zfpx_encode_fixed_rate(src: torch.Tensor, rate: int, out: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
    """Encode a (nz, ny, nx) float32 device tensor (any strides)."""
    nz, ny, nx = src.shape
    sz, sy, sx = src.stride()
    nbytes = zfpx_fixed_rate_bytes(nx, ny, nz, rate)
    if out is None:
        out = torch.empty(nbytes // 8, dtype=torch.int64, device=src.device)
    _check(_lib.zfpx_encode_fixed_rate(_dev(src, torch.float32), nx, ny, nz, sx, sy, sz, rate,
                                       _dev(out), _nbytes(out), _stream(stream)),
           "zfpx_encode_fixed_rate")
    return out


def zfpx_decode_fixed_rate(words: torch.Tensor, rate: int, out: torch.Tensor, stream=None):
    """Decode into `out`, a (nz, ny, nx) float32 device tensor (any strides)."""
    nz, ny, nx = out.shape
    sz, sy, sx = out.stride()
    _check(_lib.zfpx_decode_fixed_rate(_dev(words), _nbytes(words), nx, ny, nz, sx, sy, sz, rate,
                                       _dev(out, torch.float32), _stream(stream)),
           "zfpx_decode_fixed_rate")
    return out


# ---------------------------------------------------------------------------
# Plans
# ---------------------------------------------------------------------------

def _arr(a, ctype):
    import numpy as np
    dt = np.int64 if ctype is _c.c_int64 else np.int32
    a = np.ascontiguousarray(a, dtype=dt)
    return a, a.ctypes.data_as(_c.POINTER(ctype))


class Plan:
    """Owns a zfpx_plan built from chunk tables (see include/zfpx.h)."""

    def __init__(self, chunk_base, level_stride, levels, row_start, row_offset, row_len):
        keep = []
        args = []
        for a, ct in ((chunk_base, _I64), (level_stride, _I64), (levels, _I32),
                      (row_start, _I32), (row_offset, _I64), (row_len, _I32)):
            arr, ptr = _arr(a, ct)
            keep.append(arr)
            args.append(ptr)
        self.nchunks = int(keep[0].size)
        h = _P()
        _check(_lib.zfpx_plan_create(self.nchunks, *args, _c.byref(h)), "zfpx_plan_create")
        self._h = h
        nb, nv, ne = _I64(), _I64(), _I64()
        _check(_lib.zfpx_plan_info(h, _c.byref(nb), _c.byref(nv), _c.byref(ne)), "zfpx_plan_info")
        self.nblocks, self.nvalues, self.min_buffer_elems = nb.value, nv.value, ne.value

    @classmethod
    def from_chunkset(cls, cs) -> "Plan":
        return cls(cs.chunk_base, cs.level_stride, cs.levels, cs.row_start, cs.row_offset,
                   cs.row_len)

    @property
    def handle(self):
        return self._h

    def sizes(self, rate: int):
        """(per-chunk bytes, per-chunk offsets, total bytes)."""
        import numpy as np
        b = np.zeros(max(self.nchunks, 1), np.int64)
        o = np.zeros(max(self.nchunks, 1), np.int64)
        t = _I64()
        _check(_lib.zfpx_plan_sizes(self._h, rate, b.ctypes.data_as(_PI64),
                                    o.ctypes.data_as(_PI64), _c.byref(t)), "zfpx_plan_sizes")
        return b[: self.nchunks], o[: self.nchunks], t.value

    def total_bytes(self, rate: int) -> int:
        return self.nblocks * 8 * rate

    def close(self):
        if getattr(self, "_h", None):
            _lib.zfpx_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def zfpx_plan_create(chunks) -> Plan:
    return Plan.from_chunkset(chunks)


def zfpx_pack_encode(plan: Plan, src: torch.Tensor, rate: int, send: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    if send is None:
        send = torch.empty(plan.nblocks * rate, dtype=torch.int64, device=src.device)
    _check(_lib.zfpx_pack_encode(plan.handle, _dev(src, torch.float32), src.numel(), rate,
                                 _dev(send), _nbytes(send), _stream(stream)), "zfpx_pack_encode")
    return send


def zfpx_decode_unpack(plan: Plan, recv: torch.Tensor, rate: int, dst: torch.Tensor,
                       stream=None) -> torch.Tensor:
    _check(_lib.zfpx_decode_unpack(plan.handle, _dev(recv), _nbytes(recv), rate,
                                   _dev(dst, torch.float32), dst.numel(), _stream(stream)),
           "zfpx_decode_unpack")
    return dst


def zfpx_pack_encode_chunks(plan: Plan, first: int, count: int, src: torch.Tensor, rate: int,
                            send: torch.Tensor, stream=None) -> torch.Tensor:
    _check(_lib.zfpx_pack_encode_chunks(plan.handle, first, count, _dev(src, torch.float32),
                                        src.numel(), rate, _dev(send), _nbytes(send),
                                        _stream(stream)), "zfpx_pack_encode_chunks")
    return send


def zfpx_decode_unpack_chunks(plan: Plan, first: int, count: int, recv: torch.Tensor, rate: int,
                              dst: torch.Tensor, stream=None) -> torch.Tensor:
    _check(_lib.zfpx_decode_unpack_chunks(plan.handle, first, count, _dev(recv), _nbytes(recv),
                                          rate, _dev(dst, torch.float32), dst.numel(),
                                          _stream(stream)), "zfpx_decode_unpack_chunks")
    return dst


# ---------------------------------------------------------------------------
# Chunk-wise pipeline over a link (host memory standing in for it)
# ---------------------------------------------------------------------------

class Pipeline:
    """zfpx_pipeline_*: encode chunk groups on one stream while the previous
    group is copied to pinned host memory on another (and the reverse)."""

    def __init__(self, plan: Plan, rate: int, groups: int):
        self.plan, self.rate = plan, rate
        h = _P()
        _check(_lib.zfpx_pipeline_create(plan.handle, rate, groups, _c.byref(h)),
               "zfpx_pipeline_create")
        self._h = h

    def send(self, src: torch.Tensor, send: torch.Tensor, link: torch.Tensor,
             compute_stream, copy_stream) -> None:
        if link.is_cuda or not link.is_pinned():
            raise ValueError("link must be pinned host memory")
        _check(_lib.zfpx_pipeline_send(self._h, _dev(src, torch.float32), src.numel(),
                                       _dev(send), _nbytes(send), link.data_ptr(), _nbytes(link),
                                       _stream(compute_stream), _stream(copy_stream)),
               "zfpx_pipeline_send")

    def recv(self, link: torch.Tensor, recv: torch.Tensor, dst: torch.Tensor,
             compute_stream, copy_stream) -> None:
        if link.is_cuda or not link.is_pinned():
            raise ValueError("link must be pinned host memory")
        _check(_lib.zfpx_pipeline_recv(self._h, link.data_ptr(), _nbytes(link), _dev(recv),
                                       _nbytes(recv), _dev(dst, torch.float32), dst.numel(),
                                       _stream(compute_stream), _stream(copy_stream)),
               "zfpx_pipeline_recv")

    def close(self):
        if getattr(self, "_h", None):
            _lib.zfpx_pipeline_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def zfpx_pipeline_create(plan: Plan, rate: int, groups: int) -> Pipeline:
    return Pipeline(plan, rate, groups)


# ---------------------------------------------------------------------------
# Variable-size modes (fixed precision / fixed accuracy)
# ---------------------------------------------------------------------------

MINEXP_NONE = -1074  # ZFPX_MINEXP_NONE: precision mode (no exponent floor)


def zfpx_accuracy_minexp(tolerance: float) -> int:
    return _lib.zfpx_accuracy_minexp(float(tolerance))


def zfpx_plan_var_sizes(plan: Plan, rate_cap: int):
    """(largest stream in 32-bit words, tiles, scratch bytes)."""
    mw, nt, wb = _I64(), _I64(), _SZ()
    _check(_lib.zfpx_plan_var_sizes(plan.handle, rate_cap, _c.byref(mw), _c.byref(nt),
                                    _c.byref(wb)), "zfpx_plan_var_sizes")
    return mw.value, nt.value, wb.value


def zfpx_plan_encode_var(plan: Plan, src: torch.Tensor, maxprec: int, minexp: int,
                         rate_cap: int, words: torch.Tensor | None = None,
                         nd: torch.Tensor | None = None, tile_off: torch.Tensor | None = None,
                         work: torch.Tensor | None = None, stream=None):
    """Returns (words int32, nd uint8, tile_off int64); the stream's length is
    tile_off[-1] words (read it after synchronising)."""
    mw, nt, wb = zfpx_plan_var_sizes(plan, rate_cap)
    dev = src.device
    if words is None:
        words = torch.empty(max(mw, 1), dtype=torch.int32, device=dev)
    if nd is None:
        nd = torch.empty(max(plan.nblocks, 1), dtype=torch.uint8, device=dev)
    if tile_off is None:
        tile_off = torch.empty(nt + 1, dtype=torch.int64, device=dev)
    if work is None:
        work = torch.empty((wb + 7) // 8, dtype=torch.int64, device=dev)
    _check(_lib.zfpx_plan_encode_var(plan.handle, _dev(src, torch.float32), src.numel(),
                                     maxprec, minexp, rate_cap, _dev(words), _nbytes(words),
                                     _dev(nd, torch.uint8), _dev(tile_off, torch.int64),
                                     _dev(work), _nbytes(work), _stream(stream)),
           "zfpx_plan_encode_var")
    return words, nd, tile_off


def zfpx_plan_encode_var_noalloc(plan: Plan, src: torch.Tensor, maxprec: int, minexp: int,
                                 rate_cap: int, words: torch.Tensor, nd: torch.Tensor,
                                 tile_off: torch.Tensor, stream=None) -> None:
    """zfpx_plan_encode_var with the library's own device scratch instead of
    a workspace: no allocation on the call (outputs are the caller's)."""
    _check(_lib.zfpx_plan_encode_var_noalloc(plan.handle, _dev(src, torch.float32), src.numel(),
                                             maxprec, minexp, rate_cap, _dev(words),
                                             _nbytes(words), _dev(nd, torch.uint8),
                                             _dev(tile_off, torch.int64), _stream(stream)),
           "zfpx_plan_encode_var_noalloc")


def zfpx_noalloc_scratch_bytes() -> int:
    return int(_lib.zfpx_noalloc_scratch_bytes())


def zfpx_plan_decode_var(plan: Plan, words: torch.Tensor, nd: torch.Tensor,
                         tile_off: torch.Tensor, maxprec: int, minexp: int, rate_cap: int,
                         dst: torch.Tensor, stream=None) -> torch.Tensor:
    _check(_lib.zfpx_plan_decode_var(plan.handle, _dev(words), _nbytes(words),
                                     _dev(nd, torch.uint8), _dev(tile_off, torch.int64),
                                     maxprec, minexp, rate_cap, _dev(dst, torch.float32),
                                     dst.numel(), _stream(stream)), "zfpx_plan_decode_var")
    return dst


def zfpx_plan_var_chunk_offsets(plan: Plan, nd: torch.Tensor, tile_off: torch.Tensor,
                                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(plan.nchunks + 1, dtype=torch.int64, device=tile_off.device)
    _check(_lib.zfpx_plan_var_chunk_offsets(plan.handle, _dev(nd, torch.uint8),
                                            _dev(tile_off, torch.int64),
                                            _dev(out, torch.int64), _stream(stream)),
           "zfpx_plan_var_chunk_offsets")
    return out


def zfpx_plan_set_config(plan: Plan, op: int, rate: int, wg_threads: int, grid_wgs: int) -> None:
    _check(_lib.zfpx_plan_set_config(plan.handle, op, rate, wg_threads, grid_wgs),
           "zfpx_plan_set_config")


def zfpx_plan_get_config(plan: Plan, op: int, rate: int):
    wg, grid = _INT(), _INT()
    _check(_lib.zfpx_plan_get_config(plan.handle, op, rate, _c.byref(wg), _c.byref(grid)),
           "zfpx_plan_get_config")
    return wg.value, grid.value


def zfpx_autotune(plan: Plan, op: int, rate: int, src: torch.Tensor, stream_buf: torch.Tensor,
                  dst: torch.Tensor, cache_path: str | None = None, stream=None) -> float:
    us = _c.c_double()
    _check(_lib.zfpx_autotune(plan.handle, op, rate, _dev(src, torch.float32), src.numel(),
                              _dev(stream_buf), _nbytes(stream_buf), _dev(dst, torch.float32),
                              dst.numel(), cache_path.encode() if cache_path else None,
                              _stream(stream), _c.byref(us)), "zfpx_autotune")
    return us.value


class Graph:
    """pack_encode + decode_unpack over a whole plan, captured in a HIP graph."""

    def __init__(self, plan: Plan, rate: int, src: torch.Tensor, send: torch.Tensor,
                 dst: torch.Tensor):
        h = _P()
        _check(_lib.zfpx_graph_create(plan.handle, rate, _dev(src, torch.float32), src.numel(),
                                      _dev(send), _nbytes(send), _dev(dst, torch.float32),
                                      dst.numel(), _c.byref(h)), "zfpx_graph_create")
        self._h = h
        self._keep = (plan, src, send, dst)

    def launch(self, stream=None) -> None:
        _check(_lib.zfpx_graph_launch(self._h, _stream(stream)), "zfpx_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            _lib.zfpx_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def zfpx_graph_create(plan, rate, src, send, dst) -> Graph:
    return Graph(plan, rate, src, send, dst)


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------

class zfpx_request(_c.Structure):
    _fields_ = [("op", _c.c_int32), ("rate", _c.c_int32),
                ("nx", _c.c_int64), ("ny", _c.c_int64), ("nz", _c.c_int64),
                ("sx", _c.c_int64), ("sy", _c.c_int64), ("sz", _c.c_int64),
                ("d_in", _c.c_void_p), ("d_out", _c.c_void_p), ("tag", _c.c_uint64)]


def make_request(op: int, rate: int, array: torch.Tensor, words: torch.Tensor,
                 tag: int = 0) -> zfpx_request:
    """A request on a (nz, ny, nx) float32 view `array` and its coded `words`:
    op 0 encodes array -> words, op 1 decodes words -> array."""
    nz, ny, nx = array.shape
    sz, sy, sx = array.stride()
    fin, fout = (array, words) if op == 0 else (words, array)
    return zfpx_request(op, rate, nx, ny, nz, sx, sy, sz, _dev(fin), _dev(fout), tag)


class Server:
    """Continuous-batching server around the device-resident loop."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, workgroups: int = 0):
        h = _P()
        _check(_lib.zfpx_server_create(hbm_budget_bytes, max_slots, workgroups, _c.byref(h)),
               "zfpx_server_create")
        self._h = h

    def submit(self, rq: zfpx_request) -> int:
        t = _c.c_uint64()
        _check(_lib.zfpx_server_submit(self._h, _c.byref(rq), _c.byref(t)), "zfpx_server_submit")
        return t.value

    def poll(self, ticket: int):
        done, lat = _INT(), _c.c_double()
        _check(_lib.zfpx_server_poll(self._h, ticket, _c.byref(done), _c.byref(lat)),
               "zfpx_server_poll")
        return bool(done.value), lat.value

    def drain(self, timeout_s: float = 60.0) -> None:
        _check(_lib.zfpx_server_drain(self._h, timeout_s), "zfpx_server_drain")

    def set_max_queue(self, max_queued: int) -> None:
        _check(_lib.zfpx_server_set_max_queue(self._h, max_queued), "zfpx_server_set_max_queue")

    def set_idle_us(self, idle_us: int) -> None:
        _check(_lib.zfpx_server_set_idle_us(self._h, idle_us), "zfpx_server_set_idle_us")

    def stats(self):
        a, m, l = _c.c_uint64(), _SZ(), _c.c_uint64()
        _check(_lib.zfpx_server_stats(self._h, _c.byref(a), _c.byref(m), _c.byref(l)),
               "zfpx_server_stats")
        return {"admitted": a.value, "max_inflight_bytes": m.value, "loop_launches": l.value}

    def replay(self, requests, arrival_s, timeout_s: float = 120.0):
        import numpy as np
        n = len(requests)
        arr = (zfpx_request * n)(*requests)
        t = np.ascontiguousarray(arrival_s, dtype=np.float64)
        lat = np.zeros(n, np.float64)
        _check(_lib.zfpx_server_replay(self._h, _c.cast(arr, _P), t.ctypes.data, n, timeout_s,
                                       lat.ctypes.data), "zfpx_server_replay")
        return lat

    def close(self):
        if getattr(self, "_h", None):
            _lib.zfpx_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def zfpx_plain_replay(requests, arrival_s, timeout_s: float = 120.0, stream=None):
    import numpy as np
    n = len(requests)
    arr = (zfpx_request * n)(*requests)
    t = np.ascontiguousarray(arrival_s, dtype=np.float64)
    lat = np.zeros(n, np.float64)
    _check(_lib.zfpx_plain_replay(_c.cast(arr, _P), t.ctypes.data, n, timeout_s,
                                  _stream(stream), lat.ctypes.data), "zfpx_plain_replay")
    return lat


# ---------------------------------------------------------------------------
# float16 comparator
# ---------------------------------------------------------------------------

def f16_truncate(x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
    _check(_lib.f16_truncate(_dev(x, torch.float32), x.numel(), _dev(out), _stream(stream)),
           "f16_truncate")
    return out


def f16_restore(h: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(h.numel(), dtype=torch.float32, device=h.device)
    _check(_lib.f16_restore(_dev(h), h.numel(), _dev(out, torch.float32), _stream(stream)),
           "f16_restore")
    return out
