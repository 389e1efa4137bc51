"""CPU oracle for ZFP fixed-rate coding and float16 truncation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_2609_24294_amd``) never imports it, and the two share no code.

The codec itself is plain C (``zfp_oracle.c``), compiled with gcc into
``liboracle.so``; this module only marshals numpy arrays through ctypes.  The
float16 comparator is numpy's own IEEE binary16 conversion (round to nearest,
ties to even, subnormals kept, overflow to infinity), which is the definition
the paper's comparator uses (Section IV-F: cast to float16 and back).

Parity unpinned: byte compatibility with the ZFP library (not available), and
the paper's error figures (its input data are not available).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zfp_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the C oracle (always recompiles) and return the library path."""
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           _SRC, "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U32P = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_U64P = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_F32P = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_U8P = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_I64 = ctypes.c_int64
_INT = ctypes.c_int

_CHUNK_ARGS = [_INT, _I64P, _I64P, _I32P, _I32P, _I64P, _I32P]

_SIGS = {
    "orc_block_exponent": (_INT, [_F32P, ctypes.POINTER(_INT)]),
    "orc_cast_forward": (None, [_F32P, _INT, _I32P]),
    "orc_cast_inverse": (None, [_I32P, _INT, _F32P]),
    "orc_lift_forward": (None, [_I32P, _INT]),
    "orc_lift_inverse": (None, [_I32P, _INT]),
    "orc_transform_forward": (None, [_I32P]),
    "orc_transform_inverse": (None, [_I32P]),
    "orc_sequency_order": (None, [_I32P]),
    "orc_to_negabinary": (ctypes.c_uint32, [ctypes.c_int32]),
    "orc_from_negabinary": (ctypes.c_int32, [ctypes.c_uint32]),
    "orc_encode_planes": (_I64, [_U32P, _I64, _U64P, _I64]),
    "orc_decode_planes": (_I64, [_U64P, _I64, _I64, _U32P]),
    "orc_encode_block": (None, [_F32P, _INT, _U64P]),
    "orc_decode_block": (None, [_U64P, _INT, _F32P]),
    "orc_regular_blocks": (_I64, [_I64, _I64, _I64]),
    "orc_encode_regular": (None, [_F32P, _I64, _I64, _I64, _I64, _I64, _I64, _INT, _U64P]),
    "orc_decode_regular": (None, [_U64P, _I64, _I64, _I64, _I64, _I64, _I64, _INT, _F32P]),
    "orc_chunk_blocks": (None, _CHUNK_ARGS + [_I64P]),
    "orc_pack_encode": (None, _CHUNK_ARGS + [_F32P, _INT, _U64P]),
    "orc_decode_unpack": (None, _CHUNK_ARGS + [_U64P, _INT, _F32P]),
    "orc_pack_encode_sample": (None, _CHUNK_ARGS + [_F32P, _INT, _I64P, _I64, _U64P]),
    "orc_decode_sample": (None, _CHUNK_ARGS + [_U64P, _INT, _I64P, _I64, _F32P, _I64P, _I32P]),
    "orc_decode_blocks": (None, [_U64P, _I64, _INT, _F32P]),
    "orc_encode_blocks": (None, [_F32P, _I64, _INT, _U64P]),
    "orc_encode_planes_from": (_I64, [_U32P, _INT, _I64, _U64P, _I64]),
    "orc_decode_planes_from": (_I64, [_U64P, _I64, _INT, _I64, _U32P]),
    "orc_block_precision": (_INT, [_INT, _INT, _INT]),
    "orc_encode_block_var": (_I64, [_F32P, _INT, _INT, _I64, _U64P]),
    "orc_decode_block_var": (None, [_U64P, _INT, _INT, _I64, _F32P]),
    "orc_pack_encode_var": (None, _CHUNK_ARGS + [_F32P, _INT, _INT, _INT, _U32P, _U8P, _I64P]),
    "orc_decode_unpack_var": (None, _CHUNK_ARGS + [_U32P, _U8P, _INT, _INT, _INT, _F32P]),
    "orc_set_threads": (None, [_INT]),
    "orc_pack_encode_var_sample": (None, _CHUNK_ARGS + [_F32P, _INT, _INT, _INT, _I64P, _I64,
                                                        _U64P, _I64P, _I64P, _I32P]),
}


def lib():
    """Load liboracle.so (building it first if it is missing).  The
    environment variable ZFPX_ORACLE_LIB names another build of the same
    source to load instead (the tests' sanitizer run uses it)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ZFPX_ORACLE_LIB") or LIB_PATH
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# Stage-level access (for the invariant tests)
# ---------------------------------------------------------------------------

def set_threads(n: int) -> None:
    """OpenMP threads of the C oracle's loops."""
    lib().orc_set_threads(int(n))


def block_exponent(v):
    v = np.ascontiguousarray(v, dtype=np.float32)
    e = _INT(0)
    nonempty = lib().orc_block_exponent(v, ctypes.byref(e))
    return bool(nonempty), int(e.value)


def cast_forward(v, emax):
    v = np.ascontiguousarray(v, dtype=np.float32)
    q = np.zeros(64, np.int32)
    lib().orc_cast_forward(v, int(emax), q)
    return q


def cast_inverse(q, emax):
    q = np.ascontiguousarray(q, dtype=np.int32)
    v = np.zeros(64, np.float32)
    lib().orc_cast_inverse(q, int(emax), v)
    return v


def lift_forward(x4):
    p = np.ascontiguousarray(x4, dtype=np.int32).copy()
    lib().orc_lift_forward(p, 1)
    return p


def lift_inverse(x4):
    p = np.ascontiguousarray(x4, dtype=np.int32).copy()
    lib().orc_lift_inverse(p, 1)
    return p


def transform_forward(q64):
    p = np.ascontiguousarray(q64, dtype=np.int32).copy()
    lib().orc_transform_forward(p)
    return p


def transform_inverse(q64):
    p = np.ascontiguousarray(q64, dtype=np.int32).copy()
    lib().orc_transform_inverse(p)
    return p


def sequency_order():
    p = np.zeros(64, np.int32)
    lib().orc_sequency_order(p)
    return p


def to_negabinary(q: int) -> int:
    return int(lib().orc_to_negabinary(int(q)))


def from_negabinary(u: int) -> int:
    return int(lib().orc_from_negabinary(int(u)))


def encode_planes(u64, budget, nwords=None):
    """Code 64 negabinary coefficients under `budget` bits; returns (words, nbits)."""
    u = np.ascontiguousarray(u64, dtype=np.uint32)
    if nwords is None:
        nwords = (int(budget) + 63) // 64 + 1
    w = np.zeros(nwords, np.uint64)
    nbits = lib().orc_encode_planes(u, int(budget), w, 0)
    return w, int(nbits)


def decode_planes(words, budget):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    u = np.zeros(64, np.uint32)
    nbits = lib().orc_decode_planes(w, 0, int(budget), u)
    return u, int(nbits)


# ---------------------------------------------------------------------------
# Blocks and arrays
# ---------------------------------------------------------------------------

def encode_block(v64, rate):
    v = np.ascontiguousarray(v64, dtype=np.float32)
    w = np.zeros(int(rate), np.uint64)
    lib().orc_encode_block(v, int(rate), w)
    return w


def decode_block(words, rate):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    v = np.zeros(64, np.float32)
    lib().orc_decode_block(w, int(rate), v)
    return v


def encode_blocks(vals, rate):
    """vals: (nblocks, 64) float32 -> (nblocks, rate) uint64."""
    vals = np.ascontiguousarray(vals, dtype=np.float32).reshape(-1, 64)
    out = np.zeros((vals.shape[0], int(rate)), np.uint64)
    lib().orc_encode_blocks(vals.reshape(-1), vals.shape[0], int(rate), out.reshape(-1))
    return out


def decode_blocks(words, rate):
    words = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, int(rate))
    vals = np.zeros((words.shape[0], 64), np.float32)
    lib().orc_decode_blocks(words.reshape(-1), words.shape[0], int(rate), vals.reshape(-1))
    return vals


def regular_blocks(nx, ny, nz):
    return int(lib().orc_regular_blocks(int(nx), int(ny), int(nz)))


def encode_regular(a, rate):
    """Encode a C-contiguous (nz, ny, nx) float32 array; x is the fastest axis."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    nz, ny, nx = a.shape
    nb = regular_blocks(nx, ny, nz)
    out = np.zeros(nb * int(rate), np.uint64)
    lib().orc_encode_regular(a.reshape(-1), nx, ny, nz, 1, nx, nx * ny, int(rate), out)
    return out


def decode_regular(words, shape, rate, fill=0.0):
    nz, ny, nx = shape
    a = np.full(nz * ny * nx, fill, np.float32)
    w = np.ascontiguousarray(words, dtype=np.uint64)
    if w.size < regular_blocks(nx, ny, nz) * int(rate):
        raise ValueError("stream shorter than rate words per block")
    lib().orc_decode_regular(w, nx, ny, nz, 1, nx, nx * ny, int(rate), a)
    return a.reshape(shape)


def _chunk_args(chunks):
    return (int(chunks.nchunks), chunks.chunk_base, chunks.level_stride, chunks.levels,
            chunks.row_start, chunks.row_offset, chunks.row_len)


def chunk_blocks(chunks):
    out = np.zeros(chunks.nchunks, np.int64)
    lib().orc_chunk_blocks(*_chunk_args(chunks), out)
    return out


def pack_encode(chunks, src, rate):
    """Encode every chunk of `chunks` (a workloads.ChunkSet) read from `src`."""
    src = np.ascontiguousarray(src, dtype=np.float32).reshape(-1)
    nb = int(chunk_blocks(chunks).sum())
    out = np.zeros(nb * int(rate), np.uint64)
    lib().orc_pack_encode(*_chunk_args(chunks), src, int(rate), out)
    return out


def decode_unpack(chunks, words, rate, dst):
    """Decode into `dst` (float32, modified in place; only chunk points written)."""
    assert dst.dtype == np.float32 and dst.flags.c_contiguous
    w = np.ascontiguousarray(words, dtype=np.uint64)
    if w.size < int(chunk_blocks(chunks).sum()) * int(rate):
        raise ValueError("stream shorter than rate words per block")
    lib().orc_decode_unpack(*_chunk_args(chunks), w, int(rate), dst.reshape(-1))
    return dst


def pack_encode_sample(chunks, src, rate, ids):
    src = np.ascontiguousarray(src, dtype=np.float32).reshape(-1)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.zeros((ids.size, int(rate)), np.uint64)
    lib().orc_pack_encode_sample(*_chunk_args(chunks), src, int(rate), ids, ids.size,
                                 out.reshape(-1))
    return out


def decode_sample(chunks, words, rate, ids):
    """Decode the listed blocks: returns (values (n,64), offsets (n,64), inside (n,64))."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    if ids.size and (ids.min() < 0 or ids.max() >= int(chunk_blocks(chunks).sum())
                     or w.size < (int(ids.max()) + 1) * int(rate)):
        raise ValueError("block id outside the plan or stream too short")
    vals = np.zeros((ids.size, 64), np.float32)
    pos = np.zeros((ids.size, 64), np.int64)
    ins = np.zeros((ids.size, 64), np.int32)
    lib().orc_decode_sample(*_chunk_args(chunks), w, int(rate), ids, ids.size,
                            vals.reshape(-1), pos.reshape(-1), ins.reshape(-1))
    return vals, pos, ins.astype(bool)


# ---------------------------------------------------------------------------
# Variable-size modes (fixed precision / fixed accuracy, with a bit cap)
# ---------------------------------------------------------------------------

# minexp that leaves every float32 block at maxprec planes (precision mode):
# the smallest double exponent, as in ZFP's description
MINEXP_NONE = -1074


def accuracy_minexp(tolerance: float) -> int:
    """minexp of accuracy mode: the largest e with 2^e <= tolerance."""
    if not tolerance > 0:
        return MINEXP_NONE
    return math.frexp(float(tolerance))[1] - 1


def block_precision(emax, maxprec, minexp):
    return int(lib().orc_block_precision(int(emax), int(maxprec), int(minexp)))


def encode_planes_from(u64, kmin, budget, nwords=None):
    u = np.ascontiguousarray(u64, dtype=np.uint32)
    if nwords is None:
        nwords = (int(budget) + 63) // 64 + 1
    w = np.zeros(nwords, np.uint64)
    nbits = lib().orc_encode_planes_from(u, int(kmin), int(budget), w, 0)
    return w, int(nbits)


def decode_planes_from(words, kmin, budget):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    u = np.zeros(64, np.uint32)
    nbits = lib().orc_decode_planes_from(w, 0, int(kmin), int(budget), u)
    return u, int(nbits)


def encode_block_var(v64, maxprec, minexp, rate_cap):
    """-> (words (rate_cap + 1 uint64, zero past the length), length in bits)."""
    v = np.ascontiguousarray(v64, dtype=np.float32)
    w = np.zeros(int(rate_cap) + 1, np.uint64)
    n = lib().orc_encode_block_var(v, int(maxprec), int(minexp), 64 * int(rate_cap), w)
    return w, int(n)


def decode_block_var(words, maxprec, minexp, rate_cap):
    w = np.zeros(int(rate_cap) + 1, np.uint64)
    words = np.asarray(words, dtype=np.uint64).reshape(-1)
    w[:min(words.size, w.size)] = words[:w.size]
    v = np.zeros(64, np.float32)
    lib().orc_decode_block_var(w, int(maxprec), int(minexp), 64 * int(rate_cap), v)
    return v


def pack_encode_var(chunks, src, maxprec, minexp, rate_cap):
    """-> (words uint32[total], nd uint8[nblocks], tile_off int64[ntiles + 1])."""
    assert 1 <= int(rate_cap) <= 32
    src = np.ascontiguousarray(src, dtype=np.float32).reshape(-1)
    nb = int(chunk_blocks(chunks).sum())
    out = np.zeros(max(1, nb * 2 * int(rate_cap)), np.uint32)
    nd = np.zeros(max(1, nb), np.uint8)
    toff = np.zeros((nb + 63) // 64 + 1, np.int64)
    lib().orc_pack_encode_var(*_chunk_args(chunks), src, int(maxprec), int(minexp),
                              int(rate_cap), out, nd, toff)
    return out[:int(toff[-1])].copy(), nd[:nb].copy(), toff


def pack_encode_var_sample(chunks, src, maxprec, minexp, rate_cap, ids):
    """Listed blocks only: (words (n, rate_cap + 1), bits (n,), offsets (n, 64),
    inside (n, 64))."""
    src = np.ascontiguousarray(src, dtype=np.float32).reshape(-1)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.zeros((ids.size, int(rate_cap) + 1), np.uint64)
    ln = np.zeros(ids.size, np.int64)
    pos = np.zeros((ids.size, 64), np.int64)
    ins = np.zeros((ids.size, 64), np.int32)
    lib().orc_pack_encode_var_sample(*_chunk_args(chunks), src, int(maxprec), int(minexp),
                                     int(rate_cap), ids, ids.size, out.reshape(-1), ln,
                                     pos.reshape(-1), ins.reshape(-1))
    return out, ln, pos, ins.astype(bool)


def decode_unpack_var(chunks, words, nd, maxprec, minexp, rate_cap, dst):
    """Decode into `dst` (float32, in place); offsets are rebuilt from nd."""
    assert dst.dtype == np.float32 and dst.flags.c_contiguous
    assert 1 <= int(rate_cap) <= 32
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.size == 0:
        w = np.zeros(1, np.uint32)
    nd = np.ascontiguousarray(nd, dtype=np.uint8)
    if nd.size == 0:
        nd = np.zeros(1, np.uint8)
    lib().orc_decode_unpack_var(*_chunk_args(chunks), w, nd, int(maxprec), int(minexp),
                                int(rate_cap), dst.reshape(-1))
    return dst


# ---------------------------------------------------------------------------
# float16 comparator
# ---------------------------------------------------------------------------

def f16_truncate(x):
    """IEEE binary16, round to nearest even; returns the 16-bit patterns."""
    with np.errstate(over="ignore"):
        return np.ascontiguousarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def f16_restore(h):
    """Exact widening of binary16 patterns back to float32."""
    return np.ascontiguousarray(h, dtype=np.uint16).view(np.float16).astype(np.float32)
