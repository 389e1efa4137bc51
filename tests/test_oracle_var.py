"""Pins of the oracle's variable-size modes (fixed precision, fixed accuracy).

The paper names these ZFP modes as the variable-size alternative to fixed
rate (Sections II-C and IV-B).  The checks: the accuracy mode's absolute
error bound, the reduction to fixed rate at full precision, exactness of the
kept bit planes, embedded prefixes across precisions, the tolerance-to-exponent
rule on exact powers of two, agreement with the independent Python writing,
and the stream layout (per-block word counts, offsets, round trip).
"""
import math

import numpy as np

import oracle
from oracle import pyblock
from paper_2609_24294_amd import workloads as W

from _blocks import block_families, blocks_to_array

NONE = oracle.MINEXP_NONE


def _bits(words):
    return np.unpackbits(np.asarray(words, np.uint64).view(np.uint8), bitorder="little")


def _coefficients(v):
    """Negabinary coefficients in sequency order, from the oracle's stages."""
    nonempty, emax = oracle.block_exponent(v)
    q = oracle.transform_forward(oracle.cast_forward(v, emax))
    perm = oracle.sequency_order()
    return emax, np.array([oracle.to_negabinary(int(q[perm[s]])) for s in range(64)], np.uint32)


def _from_coefficients(u, emax):
    perm = oracle.sequency_order()
    q = np.zeros(64, np.int32)
    for s in range(64):
        q[perm[s]] = oracle.from_negabinary(int(u[s]))
    return oracle.cast_inverse(oracle.transform_inverse(q), emax)


def test_accuracy_minexp_on_powers_of_two():
    for k in (-30, -7, -1, 0, 1, 5, 20):
        assert oracle.accuracy_minexp(2.0 ** k) == k
        assert oracle.accuracy_minexp(1.5 * 2.0 ** k) == k
        assert oracle.accuracy_minexp(np.nextafter(2.0 ** k, 0)) == k - 1
    assert oracle.accuracy_minexp(0.0) == NONE


def test_accuracy_mode_error_bound():
    # every reconstructed value within the tolerance, for any block that did
    # not reach the bit cap; tolerances from far below to far above the
    # block's magnitude (but above float32's own resolution of the block)
    rng = np.random.default_rng(40)
    checked = 0
    for v in block_families(rng, 540):
        amax = float(np.abs(v).max())
        if amax == 0 or not np.isfinite(amax):
            continue
        top = math.frexp(amax)[1]
        for j in (-22, -15, -9, -4, 0, 3, 9, 12):
            tol = math.ldexp(float(rng.uniform(1, 2)), top + j)
            if tol == 0 or not np.isfinite(tol):
                continue
            me = oracle.accuracy_minexp(tol)
            w, n = oracle.encode_block_var(v, 32, me, 32)
            if n >= 64 * 32:
                continue
            d = oracle.decode_block_var(w, 32, me, 32)
            err = np.abs(d.astype(np.float64) - v.astype(np.float64)).max()
            assert err <= tol, (j, tol, err)
            checked += 1
    assert checked > 3000


def test_blocks_far_below_tolerance_cost_one_bit():
    rng = np.random.default_rng(41)
    for k in (-10, 0, 7):
        tol = 2.0 ** k
        v = (rng.uniform(-1, 1, 64) * tol / 2 ** 9).astype(np.float32)
        w, n = oracle.encode_block_var(v, 32, oracle.accuracy_minexp(tol), 16)
        assert n == 1 and not w.any()
        assert not oracle.decode_block_var(w, 32, oracle.accuracy_minexp(tol), 16).any()


def test_full_precision_is_fixed_rate():
    # maxprec 32 with no exponent floor codes every plane: the block is the
    # fixed-rate block at rate = cap, cut at its own length
    rng = np.random.default_rng(42)
    for t, v in enumerate(block_families(rng, 270)):
        r = (1, 2, 5, 8, 13, 16, 24, 32)[t % 8]
        w, n = oracle.encode_block_var(v, 32, NONE, r)
        fixed = oracle.encode_block(v, r)
        assert 1 <= n <= 64 * r
        assert np.array_equal(w[:r], fixed) and not w[r:].any()
        if n < 64 * r:
            _, n32 = oracle.encode_block_var(v, 32, NONE, 32)
            assert n32 == n  # a larger cap changes nothing once the block fits
        d = oracle.decode_block_var(w, 32, NONE, r)
        assert np.array_equal(d.view(np.uint32), oracle.decode_block(fixed, r).view(np.uint32))


def test_precision_keeps_exactly_the_top_planes():
    rng = np.random.default_rng(43)
    for v in block_families(rng, 90):
        if not np.abs(v).max() > 0:
            continue
        emax, u = _coefficients(v)
        for p in (1, 2, 5, 9, 16, 23, 31, 32):
            w, n = oracle.encode_block_var(v, p, NONE, 32)
            if n >= 2048:
                continue
            keep = np.uint32((0xffffffff << (32 - p)) & 0xffffffff)
            want = _from_coefficients(u & keep, emax)
            got = oracle.decode_block_var(w, p, NONE, 32)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), p


def test_precisions_are_embedded_prefixes():
    rng = np.random.default_rng(44)
    for v in block_families(rng, 180):
        wf, nf = oracle.encode_block_var(v, 32, NONE, 32)
        bf = _bits(wf)
        last = 0
        for p in range(1, 33):
            w, n = oracle.encode_block_var(v, p, NONE, 32)
            assert n >= last
            last = n
            assert np.array_equal(_bits(w)[:n], bf[:n]) and not _bits(w)[n:].any()
        assert last == nf


def test_finer_tolerance_never_codes_fewer_bits():
    rng = np.random.default_rng(45)
    for v in block_families(rng, 180):
        prev = None
        for me in (20, 5, 0, -5, -12, -30, NONE):
            _, n = oracle.encode_block_var(v, 32, me, 32)
            assert prev is None or n >= prev
            prev = n


def test_c_and_python_writings_agree():
    rng = np.random.default_rng(46)
    params = [(32, NONE, 32), (12, NONE, 16), (32, -3, 32), (32, 5, 8), (20, -20, 4),
              (1, NONE, 2), (32, 0, 1)]
    for v in block_families(rng, 72):
        for mp, me, cap in params:
            w, n = oracle.encode_block_var(v, mp, me, cap)
            pw, pn = pyblock.encode_block_var([float(x) for x in v], mp, me, cap)
            assert n == pn and [int(x) for x in w] == pw
            d = oracle.decode_block_var(w, mp, me, cap)
            pd = np.array(pyblock.decode_block_var(pw, mp, me, cap), np.float32)
            assert np.array_equal(d.view(np.uint32), pd.view(np.uint32))


def test_stream_layout_of_a_chunk_set():
    rng = np.random.default_rng(47)
    blocks = block_families(rng, 200)  # 4 tiles, the last one ragged
    a = blocks_to_array(blocks)
    cs = W.regular_chunkset(*a.shape)
    for mp, me, cap in ((32, -6, 16), (10, NONE, 32), (32, NONE, 8)):
        words, nd, toff = oracle.pack_encode_var(cs, a, mp, me, cap)
        off = 0
        for b, v in enumerate(blocks):
            w, n = oracle.encode_block_var(v, mp, me, cap)
            assert nd[b] == (n + 31) // 32
            if b % 64 == 0:
                assert toff[b // 64] == off
            k = int(nd[b])
            assert np.array_equal(words[off:off + k], w.view(np.uint32)[:k])
            off += k
        assert toff[-1] == off == words.size and toff.size == 4 + 1
        dst = np.zeros(a.size, np.float32)
        oracle.decode_unpack_var(cs, words, nd, mp, me, cap, dst)
        per_block = np.stack([oracle.decode_block_var(oracle.encode_block_var(v, mp, me, cap)[0],
                                                      mp, me, cap) for v in blocks])
        assert np.array_equal(dst.reshape(a.shape).view(np.uint32),
                              blocks_to_array(per_block).view(np.uint32))


def test_ragged_chunks_round_trip_within_tolerance():
    cs = W.reduced_grid_chunkset(n_half=24, nlev=7, nchunks=5)
    rng = np.random.default_rng(48)
    src = np.cumsum(rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    tol = 1e-3
    me = oracle.accuracy_minexp(tol)
    words, nd, toff = oracle.pack_encode_var(cs, src, 32, me, 32)
    assert nd.size == int(oracle.chunk_blocks(cs).sum()) and (nd < 64).all()
    dst = np.full(cs.buffer_elems, np.nan, np.float32)
    oracle.decode_unpack_var(cs, words, nd, 32, me, 32, dst)
    assert not np.isnan(dst).any()
    assert np.abs(dst.astype(np.float64) - src).max() <= tol
