"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each checks a printed
value (Table 1), a closed form (the lifting matrix, the base -2 digit
expansion, the coder's length formula), an invariant (embedded prefixes,
invertibility, zero and constant blocks) or an independent writing
(``oracle/pyblock.py``) of the steps.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import pyblock
from paper_2609_24294_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Forward lifting without rounding is (1/16) M (ZFP's published transform).
M = np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]], np.int64)


# ---------------------------------------------------------------------------
# Size accounting: Table 1 of the paper
# ---------------------------------------------------------------------------

def test_table1_message_sizes():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_message_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 10
    MiB = 2.0 ** 20
    for r in rows:
        N = int(r[0])
        f32, f16, r16, r8 = map(float, r[1:])
        a, b, c = W.pencil_message_dims(N, nlon=2560, nlat=1280, nlev=137)
        blocks = oracle.regular_blocks(a, b, c)
        got = [a * b * c * 4 / MiB, a * b * c * 2 / MiB, blocks * 8 * 16 / MiB,
               blocks * 8 * 8 / MiB]
        for g, want in zip(got, (f32, f16, r16, r8)):
            # the table prints two decimals (rounded half up)
            assert abs(g - want) <= 0.005 + 1e-9, (N, got, (f32, f16, r16, r8))


def test_table1_worked_example_n9():
    a, b, c = W.pencil_message_dims(9)
    assert (a, b, c) == (853, 426, 45)
    assert oracle.regular_blocks(a, b, c) == 274776


# ---------------------------------------------------------------------------
# Lifting transform
# ---------------------------------------------------------------------------

def test_lifting_matches_matrix_on_exact_inputs():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        y = rng.integers(-2 ** 20, 2 ** 20, 4)
        got = oracle.lift_forward((16 * y).astype(np.int32)).astype(np.int64)
        assert np.array_equal(got, M @ y)


def test_inverse_lifting_matches_matrix_inverse():
    rng = np.random.default_rng(12)
    for _ in range(2000):
        y = rng.integers(-2 ** 20, 2 ** 20, 4)
        got = oracle.lift_inverse((M @ y).astype(np.int32)).astype(np.int64)
        assert np.array_equal(got, 16 * y)


def test_3d_transform_is_separable_product():
    """fwd(4096 Y) = (M x M x M) Y with block index 16 z + 4 y + x."""
    rng = np.random.default_rng(13)
    for _ in range(200):
        Y = rng.integers(-2 ** 8, 2 ** 8, (4, 4, 4))  # [z, y, x]
        want = np.einsum("az,by,cx,zyx->abc", M, M, M, Y)
        got = oracle.transform_forward((4096 * Y).reshape(-1).astype(np.int32))
        assert np.array_equal(got.astype(np.int64).reshape(4, 4, 4), want)
        back = oracle.transform_inverse(want.reshape(-1).astype(np.int32))
        assert np.array_equal(back.astype(np.int64).reshape(4, 4, 4), 4096 * Y)


def test_forward_after_inverse_is_identity():
    rng = np.random.default_rng(14)
    for _ in range(5000):
        c = rng.integers(-2 ** 29, 2 ** 29, 4).astype(np.int32)
        assert np.array_equal(oracle.lift_forward(oracle.lift_inverse(c)), c)
    for _ in range(500):
        c = rng.integers(-2 ** 24, 2 ** 24, 64).astype(np.int32)
        assert np.array_equal(oracle.transform_forward(oracle.transform_inverse(c)), c)


def test_inverse_after_forward_small_error_bruteforce():
    # the lifting steps drop one parity bit per average: not exactly invertible
    worst = 0
    for x in itertools.product(range(-8, 9), repeat=4):
        x = np.array(x, np.int32)
        worst = max(worst, int(np.abs(oracle.lift_inverse(oracle.lift_forward(x)) - x).max()))
    assert worst == 2


def test_constant_line_goes_to_dc():
    for c in (-(2 ** 30) + 1, -7, 0, 1, 12345, 2 ** 30 - 1):
        assert list(oracle.lift_forward(np.full(4, c, np.int32))) == [c, 0, 0, 0]
        got = oracle.transform_forward(np.full(64, c, np.int32))
        assert got[0] == c and not got[1:].any()


# ---------------------------------------------------------------------------
# Negabinary and sequency order
# ---------------------------------------------------------------------------

def test_negabinary_hand_values():
    assert oracle.to_negabinary(0) == 0
    assert oracle.to_negabinary(1) == 0b1
    assert oracle.to_negabinary(-1) == 0b11
    assert oracle.to_negabinary(2) == 0b110
    assert oracle.to_negabinary(-2) == 0b10
    assert oracle.to_negabinary(3) == 0b111


def test_negabinary_is_base_minus_two():
    rng = np.random.default_rng(15)
    for q in list(rng.integers(-2 ** 31, 2 ** 31, 3000)) + [-(2 ** 31), 2 ** 31 - 1]:
        q = int(q)
        u = oracle.to_negabinary(q)
        val = sum(((u >> i) & 1) * (-2) ** i for i in range(32))
        assert (val - q) % 2 ** 32 == 0
        assert oracle.from_negabinary(u) == q


def test_sequency_order():
    p = oracle.sequency_order()
    assert sorted(p) == list(range(64))
    assert list(p[:10]) == [0, 1, 4, 16, 5, 17, 20, 2, 8, 32]
    tot = [(i & 3) + ((i >> 2) & 3) + (i >> 4) for i in p]
    assert tot == sorted(tot)
    assert p[-1] == 63


# ---------------------------------------------------------------------------
# Exponent and cast
# ---------------------------------------------------------------------------

def test_block_exponent_cases():
    z = np.zeros(64, np.float32)
    assert oracle.block_exponent(z) == (False, -126)
    assert oracle.block_exponent(-z) == (False, -126)
    for val, e in [(1.0, 1), (0.75, 0), (0.5, 0), (-3.0, 2), (2.0 ** -126, -125),
                   (2.0 ** -130, -126), (2.0 ** -149, -126), (3.0e38, 128)]:
        v = z.copy()
        v[17] = val
        assert oracle.block_exponent(v) == (True, e), val


def test_cast_is_exact_truncation():
    rng = np.random.default_rng(16)
    for _ in range(200):
        v = (rng.standard_normal(64) * 2.0 ** rng.integers(-140, 120, 64)).astype(np.float32)
        _, emax = oracle.block_exponent(v)
        q = oracle.cast_forward(v, emax)
        for i in range(64):
            exact = Fraction(float(v[i])) * Fraction(2) ** (30 - emax)
            want = math.floor(exact) if exact >= 0 else -math.floor(-exact)
            assert q[i] == want
            assert abs(q[i]) < 2 ** 30


def test_inverse_cast_single_rounding():
    rng = np.random.default_rng(17)
    for emax in (-130, -126, -110, -96, 0, 50, 128):
        q = rng.integers(-2 ** 30, 2 ** 30, 64).astype(np.int32)
        v = oracle.cast_inverse(q, emax)
        for i in range(64):
            exact = Fraction(int(q[i])) * Fraction(2) ** (emax - 30)
            # round half even to float32, via the spacing at that magnitude
            assert float(v[i]) == _rne_f32(exact)


def _rne_f32(x: Fraction) -> float:
    if x == 0:
        return 0.0
    s = -1 if x < 0 else 1
    a = abs(x)
    e = math.floor(math.log2(a)) if a.numerator.bit_length() > 0 else 0
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    ulp_e = max(e, -126) - 23
    k = a / Fraction(2) ** ulp_e
    n = math.floor(k)
    r = k - n
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and n % 2 == 1):
        n += 1
    val = n * Fraction(2) ** ulp_e
    if val >= Fraction(2) ** 128:
        return s * math.inf
    return s * float(val)


# ---------------------------------------------------------------------------
# Embedded coder
# ---------------------------------------------------------------------------

def _closed_form_length(u):
    """Unlimited-budget length from the coder's description, plane by plane."""
    n = 0
    total = 0
    for k in range(31, -1, -1):
        x = sum(((int(u[s]) >> k) & 1) << s for s in range(64))
        total += n
        prev = n
        ones = [p for p in range(n, 64) if (x >> p) & 1]
        for p in ones:
            total += 2 + p - prev - (1 if p == 63 else 0)
            prev = p + 1
        if prev < 64:
            total += 1
        n = prev
    return total


def _random_coefficients(rng, kind):
    if kind == 0:
        return rng.integers(0, 2 ** 32, 64, dtype=np.uint64).astype(np.uint32)
    if kind == 1:  # decaying magnitudes, like transformed smooth data
        mags = (2.0 ** (30 - np.arange(64) / 2.5)) * rng.standard_normal(64)
        q = mags.astype(np.int64).astype(np.int32)
        return np.array([oracle.to_negabinary(int(x)) for x in q], np.uint32)
    if kind == 2:  # sparse
        u = np.zeros(64, np.uint32)
        idx = rng.integers(0, 64, rng.integers(1, 6))
        u[idx] = rng.integers(1, 2 ** 32, idx.size, dtype=np.uint64).astype(np.uint32)
        return u
    u = np.zeros(64, np.uint32)  # only the last position
    u[63] = rng.integers(1, 2 ** 32, dtype=np.uint64)
    return u


def test_plane_coder_roundtrip_and_length():
    rng = np.random.default_rng(18)
    for t in range(400):
        u = _random_coefficients(rng, t % 4)
        w, nbits = oracle.encode_planes(u, 10 ** 6, nwords=80)
        assert nbits == _closed_form_length(u)
        back, nread = oracle.decode_planes(w, 10 ** 6)
        assert nread == nbits
        assert np.array_equal(back, u)


def test_plane_coder_budget_is_prefix():
    rng = np.random.default_rng(19)
    for t in range(300):
        u = _random_coefficients(rng, t % 4)
        full, nfull = oracle.encode_planes(u, 10 ** 6, nwords=80)
        B = int(rng.integers(1, nfull + 40))
        part, npart = oracle.encode_planes(u, B, nwords=80)
        assert npart == min(B, nfull)
        bits_full = np.unpackbits(full.view(np.uint8), bitorder="little")
        bits_part = np.unpackbits(part.view(np.uint8), bitorder="little")
        assert np.array_equal(bits_part[:npart], bits_full[:npart])
        assert not bits_part[npart:].any()


# ---------------------------------------------------------------------------
# Whole blocks
# ---------------------------------------------------------------------------

def _blocks(rng, count):
    out = []
    for t in range(count):
        k = t % 7
        if k == 0:
            v = 280 + 15 * rng.standard_normal(64)
        elif k == 1:
            g = np.cumsum(np.cumsum(rng.standard_normal((4, 4, 4)), 0), 2)
            v = g.reshape(-1)
        elif k == 2:
            v = rng.standard_normal(64) * 10.0 ** rng.uniform(-40, 38, 64)
        elif k == 3:
            v = np.zeros(64)
            v[rng.integers(64)] = rng.standard_normal() * 2.0 ** rng.integers(-149, 127)
        elif k == 4:
            v = rng.choice([0.0, 1.0, -1.0, 2.0, -2.0], 64) * 2.0 ** rng.integers(-20, 20)
        elif k == 5:
            v = rng.standard_normal(64) * 2.0 ** -135  # subnormal range
        else:
            v = np.exp(rng.standard_normal(64))
        out.append(np.asarray(v, np.float32))
    return out


def _bits(words):
    return np.unpackbits(np.asarray(words, np.uint64).view(np.uint8), bitorder="little")


def test_embedded_prefix_across_rates():
    rng = np.random.default_rng(20)
    for v in _blocks(rng, 700):
        s8, s16, s32 = (_bits(oracle.encode_block(v, r)) for r in (8, 16, 32))
        assert np.array_equal(s8, s16[:512])
        assert np.array_equal(s16, s32[:1024])
        s1, s3 = _bits(oracle.encode_block(v, 1)), _bits(oracle.encode_block(v, 3))
        assert np.array_equal(s1, s3[:64])


def test_zero_block():
    for v in (np.zeros(64, np.float32), -np.zeros(64, np.float32)):
        for r in (1, 8, 16, 32):
            w = oracle.encode_block(v, r)
            assert w.shape == (r,) and not w.any()
            d = oracle.decode_block(w, r)
            assert not d.view(np.uint32).any()  # +0.0 everywhere


def test_constant_block_roundtrips_exactly_for_rate_ge_2():
    rng = np.random.default_rng(21)
    vals = list(rng.standard_normal(40) * 10.0 ** rng.uniform(-38, 38, 40))
    vals += [2.0 ** -149, -(2.0 ** -140), 3.0e38, 1.0, -1.0, 280.0]
    for c in vals:
        v = np.full(64, c, np.float32)
        for r in (2, 3, 8, 16, 32):
            d = oracle.decode_block(oracle.encode_block(v, r), r)
            assert np.array_equal(d.view(np.uint32), v.view(np.uint32)), (c, r)


def test_rate32_near_lossless():
    rng = np.random.default_rng(22)
    for v in _blocks(rng, 700):
        nonempty, emax = oracle.block_exponent(v)
        d = oracle.decode_block(oracle.encode_block(v, 32), 32)
        err = np.abs(d.astype(np.float64) - v.astype(np.float64))
        # measured worst case is 32 units of 2^(emax-30); allow 64
        assert err.max() <= 64 * 2.0 ** (emax - 30), (err.max(), emax)


def test_single_spike_blocks_all_rates():
    for pos in range(64):
        for val in (1.0, -3.5, 2.0 ** -140, 1.0e30):
            v = np.zeros(64, np.float32)
            v[pos] = val
            for r in (1, 2, 4, 8, 16, 32):
                w = oracle.encode_block(v, r)
                d = oracle.decode_block(w, r)
                assert np.array_equal(w, np.array(pyblock.encode_block(list(v), r), np.uint64))
                if r == 32:  # a spike spreads over all 64 coefficients: near-lossless only
                    _, emax = oracle.block_exponent(v)
                    err = np.abs(d.astype(np.float64) - v.astype(np.float64)).max()
                    assert err <= 64 * 2.0 ** (emax - 30), (pos, val, r)


def test_c_and_python_oracles_agree():
    rng = np.random.default_rng(23)
    for t, v in enumerate(_blocks(rng, 350)):
        for r in (1, 5, 8, 16, 32):
            w = oracle.encode_block(v, r)
            assert np.array_equal(w, np.array(pyblock.encode_block(list(v), r), np.uint64))
            d = oracle.decode_block(w, r)
            dp = np.array(pyblock.decode_block([int(x) for x in w], r), np.float32)
            assert np.array_equal(d.view(np.uint32), dp.view(np.uint32))


def test_c_and_python_decoders_agree_on_random_words():
    rng = np.random.default_rng(24)
    for t in range(300):
        r = int(rng.choice([1, 2, 8, 16, 32]))
        w = rng.integers(0, 2 ** 63, r, dtype=np.int64).astype(np.uint64) * 2 + rng.integers(0, 2, r).astype(np.uint64)
        d = oracle.decode_block(w, r)
        dp = np.array(pyblock.decode_block([int(x) for x in w], r), np.float32)
        assert np.array_equal(d.view(np.uint32), dp.view(np.uint32))


# ---------------------------------------------------------------------------
# Arrays and chunk geometry
# ---------------------------------------------------------------------------

def test_partial_blocks_use_edge_padding():
    rng = np.random.default_rng(25)
    a = rng.standard_normal((6, 5, 7)).astype(np.float32)  # (nz, ny, nx)
    words = oracle.encode_regular(a, 16).reshape(-1, 16)
    padded = np.pad(a, ((0, 2), (0, 3), (0, 1)), mode="edge")
    b = 0
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                blk = padded[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4]
                assert np.array_equal(words[b], oracle.encode_block(blk.reshape(-1), 16))
                b += 1
    # decoding takes the stream of its own rate (a rate-32 stream here)
    back = oracle.decode_regular(oracle.encode_regular(a, 32), a.shape, 32)
    emax = np.frexp(np.abs(a).max())[1]
    assert np.abs(back.astype(np.float64) - a).max() <= 2.0 ** (emax - 20)


def test_chunk_view_of_regular_array_matches_regular_coder():
    rng = np.random.default_rng(26)
    a = rng.standard_normal((9, 10, 13)).astype(np.float32)
    cs = W.regular_chunkset(9, 10, 13)
    for r in (8, 16):
        assert np.array_equal(oracle.pack_encode(cs, a, r), oracle.encode_regular(a, r))


def test_ragged_chunks_cover_every_point_once():
    cs = W.reduced_grid_chunkset(n_half=24, nlev=7, nchunks=5)
    rng = np.random.default_rng(27)
    src = rng.standard_normal(cs.buffer_elems).astype(np.float32)
    words = oracle.pack_encode(cs, src, 32)
    assert words.size == int(oracle.chunk_blocks(cs).sum()) * 32
    dst = np.full(cs.buffer_elems, np.nan, np.float32)
    oracle.decode_unpack(cs, words, 32, dst)
    assert not np.isnan(dst).any()  # the chunks tile the whole buffer
    assert np.allclose(dst, src, rtol=0, atol=1e-5 * np.abs(src).max())


def test_ragged_block_count_formula():
    # a chunk of two 4-row groups: rows of lengths 20..32 and 36..48 points
    cs = W.ChunkSet(np.array([0]), np.array([1000]), np.array([5]), np.array([0, 8]),
                    np.arange(8) * 50, 20 + 4 * np.arange(8), 5000)
    # ceil(5/4) level blocks x (ceil(32/4) + ceil(48/4)) x-blocks
    assert list(oracle.chunk_blocks(cs)) == [2 * (8 + 12)]


def test_sampled_encode_matches_full_encode():
    cs = W.reduced_grid_chunkset(n_half=16, nlev=9, nchunks=3)
    rng = np.random.default_rng(28)
    src = rng.standard_normal(cs.buffer_elems).astype(np.float32)
    full = oracle.pack_encode(cs, src, 8).reshape(-1, 8)
    ids = rng.choice(full.shape[0], 50, replace=False)
    assert np.array_equal(oracle.pack_encode_sample(cs, src, 8, ids), full[ids])


# ---------------------------------------------------------------------------
# float16 comparator (IEEE binary16, round to nearest even)
# ---------------------------------------------------------------------------

def test_f16_hand_values():
    cases = {
        1.0: 0x3C00, -2.0: 0xC000, 65504.0: 0x7BFF, 65519.996: 0x7BFF, 65520.0: 0x7C00,
        2.0 ** -24: 0x0001, 2.0 ** -25: 0x0000, 1.5 * 2.0 ** -24: 0x0002,
        2.0 ** -14: 0x0400, 1.0 + 2.0 ** -11: 0x3C00, 1.0 + 3 * 2.0 ** -11: 0x3C02,
        -0.0: 0x8000, math.inf: 0x7C00, -math.inf: 0xFC00, 1.0e6: 0x7C00,
    }
    x = np.array(list(cases), np.float32)
    got = oracle.f16_truncate(x)
    assert [int(g) for g in got] == list(cases.values())
    back = oracle.f16_restore(got)
    assert back[0] == 1.0 and back[5] == 2.0 ** -24 and np.isinf(back[4])


# ---------------------------------------------------------------------------
# Scatter and sampling helpers of the oracle, each against an independent
# formulation: numpy slicing of the per-block decode, or the whole-buffer
# functions pinned above
# ---------------------------------------------------------------------------

def _scatter_blocks(blocks, shape):
    """Place per-block values (nb, 64; index 16 z + 4 y + x) into an array of
    `shape` (nz, ny, nx) by numpy reshapes, blocks x-fastest; padding dropped."""
    nz, ny, nx = shape
    nbz, nby, nbx = -(-nz // 4), -(-ny // 4), -(-nx // 4)
    full = blocks.reshape(nbz, nby, nbx, 4, 4, 4).transpose(0, 3, 1, 4, 2, 5)
    return full.reshape(4 * nbz, 4 * nby, 4 * nbx)[:nz, :ny, :nx]


@pytest.mark.parametrize("shape", [(6, 9, 7), (4, 4, 4), (1, 5, 13), (9, 1, 2)])
def test_regular_decode_scatter_and_sentinels(shape):
    """orc_decode_regular puts every real value where numpy slicing of the
    per-block decode puts it (no axis swap, no padding written over edge
    values) and writes nothing else: in a strided destination every element
    between and around the view keeps its sentinel."""
    rng = np.random.default_rng(sum(shape) + 31)
    nz, ny, nx = shape
    a = (280 + 15 * rng.standard_normal(shape)).astype(np.float32)
    sx, sy = 2, 2 * nx + 3
    sz = sy * (ny + 1) + 5
    L = oracle.lib()
    for rate in (8, 32):
        words = oracle.encode_regular(a, rate)
        want = _scatter_blocks(oracle.decode_blocks(words, rate), shape)
        buf = np.full(sz * nz + 7, -7.0, np.float32)
        L.orc_decode_regular(words, nx, ny, nz, sx, sy, sz, rate, buf)
        idx = (np.arange(nz)[:, None, None] * sz + np.arange(ny)[None, :, None] * sy
               + np.arange(nx)[None, None, :] * sx)
        assert np.array_equal(buf[idx].view(np.uint32), want.view(np.uint32)), rate
        outside = np.ones(buf.size, bool)
        outside[idx.reshape(-1)] = False
        assert (buf[outside] == -7.0).all(), rate
        if rate == 32:
            # near-lossless at rate 32 (every value within 2^(emax-20) of its input)
            emax = np.frexp(np.abs(a).max())[1]
            assert np.abs(buf[idx].astype(np.float64) - a).max() <= 2.0 ** (emax - 20)


def test_decode_sample_matches_decode_unpack():
    """Every block decoded on its own (with the destination offset of each of
    its values and an in-range flag) agrees with the whole-buffer decode, and
    the in-range values cover every point of the chunks exactly once."""
    cs = W.reduced_grid_chunkset(n_half=20, nlev=6, nchunks=4)
    rng = np.random.default_rng(32)
    src = (280 + 15 * rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    for rate in (8, 16):
        words = oracle.pack_encode(cs, src, rate)
        dst = np.full(cs.buffer_elems, np.nan, np.float32)
        oracle.decode_unpack(cs, words, rate, dst)
        nb = int(oracle.chunk_blocks(cs).sum())
        vals, pos, inside = oracle.decode_sample(cs, words, rate, np.arange(nb))
        assert int(inside.sum()) == cs.buffer_elems == cs.values()
        p = pos[inside]
        assert np.array_equal(np.sort(p), np.arange(cs.buffer_elems))
        assert np.array_equal(vals[inside].view(np.uint32), dst[p].view(np.uint32))
        # each block's values in block order equal the per-block decoder's
        per_block = oracle.decode_blocks(words, rate).reshape(nb, 64)
        assert np.array_equal(vals.view(np.uint32), per_block.view(np.uint32))


def test_pack_encode_var_sample_matches_whole_stream():
    """Sampled variable-size blocks equal the same blocks cut out of the whole
    stream at the offsets its per-block word counts give."""
    cs = W.reduced_grid_chunkset(n_half=20, nlev=6, nchunks=4)
    rng = np.random.default_rng(33)
    src = np.cumsum(rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    for mp, me, cap in ((32, oracle.accuracy_minexp(1e-2), 16), (12, oracle.MINEXP_NONE, 32)):
        words, nd, toff = oracle.pack_encode_var(cs, src, mp, me, cap)
        start = np.concatenate([[0], np.cumsum(nd.astype(np.int64))])
        ids = np.unique(np.concatenate([rng.integers(0, nd.size, 60), [0, nd.size - 1]]))
        sw, bits, pos, inside = oracle.pack_encode_var_sample(cs, src, mp, me, cap, ids)
        for j, b in enumerate(ids):
            k = int(nd[b])
            assert (int(bits[j]) + 31) // 32 == k
            got = sw[j].view(np.uint32)
            assert np.array_equal(got[:k], words[start[b]:start[b] + k]), (mp, b)
            assert not got[k:].any()
        assert (inside.sum(1) > 0).all()
        assert np.isin(pos[inside], np.arange(cs.buffer_elems)).all()


def test_in_range_counts_from_geometry():
    """The test-side geometry count of real values per block (written from the
    chunk layout) agrees with the in-range flags the oracle's sampler reports,
    on ragged reduced-grid chunks and on a regular array with partial blocks."""
    from _blocks import real_values
    lens = np.array([5, 9, 3, 11, 7, 2, 6])
    offs = np.concatenate([[1], 1 + np.cumsum(lens)[:-1] + 3 * np.arange(1, 7)])
    odd = W.ChunkSet(np.array([0, 2]), np.array([200, 203]), np.array([6, 3]),
                     np.array([0, 5, 7]), np.concatenate([offs[:5], offs[5:] - 2]), lens, 1300)
    for cs in (W.reduced_grid_chunkset(n_half=20, nlev=6, nchunks=4),
               W.reduced_grid_chunkset(n_half=12, nlev=5, nchunks=3), odd,
               W.regular_chunkset(7, 10, 13)):
        nb = int(oracle.chunk_blocks(cs).sum())
        words = np.zeros(nb * 8, np.uint64)
        _, _, inside = oracle.decode_sample(cs, words, 8, np.arange(nb))
        assert np.array_equal(inside.sum(1), real_values(cs, np.arange(nb)))
        assert int(real_values(cs, np.arange(nb)).sum()) == cs.values()
