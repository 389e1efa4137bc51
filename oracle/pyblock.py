"""Second, independent writing of the single-block ZFP fixed-rate codec.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Pure Python integers
and lists of bits, written separately from ``zfp_oracle.c`` so that a slip in
either shows up as a disagreement on random blocks.  It follows the same
steps (ZFP's published algorithm description as used by the paper, Section
II-C) and the same readings of the open conventions.  Slow: small cases only.
"""
from __future__ import annotations

import math
import struct

MASK32 = (1 << 32) - 1
NB = 0xAAAAAAAA


def _s32(x: int) -> int:
    """Two's-complement int32 value of x modulo 2^32."""
    x &= MASK32
    return x - (1 << 32) if x >> 31 else x


def _f32(x: float) -> float:
    """Round a double to float32 (nearest, ties to even; overflow to infinity)."""
    try:
        return struct.unpack("<f", struct.pack("<f", x))[0]
    except OverflowError:
        return math.copysign(math.inf, x)


def exponent(v: list[float]):
    """(nonempty, emax): emax = max frexp exponent over nonzero values, >= -126."""
    es = [max(math.frexp(abs(x))[1], -126) for x in v if x != 0.0]
    return (len(es) > 0, max(es) if es else -126)


def lift(xs: list[int]) -> list[int]:
    x, y, z, w = xs
    x = _s32(x + w) >> 1; w = _s32(w - x)
    z = _s32(z + y) >> 1; y = _s32(y - z)
    x = _s32(x + z) >> 1; z = _s32(z - x)
    w = _s32(w + y) >> 1; y = _s32(y - w)
    w = _s32(w + (y >> 1)); y = _s32(y - (w >> 1))
    return [x, y, z, w]


def unlift(xs: list[int]) -> list[int]:
    x, y, z, w = xs
    y = _s32(y + (w >> 1)); w = _s32(w - (y >> 1))
    y = _s32(y + w); w = _s32((w << 1) - y)
    z = _s32(z + x); x = _s32((x << 1) - z)
    y = _s32(y + z); z = _s32((z << 1) - y)
    w = _s32(w + x); x = _s32((x << 1) - w)
    return [x, y, z, w]


def _apply_lines(q: list[int], f, stride: int, starts: list[int]) -> None:
    for s0 in starts:
        idx = [s0 + t * stride for t in range(4)]
        out = f([q[i] for i in idx])
        for i, o in zip(idx, out):
            q[i] = o


_X_STARTS = [16 * z + 4 * y for z in range(4) for y in range(4)]
_Y_STARTS = [16 * z + x for z in range(4) for x in range(4)]
_Z_STARTS = [4 * y + x for y in range(4) for x in range(4)]


def forward(q: list[int]) -> list[int]:
    q = list(q)
    _apply_lines(q, lift, 1, _X_STARTS)
    _apply_lines(q, lift, 4, _Y_STARTS)
    _apply_lines(q, lift, 16, _Z_STARTS)
    return q


def inverse(q: list[int]) -> list[int]:
    q = list(q)
    _apply_lines(q, unlift, 16, _Z_STARTS)
    _apply_lines(q, unlift, 4, _Y_STARTS)
    _apply_lines(q, unlift, 1, _X_STARTS)
    return q


def sequency() -> list[int]:
    def key(i):
        x, y, z = i & 3, (i >> 2) & 3, i >> 4
        return (x + y + z, x * x + y * y + z * z, i)
    return sorted(range(64), key=key)


def _plane(u: list[int], k: int) -> list[int]:
    return [(c >> k) & 1 for c in u]


def code(u: list[int], budget: int, kmin: int = 0) -> list[int]:
    """Embedded coding of 64 negabinary words, planes 31 down to kmin;
    returns the emitted bits."""
    out: list[int] = []
    n = 0
    for k in range(31, kmin - 1, -1):
        if len(out) >= budget:
            break
        p = _plane(u, k)
        for s in range(n):
            if len(out) >= budget:
                break
            out.append(p[s])
        # group tests and unary scans over positions >= n
        while n < 64 and len(out) < budget:
            g = 1 if any(p[n:]) else 0
            out.append(g)
            if not g:
                break
            while n < 63 and len(out) < budget:
                out.append(p[n])
                if p[n]:
                    break
                n += 1
            n += 1
    return out


def uncode(bits: list[int], budget: int, kmin: int = 0) -> list[int]:
    u = [0] * 64
    pos = 0
    n = 0

    def take():
        nonlocal pos
        b = bits[pos]
        pos += 1
        return b

    for k in range(31, kmin - 1, -1):
        if pos >= budget:
            break
        p = [0] * 64
        for s in range(min(n, budget - pos)):
            p[s] = take()
        while n < 64 and pos < budget:
            if not take():
                break
            while n < 63 and pos < budget:
                if take():
                    break
                n += 1
            p[n] = 1
            n += 1
        for s in range(64):
            u[s] |= p[s] << k
    return u


def _bits_to_words(bits: list[int], nwords: int) -> list[int]:
    words = [0] * nwords
    for i, b in enumerate(bits):
        if b:
            words[i // 64] |= 1 << (i % 64)
    return words


def _words_to_bits(words: list[int]) -> list[int]:
    return [(w >> i) & 1 for w in words for i in range(64)]


def encode_block(v: list[float], rate: int) -> list[int]:
    """64 float32 values (block-local index 16z+4y+x) -> `rate` 64-bit words."""
    v = [_f32(float(x)) for x in v]
    nonempty, emax = exponent(v)
    if not nonempty:
        return [0] * rate
    bits = [1] + [((emax + 127) >> i) & 1 for i in range(8)]
    q = [int(math.ldexp(x, 30 - emax)) for x in v]  # int() truncates toward zero
    c = forward(q)
    perm = sequency()
    u = [(_s32(c[perm[s]]) + NB) & MASK32 ^ NB for s in range(64)]
    bits += code(u, 64 * rate - 9)
    return _bits_to_words(bits, rate)


def decode_block(words: list[int], rate: int) -> list[float]:
    bits = _words_to_bits(words)
    if not bits[0]:
        return [0.0] * 64
    emax = sum(bits[1 + i] << i for i in range(8)) - 127
    u = uncode(bits[9:], 64 * rate - 9)
    perm = sequency()
    c = [0] * 64
    for s in range(64):
        c[perm[s]] = _s32((u[s] ^ NB) - NB)
    q = inverse(c)
    # math.ldexp is exact here; struct packing rounds once, to nearest even
    return [_f32(math.ldexp(float(x), emax - 30)) for x in q]


# Variable-size modes: the same coder stopped after p bit planes, where
# p = min(maxprec, max(0, emax - minexp + 2 (d + 1))) for d = 3 dimensions;
# p = 0 gives the single bit 0; the length is capped at 64 rate_cap bits.

def planes_for(emax: int, maxprec: int, minexp: int) -> int:
    return max(0, min(maxprec, emax - minexp + 2 * (3 + 1)))


def encode_block_var(v: list[float], maxprec: int, minexp: int, rate_cap: int):
    """-> (rate_cap + 1 words, length in bits)."""
    v = [_f32(float(x)) for x in v]
    nonempty, emax = exponent(v)
    p = planes_for(emax, maxprec, minexp) if nonempty else 0
    if p == 0:
        return [0] * (rate_cap + 1), 1
    bits = [1] + [((emax + 127) >> i) & 1 for i in range(8)]
    q = [int(math.ldexp(x, 30 - emax)) for x in v]
    c = forward(q)
    perm = sequency()
    u = [(_s32(c[perm[s]]) + NB) & MASK32 ^ NB for s in range(64)]
    bits += code(u, 64 * rate_cap - 9, 32 - p)
    return _bits_to_words(bits, rate_cap + 1), len(bits)


def decode_block_var(words: list[int], maxprec: int, minexp: int, rate_cap: int) -> list[float]:
    bits = _words_to_bits(list(words) + [0])
    if not bits[0]:
        return [0.0] * 64
    emax = sum(bits[1 + i] << i for i in range(8)) - 127
    p = planes_for(emax, maxprec, minexp)
    u = uncode(bits[9:], 64 * rate_cap - 9, 32 - p)
    perm = sequency()
    c = [0] * 64
    for s in range(64):
        c[perm[s]] = _s32((u[s] ^ NB) - NB)
    q = inverse(c)
    return [_f32(math.ldexp(float(x), emax - 30)) for x in q]

