"""Seeded families of 4x4x4 test blocks, and the in-range value count of a
chunk block from the chunk geometry (inputs and geometry only)."""
import numpy as np


def block_families(rng, count):
    """`count` float32 blocks cycling through smooth, noisy, wide-range,
    single-spike, tiny-integer, subnormal, constant, lognormal and zero cases."""
    out = []
    for t in range(count):
        k = t % 9
        if k == 0:
            v = 280 + 15 * rng.standard_normal(64)
        elif k == 1:
            v = np.cumsum(np.cumsum(rng.standard_normal((4, 4, 4)), 0), 2).reshape(-1)
        elif k == 2:
            v = rng.standard_normal(64) * 10.0 ** rng.uniform(-40, 38, 64)
        elif k == 3:
            v = np.zeros(64)
            v[rng.integers(64)] = rng.standard_normal() * 2.0 ** rng.integers(-149, 127)
        elif k == 4:
            v = rng.choice([0.0, 1.0, -1.0, 2.0, -2.0], 64) * 2.0 ** rng.integers(-20, 20)
        elif k == 5:
            v = rng.standard_normal(64) * 2.0 ** -135
        elif k == 6:
            v = np.full(64, rng.standard_normal() * 2.0 ** rng.integers(-100, 100))
        elif k == 7:
            v = np.exp(rng.standard_normal(64))
        else:
            v = np.zeros(64) * (-1.0 if t % 2 else 1.0)
        # finite inputs only (non-finite values are outside the codec's contract)
        fmax = float(np.finfo(np.float32).max)
        out.append(np.asarray(np.clip(v, -fmax, fmax), np.float32))
    return np.stack(out)


def blocks_to_array(blocks):
    """Lay out (n, 64) blocks as a (4, 4, 4 n) array whose x-block b is block b."""
    n = blocks.shape[0]
    return np.ascontiguousarray(blocks.reshape(n, 4, 4, 4).transpose(1, 2, 0, 3).reshape(4, 4, 4 * n))


def array_to_blocks(a):
    n = a.shape[2] // 4
    return np.ascontiguousarray(a.reshape(4, 4, n, 4).transpose(2, 0, 1, 3).reshape(n, 64))


def real_values(cs, ids):
    """In-range values of each listed block, from the chunk geometry alone:
    blocks are numbered by chunk, then level block, then row group (rows in
    fours), then x block; a group is as wide as its longest row."""
    first, per_chunk = [0], []
    for c in range(cs.nchunks):
        r0, r1 = int(cs.row_start[c]), int(cs.row_start[c + 1])
        lens = cs.row_len[r0:r1].astype(np.int64)
        widths = [-(-int(lens[g:g + 4].max()) // 4) for g in range(0, lens.size, 4)]
        per_lb = int(sum(widths))
        per_chunk.append((lens, np.cumsum([0] + widths), per_lb, int(cs.levels[c])))
        first.append(first[-1] + per_lb * -(-int(cs.levels[c]) // 4))
    first = np.array(first)
    out = np.zeros(len(ids), np.int64)
    for j, b in enumerate(ids):
        c = int(np.searchsorted(first, b, side="right") - 1)
        lens, gstart, per_lb, nlev = per_chunk[c]
        rem = int(b - first[c])
        bz, rem = divmod(rem, per_lb)
        g = int(np.searchsorted(gstart, rem, side="right") - 1)
        bx = rem - int(gstart[g])
        rows = lens[4 * g: 4 * g + 4]
        out[j] = min(4, nlev - 4 * bz) * int(np.clip(rows - 4 * bx, 0, 4).sum())
    return out
