"""Seeded families of 4x4x4 test blocks (inputs only)."""
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
