"""The Fourier-space lambda->theta buffer (inputs only): layout, chunk
coverage and the structure of the generated coefficients."""
import numpy as np

import oracle
from paper_2609_24294_amd import workloads as W


def test_chunks_cover_every_coefficient_once():
    cs = W.fourier_chunkset(nlev=5, nrows=6, mmax=40, ndest=3)
    seen = np.zeros(cs.buffer_elems, np.int32)
    for c in range(cs.nchunks):
        for z in range(int(cs.levels[c])):
            for r in range(int(cs.row_start[c]), int(cs.row_start[c + 1])):
                o = int(cs.chunk_base[c] + z * cs.level_stride[c] + cs.row_offset[r])
                seen[o:o + int(cs.row_len[r])] += 1
    assert (seen == 1).all()
    # destination d's message is its real chunk followed by its imaginary chunk
    assert list(cs.chunk_base[:4]) == [0, 5 * 6 * 41, 13, 5 * 6 * 41 + 13]


def test_round_trip_through_the_oracle_covers_the_buffer():
    cs = W.fourier_chunkset(nlev=5, nrows=6, mmax=40, ndest=3)
    f32, _ = W.fourier_buffer(L=40, nlev=5, nrows=6)
    words = oracle.pack_encode(cs, f32, 32)
    dst = np.full(cs.buffer_elems, np.nan, np.float32)
    oracle.decode_unpack(cs, words, 32, dst)
    assert not np.isnan(dst).any()
    assert np.abs(dst - f32.reshape(-1)).max() <= 1e-5 * np.abs(f32).max()


def test_coefficients_structure():
    f32, f64 = W.fourier_buffer(L=95, nlev=7, nrows=8)
    assert f32.shape == (2, 7, 8, 96)
    assert not f64[1, :, :, 0].any()            # m = 0 is real
    assert abs(np.mean(f64 * f64) - 1.0) < 1e-12  # unit RMS
    power = (f64 * f64).mean(axis=(0, 1, 2))
    assert power[:8].mean() > 100 * power[-8:].mean()  # energy falls off with m
    # levels are correlated (AR(1), 0.9) and rows vary smoothly at low m
    c = np.corrcoef(f64[0, :-1, :, 1:6].ravel(), f64[0, 1:, :, 1:6].ravel())[0, 1]
    assert c > 0.7
