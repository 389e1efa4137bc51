"""The codec on the Fourier-space lambda->theta buffer (real and imaginary
planes, chunked by wavenumber range) against the oracle: bit-exact streams
and floats at fixed rate and in the variable-size modes."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_24294_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def f32bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def test_small_buffer_fixed_and_variable(zfpx_lib):
    Z = zfpx_lib
    nlev, nrows, mmax, ndest = 9, 12, 127, 4
    cs = W.fourier_chunkset(nlev, nrows, mmax, ndest)
    f32, _ = W.fourier_buffer(L=mmax, nlev=nlev, nrows=nrows)
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(f32.reshape(-1)).to(DEV)
    for rate in (8, 16, 32):
        words = Z.zfpx_pack_encode(plan, d, rate)
        want = oracle.pack_encode(cs, f32, rate)
        assert np.array_equal(words.cpu().numpy().view(np.uint64), want), rate
        out = torch.full_like(d, float("nan"))
        Z.zfpx_decode_unpack(plan, words, rate, out)
        back = np.full(cs.buffer_elems, np.nan, np.float32)
        oracle.decode_unpack(cs, want, rate, back)
        assert np.array_equal(f32bits(out.cpu()), f32bits(back)), rate
    for maxprec, minexp, cap in ((16, -1074, 16), (32, oracle.accuracy_minexp(1e-3), 32)):
        w, nd, toff = Z.zfpx_plan_encode_var(plan, d, maxprec, minexp, cap)
        torch.cuda.synchronize()
        ow, ond, otoff = oracle.pack_encode_var(cs, f32, maxprec, minexp, cap)
        assert np.array_equal(toff.cpu().numpy(), otoff)
        assert np.array_equal(nd.cpu().numpy()[:ond.size], ond)
        assert np.array_equal(w[:int(otoff[-1])].cpu().numpy().view(np.uint32), ow)


def test_full_share_sampled(zfpx_lib):
    Z = zfpx_lib
    c = W.FOURIER
    cs = W.fourier_chunkset(c["nlev"], c["nrows"], c["mmax"], c["ndest"])
    f32, _ = W.fourier_buffer()
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(f32.reshape(-1)).to(DEV)
    rng = np.random.default_rng(500)
    for rate in (8, 16):
        words = Z.zfpx_pack_encode(plan, d, rate).cpu().numpy().view(np.uint64).reshape(-1, rate)
        ids = np.unique(np.concatenate([rng.choice(plan.nblocks, 3000, replace=False),
                                        [0, plan.nblocks - 1]]))
        want = oracle.pack_encode_sample(cs, f32, rate, ids)
        assert np.array_equal(words[ids], want), rate
