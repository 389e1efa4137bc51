"""Chunk-wise pipeline over a host link: the bytes that reach the link are
the fixed-rate stream, and the receive side decodes them as the direct call
does, for any number of chunk groups."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_24294_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("groups", [1, 5, 64, 1000])
def test_send_and_recv_match_direct_calls(zfpx_lib, groups):
    Z = zfpx_lib
    cs = W.zlambda_chunkset(nfields=2, nlev=21, nrows=32, npts=613, nchunks=16)
    rng = np.random.default_rng(400 + groups)
    src_h = (280 + np.cumsum(rng.standard_normal(cs.buffer_elems))).astype(np.float32)
    plan = Z.Plan.from_chunkset(cs)
    src = torch.from_numpy(src_h).to(DEV)
    cstream, xstream = torch.cuda.Stream(), torch.cuda.Stream()
    for rate in (8, 16):
        nbytes = plan.nblocks * 8 * rate
        pipe = Z.Pipeline(plan, rate, groups)
        send = torch.empty(nbytes // 8, dtype=torch.int64, device=DEV)
        link = torch.zeros(nbytes // 8, dtype=torch.int64).pin_memory()
        torch.cuda.synchronize()
        pipe.send(src, send, link, cstream, xstream)
        xstream.synchronize()
        want = oracle.pack_encode(cs, src_h, rate)
        assert np.array_equal(link.numpy().view(np.uint64), want)
        recv = torch.empty_like(send)
        dst = torch.full_like(src, float("nan"))
        pipe.recv(link, recv, dst, cstream, xstream)
        cstream.synchronize()
        direct = torch.full_like(src, float("nan"))
        Z.zfpx_decode_unpack(plan, send, rate, direct)
        torch.cuda.synchronize()
        assert torch.equal(dst.view(torch.int32), direct.view(torch.int32))
        pipe.close()
