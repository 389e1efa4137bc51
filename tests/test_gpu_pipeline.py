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


def test_back_to_back_calls_without_host_sync(zfpx_lib):
    # three sends and three receives enqueued in a row on the same buffers:
    # each waits on the device for the previous one's use of them
    Z = zfpx_lib
    cs = W.zlambda_chunkset(nfields=1, nlev=17, nrows=16, npts=401, nchunks=4)
    rng = np.random.default_rng(410)
    plan = Z.Plan.from_chunkset(cs)
    srcs = [torch.from_numpy((280 + np.cumsum(rng.standard_normal(cs.buffer_elems)))
                             .astype(np.float32)).to(DEV) for _ in range(3)]
    cstream, xstream = torch.cuda.Stream(), torch.cuda.Stream()
    rate = 16
    pipe = Z.Pipeline(plan, rate, 4)
    nbytes = plan.nblocks * 8 * rate
    send = torch.empty(nbytes // 8, dtype=torch.int64, device=DEV)
    recv = torch.empty_like(send)
    links = [torch.zeros(nbytes // 8, dtype=torch.int64).pin_memory() for _ in range(3)]
    dsts = [torch.full_like(srcs[0], float("nan")) for _ in range(3)]
    torch.cuda.synchronize()
    for k in range(3):
        pipe.send(srcs[k], send, links[k], cstream, xstream)
    xstream.synchronize()
    for k in range(3):
        pipe.recv(links[k], recv, dsts[k], cstream, xstream)
    cstream.synchronize()
    for k in range(3):
        want = oracle.pack_encode(cs, srcs[k].cpu().numpy(), rate)
        assert np.array_equal(links[k].numpy().view(np.uint64), want), k
        back = np.full(cs.buffer_elems, np.nan, np.float32)
        oracle.decode_unpack(cs, want, rate, back)
        assert np.array_equal(dsts[k].cpu().numpy().view(np.uint32), back.view(np.uint32)), k
    pipe.close()
