"""Variable-size modes on the GPU against the oracle: the stream (words,
per-block word counts, tile offsets) bit for bit, decoded floats bit for bit,
chunk offsets, the capacity limit and arbitrary decoder input."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_24294_amd import workloads as W

from _blocks import array_to_blocks, block_families, blocks_to_array

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NONE = -1074

PARAMS = [  # (maxprec, minexp, rate_cap)
    (32, NONE, 32), (32, NONE, 16), (16, NONE, 16), (8, NONE, 8), (1, NONE, 1),
    (32, -7, 32), (32, -20, 16), (32, 0, 5), (20, -20, 24), (12, 3, 11),
]


def f32bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def _stream(words, nd, toff):
    torch.cuda.synchronize()
    toff = toff.cpu().numpy()
    total = int(toff[-1])
    return words[:total].cpu().numpy().view(np.uint32), nd.cpu().numpy(), toff


@pytest.mark.parametrize("maxprec,minexp,cap", PARAMS)
def test_block_families(zfpx_lib, maxprec, minexp, cap):
    Z = zfpx_lib
    rng = np.random.default_rng(300 + cap + maxprec)
    blocks = block_families(rng, 900)  # 15 tiles, the last one ragged
    a = blocks_to_array(blocks)
    cs = W.regular_chunkset(*a.shape)
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(a.reshape(-1)).to(DEV)
    words, nd, toff = Z.zfpx_plan_encode_var(plan, d, maxprec, minexp, cap)
    gw, gnd, gtoff = _stream(words, nd, toff)
    ow, ond, otoff = oracle.pack_encode_var(cs, a, maxprec, minexp, cap)
    assert np.array_equal(gnd[:ond.size], ond)
    assert np.array_equal(gtoff, otoff)
    assert np.array_equal(gw, ow)
    out = torch.full_like(d, float("nan"))
    Z.zfpx_plan_decode_var(plan, words, nd, toff, maxprec, minexp, cap, out)
    want = np.zeros(a.size, np.float32)
    oracle.decode_unpack_var(cs, ow, ond, maxprec, minexp, cap, want)
    assert np.array_equal(f32bits(out.cpu()), f32bits(want))


def test_ragged_chunks_and_chunk_offsets(zfpx_lib):
    Z = zfpx_lib
    cs = W.reduced_grid_chunkset(n_half=40, nlev=9, nchunks=7)
    rng = np.random.default_rng(310)
    src = np.cumsum(rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(src).to(DEV)
    for maxprec, minexp, cap in ((32, oracle.accuracy_minexp(1e-3), 32), (14, NONE, 16)):
        words, nd, toff = Z.zfpx_plan_encode_var(plan, d, maxprec, minexp, cap)
        coff = Z.zfpx_plan_var_chunk_offsets(plan, nd, toff)
        gw, gnd, gtoff = _stream(words, nd, toff)
        ow, ond, otoff = oracle.pack_encode_var(cs, src, maxprec, minexp, cap)
        assert np.array_equal(gnd, ond) and np.array_equal(gtoff, otoff)
        assert np.array_equal(gw, ow)
        first = np.concatenate([[0], np.cumsum(oracle.chunk_blocks(cs))])
        off = np.concatenate([[0], np.cumsum(ond.astype(np.int64))])
        assert np.array_equal(coff.cpu().numpy(), off[first])
        out = torch.full_like(d, float("nan"))
        Z.zfpx_plan_decode_var(plan, words, nd, toff, maxprec, minexp, cap, out)
        want = np.full(src.size, np.nan, np.float32)
        oracle.decode_unpack_var(cs, ow, ond, maxprec, minexp, cap, want)
        assert np.array_equal(f32bits(out.cpu()), f32bits(want))
        if maxprec == 32:
            assert np.abs(out.cpu().numpy().astype(np.float64) - src).max() <= 1e-3


def test_full_precision_matches_fixed_rate_stream(zfpx_lib):
    # maxprec 32 without an exponent floor is fixed rate cut at each block's length
    Z = zfpx_lib
    cs = W.zlambda_chunkset(nfields=1, nlev=13, nrows=8, npts=301, nchunks=2)
    rng = np.random.default_rng(311)
    src = (280 + np.cumsum(rng.standard_normal(cs.buffer_elems))).astype(np.float32)
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(src).to(DEV)
    for r in (8, 16):
        words, nd, toff = Z.zfpx_plan_encode_var(plan, d, 32, NONE, r)
        fixed = Z.zfpx_pack_encode(plan, d, r).cpu().numpy().view(np.uint32).reshape(-1, 2 * r)
        gw, gnd, gtoff = _stream(words, nd, toff)
        off = np.concatenate([[0], np.cumsum(gnd.astype(np.int64))])
        for b in range(gnd.size):
            k = int(gnd[b])
            assert np.array_equal(gw[off[b]:off[b] + k], fixed[b, :k])
            assert not fixed[b, k:].any()


def test_capacity_is_never_exceeded(zfpx_lib):
    Z = zfpx_lib
    rng = np.random.default_rng(312)
    blocks = block_families(rng, 300)
    a = blocks_to_array(blocks)
    plan = Z.Plan.from_chunkset(W.regular_chunkset(*a.shape))
    d = torch.from_numpy(a.reshape(-1)).to(DEV)
    full_w, full_nd, full_toff = Z.zfpx_plan_encode_var(plan, d, 32, NONE, 16)
    total = int(full_toff[-1].item())
    cap_words = total // 2
    buf = torch.full((total + 256,), -7, dtype=torch.int32, device=DEV)
    w, nd, toff = Z.zfpx_plan_encode_var(plan, d, 32, NONE, 16, words=buf[:cap_words])
    torch.cuda.synchronize()
    assert int(toff[-1].item()) == total  # the full size is still reported
    assert torch.equal(buf[:cap_words], full_w[:cap_words])
    assert bool((buf[cap_words:] == -7).all())


def test_scratch_reused_across_calls(zfpx_lib):
    Z = zfpx_lib
    rng = np.random.default_rng(313)
    blocks = block_families(rng, 700)
    a = blocks_to_array(blocks)
    cs = W.regular_chunkset(*a.shape)
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(a.reshape(-1)).to(DEV)
    _, _, wb = Z.zfpx_plan_var_sizes(plan, 32)
    work = torch.full(((wb + 7) // 8,), 12345, dtype=torch.int64, device=DEV)  # stale content
    for maxprec, minexp, cap in ((32, -5, 32), (9, NONE, 8), (32, -5, 32)):
        words, nd, toff = Z.zfpx_plan_encode_var(plan, d, maxprec, minexp, cap, work=work)
        gw, gnd, gtoff = _stream(words, nd, toff)
        ow, ond, otoff = oracle.pack_encode_var(cs, a, maxprec, minexp, cap)
        assert np.array_equal(gw, ow) and np.array_equal(gtoff, otoff)


def test_decoder_on_arbitrary_content(zfpx_lib):
    # random words and counts with consistent offsets: same floats as the
    # oracle; then counts past the cap and arbitrary offsets: no fault
    Z = zfpx_lib
    rng = np.random.default_rng(314)
    nb, cap = 1000, 8
    a = np.zeros((4, 4, 4 * nb), np.float32)
    cs = W.regular_chunkset(*a.shape)
    plan = Z.Plan.from_chunkset(cs)
    nd = rng.integers(0, 2 * cap + 1, nb).astype(np.uint8)
    off = np.concatenate([[0], np.cumsum(nd.astype(np.int64))])
    words = rng.integers(0, 2 ** 32, int(off[-1]) + 1, dtype=np.uint64).astype(np.uint32)
    toff = off[::64].copy()
    toff = np.concatenate([toff, [off[-1]]]) if toff.size == (nb + 63) // 64 else toff
    for maxprec, minexp in ((32, NONE), (32, -3), (11, NONE)):
        out = torch.full((a.size,), float("nan"), device=DEV)
        Z.zfpx_plan_decode_var(plan, torch.from_numpy(words.view(np.int32)).to(DEV),
                               torch.from_numpy(nd).to(DEV), torch.from_numpy(toff).to(DEV),
                               maxprec, minexp, cap, out)
        want = np.zeros(a.size, np.float32)
        oracle.decode_unpack_var(cs, words, nd, maxprec, minexp, cap, want)
        assert np.array_equal(f32bits(out.cpu()), f32bits(want))
    bad_nd = rng.integers(0, 256, nb).astype(np.uint8)
    bad_toff = rng.integers(-2 ** 62, 2 ** 62, toff.size)
    bad_toff[::3] = rng.integers(0, int(off[-1]) + 1, bad_toff[::3].size)
    out = torch.empty((a.size,), device=DEV)
    Z.zfpx_plan_decode_var(plan, torch.from_numpy(words.view(np.int32)).to(DEV),
                           torch.from_numpy(bad_nd).to(DEV), torch.from_numpy(bad_toff).to(DEV),
                           32, NONE, cap, out)
    torch.cuda.synchronize()


def test_zlambda_share_full_size_sampled(zfpx_lib):
    # the 4 x 137 x 64 x 1612 share in one launch: offsets are an exclusive
    # scan of the counts, and sampled blocks match the oracle (stream and
    # decoded floats)
    Z = zfpx_lib
    x32, _ = W.zlambda_fields(want_f64=False)
    cs = W.zlambda_chunkset()
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(x32.reshape(-1)).to(DEV)
    rng = np.random.default_rng(315)
    for maxprec, minexp, cap in ((16, NONE, 16), (32, oracle.accuracy_minexp(0.05), 32)):
        words, nd, toff = Z.zfpx_plan_encode_var(plan, d, maxprec, minexp, cap)
        out = torch.empty_like(d)
        Z.zfpx_plan_decode_var(plan, words, nd, toff, maxprec, minexp, cap, out)
        gw, gnd, gtoff = _stream(words, nd, toff)
        off = np.concatenate([[0], np.cumsum(gnd.astype(np.int64))])
        assert np.array_equal(gtoff, np.concatenate([off[:-1][::64], off[-1:]]))
        ids = np.unique(np.concatenate([rng.choice(gnd.size, 3000, replace=False),
                                        [0, 63, 64, gnd.size - 1]]))
        ow, ol, pos, ins = oracle.pack_encode_var_sample(cs, x32, maxprec, minexp, cap, ids)
        assert np.array_equal(gnd[ids], (ol + 31) // 32)
        host_out = out.cpu().numpy()
        for j, b in enumerate(ids):
            k = int(gnd[b])
            assert np.array_equal(gw[off[b]:off[b] + k], ow[j].view(np.uint32)[:k]), b
            v = oracle.decode_block_var(ow[j], maxprec, minexp, cap)
            assert np.array_equal(f32bits(host_out[pos[j][ins[j]]]), f32bits(v[ins[j]])), b


def test_encode_decode_captured_in_a_graph(zfpx_lib):
    # the variable-size calls only enqueue kernels (no memset, no allocation):
    # captured once, each replay on new input matches the eager calls
    Z = zfpx_lib
    cs = W.zlambda_chunkset(nfields=1, nlev=21, nrows=16, npts=501, nchunks=4)
    plan = Z.Plan.from_chunkset(cs)
    rng = np.random.default_rng(316)
    maxprec, minexp, cap = 32, oracle.accuracy_minexp(1e-3), 16
    src = torch.empty(cs.buffer_elems, dtype=torch.float32, device=DEV)
    out = torch.empty_like(src)
    mw, nt, wb = Z.zfpx_plan_var_sizes(plan, cap)
    words = torch.empty(mw, dtype=torch.int32, device=DEV)
    nd = torch.empty(plan.nblocks, dtype=torch.uint8, device=DEV)
    toff = torch.empty(nt + 1, dtype=torch.int64, device=DEV)
    work = torch.empty((wb + 7) // 8, dtype=torch.int64, device=DEV)
    src.copy_(torch.from_numpy(np.cumsum(rng.standard_normal(cs.buffer_elems)).astype(np.float32)))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            Z.zfpx_plan_encode_var(plan, src, maxprec, minexp, cap, words, nd, toff, work)
            Z.zfpx_plan_decode_var(plan, words, nd, toff, maxprec, minexp, cap, out)
    for rep in range(3):
        host = np.cumsum(rng.standard_normal(cs.buffer_elems)).astype(np.float32)
        src.copy_(torch.from_numpy(host))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_words = words[:int(toff[-1].item())].clone()
        got_out = out.clone()
        ew, end_, eto = Z.zfpx_plan_encode_var(plan, src, maxprec, minexp, cap)
        eo = torch.empty_like(src)
        Z.zfpx_plan_decode_var(plan, ew, end_, eto, maxprec, minexp, cap, eo)
        torch.cuda.synchronize()
        assert torch.equal(toff, eto) and torch.equal(nd, end_[:plan.nblocks])
        assert torch.equal(got_words, ew[:int(eto[-1].item())]), rep
        assert torch.equal(got_out.view(torch.int32), eo.view(torch.int32)), rep
        ow, ond, otoff = oracle.pack_encode_var(cs, host, maxprec, minexp, cap)
        assert np.array_equal(got_words.cpu().numpy().view(np.uint32), ow), rep


def test_large_buffer_full_size_sampled(zfpx_lib):
    # O2560 x 90 levels (9.47 GB, 37,859,840 blocks) in one launch: offsets are
    # the exclusive scan of the counts over 591,560 tiles, and sampled blocks
    # match the oracle (stream words and decoded floats)
    Z = zfpx_lib
    cs = W.large_chunkset()
    x32 = W.large_field_repeated(W.large_field_levels(8))
    plan = Z.Plan.from_chunkset(cs)
    d = torch.from_numpy(x32.reshape(-1)).to(DEV)
    maxprec, minexp, cap = 16, NONE, 16
    words, nd, toff = Z.zfpx_plan_encode_var(plan, d, maxprec, minexp, cap)
    out = torch.empty_like(d)
    Z.zfpx_plan_decode_var(plan, words, nd, toff, maxprec, minexp, cap, out)
    torch.cuda.synchronize()
    gnd = nd.cpu().numpy()
    gtoff = toff.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(gnd.astype(np.int64))])
    assert gtoff.size == 591560 + 1
    assert np.array_equal(gtoff, np.concatenate([off[:-1][::64], off[-1:]]))
    rng = np.random.default_rng(317)
    ids = np.unique(np.concatenate([rng.choice(plan.nblocks, 1500, replace=False),
                                    [0, 63, 64, plan.nblocks - 1]]))
    ow, ol, pos, ins = oracle.pack_encode_var_sample(cs, x32, maxprec, minexp, cap, ids)
    assert np.array_equal(gnd[ids], (ol + 31) // 32)
    flat = out.view(-1)
    for j, b in enumerate(ids):
        k = int(gnd[b])
        got = words[int(off[b]):int(off[b]) + k].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ow[j].view(np.uint32)[:k]), b
        v = oracle.decode_block_var(ow[j], maxprec, minexp, cap)
        p = torch.from_numpy(pos[j][ins[j]]).to(DEV)
        assert np.array_equal(flat[p].cpu().numpy().view(np.uint32), v[ins[j]].view(np.uint32)), b
