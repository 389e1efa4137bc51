"""GPU (HIP) path against the CPU oracle: bit-exact streams and floats."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_24294_amd import workloads as W

from _blocks import array_to_blocks, block_families, blocks_to_array, real_values

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def f32bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def test_small_field_all_rates(zfpx_lib):
    x32, _ = W.small_field()
    d = torch.from_numpy(x32).to(DEV)
    for rate in (8, 16, 32):
        words = zfpx_lib.zfpx_encode_fixed_rate(d, rate)
        want = oracle.encode_regular(x32, rate)
        assert np.array_equal(u64(words), want), rate
        out = torch.full_like(d, float("nan"))
        zfpx_lib.zfpx_decode_fixed_rate(words, rate, out)
        back = oracle.decode_regular(want, x32.shape, rate)
        assert np.array_equal(f32bits(out.cpu()), f32bits(back)), rate


@pytest.mark.parametrize("rate", [1, 2, 3, 5, 8, 11, 16, 24, 31, 32])
def test_block_families_every_rate(zfpx_lib, rate):
    rng = np.random.default_rng(100 + rate)
    blocks = block_families(rng, 900)
    a = blocks_to_array(blocks)
    d = torch.from_numpy(a).to(DEV)
    words = zfpx_lib.zfpx_encode_fixed_rate(d, rate)
    want = oracle.encode_blocks(blocks, rate)
    got = u64(words).reshape(-1, rate)
    bad = np.nonzero((got != want).any(1))[0]
    assert bad.size == 0, f"rate {rate}: {bad.size} blocks differ, first {bad[:5]}"
    out = torch.empty_like(d)
    zfpx_lib.zfpx_decode_fixed_rate(words, rate, out)
    dec = array_to_blocks(out.cpu().numpy())
    assert np.array_equal(f32bits(dec), f32bits(oracle.decode_blocks(want, rate)))


@pytest.mark.parametrize("rate", [1, 8, 16, 32])
def test_decoder_on_random_words(zfpx_lib, rate):
    rng = np.random.default_rng(200 + rate)
    nb = 3000
    w = rng.integers(-2 ** 63, 2 ** 63 - 1, nb * rate, dtype=np.int64, endpoint=True)
    dw = torch.from_numpy(w).to(DEV)
    out = torch.empty((4, 4, 4 * nb), dtype=torch.float32, device=DEV)
    zfpx_lib.zfpx_decode_fixed_rate(dw, rate, out)
    got = array_to_blocks(out.cpu().numpy())
    want = oracle.decode_blocks(w.view(np.uint64), rate)
    assert np.array_equal(f32bits(got), f32bits(want))


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 9), (3, 130, 6), (17, 4, 65), (8, 1, 1031)])
def test_odd_shapes_and_strides(zfpx_lib, shape):
    rng = np.random.default_rng(sum(shape))
    nz, ny, nx = shape
    base = rng.standard_normal((nz + 1, ny + 2, 2 * nx + 3)).astype(np.float32)
    dbase = torch.from_numpy(base).to(DEV)
    views = {
        "contiguous": (dbase[:nz, :ny, :nx].contiguous(), None),
        "x-stride 2": (dbase[1:, 2:, 3::2], None),
        "permuted": (torch.from_numpy(np.ascontiguousarray(
            base[:nz, :ny, :nx].transpose(2, 1, 0))).to(DEV).permute(2, 1, 0), None),
    }
    for name, (view, _) in views.items():
        host = np.ascontiguousarray(view.cpu().numpy())
        for rate in (3, 8, 16, 32):
            words = zfpx_lib.zfpx_encode_fixed_rate(view, rate)
            want = oracle.encode_regular(host, rate)
            assert np.array_equal(u64(words), want), (name, rate)
            full = torch.full((nz, ny, 2 * nx), 7.0, device=DEV)
            out = full[:, :, ::2]
            zfpx_lib.zfpx_decode_fixed_rate(words, rate, out)
            back = oracle.decode_regular(want, host.shape, rate)
            assert np.array_equal(f32bits(out.cpu().numpy()), f32bits(back)), (name, rate)
            assert (full[:, :, 1::2] == 7.0).all(), "decode wrote outside the array"


def _check_plan(zfpx_lib, cs, src, rates, full=True, sample=0, seed=0):
    plan = zfpx_lib.Plan.from_chunkset(cs)
    dsrc = torch.from_numpy(src.reshape(-1)).to(DEV)
    for rate in rates:
        send = zfpx_lib.zfpx_pack_encode(plan, dsrc, rate)
        dst = torch.full_like(dsrc, float("nan"))
        zfpx_lib.zfpx_decode_unpack(plan, send, rate, dst)
        got = u64(send)
        if full:
            want = oracle.pack_encode(cs, src, rate)
            assert np.array_equal(got, want), rate
            back = np.full(src.size, np.nan, np.float32)
            oracle.decode_unpack(cs, want, rate, back)
            assert np.array_equal(f32bits(dst.cpu().numpy()), f32bits(back)), rate
        if sample:
            rng = np.random.default_rng(seed + rate)
            ids = np.unique(np.concatenate([rng.integers(0, plan.nblocks, sample),
                                            [0, plan.nblocks - 1]]))
            want = oracle.pack_encode_sample(cs, src, rate, ids)
            assert np.array_equal(got.reshape(-1, rate)[ids], want), rate
            vals, pos, inside = oracle.decode_sample(cs, got, rate, ids)
            assert int(inside.sum()) == int(real_values(cs, ids).sum()), rate
            dh = dst.cpu().numpy()
            assert np.array_equal(f32bits(dh[pos[inside]]), f32bits(vals[inside])), rate
    return plan


def test_zlambda_share_full_parity(zfpx_lib):
    cs = W.zlambda_chunkset()
    x32, _ = W.zlambda_fields()
    plan = _check_plan(zfpx_lib, cs, x32, (8, 16, 32))
    _, offs, total = plan.sizes(16)
    assert total == 902720 * 128 and offs[1] == 14105 * 128


def test_ragged_plans_small(zfpx_lib):
    rng = np.random.default_rng(5)
    cs = W.reduced_grid_chunkset(n_half=24, nlev=7, nchunks=5)
    src = (280 + 15 * rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    _check_plan(zfpx_lib, cs, src, (1, 7, 8, 16, 32))
    # odd row lengths, partial row groups, unaligned rows: the scalar path
    lens = np.array([5, 9, 3, 11, 7, 2, 6])
    offs = np.concatenate([[1], 1 + np.cumsum(lens)[:-1] + 3 * np.arange(1, 7)])
    cs2 = W.ChunkSet(np.array([0, 2]), np.array([200, 203]), np.array([6, 3]),
                     np.array([0, 5, 7]), np.concatenate([offs[:5], offs[5:] - 2]),
                     lens, 1300)
    src2 = rng.standard_normal(cs2.buffer_elems).astype(np.float32)
    _check_plan(zfpx_lib, cs2, src2, (2, 8, 16, 32))


def test_per_chunk_launches_equal_one_launch(zfpx_lib):
    cs = W.reduced_grid_chunkset(n_half=48, nlev=9, nchunks=12)
    rng = np.random.default_rng(6)
    host = rng.standard_normal(cs.buffer_elems).astype(np.float32)
    src = torch.from_numpy(host).to(DEV)
    plan = zfpx_lib.Plan.from_chunkset(cs)
    for rate in (8, 16):
        want = oracle.pack_encode(cs, host, rate)
        back = np.zeros(cs.buffer_elems, np.float32)
        oracle.decode_unpack(cs, want, rate, back)
        whole = zfpx_lib.zfpx_pack_encode(plan, src, rate)
        assert np.array_equal(u64(whole), want), rate
        parts = torch.zeros_like(whole)
        for c in range(cs.nchunks):
            zfpx_lib.zfpx_pack_encode_chunks(plan, c, 1, src, rate, parts)
        assert np.array_equal(u64(parts), want), rate
        d1 = torch.zeros_like(src)
        d2 = torch.zeros_like(src)
        zfpx_lib.zfpx_decode_unpack(plan, whole, rate, d1)
        for c in range(cs.nchunks):
            zfpx_lib.zfpx_decode_unpack_chunks(plan, c, 1, whole, rate, d2)
        assert np.array_equal(f32bits(d1.cpu().numpy()), f32bits(back)), rate
        assert np.array_equal(f32bits(d2.cpu().numpy()), f32bits(back)), rate


def test_every_launch_config_gives_identical_bytes(zfpx_lib):
    cs = W.reduced_grid_chunkset(n_half=64, nlev=11, nchunks=16)
    rng = np.random.default_rng(7)
    host = (280 + 15 * rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    src = torch.from_numpy(host).to(DEV)
    plan = zfpx_lib.Plan.from_chunkset(cs)
    for rate in (8, 32):
        # the reference is the oracle's stream and decode, moved to the device
        want = oracle.pack_encode(cs, host, rate)
        back = np.zeros(cs.buffer_elems, np.float32)
        oracle.decode_unpack(cs, want, rate, back)
        ref = torch.from_numpy(want.view(np.int64)).to(DEV)
        dref = torch.from_numpy(back).to(DEV)
        for wg in (64, 128, 256):
            for grid in (0, 1, 3, 64):
                for op in (0, 1):
                    try:
                        zfpx_lib.zfpx_plan_set_config(plan, op, rate, wg, grid)
                    except zfpx_lib.ZfpxError:
                        continue  # does not fit in LDS at this rate
                w = zfpx_lib.zfpx_pack_encode(plan, src, rate)
                d = torch.zeros_like(src)
                zfpx_lib.zfpx_decode_unpack(plan, w, rate, d)
                assert torch.equal(w, ref), (wg, grid)
                assert torch.equal(d.view(torch.int32), dref.view(torch.int32)), (wg, grid)
        # and the configuration the autotuner picks
        for op in (0, 1):
            zfpx_lib.zfpx_autotune(plan, op, rate, src, torch.empty_like(ref), torch.empty_like(src))
        w = zfpx_lib.zfpx_pack_encode(plan, src, rate)
        d = torch.zeros_like(src)
        zfpx_lib.zfpx_decode_unpack(plan, w, rate, d)
        assert torch.equal(w, ref), "autotuned"
        assert torch.equal(d.view(torch.int32), dref.view(torch.int32)), "autotuned"


def test_graph_replays_match_eager(zfpx_lib):
    cs = W.reduced_grid_chunkset(n_half=80, nlev=13, nchunks=20)
    rng = np.random.default_rng(8)
    host = (280 + 15 * rng.standard_normal(cs.buffer_elems)).astype(np.float32)
    src = torch.from_numpy(host).to(DEV)
    plan = zfpx_lib.Plan.from_chunkset(cs)
    rate = 16
    want = oracle.pack_encode(cs, host, rate)
    back = np.zeros(cs.buffer_elems, np.float32)
    oracle.decode_unpack(cs, want, rate, back)
    send_e = torch.from_numpy(want.view(np.int64)).to(DEV)
    dst_e = torch.from_numpy(back).to(DEV)
    send = torch.zeros_like(send_e)
    dst = torch.zeros_like(src)
    g = zfpx_lib.Graph(plan, rate, src, send, dst)
    for rep in range(4):
        send.zero_()
        dst.fill_(-1.0)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(send, send_e), rep
        assert torch.equal(dst, dst_e), rep
    g.close()


def test_f16_matches_numpy(zfpx_lib):
    rng = np.random.default_rng(9)
    specials = np.array([0.0, -0.0, 1.0, -2.0, 65504.0, 65519.996, 65520.0, 1e6, -1e6,
                         2.0 ** -24, 2.0 ** -25, 1.5 * 2.0 ** -24, 2.0 ** -14, 2.0 ** -149,
                         1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, np.inf, -np.inf], np.float32)
    bits = rng.integers(0, 2 ** 32, 300000, dtype=np.uint64).astype(np.uint32).view(np.float32)
    x = np.concatenate([specials, bits, (280 + 15 * rng.standard_normal(100003)).astype(np.float32)])
    dall = torch.from_numpy(x).to(DEV)
    for off in (0, 1, 3):  # aligned and unaligned device starts, ragged tails
        xs = x[off:]
        d = dall[off:]  # a view: off > 0 is not 16-byte aligned (element-wise path)
        h = zfpx_lib.f16_truncate(d)
        want = oracle.f16_truncate(xs)
        got = h.cpu().numpy().view(np.uint16)
        nan = np.isnan(xs)
        assert np.array_equal(got[~nan], want[~nan])
        assert np.isnan(got[nan].view(np.float16)).all()
        back = zfpx_lib.f16_restore(h)
        hv = torch.empty(h.numel() + 1, dtype=h.dtype, device=DEV)
        hv[1:] = h  # an unaligned float16 input as well
        back2 = zfpx_lib.f16_restore(hv[1:])
        assert torch.equal(back2.view(torch.int32), back.view(torch.int32))  # NaNs too
        wantb = oracle.f16_restore(want)
        gb = back.cpu().numpy()
        assert np.array_equal(f32bits(gb[~nan]), f32bits(wantb[~nan]))
        assert np.isnan(gb[nan]).all()


def test_empty_inputs(zfpx_lib):
    e = torch.empty((0, 4, 4), dtype=torch.float32, device=DEV)
    w = zfpx_lib.zfpx_encode_fixed_rate(e, 8)
    assert w.numel() == 0
    zfpx_lib.zfpx_decode_fixed_rate(w, 8, e)
    h = zfpx_lib.f16_truncate(torch.empty(0, device=DEV))
    assert h.numel() == 0
    plan = zfpx_lib.Plan([0, 0], [16, 16], [0, 3], [0, 1, 1], [0], [4])
    assert plan.nblocks == 0
    src = torch.zeros(64, device=DEV)
    send = zfpx_lib.zfpx_pack_encode(plan, src, 8)
    assert send.numel() == 0


def _full_parity(zfpx_lib, cs, host, dsrc, plan, rate):
    """Whole-buffer stream and decode of the default launch against the
    oracle; returns the device stream and decode for further comparisons."""
    send = zfpx_lib.zfpx_pack_encode(plan, dsrc, rate)
    dst = torch.full_like(dsrc, float("nan"))
    zfpx_lib.zfpx_decode_unpack(plan, send, rate, dst)
    torch.cuda.synchronize()
    want = oracle.pack_encode(cs, host, rate)
    got = u64(send)
    bad = np.nonzero((got != want).reshape(-1, rate).any(1))[0]
    assert bad.size == 0, f"rate {rate}: {bad.size} blocks differ, first {bad[:5]}"
    del got
    back = np.full(host.size, np.nan, np.float32)
    oracle.decode_unpack(cs, want, rate, back)
    del want
    dh = dst.cpu().numpy()
    diff = np.nonzero(f32bits(dh) != f32bits(back))[0]
    assert diff.size == 0, f"rate {rate}: {diff.size} values differ, first {diff[:5]}"
    return send, dst


@pytest.fixture(scope="module")
def large_buffer(zfpx_lib):
    """O2560 x 90 levels (9.47 GB, one chunk, 37,859,840 blocks); levels
    8..89 repeat the generated levels 0..7."""
    cs = W.large_chunkset()
    host = W.large_field_repeated(W.large_field_levels(8)).reshape(-1)
    assert host.size == cs.buffer_elems == 2367590400
    plan = zfpx_lib.Plan.from_chunkset(cs)
    assert plan.nblocks == 37859840
    dsrc = torch.from_numpy(host).to(DEV)
    yield cs, host, dsrc, plan
    del dsrc
    torch.cuda.empty_cache()


@pytest.mark.parametrize("rate", [8, 16])
def test_large_full_buffer_parity(zfpx_lib, large_buffer, rate):
    """Every block of the O2560 x 90 buffer, streams and decoded floats, in
    the launch configuration the benchmark times."""
    cs, host, dsrc, plan = large_buffer
    _, _, total = plan.sizes(rate)
    assert total == 37859840 * 8 * rate
    send, dst = _full_parity(zfpx_lib, cs, host, dsrc, plan, rate)
    del send, dst
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def ltheta_buffer(zfpx_lib):
    cs = W.ltheta_chunkset()
    host = W.ltheta_field().reshape(-1)
    plan = zfpx_lib.Plan.from_chunkset(cs)
    dsrc = torch.from_numpy(host).to(DEV)
    yield cs, host, dsrc, plan
    del dsrc
    torch.cuda.empty_cache()


@pytest.mark.parametrize("rate", [8, 16, 32])
def test_ltheta_full_buffer_parity(zfpx_lib, ltheta_buffer, rate):
    """The O1280 x 137 lambda->theta buffer (256 uneven chunks, 3.617 GB),
    every block against the oracle; at rate 16 also the forms the benchmark
    compares: autotuned launches captured in a graph, and one launch per
    chunk."""
    cs, host, dsrc, plan = ltheta_buffer
    b, o, total = plan.sizes(rate)
    assert b.size == 256 and total == 14470400 * 8 * rate
    send, dst = _full_parity(zfpx_lib, cs, host, dsrc, plan, rate)
    if rate == 16:
        s2 = torch.empty_like(send)
        d2 = torch.empty_like(dst)
        for op in (0, 1):
            zfpx_lib.zfpx_autotune(plan, op, rate, dsrc, s2, d2)
        s2.zero_()
        d2.fill_(-1.0)
        g = zfpx_lib.Graph(plan, rate, dsrc, s2, d2)
        for rep in range(2):
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(s2, send), ("graph", rep)
            assert torch.equal(d2.view(torch.int32), dst.view(torch.int32)), ("graph", rep)
            s2.zero_()
            d2.fill_(-1.0)
        g.close()
        for c in range(cs.nchunks):
            zfpx_lib.zfpx_pack_encode_chunks(plan, c, 1, dsrc, rate, s2)
        for c in range(cs.nchunks):
            zfpx_lib.zfpx_decode_unpack_chunks(plan, c, 1, s2, rate, d2)
        torch.cuda.synchronize()
        assert torch.equal(s2, send), "per-chunk launches"
        assert torch.equal(d2.view(torch.int32), dst.view(torch.int32)), "per-chunk launches"
        # sampled blocks through the sampling helpers, with their in-range counts
        rng = np.random.default_rng(11)
        ids = np.unique(np.concatenate([rng.integers(0, plan.nblocks, 2000),
                                        [0, plan.nblocks - 1]]))
        vals, pos, inside = oracle.decode_sample(cs, u64(send), rate, ids)
        assert int(inside.sum()) == int(real_values(cs, ids).sum())
        del s2, d2
    del send, dst
    torch.cuda.empty_cache()
