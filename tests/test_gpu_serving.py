"""Serving loop: every result in the mix equals the request run alone and
the CPU oracle's result for the same view (tolerance 0), admission respects
the HBM budget, errors are reported."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2609_24294_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _oracle_ref(op, rate, view, words=None):
    """The oracle's output for a request: the stream of the host copy of the
    float32 view (op 0), or the decode of the request's input stream (op 1)."""
    if op == 0:
        host = view.contiguous().cpu().numpy()
        return torch.from_numpy(oracle.encode_regular(host, rate).view(np.int64)).to(DEV)
    w = words.cpu().numpy().view(np.uint64)
    return torch.from_numpy(oracle.decode_regular(w, tuple(view.shape), rate)).to(DEV)


def _same(a, b):
    return torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else a,
                       b.view(torch.int32) if b.dtype == torch.float32 else b)


def _requests(zfpx, pool, rng, count):
    """Mixed encode/decode requests on views of `pool`, each with its own
    output buffer, plus the expected outputs: the oracle's, which the same
    request run alone in one launch reproduces."""
    reqs, outs, refs = [], [], []
    for i in range(count):
        op = int(rng.integers(0, 2))
        rate = int(rng.choice([1, 7, 8, 16, 32]))
        nx = int(rng.choice([4, 12, 64, 300, 1028, 4096]))
        view = pool[:, :, :nx]
        if i % 7 == 3:  # a strided view takes the generic path
            view = pool[:, ::2, : 2 * nx : 2]
        nbytes = zfpx.zfpx_fixed_rate_bytes(view.shape[2], view.shape[1], view.shape[0], rate)
        if op == 0:
            words = torch.zeros(nbytes // 8, dtype=torch.int64, device=DEV)
            ref = _oracle_ref(0, rate, view)
            assert _same(zfpx.zfpx_encode_fixed_rate(view, rate), ref), (i, "alone")
            reqs.append(zfpx.make_request(0, rate, view, words, tag=i))
            outs.append(words)
        else:
            src_words = zfpx.zfpx_encode_fixed_rate(view, rate)
            arr = torch.full(view.shape, -7.0, device=DEV)
            ref = _oracle_ref(1, rate, view, src_words)
            alone = torch.full(view.shape, -7.0, device=DEV)
            zfpx.zfpx_decode_fixed_rate(src_words, rate, alone)
            assert _same(alone, ref), (i, "alone")
            reqs.append(zfpx.make_request(1, rate, arr, src_words, tag=i))
            outs.append((arr, src_words))
        refs.append(ref)
    torch.cuda.synchronize()
    return reqs, outs, refs


def _check(outs, refs):
    for i, (o, r) in enumerate(zip(outs, refs)):
        got = o if isinstance(o, torch.Tensor) else o[0]
        assert _same(got, r), f"request {i} differs from the oracle and its one-launch result"


def test_server_mix_equals_alone(zfpx_lib):
    rng = np.random.default_rng(40)
    pool = torch.from_numpy(W.serving_pool(nx_max=8192)).to(DEV)
    reqs, outs, refs = _requests(zfpx_lib, pool, rng, 60)
    sv = zfpx_lib.Server(64 << 30, max_slots=16)
    tickets = []
    for i, rq in enumerate(reqs):
        tickets.append(sv.submit(rq))
        if i % 10 == 9:
            time.sleep(0.002)  # some requests arrive while others run
    sv.drain(60.0)
    for t in tickets:
        done, lat = sv.poll(t)
        assert done and lat > 0
    st = sv.stats()
    sv.close()
    torch.cuda.synchronize()
    assert st["admitted"] == len(reqs)
    _check(outs, refs)


def test_server_few_workgroups(zfpx_lib):
    """The smallest loops: 1 (raised to 2: workgroup 0 only dispatches, so one
    worker) and 3 workgroups code every tile of a mix, each equal to the
    oracle's."""
    rng = np.random.default_rng(43)
    pool = torch.from_numpy(W.serving_pool(nx_max=8192)).to(DEV)
    for wg in (1, 3):
        reqs, outs, refs = _requests(zfpx_lib, pool, rng, 20)
        sv = zfpx_lib.Server(64 << 30, max_slots=8, workgroups=wg)
        for rq in reqs:
            sv.submit(rq)
        sv.drain(60.0)
        st = sv.stats()
        sv.close()
        torch.cuda.synchronize()
        assert st["admitted"] == len(reqs)
        _check(outs, refs)


def test_server_budget_admission(zfpx_lib):
    rng = np.random.default_rng(41)
    pool = torch.from_numpy(W.serving_pool(nx_max=8192)).to(DEV)
    reqs, outs, refs = _requests(zfpx_lib, pool, rng, 30)
    sizes = []
    for rq in reqs:
        nb = -(-rq.nx // 4) * -(-rq.ny // 4) * -(-rq.nz // 4)
        sizes.append(rq.nx * rq.ny * rq.nz * 4 + nb * 8 * rq.rate)
    budget = 2 * max(sizes)
    sv = zfpx_lib.Server(budget, max_slots=64)
    for rq in reqs:
        sv.submit(rq)
    sv.drain(60.0)
    st = sv.stats()
    sv.close()
    torch.cuda.synchronize()
    assert st["max_inflight_bytes"] <= budget
    _check(outs, refs)


def test_server_rejects_bad_requests(zfpx_lib):
    pool = torch.from_numpy(W.serving_pool(nx_max=1024)).to(DEV)
    words = torch.zeros(1 << 16, dtype=torch.int64, device=DEV)
    sv = zfpx_lib.Server(1 << 20, max_slots=4)
    big = zfpx_lib.make_request(0, 8, pool, words)  # more bytes than the whole budget
    with pytest.raises(zfpx_lib.ZfpxError) as e:
        sv.submit(big)
    assert e.value.status == zfpx_lib.EINVAL
    bad = zfpx_lib.make_request(0, 0, pool[:, :4, :4], words)
    with pytest.raises(zfpx_lib.ZfpxError):
        sv.submit(bad)
    sv.close()


def test_server_queue_full_is_eagain(zfpx_lib):
    """The budget holds one 64 MB request, so the others wait in the host
    queue; with a queue of two, a submit while the queue is full gets EAGAIN
    and the request is not taken (it can be submitted again later); every
    request taken completes with the oracle's result."""
    pool = torch.from_numpy(W.serving_pool(nx_max=32768)).to(DEV)
    rate = 16
    ref = _oracle_ref(0, rate, pool)
    nbytes = pool.numel() * 4 + ref.numel() * 8
    bufs = [torch.empty_like(ref) for _ in range(8)]
    torch.cuda.synchronize()
    sv = zfpx_lib.Server(nbytes, max_slots=4)
    sv.set_max_queue(2)
    outs, tickets, rejected = [], [], None
    for i, out in enumerate(bufs):  # a submit takes microseconds, a 64 MB request far longer
        rq = zfpx_lib.make_request(0, rate, pool, out, tag=i)
        try:
            tickets.append(sv.submit(rq))
        except zfpx_lib.ZfpxError as e:
            assert e.status == zfpx_lib.EAGAIN
            rejected = (rq, out)
            break
        outs.append(out)
    # one in flight and two queued at most when the rejection came
    assert rejected is not None and len(outs) <= 3
    sv.drain(60.0)
    tickets.append(sv.submit(rejected[0]))  # taken now that the queue has room
    outs.append(rejected[1])
    sv.drain(60.0)
    for tk in tickets:
        done, _ = sv.poll(tk)
        assert done
    for pol in (-1, 0, (1 << 20) + 1):
        with pytest.raises(zfpx_lib.ZfpxError):
            sv.set_max_queue(pol)
    sv.close()
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref)


def test_server_idle_setting(zfpx_lib):
    """Requests 5 ms apart: with the default 2 ms idle spell the loop leaves
    and is launched again for each; with a 50 ms spell one launch serves all.
    Out-of-range settings are rejected; outputs equal the oracle's."""
    pool = torch.from_numpy(W.serving_pool(nx_max=512)).to(DEV)
    view = pool[:, :, :256]
    ref = _oracle_ref(0, 16, view)
    arrival = np.arange(6) * 5e-3
    launches = {}
    for idle in (None, 50000):
        outs = [torch.empty_like(ref) for _ in arrival]
        torch.cuda.synchronize()
        reqs = [zfpx_lib.make_request(0, 16, view, o) for o in outs]
        sv = zfpx_lib.Server(64 << 30, max_slots=8)
        try:
            if idle is not None:
                sv.set_idle_us(idle)
            lat = sv.replay(reqs, arrival, timeout_s=30.0)
            launches[idle] = sv.stats()["loop_launches"]
            for bad in (0, 99, 10000001):
                with pytest.raises(RuntimeError):
                    sv.set_idle_us(bad)
        finally:
            sv.close()
        torch.cuda.synchronize()
        assert (lat > 0).all()
        for o in outs:
            assert _same(o, ref)
    # (two requests may share a launch if the host thread falls behind the
    # schedule by milliseconds)
    assert launches[None] >= len(arrival) - 2
    assert launches[50000] == 1


def test_server_relaunch_races(zfpx_lib):
    """A 200 us idle spell and arrivals 100-400 us apart: the loop leaves and is
    launched again many times, requests often arriving while it is leaving.
    Every request completes with the oracle's output."""
    rng = np.random.default_rng(44)
    pool = torch.from_numpy(W.serving_pool(nx_max=512)).to(DEV)
    views = [pool[:, :, :nx] for nx in (64, 128, 256)]
    refs = [_oracle_ref(0, 16, v) for v in views]
    n = 150
    which = rng.integers(0, len(views), n)
    outs = [torch.empty_like(refs[k]) for k in which]
    torch.cuda.synchronize()
    reqs = [zfpx_lib.make_request(0, 16, views[k], o) for k, o in zip(which, outs)]
    arrival = np.cumsum(rng.uniform(100e-6, 400e-6, n))
    sv = zfpx_lib.Server(64 << 30, max_slots=16)
    try:
        sv.set_idle_us(200)
        lat = sv.replay(reqs, arrival, timeout_s=60.0)
        launches = sv.stats()["loop_launches"]
    finally:
        sv.close()
    torch.cuda.synchronize()
    assert (lat > 0).all()
    assert launches > 1
    for k, o in zip(which, outs):
        assert _same(o, refs[k])


def test_replay_forms_agree(zfpx_lib):
    rng = np.random.default_rng(42)
    pool = torch.from_numpy(W.serving_pool(nx_max=4096)).to(DEV)
    reqs, outs, refs = _requests(zfpx_lib, pool, rng, 40)
    arrival = np.cumsum(rng.exponential(50e-6, len(reqs)))
    arrival -= arrival[0]
    sv = zfpx_lib.Server(64 << 30, max_slots=32)
    lat = sv.replay(reqs, arrival, timeout_s=60.0)
    sv.close()
    torch.cuda.synchronize()
    assert (lat > 0).all()
    _check(outs, refs)
    for o in outs:  # scribble, then the plain form must rebuild the same outputs
        (o if isinstance(o, torch.Tensor) else o[0]).fill_(0)
    lat2 = zfpx_lib.zfpx_plain_replay(reqs, arrival, timeout_s=60.0)
    torch.cuda.synchronize()
    assert (lat2 > 0).all()
    _check(outs, refs)


def test_server_large_requests_in_runs(zfpx_lib):
    """Requests of 1024+ tiles are handed out in runs of several tiles per
    claim (the last run of a request cut short); mixed with small requests,
    every result still equals its one-launch form."""
    rng = np.random.default_rng(43)
    pool = torch.from_numpy(W.serving_pool(nx_max=32768)).to(DEV)
    reqs, outs, refs = [], [], []
    for i, nx in enumerate([32764, 12, 16384, 300, 32768, 4, 20001, 64]):
        view = pool[:, :, :nx]
        rate = int(rng.choice([8, 16, 32]))
        words = _oracle_ref(0, rate, view)
        assert _same(zfpx_lib.zfpx_encode_fixed_rate(view, rate), words), (i, "alone")
        if i % 2 == 0:
            out = torch.zeros_like(words)
            reqs.append(zfpx_lib.make_request(0, rate, view, out, tag=i))
            outs.append(out)
            refs.append(words)
        else:
            arr = torch.full(view.shape, -7.0, device=DEV)
            ref = _oracle_ref(1, rate, view, words)
            reqs.append(zfpx_lib.make_request(1, rate, arr, words, tag=i))
            outs.append((arr, words))  # requests hold raw pointers: keep inputs alive
            refs.append(ref)
        # decoding the large ones too (runs on the decode path)
        if nx >= 16384:
            arr = torch.full(view.shape, -7.0, device=DEV)
            ref = _oracle_ref(1, rate, view, words)
            reqs.append(zfpx_lib.make_request(1, rate, arr, words, tag=100 + i))
            outs.append((arr, words))
            refs.append(ref)
    torch.cuda.synchronize()
    tiles = [-(-(-(-rq.nx // 4) * -(-rq.ny // 4) * -(-rq.nz // 4)) // 64) for rq in reqs]
    assert max(tiles) >= 4096 and any(t >= 1024 and t % 8 for t in tiles)
    sv = zfpx_lib.Server(64 << 30, max_slots=8)
    for rq in reqs:
        sv.submit(rq)
    sv.drain(60.0)
    sv.close()
    torch.cuda.synchronize()
    _check(outs, refs)


def test_server_array_beyond_4gib(zfpx_lib):
    """A request whose float32 array spans more than 4 GiB takes the
    element-wise coherent path; its results equal the one-launch form."""
    nx, ny, sz = 64, 8, (1 << 30) + 64  # two levels 4 GiB + 256 B apart
    base = torch.empty(sz + ny * nx, dtype=torch.float32, device=DEV)
    rng = np.random.default_rng(44)
    lev = torch.from_numpy((280 + 15 * rng.standard_normal((2, ny, nx))).astype(np.float32)).to(DEV)
    base[:ny * nx] = lev[0].reshape(-1)
    base[sz: sz + ny * nx] = lev[1].reshape(-1)
    view = torch.as_strided(base, (2, ny, nx), (sz, nx, 1))
    rate = 16
    words = _oracle_ref(0, rate, view)
    assert _same(zfpx_lib.zfpx_encode_fixed_rate(view, rate), words)
    ref = _oracle_ref(1, rate, view, words)
    out_words = torch.zeros_like(words)
    out_view = torch.as_strided(base, (2, ny, nx), (sz, nx, 1))
    sv = zfpx_lib.Server(64 << 30, max_slots=4)
    sv.submit(zfpx_lib.make_request(0, rate, view, out_words))
    sv.drain(60.0)
    base.fill_(-7.0)  # the decode writes back into the same strided layout
    torch.cuda.synchronize()  # the server's loop runs on its own stream
    sv.submit(zfpx_lib.make_request(1, rate, out_view, words))
    sv.drain(60.0)
    sv.close()
    torch.cuda.synchronize()
    assert torch.equal(out_words, words)
    got = torch.stack([base[:ny * nx].reshape(ny, nx), base[sz: sz + ny * nx].reshape(ny, nx)])
    assert _same(got, ref)
