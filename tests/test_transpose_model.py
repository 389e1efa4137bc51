"""Transposition-time model (host only): Table 1 message sizes, the
alpha-beta exchange, codec times and the serial / pipelined totals."""
import math
import os

import pytest

from paper_2609_24294_amd import transpose_model as TM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_message_sizes_match_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_message_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    MiB = 2.0 ** 20
    for r in rows:
        n = int(r[0])
        for strategy, want in zip(TM.STRATEGIES, map(float, r[1:])):
            got = TM.message_bytes(n, strategy) / MiB
            assert abs(got - want) <= 0.005 + 1e-9, (n, strategy, got, want)


def test_message_dims_need_square_node_counts():
    assert TM.message_dims(9) == (853, 426, 45)
    with pytest.raises(ValueError):
        TM.message_dims(10)


def test_comm_time_is_alpha_beta_by_hand():
    net = TM.Network(link_gbps=200.0, hop_us=1.0, hops=5)
    m = TM.message_bytes(9, "float32")
    # 3 ranks per row communicator: 2 remote messages, each 5 us + m / 25 GB/s
    assert TM.comm_time(9, m, net) == pytest.approx(2 * (5e-6 + m / 25e9), rel=1e-12)


def test_without_codec_cost_speedups_are_size_ratios():
    rows = TM.table(None, nodes=(4,))
    r = rows[0]
    net = TM.Network()
    m32 = TM.message_bytes(4, "float32")
    for s in TM.STRATEGIES:
        ms = TM.message_bytes(4, s)
        exact = (net.alpha + m32 / net.beta) / (net.alpha + ms / net.beta)
        assert r[s]["speedup_serial"] == pytest.approx(exact, rel=1e-12)
        # one remote message of 53-222 MB: the 5 us latency moves the ratio
        # of the byte counts by less than 0.3%
        assert r[s]["speedup_serial"] == pytest.approx(m32 / ms, rel=3e-3)


def test_codec_times_use_the_whole_outgoing_buffer():
    rates = TM.CodecRates(encode16=2000, decode16=1000, encode8=2000, decode8=1000,
                          f16_truncate=4000, f16_restore=4000)
    tc, td = TM.codec_times(16, "zfp_rate16", rates)
    buf = 4 * TM.message_bytes(16, "float32")  # sqrt(16) messages of float32
    assert tc == pytest.approx(buf / 2000e9) and td == pytest.approx(buf / 1000e9)
    assert TM.codec_times(16, "float32", rates) == (0.0, 0.0)
    assert TM.codec_times(16, "float16", rates, f16_cast_free=True) == (0.0, 0.0)
    tc, td = TM.codec_times(16, "float16", rates)
    assert tc == pytest.approx(buf / 4000e9) and td == pytest.approx(buf / 4000e9)


def test_summary_at_121_nodes_with_free_codecs():
    # with free codecs the N = 121 speedups are the alpha-beta ratios: 1.29 MB
    # float32 messages take 52 us at 25 GB/s, so the 5 us latency keeps them
    # below the size ratios of Table 1 (2, 2 and 4)
    rates = TM.CodecRates(1e9, 1e9, 1e9, 1e9, 1e9, 1e9)
    row = TM.summary(rates)["rows"][-1]
    assert row["N"] == 121
    net = TM.Network()
    m32 = TM.message_bytes(121, "float32")
    for s in ("float16", "zfp_rate16", "zfp_rate8"):
        ms = TM.message_bytes(121, s)
        want = (net.alpha + m32 / net.beta) / (net.alpha + ms / net.beta)
        assert row[s][0] == pytest.approx(want, abs=1e-3)
        assert row[s][0] < m32 / ms
    assert row["zfp_rate8"][0] > row["zfp_rate16"][0] == row["float16"][0] > 1.8


def test_serial_and_pipelined_bounds():
    rates = TM.CodecRates(1500, 1200, 1800, 1500, 3000, 3500)
    for free in (True, False):
        for row in TM.table(rates, f16_cast_free=free):
            for s in TM.STRATEGIES:
                b = row[s]
                stages = (b["compress_s"], b["comm_s"], b["decompress_s"])
                assert b["serial_s"] == pytest.approx(sum(stages))
                assert max(stages) <= b["pipelined_s"] <= b["serial_s"]


def test_codec_overhead_shrinks_with_more_remote_messages():
    # codec time and traffic both scale with the node's share; the share of
    # it that leaves the node, (p - 1) / p, grows with N, so the codec's
    # relative cost falls (the paper's trend, here without contention)
    rates = TM.CodecRates(1500, 1200, 1800, 1500, 3000, 3500)
    frac = []
    for row in TM.table(rates):
        b = row["zfp_rate16"]
        frac.append((b["compress_s"] + b["decompress_s"]) / b["serial_s"])
    assert frac[0] > frac[-1]
    assert all(math.isfinite(f) and 0 < f < 1 for f in frac)
