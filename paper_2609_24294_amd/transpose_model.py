"""Transposition-time model for the row all-to-all of the SHT.

The paper (Section IV-D, network simulation and time model) adds the measured
compression time before and the measured decompression time after the
simulated all-to-all: t = t_compress + t_comm + t_decompress, a serial model
it calls a conservative upper bound.  Its network is a simulated Dragonfly
(200 Gb/s links, 1 us per hop, N = 4 ... 121 nodes; Table 1 gives the
per-rank-pair message sizes of the row transposition).

Here the all-to-all is an alpha-beta exchange instead of a packet-level
simulation: each of the sqrt(N) ranks of a row communicator sends its
sqrt(N) - 1 remote messages one after another over its injection link,
t_comm = (sqrt(N) - 1) * (alpha + m / beta), with alpha = path hops x 1 us and
beta = the link bandwidth.  Codec times come from rates measured on this GPU
(GB/s of float32 input), applied to the node's whole outgoing buffer of
sqrt(N) messages.  As in the paper, the float16 cast is taken as free by
default (it is a register operation fused into the copy); the measured
truncate/restore rates can be charged instead.  A pipelined variant (the overlap the paper leaves to
future work) is reported beside the serial one: with the buffer cut into
chunks, time = the slowest of the three stages plus one chunk of each of the
other two.

Host-only; no GPU code runs here.
"""
from __future__ import annotations

import dataclasses
import math

# The paper's grid for Table 1 (DYAMOND, 2560 x 1280 points, 137 levels; the
# table's sizes are reproduced with 1280 latitudes) and its network.
GRID = (2560, 1280, 137)
NODES = (4, 9, 16, 25, 36, 49, 64, 81, 100, 121)
STRATEGIES = ("float32", "float16", "zfp_rate16", "zfp_rate8")


@dataclasses.dataclass
class Network:
    link_gbps: float = 200.0   # link bandwidth, Gbit/s
    hop_us: float = 1.0        # latency per hop
    hops: int = 5              # router hops of an inter-group path of the Dragonfly

    @property
    def beta(self) -> float:   # bytes per second
        return self.link_gbps * 1e9 / 8.0

    @property
    def alpha(self) -> float:  # seconds per message
        return self.hops * self.hop_us * 1e-6


@dataclasses.dataclass
class CodecRates:
    """Measured rates in GB/s of float32 input (1e9 bytes/s)."""
    encode16: float
    decode16: float
    encode8: float
    decode8: float
    f16_truncate: float
    f16_restore: float


def message_dims(nodes: int, grid=GRID):
    """Per-rank-pair sub-array of the row transposition: each axis of the
    grid split sqrt(N) ways, rounded down (Table 1)."""
    p = math.isqrt(nodes)
    if p * p != nodes:
        raise ValueError("N must be a square")
    return tuple(n // p for n in grid)


def message_bytes(nodes: int, strategy: str, grid=GRID) -> int:
    """Bytes of one rank-pair message for a strategy.  Fixed-rate ZFP
    messages hold whole 4x4x4 blocks: ceil(a/4) ceil(b/4) ceil(c/4) blocks
    of 8 * rate bytes."""
    a, b, c = message_dims(nodes, grid)
    if strategy == "float32":
        return 4 * a * b * c
    if strategy == "float16":
        return 2 * a * b * c
    if strategy.startswith("zfp_rate"):
        rate = int(strategy[len("zfp_rate"):])
        blocks = -(-a // 4) * -(-b // 4) * -(-c // 4)
        return blocks * 8 * rate
    raise ValueError(strategy)


def comm_time(nodes: int, msg: int, net: Network) -> float:
    p = math.isqrt(nodes)
    return (p - 1) * (net.alpha + msg / net.beta)


def codec_times(nodes: int, strategy: str, rates: CodecRates | None, grid=GRID,
                f16_cast_free: bool = False):
    """(compress, decompress) seconds for the node's outgoing buffer of
    sqrt(N) messages; zero for float32, when no rates are given, and for
    float16 when its cast is taken as free."""
    if strategy == "float32" or rates is None or (strategy == "float16" and f16_cast_free):
        return 0.0, 0.0
    p = math.isqrt(nodes)
    f32 = p * message_bytes(nodes, "float32", grid)
    enc, dec = {"float16": (rates.f16_truncate, rates.f16_restore),
                "zfp_rate16": (rates.encode16, rates.decode16),
                "zfp_rate8": (rates.encode8, rates.decode8)}[strategy]
    return f32 / (enc * 1e9), f32 / (dec * 1e9)


def breakdown(nodes: int, strategy: str, rates: CodecRates | None, net: Network | None = None,
              chunks: int = 16, grid=GRID, f16_cast_free: bool = True) -> dict:
    """Serial and pipelined time of one row transposition."""
    net = net or Network()
    msg = message_bytes(nodes, strategy, grid)
    tc, td = codec_times(nodes, strategy, rates, grid, f16_cast_free)
    tm = comm_time(nodes, msg, net)
    stages = (tc, tm, td)
    pipelined = max(stages) + (sum(stages) - max(stages)) / chunks
    return {"message_bytes": msg, "compress_s": tc, "comm_s": tm, "decompress_s": td,
            "serial_s": tc + tm + td, "pipelined_s": pipelined}


def table(rates: CodecRates | None, net: Network | None = None, nodes=NODES, grid=GRID,
          f16_cast_free: bool = True) -> list:
    """One row per node count: each strategy's breakdown and its speedup
    over float32 (serial and pipelined)."""
    out = []
    for n in nodes:
        row = {"nodes": n}
        base = breakdown(n, "float32", rates, net, grid=grid)
        for s in STRATEGIES:
            b = breakdown(n, s, rates, net, grid=grid, f16_cast_free=f16_cast_free)
            b["speedup_serial"] = base["serial_s"] / b["serial_s"]
            b["speedup_pipelined"] = base["pipelined_s"] / b["pipelined_s"]
            row[s] = b
        out.append(row)
    return out


def summary(rates: CodecRates, net: Network | None = None, nodes=NODES) -> dict:
    """Compact report: per node count the serial and pipelined speedup of
    each strategy over float32 and the codec's share of the serial time;
    float16 is given once with a free cast and once at its measured rates."""
    free = table(rates, net, nodes)
    charged = table(rates, net, nodes, f16_cast_free=False)
    rows = []
    for a, b in zip(free, charged):
        r = {"N": a["nodes"], "float32_ms": round(1e3 * a["float32"]["serial_s"], 4)}
        for s in STRATEGIES[1:]:
            x = a[s]
            r[s] = [round(x["speedup_serial"], 3), round(x["speedup_pipelined"], 3),
                    round((x["compress_s"] + x["decompress_s"]) / x["serial_s"], 4)]
        r["float16_measured_cast"] = [round(b["float16"]["speedup_serial"], 3),
                                      round(b["float16"]["speedup_pipelined"], 3)]
        rows.append(r)
    return {"columns": "[speedup serial, speedup pipelined, codec share of serial time]",
            "rows": rows}
