"""Benchmark: fixed-rate ZFP pack+encode / decode+unpack of one GPU's
z->lambda transpose buffer on one MI355X.

Workload (default): one GPU's share of a 64-rank z->lambda transposition at
O1280-like resolution -- 4 float32 fields (u, v, T, q) x 137 levels x 64
latitude rows x 1612 points = 56,536,064 values (226.1 MB), cut into 64
per-destination chunks, synthetic T42 spectral fields (seeded).

A step is one pass of the method over that buffer at rate 16: fused
pack+encode into the send buffer, then fused decode+unpack into the receive
layout.  `value` = float32 input bytes / step time (encode + decode), with the
inputs resident in HBM.  Several input/output buffer sets are rotated so that
the 256 MB last-level cache cannot hold a step's working set.  Rate 8 and the
float16 comparator are timed the same way and reported beside it.

One JSON line on stdout.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg: str) -> None:
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rate", type=int, default=16)
    ap.add_argument("--sets", type=int, default=3, help="rotated buffer sets")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip rate-8 and f16 legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter calibration)")
    return ap.parse_args()


def timed_loop(fn_list, steps, warmup, torch):
    """Run warmup + steps iterations of a list of launch callables on the
    current stream; per callable, the mean event-timed duration (ms)."""
    s = torch.cuda.current_stream()
    for i in range(warmup):
        for f in fn_list:
            f(i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(fn_list) + 1)]
           for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        e = evs[i]
        e[0].record(s)
        for j, f in enumerate(fn_list):
            f(i)
            e[j + 1].record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [sum(evs[i][j].elapsed_time(evs[i][j + 1]) for i in range(steps)) / steps
           for j in range(len(fn_list))]
    return wall, per


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2609_24294_amd import workloads as W
    from paper_2609_24294_amd import zfpx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rate = args.rate
    log("generating the z->lambda share (4 fields x 137 x 64 x 1612)")
    x32, _ = W.zlambda_fields(want_f64=False)
    cs = W.zlambda_chunkset()
    plan = zfpx.Plan.from_chunkset(cs)
    nvals = plan.nvalues
    nblocks = plan.nblocks
    in_bytes = 4 * nvals
    nsets = max(1, args.sets)
    src = [torch.from_numpy(x32.reshape(-1)).to(dev) for _ in range(nsets)]
    del x32
    send = {r: [torch.empty(nblocks * r, dtype=torch.int64, device=dev) for _ in range(nsets)]
            for r in (rate, 8) if r}
    dst = [torch.empty_like(src[0]) for _ in range(nsets)]

    def enc(r):
        return lambda i: zfpx.zfpx_pack_encode(plan, src[i % nsets], r, send[r][i % nsets])

    def dec(r):
        return lambda i: zfpx.zfpx_decode_unpack(plan, send[r][i % nsets], r, dst[i % nsets])

    log(f"timing rate {rate}: {args.warmup} warmup + {args.steps} steps")
    wall, (t_enc, t_dec) = timed_loop([enc(rate), dec(rate)], args.steps, args.warmup, torch)
    ms_per_step = 1000.0 * wall / args.steps
    value = in_bytes * args.steps / wall / 1e9

    coded = nblocks * 8 * rate
    alg_enc = in_bytes + coded   # read float32, write the stream
    alg_dec = coded + in_bytes   # read the stream, write float32
    enc_gbs = alg_enc / (t_enc * 1e-3) / 1e9
    dec_gbs = alg_dec / (t_dec * 1e-3) / 1e9
    dominant = "pack_encode" if t_enc >= t_dec else "decode_unpack"
    t_dom = max(t_enc, t_dec)
    alg_dom = alg_enc if t_enc >= t_dec else alg_dec
    achieved = alg_dom / (t_dom * 1e-3) / 1e9

    # bit-exact round trip is checked by the tests; here only a cheap sanity check
    torch.cuda.synchronize()

    extras = {}
    if not args.no_extras:
        log("timing rate 8 and the float16 comparator")
        _, (e8, d8) = timed_loop([enc(8), dec(8)], max(5, args.steps // 2), 2, torch)
        c8 = nblocks * 8 * 8
        h = [torch.empty(nvals, dtype=torch.int16, device=dev) for _ in range(nsets)]
        ft = lambda i: zfpx.f16_truncate(src[i % nsets], h[i % nsets])
        fr = lambda i: zfpx.f16_restore(h[i % nsets], dst[i % nsets])
        _, (tt, tr) = timed_loop([ft, fr], max(5, args.steps // 2), 2, torch)
        extras = {
            "rate8": {"encode_ms": round(e8, 4), "decode_ms": round(d8, 4),
                      "gbs_fp32_input": round(in_bytes / ((e8 + d8) * 1e-3) / 1e9, 1),
                      "encode_hbm_frac": round((in_bytes + c8) / (e8 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "decode_hbm_frac": round((in_bytes + c8) / (d8 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "bytes_reduction": round(in_bytes / c8, 3)},
            "f16": {"truncate_ms": round(tt, 4), "restore_ms": round(tr, 4),
                    "gbs_fp32_input": round(in_bytes / ((tt + tr) * 1e-3) / 1e9, 1),
                    "truncate_hbm_frac": round(6 * nvals / (tt * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "bytes_reduction": 2.0},
        }
        del h

    if args.copy_calibration:
        log("plain 1 GiB device copy (counter calibration)")
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cs, rate)

    out = {
        "metric": "encode+decode GB/s of fp32 input and % HBM peak at rate 8/16; p99 request latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32->int32 codec",
        "data": "synthetic T42 spherical-harmonic fields (seeded); DYAMOND not available",
        "config": {"workload": "z->lambda transpose share, 4x137x64x1612 f32 (226.1 MB), "
                               "64 chunks", "rate": rate, "values": nvals, "blocks": nblocks,
                   "buffer_sets": nsets},
        "encode_ms": round(t_enc, 4),
        "decode_ms": round(t_dec, 4),
        "encode_hbm_frac": round(enc_gbs / HBM_PEAK_GBS, 4),
        "decode_hbm_frac": round(dec_gbs / HBM_PEAK_GBS, 4),
        "bytes_reduction": round(in_bytes / coded, 3),
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes": alg_dom, "traffic": None},
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(cs, rate):
    """The CPU oracle (plain C, OpenMP over blocks) on the same workload."""
    import numpy as np

    import oracle
    from paper_2609_24294_amd import workloads as W

    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or W.cpu_count()
    log(f"cpu baseline: oracle on the whole share at rate {rate}, {cores} threads")
    x32, _ = W.zlambda_fields(want_f64=False)
    oracle.lib()
    times = []
    for _ in range(2):
        t0 = time.perf_counter()
        words = oracle.pack_encode(cs, x32, rate)
        t1 = time.perf_counter()
        back = np.empty(x32.size, np.float32)
        oracle.decode_unpack(cs, words, rate, back)
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    te, td = min(times, key=lambda t: t[0] + t[1])
    nvals = cs.values()
    return {"value": round(4 * nvals / (te + td) / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"whole z->lambda share ({nvals} values), pack+encode then decode+unpack "
                      f"at rate {rate}, best of 2",
            "encode_s": round(te, 3), "decode_s": round(td, 3)}


if __name__ == "__main__":
    main()
