"""Benchmark: fixed-rate ZFP pack+encode / decode+unpack of one GPU's
transpose buffers on one MI355X.

Headline workload: the large single-GPU buffer -- one float32 field on the
O2560-like reduced octahedral grid (5120 latitude rows, 26,306,560 points per
level) x 90 levels = 2,367,590,400 values (9.47 GB), one chunk, synthetic
T42 spectral field (seeded; levels 8..89 repeat the generated levels 0..7).

A step is one pass of the method over that buffer at rate 16: fused
pack+encode into the send buffer, then fused decode+unpack into the receive
layout.  Each step decodes the stream the previous step encoded (two stream
buffers alternate), as a receiver decodes a message that arrived from the
network.  `value` = float32 input bytes x steps / wall time of the timed
steps, with the inputs resident in HBM.  Rate 8 and the float16 comparator
are timed on the same buffer; the z->lambda share (226 MB, 64 chunks), the
small regular field (256 KiB) and the other legs are reported beside it.

One JSON line on stdout.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
VALU_SIMD_CYCLES_PER_S = 1024 * 2.4e9  # 256 CUs x 4 SIMDs at 2.4 GHz


KERNEL_SOURCES = ("paper_2609_24294_amd/csrc/kernels.hip",
                  "paper_2609_24294_amd/csrc/block_codec.hpp",
                  "paper_2609_24294_amd/csrc/internal.hpp")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "o2560_l90_hbm_traffic.md")

LEGS = ("share", "small", "accuracy", "variable", "sensitivity", "pipeline", "fourier",
        "batching", "serving", "cpu")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, rate: int, path: str = TRAFFIC_PROFILE):
    """HBM bytes per launch of `kernel` at `rate` from the committed counter
    passes (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    or None when there are none or the kernel sources changed since."""
    try:
        text = open(path).read()
        block = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if kernel_source_hash() != block["source_hash"]:
            return None
        k = block["kernels"][kernel][str(rate)]
        return {"bytes": k["read_bytes"] + k["write_bytes"], "read": k["read_bytes"],
                "write": k["write_bytes"], "valu": k.get("valu_insts"),
                "waves": k.get("waves")}
    except (OSError, IndexError, KeyError, ValueError):
        return None


def log(msg: str) -> None:
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rate", type=int, default=16)
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs besides the headline (" + ",".join(LEGS) +
                         "), 'all' or 'none'")
    ap.add_argument("--sets", type=int, default=3, help="rotated buffer sets (z->lambda share)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for counter calibration)")
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--serving-workgroups", type=int, default=0,
                    help="workgroups of the serving loop (0: the library's default)")
    return ap.parse_args()


def timed_loop(fn_list, steps, warmup, torch, detail=False):
    """Run warmup + steps iterations of a list of launch callables on the
    current stream (the stream the library launches on); per callable, the
    mean event-timed duration (ms) (and, with detail, the per-step
    durations).  Step i of a callable list runs f(i) for each f in order."""
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
            f(warmup + i)
            e[j + 1].record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    each = [[evs[i][j].elapsed_time(evs[i][j + 1]) for i in range(steps)]
            for j in range(len(fn_list))]
    per = [sum(e) / steps for e in each]
    if detail:
        return wall, per, each
    return wall, per


def hbm_frac(nbytes, ms):
    return round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)


def large_buffer(torch, W):
    """The O2560 x 90 field on the device (levels 8..89 repeat 0..7: a
    4-level block never straddles a repeat, so every block has the
    generator's level-to-level statistics)."""
    log("generating the O2560 x 90 field (8 levels, repeated on the device)")
    base = W.large_field_levels(8)
    cs = W.large_chunkset()
    npts = base.shape[1]
    nlev = cs.buffer_elems // npts
    dev = torch.device("cuda:0")
    b = torch.from_numpy(base.reshape(-1)).to(dev)
    src = torch.empty(cs.buffer_elems, dtype=torch.float32, device=dev)
    for k in range(0, nlev, 8):
        n = min(8, nlev - k) * npts
        src[k * npts: k * npts + n] = b[:n]
    del b
    return cs, src, base, npts, nlev


def headline_report(args, torch, zfpx, W):
    """O2560 x 90 levels (9.47 GB, one chunk): `steps` timed steps of encode
    then decode at the headline rate, each decoding the previous step's
    stream; rate 8 and float16 on the same buffer."""
    cs, src, base, npts, nlev = large_buffer(torch, W)
    del base
    plan = zfpx.Plan.from_chunkset(cs)
    nvals, nblocks = plan.nvalues, plan.nblocks
    in_bytes = 4 * nvals
    dev = src.device
    dst = torch.empty_like(src)
    out = {"workload": f"O2560 reduced grid ({npts} points/level, 5120 rows) x {nlev} levels "
                       f"f32 ({in_bytes / 1e9:.2f} GB), one chunk",
           "values": nvals, "blocks": nblocks,
           "data": "synthetic T42 field; levels 8..89 repeat the generated levels 0..7"}
    res = {}
    for rate in ((args.rate, 8) if args.rate != 8 else (8,)):
        send = [torch.empty(nblocks * rate, dtype=torch.int64, device=dev) for _ in range(2)]
        enc = lambda i, r=rate, sd=send: zfpx.zfpx_pack_encode(plan, src, r, sd[i % 2])
        dec = lambda i, r=rate, sd=send: zfpx.zfpx_decode_unpack(plan, sd[(i - 1) % 2], r, dst)
        steps = args.steps if rate == args.rate else max(5, args.steps // 2)
        log(f"headline: rate {rate}, {max(2, args.warmup)} warmup + {steps} steps")
        wall, (te, td), each = timed_loop([enc, dec], steps, max(2, args.warmup), torch,
                                          detail=True)
        alg = in_bytes + nblocks * 8 * rate
        res[rate] = dict(wall=wall, steps=steps, te=te, td=td, alg=alg)
        out[f"rate{rate}"] = {
            "encode_ms": round(te, 4), "decode_ms": round(td, 4),
            **{f"{name}_ms_{stat}": round(float(f(each[j])), 4)
               for j, name in enumerate(("encode", "decode"))
               for stat, f in (("median", statistics.median), ("min", min))},
            "gbs_fp32_input": round(in_bytes / ((te + td) * 1e-3) / 1e9, 1),
            "encode_gbs_fp32": round(in_bytes / (te * 1e-3) / 1e9, 1),
            "decode_gbs_fp32": round(in_bytes / (td * 1e-3) / 1e9, 1),
            "encode_hbm_frac": hbm_frac(alg, te), "decode_hbm_frac": hbm_frac(alg, td),
            "algorithmic_bytes_per_launch": alg,
            "bytes_reduction": round(in_bytes / (nblocks * 8 * rate), 3)}
        del send
    h = torch.empty(nvals, dtype=torch.int16, device=dev)
    ft = lambda i: zfpx.f16_truncate(src, h)
    fr = lambda i: zfpx.f16_restore(h, dst)
    _, (tt, tr) = timed_loop([ft, fr], max(5, args.steps // 2), 2, torch)
    out["f16"] = {"truncate_ms": round(tt, 4), "restore_ms": round(tr, 4),
                  "gbs_fp32_input": round(in_bytes / ((tt + tr) * 1e-3) / 1e9, 1),
                  "truncate_hbm_frac": hbm_frac(6 * nvals, tt),
                  "restore_hbm_frac": hbm_frac(6 * nvals, tr), "bytes_reduction": 2.0}
    del h
    if args.copy_calibration:
        # known traffic for the counter passes: 256 MiB read and 256 MiB
        # written by a plain elementwise kernel (and by the runtime's copy)
        log("plain 256 MiB device copies (counter calibration)")
        a = torch.empty(1 << 26, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    # precision mode 16 (cap 16): three encode launches, one decode launch
    log("headline buffer: precision 16 (variable size)")
    w, nd, to = zfpx.zfpx_plan_encode_var(plan, src, 16, zfpx.MINEXP_NONE, 16)
    enc = lambda i: zfpx.zfpx_plan_encode_var(plan, src, 16, zfpx.MINEXP_NONE, 16, w, nd, to)
    dec = lambda i: zfpx.zfpx_plan_decode_var(plan, w, nd, to, 16, zfpx.MINEXP_NONE, 16, dst)
    _, (te, td) = timed_loop([enc, dec], 5, 1, torch)
    torch.cuda.synchronize()
    coded = 4 * int(to[-1].item()) + plan.nblocks + 8 * to.numel()
    out["precision16"] = {"encode_ms": round(te, 3), "decode_ms": round(td, 3),
                          "bits_per_value": round(8 * coded / nvals, 3),
                          "encode_hbm_frac": hbm_frac(in_bytes + coded, te),
                          "decode_hbm_frac": hbm_frac(in_bytes + coded, td)}
    del w, nd, to, src, dst
    torch.cuda.empty_cache()
    return out, res, in_bytes


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    legs = (set(LEGS) if args.legs == "all" else
            set() if args.legs == "none" else set(args.legs.split(",")))
    unknown = legs - set(LEGS)
    if unknown:
        print(f"unknown legs {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2609_24294_amd import workloads as W
    from paper_2609_24294_amd import zfpx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rate = args.rate

    head, res, in_bytes = headline_report(args, torch, zfpx, W)
    r = res[rate]
    ms_per_step = 1000.0 * r["wall"] / r["steps"]
    value = in_bytes * r["steps"] / r["wall"] / 1e9
    t_enc, t_dec = r["te"], r["td"]
    dominant = "pack_encode" if t_enc >= t_dec else "decode_unpack"
    t_dom = max(t_enc, t_dec)
    achieved = r["alg"] / (t_dom * 1e-3) / 1e9
    traffic = measured_traffic(dominant, rate)

    share = small = accuracy = variable = sensitivity = pipeline = fourier = None
    batching = serving = cpu = model = None
    if "share" in legs or "variable" in legs or "pipeline" in legs or "sensitivity" in legs \
            or "accuracy" in legs:
        share_ctx = share_buffers(args, torch, zfpx, W)
        if "share" in legs:
            share = share_report(args, share_ctx, torch, zfpx)
        if "variable" in legs:
            variable = variable_report(share_ctx["plan"], share_ctx["src"], share_ctx["dst"],
                                       share_ctx["nvals"], share_ctx["nblocks"],
                                       max(5, args.steps // 2), torch, zfpx, W)
        if "pipeline" in legs:
            pipeline = pipeline_report(share_ctx["plan"], share_ctx["src"][0], share_ctx["nvals"],
                                       share_ctx["nblocks"], torch, zfpx)
        if "accuracy" in legs:
            accuracy = accuracy_report(share_ctx["plan"], share_ctx["src"][0],
                                       share_ctx["dst"][0], share_ctx["nvals"],
                                       share_ctx["nblocks"], torch, zfpx, W)
        # last user of the share's buffers: it overwrites them with other data
        if "sensitivity" in legs:
            sensitivity = sensitivity_report(share_ctx["plan"], share_ctx["src"], share_ctx["dst"],
                                             share_ctx["nblocks"], max(5, args.steps // 2),
                                             torch, zfpx, W)
        del share_ctx
        torch.cuda.empty_cache()
    if "small" in legs:
        small = small_report(torch, zfpx, W)
    if "fourier" in legs:
        fourier = fourier_report(max(5, args.steps // 2), torch, zfpx, W)
    if rate == 16 and 8 in res:
        r8 = res[8]
        f16 = head["f16"]
        model = transpose_model_report(in_bytes, t_enc, t_dec, r8["te"], r8["td"],
                                       f16["truncate_ms"], f16["restore_ms"])
    if "batching" in legs:
        torch.cuda.empty_cache()
        batching = batching_report(torch, zfpx, W)
    if "serving" in legs:
        torch.cuda.empty_cache()
        try:
            serving = serving_report(torch, zfpx, W, args.serving_requests,
                                     args.serving_workgroups)
        except zfpx.ZfpxError as e:
            serving = {"error": str(e)}
    if "cpu" in legs:
        cpu = cpu_baseline(rate)

    out = {
        "metric": "encode+decode GB/s of fp32 input and % HBM peak at rate 8/16; p99 request latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": max(2, args.warmup),
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32->int32 codec",
        "data": "synthetic T42 spherical-harmonic fields (seeded); DYAMOND not available",
        "config": {"workload": "O2560 reduced octahedral grid x 90 levels, one float32 field "
                               "(2,367,590,400 values, 9.47 GB), one chunk", "rate": rate,
                   "values": head["values"], "blocks": head["blocks"],
                   "stream_buffers": 2},
        "encode_ms": round(t_enc, 4),
        "decode_ms": round(t_dec, 4),
        "encode_hbm_frac": hbm_frac(r["alg"], t_enc),
        "decode_hbm_frac": hbm_frac(r["alg"], t_dec),
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes": r["alg"],
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_read_write": [traffic["read"], traffic["write"]] if traffic else None,
                     # the same kernel against its instruction-issue ceiling: VALU
                     # wavefront instructions (counter pass) x 4 cycles each on a
                     # 16-lane SIMD, over 1024 SIMDs x 2.4 GHz x the launch time
                     "valu_per_tile": (round(traffic["valu"] / traffic["waves"], 1)
                                       if traffic and traffic.get("valu") and traffic.get("waves")
                                       else None),
                     "valu_issue_frac": (round(traffic["valu"] * 4 / (VALU_SIMD_CYCLES_PER_S
                                                                     * t_dom * 1e-3), 4)
                                         if traffic and traffic["valu"] else None)},
        "cpu_baseline": cpu,
        "headline": head,
        "share": share,
        "small": small,
        "transpose_model": model,
        "accuracy": accuracy,
        "variable": variable,
        "sensitivity": sensitivity,
        "pipeline": pipeline,
        "fourier": fourier,
        "batching": batching,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


def share_buffers(args, torch, zfpx, W):
    """The z->lambda share on the device, in `sets` rotated buffer sets."""
    log("generating the z->lambda share (4 fields x 137 x 64 x 1612)")
    x32, _ = W.zlambda_fields(want_f64=False)
    cs = W.zlambda_chunkset()
    plan = zfpx.Plan.from_chunkset(cs)
    dev = torch.device("cuda:0")
    nsets = max(2, args.sets)
    src = [torch.from_numpy(x32.reshape(-1)).to(dev) for _ in range(nsets)]
    dst = [torch.empty_like(src[0]) for _ in range(nsets)]
    return {"cs": cs, "plan": plan, "src": src, "dst": dst, "nsets": nsets,
            "nvals": plan.nvalues, "nblocks": plan.nblocks}


def share_report(args, ctx, torch, zfpx):
    """z->lambda share (226.1 MB, 64 chunks): encode and decode at rates 16
    and 8 over rotated buffer sets whose combined size exceeds the 256 MB
    last-level cache; step i decodes the stream step i-1 encoded (another
    set), and float16 the same way."""
    plan, src, dst, nsets = ctx["plan"], ctx["src"], ctx["dst"], ctx["nsets"]
    nvals, nblocks = ctx["nvals"], ctx["nblocks"]
    in_bytes = 4 * nvals
    out = {"workload": "z->lambda transpose share, 4x137x64x1612 f32 (226.1 MB), 64 chunks",
           "buffer_sets": nsets}
    for rate in (16, 8):
        send = [torch.empty(nblocks * rate, dtype=torch.int64, device=src[0].device)
                for _ in range(nsets)]
        enc = lambda i, r=rate, sd=send: zfpx.zfpx_pack_encode(plan, src[i % nsets], r,
                                                              sd[i % nsets])
        dec = lambda i, r=rate, sd=send: zfpx.zfpx_decode_unpack(plan, sd[(i - 1) % nsets], r,
                                                                dst[(i - 1) % nsets])
        steps = max(10, args.steps)
        log(f"share: rate {rate}")
        _, (te, td), each = timed_loop([enc, dec], steps, max(nsets, 2), torch, detail=True)
        alg = in_bytes + nblocks * 8 * rate
        out[f"rate{rate}"] = {
            "encode_ms": round(te, 4), "decode_ms": round(td, 4),
            **{f"{name}_ms_{stat}": round(float(f(each[j])), 4)
               for j, name in enumerate(("encode", "decode"))
               for stat, f in (("median", statistics.median), ("min", min))},
            "gbs_fp32_input": round(in_bytes / ((te + td) * 1e-3) / 1e9, 1),
            "encode_hbm_frac": hbm_frac(alg, te), "decode_hbm_frac": hbm_frac(alg, td),
            "bytes_reduction": round(in_bytes / (nblocks * 8 * rate), 3)}
        del send
    h = [torch.empty(nvals, dtype=torch.int16, device=src[0].device) for _ in range(nsets)]
    ft = lambda i: zfpx.f16_truncate(src[i % nsets], h[i % nsets])
    fr = lambda i: zfpx.f16_restore(h[(i - 1) % nsets], dst[(i - 1) % nsets])
    _, (tt, tr) = timed_loop([ft, fr], max(10, args.steps), max(nsets, 2), torch)
    out["f16"] = {"truncate_ms": round(tt, 4), "restore_ms": round(tr, 4),
                  "gbs_fp32_input": round(in_bytes / ((tt + tr) * 1e-3) / 1e9, 1),
                  "truncate_hbm_frac": hbm_frac(6 * nvals, tt),
                  "restore_hbm_frac": hbm_frac(6 * nvals, tr), "bytes_reduction": 2.0}
    del h
    return out


def small_report(torch, zfpx, W, reps=200):
    """The small regular field (T42, f32[8][64][128], 65,536 values, 256 KiB)
    timed in full at rates 8/16/32 and float16: each launch is a few
    microseconds and the data stay in the last-level cache, so this is a
    launch-latency figure, not an HBM one."""
    log("small: regular 8 x 64 x 128 field, all rates")
    x32, _ = W.small_field()
    dev = torch.device("cuda:0")
    src = torch.from_numpy(x32).to(dev)
    dst = torch.empty_like(src)
    in_bytes = 4 * x32.size
    out = {"workload": "regular 64 x 128 Gauss-Legendre grid x 8 levels f32 (256 KiB), T42",
           "values": int(x32.size)}
    for rate in (8, 16, 32):
        words = zfpx.zfpx_encode_fixed_rate(src, rate)
        enc = lambda i, r=rate, w=words: zfpx.zfpx_encode_fixed_rate(src, r, w)
        dec = lambda i, r=rate, w=words: zfpx.zfpx_decode_fixed_rate(w, r, dst)
        _, (te, td) = timed_loop([enc, dec], reps, 10, torch)
        out[f"rate{rate}"] = {"encode_us": round(te * 1e3, 2), "decode_us": round(td * 1e3, 2),
                              "gbs_fp32_input": round(in_bytes / ((te + td) * 1e-3) / 1e9, 1),
                              "bytes_reduction": round(in_bytes / (words.numel() * 8), 3)}
    h = torch.empty(x32.size, dtype=torch.int16, device=dev)
    ft = lambda i: zfpx.f16_truncate(src.reshape(-1), h)
    fr = lambda i: zfpx.f16_restore(h, dst.reshape(-1))
    _, (tt, tr) = timed_loop([ft, fr], reps, 10, torch)
    out["f16"] = {"truncate_us": round(tt * 1e3, 2), "restore_us": round(tr * 1e3, 2)}
    return out


def variable_report(plan, src, dst, nvals, nblocks, steps, torch, zfpx, W):
    """Fixed-precision and fixed-accuracy modes on the same share: encode and
    decode time (rotated buffer sets, HIP events), the stream size with its
    per-block counts and tile offsets, and the error against the FP64 fields
    (untimed)."""
    import numpy as np

    from paper_2609_24294_amd import metrics
    log("variable-size modes: precision 16 and accuracy 1e-2")
    _, x64 = W.zlambda_fields(want_f64=True)
    shape = x64.shape
    names = ("u", "v", "T", "q")
    nsets = len(src)
    ntiles = (nblocks + 63) // 64
    out = {"workload": "same share and buffer sets as the headline; per-block cap 16 "
                       "bits/value (no block of either mode reaches it here)"}
    for name, maxprec, minexp, cap in (("precision16", 16, zfpx.MINEXP_NONE, 16),
                                       ("accuracy_1e-2", 32, zfpx.zfpx_accuracy_minexp(1e-2), 16)):
        sets = [zfpx.zfpx_plan_encode_var(plan, src[i], maxprec, minexp, cap) for i in range(nsets)]

        def enc(i):
            w, nd, to = sets[i % nsets]
            return zfpx.zfpx_plan_encode_var(plan, src[i % nsets], maxprec, minexp, cap, w, nd, to)

        def dec(i):  # the set the previous step encoded
            w, nd, to = sets[(i - 1) % nsets]
            return zfpx.zfpx_plan_decode_var(plan, w, nd, to, maxprec, minexp, cap,
                                             dst[(i - 1) % nsets])

        _, (te, td) = timed_loop([enc, dec], steps, nsets, torch)
        torch.cuda.synchronize()
        w, nd, to = sets[0]
        words = int(to[-1].item())
        zfpx.zfpx_plan_decode_var(plan, w, nd, to, maxprec, minexp, cap, dst[0])
        back = dst[0].cpu().numpy().reshape(shape)
        ndh = nd[:nblocks].cpu().numpy()
        payload = 4 * words
        index = nblocks + 8 * (ntiles + 1)
        alg_enc = 4 * nvals + payload + index
        r = {"maxprec": maxprec, "minexp": minexp, "rate_cap": cap,
             "encode_ms": round(te, 4), "decode_ms": round(td, 4),
             "gbs_fp32_input": round(4 * nvals / ((te + td) * 1e-3) / 1e9, 1),
             "encode_hbm_frac": round(alg_enc / (te * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "decode_hbm_frac": round(alg_enc / (td * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "bits_per_value": round(8 * (payload + index) / nvals, 3),
             "payload_bits_per_value": round(8 * payload / nvals, 3),
             "bytes_reduction": round(4 * nvals / (payload + index), 3),
             "blocks_at_cap": int((ndh >= 2 * cap).sum()),
             **{names[f]: {k: float(f"{v:.3e}") for k, v in
                           metrics.error_report(x64[f], back[f], pointwise=f in (2, 3)).items()}
                for f in range(4)}}
        if minexp != zfpx.MINEXP_NONE:
            x32 = src[0].cpu().numpy().reshape(shape)
            r["max_abs_error_vs_input"] = float(f"{np.abs(back.astype(np.float64) - x32).max():.3e}")
            r["tolerance"] = 1e-2
        out[name] = r
        del sets
    return out


def sensitivity_report(plan, src, dst, nblocks, steps, torch, zfpx, W):
    """How the codec's speed depends on the data: the same share and launch at
    rates 16 and 8 with the fields synthesised at T255 instead of T42, and
    with white noise (every coefficient significant from the first planes:
    the coder's worst case).  The headline buffers are overwritten."""
    import numpy as np

    log("sensitivity: the share at T255 and as white noise")
    nsets = len(src)
    nvals = src[0].numel()
    out = {}
    x255, _ = W.zlambda_fields(L=255, want_f64=False)
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 7))
    noise = rng.standard_normal(nvals, dtype=np.float32)
    for name, host in (("T255", x255.reshape(-1)), ("white_noise", noise)):
        for i in range(nsets):
            src[i].copy_(torch.from_numpy(host))
        r = {}
        for rate in (16, 8):
            send = [torch.empty(nblocks * rate, dtype=torch.int64, device=src[0].device)
                    for _ in range(nsets)]
            enc = lambda i: zfpx.zfpx_pack_encode(plan, src[i % nsets], rate, send[i % nsets])
            dec = lambda i: zfpx.zfpx_decode_unpack(plan, send[(i - 1) % nsets], rate,
                                                    dst[(i - 1) % nsets])
            _, (te, td) = timed_loop([enc, dec], steps, nsets, torch)
            alg = 4 * nvals + nblocks * 8 * rate
            r[f"rate{rate}"] = {"encode_ms": round(te, 4), "decode_ms": round(td, 4),
                                "encode_hbm_frac": round(alg / (te * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                "decode_hbm_frac": round(alg / (td * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del send
        out[name] = r
    torch.cuda.synchronize()
    return out


def pipeline_report(plan, src, nvals, nblocks, torch, zfpx, reps=5):
    """Send (encode + device-to-host copy) and receive (host-to-device copy +
    decode) of the share over a host link on two streams: float32 and float16
    copies, fixed rate 16 with the whole buffer coded before the copy (the
    paper's serial model) and with the copy of chunk group g overlapping the
    coding of group g+1.  Times from the first enqueue to the end of both
    streams (HIP events); inputs resident in HBM, host buffers pinned."""
    cs, xs = torch.cuda.Stream(), torch.cuda.Stream()
    log("pipeline: float32 / float16 / rate 16 serial and chunk-pipelined over a host link")

    def timed(fn):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(cs)
            xs.wait_event(e0)
            fn()
            cs.wait_stream(xs)
            e1.record(cs)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts[1:])

    dev = src.device
    link32 = torch.empty(nvals, dtype=torch.float32).pin_memory()
    out = {"link": "device <-> pinned host memory (PCIe) standing in for the network; two streams",
           "chunks": plan.nchunks}

    def f32_send():
        with torch.cuda.stream(xs):
            link32.copy_(src, non_blocking=True)

    dst = torch.empty_like(src)

    def f32_recv():
        with torch.cuda.stream(xs):
            dst.copy_(link32, non_blocking=True)

    t32s, t32r = timed(f32_send), timed(f32_recv)
    out["float32"] = {"send_ms": round(t32s, 3), "recv_ms": round(t32r, 3),
                      "link_gbs_d2h": round(4 * nvals / (t32s * 1e-3) / 1e9, 1),
                      "link_gbs_h2d": round(4 * nvals / (t32r * 1e-3) / 1e9, 1)}
    h16 = torch.empty(nvals, dtype=torch.int16, device=dev)
    link16 = torch.empty(nvals, dtype=torch.int16).pin_memory()

    def f16_send():
        with torch.cuda.stream(cs):
            zfpx.f16_truncate(src, h16, stream=cs)
        xs.wait_stream(cs)
        with torch.cuda.stream(xs):
            link16.copy_(h16, non_blocking=True)

    def f16_recv():
        with torch.cuda.stream(xs):
            h16.copy_(link16, non_blocking=True)
        cs.wait_stream(xs)
        zfpx.f16_restore(h16, dst, stream=cs)

    t16s, t16r = timed(f16_send), timed(f16_recv)
    out["float16"] = {"send_ms": round(t16s, 3), "recv_ms": round(t16r, 3),
                      "speedup_send": round(t32s / t16s, 3), "speedup_recv": round(t32r / t16r, 3)}
    del h16, link16
    for rate in (16, 8):
        nbytes = nblocks * 8 * rate
        send = torch.empty(nbytes // 8, dtype=torch.int64, device=dev)
        recv = torch.empty_like(send)
        link = torch.empty(nbytes // 8, dtype=torch.int64).pin_memory()
        for groups in (1, 8, 16, 64):
            pipe = zfpx.Pipeline(plan, rate, groups)
            ts = timed(lambda: pipe.send(src, send, link, cs, xs))
            tr = timed(lambda: pipe.recv(link, recv, dst, cs, xs))
            out[f"rate{rate}_groups{groups}"] = {
                "send_ms": round(ts, 3), "recv_ms": round(tr, 3),
                "speedup_send": round(t32s / ts, 3), "speedup_recv": round(t32r / tr, 3),
                "speedup_round_trip": round((t32s + t32r) / (ts + tr), 3)}
            pipe.close()
        del send, recv, link
    return out


def fourier_report(steps, torch, zfpx, W, nsets=3):
    """The lambda->theta share in Fourier space (real and imaginary planes of
    T1279 coefficients, 2 x 137 x 64 x 1280 f32, 32 chunks): encode/decode
    time at rates 16 and 8 and in the variable-size modes (HIP events), and
    the error of each against the FP64 coefficients, with float16 beside."""
    import numpy as np

    from paper_2609_24294_amd import metrics
    c = W.FOURIER
    log("fourier: generating the T1279 Fourier-space share (2 x 137 x 64 x 1280)")
    f32, f64 = W.fourier_buffer()
    cs = W.fourier_chunkset(c["nlev"], c["nrows"], c["mmax"], c["ndest"])
    plan = zfpx.Plan.from_chunkset(cs)
    nvals, nblocks = f32.size, plan.nblocks
    dev = torch.device("cuda:0")
    src = [torch.from_numpy(f32.reshape(-1)).to(dev) for _ in range(nsets)]
    dst = [torch.empty_like(src[0]) for _ in range(nsets)]
    ref = np.sqrt((f64 * f64).sum())

    def errors(back):
        back = back.reshape(f64.shape)
        d = back.astype(np.float64) - f64
        r = {"global": float(f"{np.sqrt((d * d).sum()) / ref:.3e}")}
        for k, name in ((0, "real"), (1, "imag")):
            e = metrics.error_report(f64[k], back[k], pointwise=False)
            r[name] = {"block_mean": float(f"{e['block_mean']:.3e}"),
                       "block_max": float(f"{e['block_max']:.3e}")}
        return r

    out = {"workload": "Fourier-space lambda->theta share: T1279 coefficients of T on rows "
                       "1024..1087 of O1280, 137 levels, real and imaginary planes, 16 destinations "
                       "x 2 chunks (synthetic, (l+1)^-3 spectrum)",
           "values": nvals, "blocks": nblocks}
    for rate in (16, 8):
        send = [torch.empty(nblocks * rate, dtype=torch.int64, device=dev) for _ in range(nsets)]
        enc = lambda i: zfpx.zfpx_pack_encode(plan, src[i % nsets], rate, send[i % nsets])
        dec = lambda i: zfpx.zfpx_decode_unpack(plan, send[(i - 1) % nsets], rate,
                                                dst[(i - 1) % nsets])
        _, (te, td) = timed_loop([enc, dec], steps, nsets, torch)
        zfpx.zfpx_decode_unpack(plan, send[0], rate, dst[0])
        alg = 4 * nvals + nblocks * 8 * rate
        out[f"rate{rate}"] = {"encode_ms": round(te, 4), "decode_ms": round(td, 4),
                              "encode_hbm_frac": round(alg / (te * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              "decode_hbm_frac": round(alg / (td * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              "bytes_reduction": round(4 * nvals / (nblocks * 8 * rate), 3),
                              **errors(dst[0].cpu().numpy())}
        del send
    h = zfpx.f16_truncate(src[0])
    out["f16"] = {"bytes_reduction": 2.0, **errors(zfpx.f16_restore(h).cpu().numpy())}
    ntiles = (nblocks + 63) // 64
    for name, maxprec, minexp, cap in (("precision16", 16, zfpx.MINEXP_NONE, 16),
                                       ("accuracy_1e-4", 32, zfpx.zfpx_accuracy_minexp(1e-4), 32)):
        sets = [zfpx.zfpx_plan_encode_var(plan, src[i], maxprec, minexp, cap) for i in range(nsets)]
        enc = lambda i: zfpx.zfpx_plan_encode_var(plan, src[i % nsets], maxprec, minexp, cap,
                                                  *sets[i % nsets])
        dec = lambda i: zfpx.zfpx_plan_decode_var(plan, *sets[(i - 1) % nsets], maxprec, minexp,
                                                  cap, dst[(i - 1) % nsets])
        _, (te, td) = timed_loop([enc, dec], steps, nsets, torch)
        torch.cuda.synchronize()
        w, nd, to = sets[0]
        zfpx.zfpx_plan_decode_var(plan, w, nd, to, maxprec, minexp, cap, dst[0])
        words = int(to[-1].item())
        index = nblocks + 8 * (ntiles + 1)
        back = dst[0].cpu().numpy()
        r = {"encode_ms": round(te, 4), "decode_ms": round(td, 4),
             "bits_per_value": round(8 * (4 * words + index) / nvals, 3),
             "blocks_at_cap": int((nd[:nblocks].cpu().numpy() >= 2 * cap).sum()),
             **errors(back)}
        if minexp != zfpx.MINEXP_NONE:
            r["max_abs_error_vs_input"] = float(f"{np.abs(back - f32.reshape(-1)).max():.3e}")
        out[name] = r
        del sets
    return out


def transpose_model_report(in_bytes, e16, d16, e8, d8, tt, tr):
    """Row-transposition time at N = 4 ... 121 nodes from the alpha-beta model
    with the paper's network parameters and the codec rates measured above
    (GB/s of float32 input)."""
    from paper_2609_24294_amd import transpose_model as TM
    gbs = lambda ms: round(in_bytes / (ms * 1e-3) / 1e9, 1)
    rates = TM.CodecRates(gbs(e16), gbs(d16), gbs(e8), gbs(d8), gbs(tt), gbs(tr))
    net = TM.Network()
    return {"network": f"alpha-beta, {net.link_gbps:g} Gb/s links, {net.hops} hops x "
                       f"{net.hop_us:g} us per message, sqrt(N)-rank row communicators",
            "codec_gbs_fp32_input": dataclasses.asdict(rates), **TM.summary(rates, net)}


def accuracy_report(plan, src, dst, nvals, nblocks, torch, zfpx, W):
    """Relative error of each rate and of float16 against the FP64 copy of the
    synthetic fields (untimed), plus the bytes reduction of the buffer: the
    share synthesised at T42 (the workload) and at T255 (rougher fields,
    where rate 16 is no longer at float32's own storage error)."""
    import numpy as np

    from paper_2609_24294_amd import metrics
    names = ("u", "v", "T", "q")
    out = {"reference": "FP64 copy of the synthetic fields; per-block L2 relative error over "
                        "4x4x4 blocks (mean/max), global L2 error, pointwise for T and q"}
    dev = src.device
    for L in (42, 255):
        log(f"accuracy: T{L}, rates 8/16/32 and float16 against the FP64 fields")
        x32, x64 = W.zlambda_fields(L=L, want_f64=True)
        shape = x64.shape
        d = torch.from_numpy(x32.reshape(-1)).to(dev)
        rep = {}
        for r in (8, 16, 32):
            send = torch.empty(nblocks * r, dtype=torch.int64, device=dev)
            zfpx.zfpx_pack_encode(plan, d, r, send)
            zfpx.zfpx_decode_unpack(plan, send, r, dst)
            back = dst.cpu().numpy().reshape(shape)
            rep[f"rate{r}"] = {
                "bytes_reduction": round(metrics.bytes_reduction(nvals, nblocks * 8 * r), 3),
                **{names[f]: {k: float(f"{v:.3e}") for k, v in
                              metrics.error_report(x64[f], back[f], pointwise=f in (2, 3)).items()}
                   for f in range(4)}}
            del send
        h = zfpx.f16_truncate(d)
        back = zfpx.f16_restore(h).cpu().numpy().reshape(shape)
        rep["f16"] = {"bytes_reduction": 2.0,
                      **{names[f]: {k: float(f"{v:.3e}") for k, v in
                                    metrics.error_report(x64[f], back[f],
                                                         pointwise=f in (2, 3)).items()}
                         for f in range(4)}}
        rep["float32_storage"] = {
            names[f]: float(f"{metrics.error_report(x64[f], x32[f], False)['block_mean']:.3e}")
            for f in range(4)}
        out[f"T{L}"] = rep
        del d, x32, x64
    return out


def batching_report(torch, zfpx, W, rate=16, reps=10):
    """The lambda->theta buffer (O1280 x 137 levels, 256 uneven chunks): one
    autotuned launch per op, the two captured in a HIP graph, against one
    launch per chunk of the same kernels."""
    import ctypes

    log("batching: generating the lambda->theta buffer (O1280 x 137 levels)")
    x = W.ltheta_field()
    cs = W.ltheta_chunkset()
    plan = zfpx.Plan.from_chunkset(cs)
    dev = torch.device("cuda:0")
    src = torch.from_numpy(x.reshape(-1)).to(dev)
    del x
    send = torch.empty(plan.nblocks * rate, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    tuned = {}
    for op in (zfpx.OP_ENCODE, zfpx.OP_DECODE):
        us = zfpx.zfpx_autotune(plan, op, rate, src, send, dst)
        tuned["encode" if op == 0 else "decode"] = {
            "config": dict(zip(("wg", "grid"), zfpx.zfpx_plan_get_config(plan, op, rate))),
            "us": round(us, 1)}
    g = zfpx.Graph(plan, rate, src, send, dst)
    L = zfpx.library()
    h, s_ = plan.handle, stream.cuda_stream
    sp, sn, dp, dn = src.data_ptr(), src.numel(), dst.data_ptr(), dst.numel()
    wp, wn = send.data_ptr(), send.numel() * 8

    def direct():
        L.zfpx_pack_encode(h, sp, sn, rate, wp, wn, s_)
        L.zfpx_decode_unpack(h, wp, wn, rate, dp, dn, s_)

    def per_chunk():
        for c in range(cs.nchunks):
            L.zfpx_pack_encode_chunks(h, c, 1, sp, sn, rate, wp, wn, s_)
        for c in range(cs.nchunks):
            L.zfpx_decode_unpack_chunks(h, c, 1, wp, wn, rate, dp, dn, s_)

    def timeit(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps * 1e3
        return round(e0.elapsed_time(e1) / reps, 4), round(wall, 4)

    log("batching: timing graph, direct and per-chunk forms")
    gpu_g, wall_g = timeit(lambda: g.launch(stream))
    gpu_d, wall_d = timeit(direct)
    gpu_c, wall_c = timeit(per_chunk)
    nvals = plan.nvalues
    g.close()
    # compressed-bytes reduction of the buffer (float32 bytes / coded bytes,
    # partial-block padding included), from the plan's chunk sizes
    reduction = {f"rate{r}": round(4 * nvals / plan.total_bytes(r), 3) for r in (8, 16, 32)}
    reduction["f16"] = 2.0
    return {"workload": "lambda->theta buffer, O1280 (2560 rows) x 137 levels f32 (3.617 GB), "
                        "256 chunks of 8 or 12 rows", "rate": rate, "values": nvals,
            "bytes_reduction": reduction,
            "graph_ms": gpu_g, "direct_ms": gpu_d, "per_chunk_ms": gpu_c,
            "wall_ms": {"graph": wall_g, "direct": wall_d, "per_chunk": wall_c},
            "speedup_graph_vs_per_chunk": round(gpu_c / gpu_g, 3),
            "graph_gbs_fp32_input": round(4 * nvals / (gpu_g * 1e-3) / 1e9, 1),
            "tuned": tuned}


def serving_report(torch, zfpx, W, count, workgroups=0):
    """Poisson arrivals of mixed compress/decompress requests (64 KB .. 64 MB of
    float32, rate 8/16/32): the saturated throughput of the serving loop and
    of one launch per request (every request at t = 0), then p50/p99 latency
    of both at 25 .. 200% of the plain form's saturated throughput.  At the
    100% point every request writes its own output buffer and each served
    output is compared bit for bit with the same request run alone in one
    launch (stopping at the first mismatch)."""
    import numpy as np

    dev = torch.device("cuda:0")
    log("serving: request pool and buffers")
    nx_max = 32768
    pool = torch.from_numpy(W.serving_pool(nx_max=nx_max)).to(dev)
    coded = {r: zfpx.zfpx_encode_fixed_rate(pool, r) for r in (8, 16, 32)}
    nsets = 32
    words_out = [torch.empty(nx_max // 4 * 16 * 2 * 32, dtype=torch.int64, device=dev)
                 for _ in range(nsets)]
    float_out = [torch.empty_like(pool) for _ in range(nsets)]
    torch.cuda.synchronize()  # inputs complete before the server's own stream reads them

    def out_words(q):
        return 16 * 2 * (q.nx // 4) * q.rate if q.op == 0 else 8 * 64 * q.nx // 2

    def build(stream, arena=None):
        reqs, nbytes, outs = [], [], []
        off = 0
        for i, q in enumerate(stream):
            k = i % nsets
            if arena is not None:
                n = out_words(q)
                o = arena[off: off + n]
                off += n
            if q.op == 0:
                view = pool[:, :, : q.nx]
                o = o if arena is not None else words_out[k]
                rq = zfpx.make_request(0, q.rate, view, o)
            else:
                o = (o.view(torch.float32).reshape(8, 64, q.nx) if arena is not None
                     else float_out[k][:, :, : q.nx])
                rq = zfpx.make_request(1, q.rate, o, coded[q.rate])
            reqs.append(rq)
            outs.append(o)
            nbytes.append(4 * 8 * 64 * q.nx)
        return reqs, np.array(nbytes, np.float64), outs

    def pct(x, p):
        return round(float(np.percentile(x, p)) * 1e6, 1)

    base = W.request_stream(count, 1.0)
    reqs, nbytes, _ = build(base)
    zero = np.zeros(count)
    log(f"serving: saturated throughput ({count} requests at t = 0), both forms")
    lat = zfpx.zfpx_plain_replay(reqs, zero, timeout_s=60.0)
    sat = nbytes.sum() / lat.max()
    sv = zfpx.Server(64 << 30, max_slots=1024, workgroups=workgroups)
    try:
        lat_s = sv.replay(reqs, zero, timeout_s=60.0)
    finally:
        sv.close()
    sat_s = nbytes.sum() / lat_s.max()
    mean_bytes = nbytes.mean()
    out = {"requests_per_point": count, "budget_bytes": 64 << 30,
           "loop_workgroups": workgroups or "library default",
           "saturated_gbs_fp32": {"server": round(sat_s / 1e9, 1),
                                  "per_request_launch": round(sat / 1e9, 1)},
           "mean_request_mb": round(mean_bytes / 1e6, 2),
           "note": "offered load is a fraction of the per-request-launch form's saturated "
                   "throughput; request buffers are drawn from 32 rotating sets except at "
                   "load 1.0, where every request has its own output; latency = completion "
                   "seen by the host minus scheduled arrival", "points": []}
    for load in (0.25, 0.5, 0.75, 0.9, 1.0, 1.25, 1.5, 2.0):
        gap = mean_bytes / (load * sat)
        stream = W.request_stream(count, gap)
        arrival = np.array([q.t_arrive for q in stream])
        arena = None
        if load == 1.0:
            arena = torch.empty(sum(out_words(q) for q in stream), dtype=torch.int64, device=dev)
        reqs, nbytes, outs = build(stream, arena)
        log(f"serving: load {load:.2f}, mean gap {gap * 1e6:.1f} us")
        sv = zfpx.Server(64 << 30, max_slots=1024, workgroups=workgroups)
        try:
            ls = sv.replay(reqs, arrival, timeout_s=60.0)
        finally:
            sv.close()
        point = {"load": load, "mean_gap_us": round(gap * 1e6, 2)}
        if arena is not None:
            torch.cuda.synchronize()
            checked, first_bad = 0, None
            for i, (q, o) in enumerate(zip(stream, outs)):
                if q.op == 0:
                    ref = zfpx.zfpx_encode_fixed_rate(pool[:, :, : q.nx], q.rate)
                    same = torch.equal(o, ref)
                else:
                    ref = torch.empty((8, 64, q.nx), dtype=torch.float32, device=dev)
                    zfpx.zfpx_decode_fixed_rate(coded[q.rate], q.rate, ref)
                    same = torch.equal(o.view(torch.int32), ref.view(torch.int32))
                if not same:
                    first_bad = i
                    break
                checked += 1
            point["served_outputs_checked"] = checked
            point["first_mismatch"] = first_bad
            del arena, outs
        lp = zfpx.zfpx_plain_replay(reqs, arrival, timeout_s=60.0)
        span_s = (arrival + ls).max()
        span_p = (arrival + lp).max()
        point["server"] = {"p50_us": pct(ls, 50), "p99_us": pct(ls, 99),
                           "gbs_fp32": round(nbytes.sum() / span_s / 1e9, 1)}
        point["per_request_launch"] = {"p50_us": pct(lp, 50), "p99_us": pct(lp, 99),
                                       "gbs_fp32": round(nbytes.sum() / span_p / 1e9, 1)}
        out["points"].append(point)
        torch.cuda.empty_cache()
    # requests 5 ms apart, past the loop's 2 ms idle spell: each one finds the
    # loop gone and pays for a new launch (the plain form beside it)
    log("serving: cold starts (requests 5 ms apart)")
    cold = [q for q in base[:400] if q.nx <= 1024][:20]
    reqs, _, _ = build(cold)
    arrival = np.arange(len(reqs)) * 5e-3
    sv = zfpx.Server(64 << 30, max_slots=1024, workgroups=workgroups)
    try:
        lc = sv.replay(reqs, arrival, timeout_s=60.0)
        launches = sv.stats()["loop_launches"]
    finally:
        sv.close()
    lp = zfpx.zfpx_plain_replay(reqs, arrival, timeout_s=60.0)
    out["cold_start"] = {"requests": len(reqs), "gap_ms": 5.0, "loop_launches": launches,
                         "server_p50_us": pct(lc, 50), "per_request_launch_p50_us": pct(lp, 50)}
    torch.cuda.synchronize()
    return out


def cpu_baseline(rate):
    """The CPU oracle (plain C, OpenMP over blocks) on a bounded sample of the
    headline workload: the first 8 levels (two 4-level blocks) of the O2560
    field, every point of each level, pack+encode then decode+unpack at
    `rate`; the throughput per byte is what the whole 90-level field would
    see (the time for it is extrapolated linearly)."""
    import numpy as np

    import oracle
    from paper_2609_24294_amd import workloads as W

    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or W.cpu_count()
    log(f"cpu baseline: oracle on the first 8 levels of the O2560 field at rate {rate}, "
        f"{cores} threads")
    x32 = W.large_field_levels(8).reshape(-1)
    cs = W.reduced_grid_chunkset(n_half=2560, nlev=8, nchunks=1)
    assert cs.buffer_elems == x32.size
    cs4 = W.reduced_grid_chunkset(n_half=2560, nlev=4, nchunks=1)
    x4 = x32[:cs4.buffer_elems]
    oracle.lib()
    oracle.set_threads(cores)
    words = oracle.pack_encode(cs4, x4, rate)  # warm-up
    times = []
    back = np.empty(x32.size, np.float32)
    for _ in range(3):
        t0 = time.perf_counter()
        words = oracle.pack_encode(cs, x32, rate)
        t1 = time.perf_counter()
        oracle.decode_unpack(cs, words, rate, back)
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    te = statistics.median(t[0] for t in times)
    td = statistics.median(t[1] for t in times)
    nvals = cs.values()
    # one thread, the first 4 levels
    oracle.set_threads(1)
    t0 = time.perf_counter()
    w4 = oracle.pack_encode(cs4, x4, rate)
    t1 = time.perf_counter()
    oracle.decode_unpack(cs4, w4, rate, back[:x4.size])
    t2 = time.perf_counter()
    oracle.set_threads(cores)
    # numpy's float16 cast and back (the comparator on the host)
    t3 = time.perf_counter()
    h = x32.astype(np.float16)
    t4 = time.perf_counter()
    _ = h.astype(np.float32)
    t5 = time.perf_counter()
    full = W.LARGE["nlev"] / 8
    return {"value": round(4 * nvals / (te + td) / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first 8 of 90 levels of the O2560 field ({nvals} values, "
                      f"{4 * nvals / 1e9:.3f} GB): pack+encode then decode+unpack at rate {rate}, "
                      f"median of 3 after a warm-up",
            "encode_s": round(te, 3), "decode_s": round(td, 3),
            "encode_gbs": round(4 * nvals / te / 1e9, 4),
            "decode_gbs": round(4 * nvals / td / 1e9, 4),
            "whole_field_s_extrapolated": round(full * (te + td), 2),
            "one_thread": {"sample": "first 4 levels", "encode_s": round(t1 - t0, 3),
                           "decode_s": round(t2 - t1, 3),
                           "gbs": round(4 * x4.size / (t2 - t0) / 1e9, 4)},
            "numpy_f16": {"truncate_s": round(t4 - t3, 3), "restore_s": round(t5 - t4, 3),
                          "gbs": round(4 * nvals / (t5 - t3) / 1e9, 4)}}


if __name__ == "__main__":
    main()
