"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

1. The plan-table builder (paper_2609_24294_amd/csrc/plan_tables.cpp, the
   host half of zfpx_plan_create) is built with g++ -fsanitize=address,
   undefined and run on the z->lambda share, the lambda->theta buffer, the
   O2560 buffer and ragged plans; its runs and tile table are checked
   against the oracle's block geometry (where each block's 64 values come
   from and which are in range).
2. The C oracle is built with gcc -fsanitize=address,undefined and the CPU
   pin suites run against that build in a subprocess.
Any sanitizer report fails the test.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2609_24294_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2609_24294_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
REPORT = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _have_asan():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                           text=True, check=True)
        return os.path.isabs(p.stdout.strip()) and os.path.exists(p.stdout.strip())
    except (OSError, subprocess.CalledProcessError):
        return False


pytestmark = pytest.mark.skipif(not _have_asan(), reason="gcc sanitizer runtimes not installed")


@pytest.fixture(scope="module")
def dump_exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / "plan_tables_dump")
    subprocess.run(["g++", "-std=c++17", *SAN, os.path.join(CSRC, "plan_tables.cpp"),
                    os.path.join(HERE, "host", "plan_tables_dump.cpp"), "-o", out], check=True)
    return out


def _run_tables(exe, cs):
    args = [cs.nchunks, *cs.chunk_base, *cs.level_stride, *cs.levels, *cs.row_start,
            *cs.row_offset, *cs.row_len]
    text = " ".join(str(int(a)) for a in args)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    p = subprocess.run([exe], input=text, capture_output=True, text=True, env=env)
    assert not any(r in p.stderr for r in REPORT), p.stderr[-2000:]
    assert p.returncode == 0, p.stderr[-2000:]
    lines = p.stdout.split("\n")
    assert lines[0] == "status 0", lines[0]
    nruns = int(lines[1].split()[1])
    runs = np.array([[int(v) for v in lines[2 + i].split()] for i in range(nruns)],
                    np.int64).reshape(nruns, 13)
    seg_block0 = np.array(lines[2 + nruns].split()[1:], np.int64)
    tile_seg = np.array(lines[3 + nruns].split()[1:], np.int64)
    totals = [int(v) for v in lines[4 + nruns].split()[1:]]
    return runs, seg_block0, tile_seg, totals


def _positions(runs, seg_block0, tile_seg, ids):
    """Element offset and in-range flag of each value of each listed block,
    found the way a device lane does: tile -> first run, forward to the run
    holding the block, then clamped row/level/point."""
    pos = np.zeros((len(ids), 64), np.int64)
    ins = np.zeros((len(ids), 64), bool)
    for j, b in enumerate(ids):
        s = int(tile_seg[b >> 6])
        while seg_block0[s + 1] <= b:
            s += 1
        block0, nbx, nlev, nrow, lstride = runs[s, :5]
        rbase, rlen = runs[s, 5:9], runs[s, 9:13]
        assert block0 <= b < block0 + nbx
        x0 = 4 * (b - block0)
        for z in range(4):
            for y in range(4):
                for x in range(4):
                    i = 16 * z + 4 * y + x
                    px = min(x0 + x, rlen[y] - 1)
                    pos[j, i] = rbase[y] + min(z, nlev - 1) * lstride + px
                    ins[j, i] = z < nlev and y < nrow and x0 + x < rlen[y]
    return pos, ins


def _odd_chunks():
    lens = np.array([5, 9, 3, 11, 7, 2, 6])
    offs = np.concatenate([[1], 1 + np.cumsum(lens)[:-1] + 3 * np.arange(1, 7)])
    return W.ChunkSet(np.array([0, 2]), np.array([200, 203]), np.array([6, 3]),
                      np.array([0, 5, 7]), np.concatenate([offs[:5], offs[5:] - 2]), lens, 1300)


@pytest.mark.parametrize("name", ["zlambda", "ltheta", "large", "ragged", "odd", "regular"])
def test_plan_tables_under_sanitizers(dump_exe, name):
    cs = {"zlambda": W.zlambda_chunkset, "ltheta": W.ltheta_chunkset,
          "large": W.large_chunkset,
          "ragged": lambda: W.reduced_grid_chunkset(n_half=24, nlev=7, nchunks=5),
          "odd": _odd_chunks, "regular": lambda: W.regular_chunkset(7, 10, 13)}[name]()
    runs, seg_block0, tile_seg, totals = _run_tables(dump_exe, cs)
    nblocks = int(oracle.chunk_blocks(cs).sum())
    assert totals[0] == nblocks == seg_block0[-1]
    assert totals[1] == cs.values()
    assert np.all(np.diff(seg_block0) == runs[:, 1])  # runs tile the block range
    assert tile_seg.size == max(1, -(-nblocks // 64))
    rng = np.random.default_rng(len(name))
    ids = np.unique(np.concatenate([rng.integers(0, nblocks, 400), [0, nblocks - 1],
                                    seg_block0[:-1][rng.integers(0, len(runs), 50)]]))
    words = np.zeros(nblocks * 8, np.uint64) if nblocks < 4_000_000 else None
    pos, ins = _positions(runs, seg_block0, tile_seg, ids)
    if words is None:  # large plans: the oracle's geometry of the listed blocks only
        words = np.zeros((int(ids.max()) + 1) * 8, np.uint64)
    _, opos, oins = oracle.decode_sample(cs, words, 8, ids)
    assert np.array_equal(ins, oins)
    assert np.array_equal(pos, opos)


def test_plan_tables_reject_bad_descriptions(dump_exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    for text in ("1 0 16 4 0 1 0 0",        # a row of zero points
                 "1 0 16 -1 0 1 0 4",       # negative levels
                 "2 0 0 16 16 4 4 0 2 1 0 0 4 4 4"):  # row_start decreasing
        p = subprocess.run([dump_exe], input=text, capture_output=True, text=True, env=env)
        assert not any(r in p.stderr for r in REPORT), p.stderr[-2000:]
        assert p.stdout.split("\n")[0] == "status -1", (text, p.stdout[:100])


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c11", *SAN, "-fopenmp", "-fPIC", "-shared",
                    os.path.join(ROOT, "oracle", "zfp_oracle.c"), "-o", lib, "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                           text=True, check=True).stdout.strip()
    env = dict(os.environ, ZFPX_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", OMP_NUM_THREADS="4")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py"),
                        os.path.join(HERE, "test_oracle_var.py"),
                        "-k", "not sanitizers"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = p.stdout + p.stderr
    assert not any(r in out for r in REPORT), out[-3000:]
    assert p.returncode == 0, out[-3000:]
    assert " passed" in out
