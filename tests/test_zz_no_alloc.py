"""The allocation-free variable-size encoder (library scratch instead of a
caller workspace) against the workspace form, through the C ABI: two calls
in a row on one GPU, the second on a smaller plan, and the size limit."""
import numpy as np
import pytest
import torch

from paper_2609_24294_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _pair(zfpx, cs, host, maxprec, minexp, cap):
    plan = zfpx.Plan.from_chunkset(cs)
    src = torch.from_numpy(host).to(DEV)
    w_ref, nd_ref, to_ref = zfpx.zfpx_plan_encode_var(plan, src, maxprec, minexp, cap)
    words = torch.full_like(w_ref, -1)
    nd = torch.full_like(nd_ref, 255)
    to = torch.full_like(to_ref, -1)
    L = zfpx.library()
    st = L.zfpx_plan_encode_var_noalloc(plan.handle, src.data_ptr(), src.numel(), maxprec, minexp,
                                        cap, words.data_ptr(), words.numel() * 4, nd.data_ptr(),
                                        to.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == 0, zfpx.zfpx_status_string(st)
    torch.cuda.synchronize()
    total = int(to_ref[-1].item())
    assert torch.equal(to, to_ref)
    assert torch.equal(nd[:plan.nblocks], nd_ref[:plan.nblocks])
    assert torch.equal(words[:total], w_ref[:total])
    return plan.nblocks


def test_noalloc_matches_workspace_form_twice(zfpx_lib):
    rng = np.random.default_rng(70)
    # first call: a ragged reduced-grid plan near the scratch limit at cap 16
    cs1 = W.reduced_grid_chunkset(n_half=160, nlev=140, nchunks=7)
    x1 = np.cumsum(rng.standard_normal(cs1.buffer_elems)).astype(np.float32)
    me = zfpx_lib.zfpx_accuracy_minexp(1e-3)
    nb1 = _pair(zfpx_lib, cs1, x1, 32, me, 16)
    # second call, smaller plan and other parameters: the scratch keeps the
    # first call's contents, which must not leak into the second stream
    cs2 = W.reduced_grid_chunkset(n_half=24, nlev=7, nchunks=5)
    x2 = (280 + 15 * rng.standard_normal(cs2.buffer_elems)).astype(np.float32)
    nb2 = _pair(zfpx_lib, cs2, x2, 12, zfpx_lib.MINEXP_NONE, 32)
    assert nb2 < nb1
    lim = zfpx_lib.zfpx_noalloc_scratch_bytes()
    assert lim == 32 << 20
    need1 = (((nb1 + 63) // 64) * 64 * 2 * 16 + (nb1 + 63) // 64) * 4
    assert need1 <= lim


def test_noalloc_rejects_plans_beyond_the_scratch(zfpx_lib):
    cs = W.reduced_grid_chunkset(n_half=320, nlev=40, nchunks=4)
    plan = zfpx_lib.Plan.from_chunkset(cs)
    need = (((plan.nblocks + 63) // 64) * 64 * 2 * 32 + (plan.nblocks + 63) // 64) * 4
    assert need > zfpx_lib.zfpx_noalloc_scratch_bytes()
    src = torch.zeros(cs.buffer_elems, device=DEV)
    mw, nt, _ = zfpx_lib.zfpx_plan_var_sizes(plan, 32)
    words = torch.empty(mw, dtype=torch.int32, device=DEV)
    nd = torch.empty(plan.nblocks, dtype=torch.uint8, device=DEV)
    to = torch.empty(nt + 1, dtype=torch.int64, device=DEV)
    with pytest.raises(zfpx_lib.ZfpxError) as e:
        zfpx_lib.zfpx_plan_encode_var_noalloc(plan, src, 32, zfpx_lib.MINEXP_NONE, 32, words, nd, to)
    assert e.value.status == zfpx_lib.ENOSPC
