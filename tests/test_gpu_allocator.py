"""Device memory from a registered allocator (tgw_set_allocator).

A C allocator (the library's counting test allocator: hipMalloc / hipFree that
record every call) is registered; covariates, panel and plan made afterwards
must take all their device memory from it and give all of it back when freed,
and the scan's outputs must be bit for bit those of handles made with the
default allocator.  The same holds for tgw_arena over one torch tensor, the
way a torch program hands the library its memory.
"""
import ctypes
import gc

import numpy as np
import pytest
import torch

from synth import cohort_spec
from tests.gpu_common import cohort_arrays, lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tgw():
    t = lib()
    t.init()
    return t


def _run(tgw, C, Y, packed, precision):
    cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
    panel = tgw.prepare_phenotypes(cov, torch.from_numpy(Y).cuda(), precision)
    plan = tgw.Plan([panel], tile=0)
    outs = tgw.scan(plan, torch.from_numpy(packed).cuda())
    plan.check()
    return {k: v.cpu() for k, v in outs[0].items()}, (cov, panel, plan)


@pytest.mark.parametrize("precision", ["split8", "fp32"])
def test_registered_allocator_supplies_all_handle_memory(tgw, precision):
    spec = cohort_spec("cfg1", n_markers=1500)
    _, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    say(f"case: counting allocator {precision}")
    want, handles = _run(tgw, C, Y, packed, precision)
    del handles
    gc.collect()

    counts = tgw.AllocCounts()
    fa, ff = tgw.debug_counting_allocator()
    tgw.set_allocator(fa, ff, ctypes.byref(counts))
    try:
        got, handles = _run(tgw, C, Y, packed, precision)
    finally:
        tgw.set_allocator()  # handles made from here on use hipMalloc again
    n_alloc, nbytes = counts.n_alloc, counts.bytes
    say(f"{n_alloc} allocations, {nbytes} bytes, {counts.n_free} freed so far")
    # the covariate fit and the panel preparation free their temporaries at once
    assert counts.n_free >= 5
    # every handle buffer came from the allocator: at least the panel operand
    n, p = spec.n_samples, Y.shape[1]
    op_bytes = ((p + 31) // 32) * ((n + 63) // 64) * (6144 if precision == "split8" else 8192)
    assert nbytes >= op_bytes + 8 * ((n + 63) // 64) * 64 * (C.shape[1] + 1)
    for k in want:
        assert torch.equal(want[k].view(torch.int32), got[k].view(torch.int32)), k
    del handles
    gc.collect()
    assert counts.n_free == counts.n_alloc == n_alloc, (counts.n_free, counts.n_alloc)


def test_torch_tensor_arena(tgw):
    """Handles made under an arena over one torch allocation live inside it;
    outputs equal the default allocator's bit for bit; everything comes back."""
    spec = cohort_spec("cfg1", n_markers=1500)
    _, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    say("case: torch tensor arena, split8")
    want, handles = _run(tgw, C, Y, packed, "split8")
    del handles
    gc.collect()

    arena = tgw.torch_arena(256 << 20)
    lo = arena.buffer.data_ptr()
    hi = lo + arena.buffer.numel()
    arena.register()
    try:
        got, handles = _run(tgw, C, Y, packed, "split8")
    finally:
        tgw.set_allocator()
    st = arena.info()
    say(f"arena: {st.n_blocks} blocks, {st.in_use} bytes in use, peak {st.peak}")
    assert st.n_blocks >= 8 and st.in_use > 0 and st.n_failed == 0 and st.n_bad_free == 0
    cov, panel, plan = handles
    # the resident panel operand and covariate basis are inside the arena
    n, p = spec.n_samples, Y.shape[1]
    op_bytes = ((p + 31) // 32) * ((n + 63) // 64) * 6144
    assert st.in_use >= op_bytes + 8 * ((n + 63) // 64) * 64 * (C.shape[1] + 1)
    assert st.in_use + st.largest_free <= hi - lo
    for k in want:
        assert torch.equal(want[k].view(torch.int32), got[k].view(torch.int32)), k
    with pytest.raises(tgw.TgwError):
        arena.close()  # handles still alive
    del handles, cov, panel, plan
    gc.collect()
    st = arena.info()
    assert (st.in_use, st.n_blocks, st.n_free_ranges, st.n_bad_free) == (0, 0, 1, 0)
    arena.close()


def test_arena_too_small_fails_cleanly(tgw):
    """A request the arena cannot hold fails the call with TGW_ERR_OUT_OF_MEMORY and
    leaves nothing allocated."""
    spec = cohort_spec("cfg1", n_markers=100)
    _, packed, C, Y = cohort_arrays(spec, np.arange(spec.n_markers))
    say("case: arena too small for the panel")
    arena = tgw.torch_arena(4 << 20).register()
    try:
        cov = tgw.fit_covariates(torch.from_numpy(C).cuda())
        with pytest.raises(tgw.TgwError) as ei:
            tgw.prepare_phenotypes(cov, torch.from_numpy(np.repeat(Y, 64, axis=1)).cuda(), "split8")
        assert ei.value.status == tgw.ERR_OUT_OF_MEMORY
    finally:
        tgw.set_allocator()
    assert arena.info().n_failed >= 1
    del cov, ei  # the exception's traceback holds the covariates handle too
    gc.collect()
    st = arena.info()
    assert (st.in_use, st.n_blocks) == (0, 0)
    arena.close()
