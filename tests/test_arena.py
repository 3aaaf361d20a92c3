"""tgw_arena, the allocator over one caller-owned device buffer, on the host.

The arena keeps its bookkeeping on the host and never touches the buffer, so
its placement can be checked without a GPU at a made-up base address: every
block lies inside the buffer, 256-byte aligned, and no two live blocks
overlap; placement is best fit (smallest free range that holds the request,
lowest address among equals), checked against an independent model of the
free ranges; freed ranges merge, so the whole buffer is one range again when
everything is freed; refused requests and stray frees are counted.
"""
import ctypes

import numpy as np
import pytest

BASE = 0x7F0000000000  # a made-up device address, 256-byte aligned
GRAIN = 256


@pytest.fixture(scope="module")
def tgw():
    from paper_2604_21095_amd import tgw as t
    return t


def _round(n):
    return GRAIN if n == 0 else -(-n // GRAIN) * GRAIN


class Model:
    """Free ranges as a sorted list of (offset, length); best fit by scanning."""

    def __init__(self, cap):
        self.free = [(0, cap)]
        self.used = {}

    def alloc(self, n):
        need = _round(n)
        fits = [(ln, off) for off, ln in self.free if ln >= need]
        if not fits:
            return None
        ln, off = min(fits)
        self.free.remove((off, ln))
        if ln > need:
            self.free.append((off + need, ln - need))
        self.free.sort()
        self.used[off] = need
        return off

    def release(self, off):
        ln = self.used.pop(off)
        self.free.append((off, ln))
        self.free.sort()
        merged = []
        for o, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self.free = merged


def test_create_validation(tgw):
    h = ctypes.c_void_p()
    assert tgw._arena_create(None, 1 << 20, ctypes.byref(h)) == tgw.ERR_INVALID_ARG
    assert tgw._arena_create(BASE, 1 << 20, None) == tgw.ERR_INVALID_ARG
    assert tgw._arena_create(BASE + 128, 1 << 20, ctypes.byref(h)) == tgw.ERR_SHAPE
    assert tgw._arena_create(BASE, 255, ctypes.byref(h)) == tgw.ERR_SHAPE
    assert tgw._arena_destroy(None) == tgw.OK
    # capacity rounds down to the grain
    a = tgw.Arena(BASE, 1000)
    st = a.info()
    assert (st.capacity, st.in_use, st.largest_free, st.n_free_ranges) == (768, 0, 768, 1)
    a.close()


def test_blocks_aligned_inside_and_merged(tgw):
    cap = 1 << 20
    a = tgw.Arena(BASE, cap)
    sizes = [1, 255, 256, 257, 4096, 0, 100_000]
    ptrs = [a.alloc(n) for n in sizes]
    assert all(p % GRAIN == 0 and BASE <= p and p + _round(n) <= BASE + cap for p, n in zip(ptrs, sizes))
    # the first requests pack from the bottom of the single free range
    assert ptrs[:4] == [BASE, BASE + 256, BASE + 512, BASE + 768]
    st = a.info()
    assert st.in_use == sum(_round(n) for n in sizes) and st.n_blocks == len(sizes)
    with pytest.raises(tgw.TgwError):
        a.close()  # blocks still in use
    for p in ptrs[::2] + ptrs[1::2]:
        a.free(p)
    st = a.info()
    assert (st.in_use, st.n_blocks, st.n_free_ranges, st.largest_free) == (0, 0, 1, cap)
    assert st.peak == sum(_round(n) for n in sizes)
    a.close()


def test_refusals_and_stray_frees_are_counted(tgw):
    a = tgw.Arena(BASE, 4096)
    p = a.alloc(4096)
    assert p == BASE
    assert a.alloc(1) == 0 and a.alloc(1 << 40) == 0
    a.free(BASE + 256)      # inside a block but not its start
    a.free(BASE - 4096)     # below the buffer
    a.free(p)
    a.free(p)               # twice
    a.free(0)               # NULL: ignored, not counted
    st = a.info()
    assert (st.n_failed, st.n_bad_free, st.in_use, st.largest_free) == (2, 3, 0, 4096)
    a.close()


def test_best_fit_against_a_model(tgw):
    rng = np.random.default_rng(5)
    cap = 64 << 20
    a = tgw.Arena(BASE, cap)
    m = Model(cap)
    live = []
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = live.pop(int(rng.integers(len(live))))
            a.free(BASE + off)
            m.release(off)
        else:
            n = int(rng.choice([rng.integers(0, 2048), rng.integers(0, 1 << 20), rng.integers(0, 8 << 20)]))
            p = a.alloc(n)
            off = m.alloc(n)
            if off is None:
                assert p == 0, step
            else:
                assert p == BASE + off, (step, n)
                live.append(off)
        if step % 100 == 0:
            st = a.info()
            assert st.in_use == sum(m.used.values())
            assert st.n_free_ranges == len(m.free)
            assert st.largest_free == max((ln for _, ln in m.free), default=0)
    # live blocks never overlap and stay inside the buffer
    spans = sorted((off, off + m.used[off]) for off in live)
    assert all(e0 <= s1 for (_, e0), (s1, _) in zip(spans, spans[1:]))
    assert not spans or spans[-1][1] <= cap
    for off in live:
        a.free(BASE + off)
    st = a.info()
    assert (st.in_use, st.n_free_ranges, st.largest_free, st.n_bad_free) == (0, 1, cap, 0)
    a.close()


def test_arena_as_registered_allocator(tgw):
    """The arena's functions are accepted by the allocator hook (no handle is made here)."""
    a = tgw.Arena(BASE, 1 << 20)
    assert tgw._set_allocator(*a.functions) == tgw.OK
    assert tgw._set_allocator(None, None, None) == tgw.OK
    a.close()
