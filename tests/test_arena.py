"""CPU: the served loop's device-memory arena (host logic, csrc/arena.h).

The arena is driven through a host-only probe over random sequences of
placements and releases and checked against what first-fit placement with
merged free extents means: every block lies inside the arena on a 4 KiB
granule and overlaps no other live block; a placement takes the lowest free
extent that holds it (an interval model of the free space decides which, or
that none does); the free extents never touch one another; used bytes equal
the rounded sizes of the live blocks and used plus free equals the arena;
peak is the largest used so far; releasing everything leaves one extent.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GRAIN = 4096


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    so = str(tmp_path_factory.mktemp("arena") / "libarena_probe.so")
    subprocess.run([gxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Werror", "-o", so,
                    os.path.join(HERE, "arena_probe.cpp")], check=True, timeout=300)
    L = ctypes.CDLL(so)
    L.arena_new.restype = ctypes.c_void_p
    L.arena_new.argtypes = [ctypes.c_size_t]
    L.arena_delete.argtypes = [ctypes.c_void_p]
    L.arena_take.restype = ctypes.c_int64
    L.arena_take.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    L.arena_give.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t]
    L.arena_used.restype = ctypes.c_size_t
    L.arena_used.argtypes = [ctypes.c_void_p]
    L.arena_peak.restype = ctypes.c_size_t
    L.arena_peak.argtypes = [ctypes.c_void_p]
    L.arena_free_extents.restype = ctypes.c_int
    L.arena_free_extents.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_int]
    return L


def _extents(L, h):
    off = (ctypes.c_int64 * 4096)()
    ln = (ctypes.c_int64 * 4096)()
    k = L.arena_free_extents(h, off, ln, 4096)
    assert k <= 4096
    return [(off[i], ln[i]) for i in range(k)]


def _rounded(n):
    return (n + GRAIN - 1) // GRAIN * GRAIN


def _model_take(free, need):
    """Lowest free extent that holds `need` bytes: its offset, or -1."""
    for off, ln in free:
        if ln >= need:
            return off
    return -1


@pytest.mark.parametrize("seed,size_pages,max_bytes", [(1, 256, 64 * 1024), (2, 64, 16 * 1024), (3, 1024, 600 * 1024)])
def test_arena_first_fit_with_merged_free_extents(probe, seed, size_pages, max_bytes):
    L = probe
    size = size_pages * GRAIN
    h = L.arena_new(size)
    rng = np.random.default_rng(seed)
    live = {}  # offset -> requested bytes
    peak = 0
    try:
        for step in range(3000):
            if live and (rng.random() < 0.45 or len(live) > 200):
                off = int(rng.choice(list(live)))
                L.arena_give(h, off, live.pop(off))
            else:
                n = int(rng.integers(1, max_bytes + 1))
                free = _extents(L, h)
                expect = _model_take(free, _rounded(n))
                got = L.arena_take(h, n)
                assert got == expect, (step, n, got, expect)
                if got >= 0:
                    live[got] = n
            free = _extents(L, h)
            used = sum(_rounded(n) for n in live.values())
            peak = max(peak, used)
            assert L.arena_used(h) == used and L.arena_peak(h) == peak
            assert used + sum(ln for _, ln in free) == size
            # live blocks: on the granule, inside the arena, disjoint
            spans = sorted((o, o + _rounded(n)) for o, n in live.items())
            assert all(o % GRAIN == 0 and 0 <= o and e <= size for o, e in spans)
            assert all(spans[i][1] <= spans[i + 1][0] for i in range(len(spans) - 1))
            # free extents: sorted, granular, merged (no two touch), disjoint from live blocks
            assert all(o % GRAIN == 0 and ln > 0 and ln % GRAIN == 0 for o, ln in free)
            assert all(free[i][0] + free[i][1] < free[i + 1][0] for i in range(len(free) - 1))
            cover = sorted(spans + [(o, o + ln) for o, ln in free])
            assert cover[0][0] == 0 and cover[-1][1] == size
            assert all(cover[i][1] == cover[i + 1][0] for i in range(len(cover) - 1))
        for off, n in list(live.items()):
            L.arena_give(h, off, n)
        assert _extents(L, h) == [(0, size)] and L.arena_used(h) == 0
    finally:
        L.arena_delete(h)


def test_arena_refuses_what_no_extent_holds(probe):
    """A request larger than every free extent fails even when the free
    total would hold it (no compaction), and succeeds once a neighbour's
    release merges two extents."""
    L = probe
    h = L.arena_new(8 * GRAIN)
    try:
        blocks = [L.arena_take(h, GRAIN) for _ in range(8)]
        assert blocks == [i * GRAIN for i in range(8)] and L.arena_take(h, 1) == -1
        L.arena_give(h, 2 * GRAIN, GRAIN)
        L.arena_give(h, 5 * GRAIN, GRAIN)
        assert L.arena_take(h, 2 * GRAIN) == -1  # two free pages, not adjacent
        L.arena_give(h, 3 * GRAIN, GRAIN)
        assert _extents(L, h) == [(2 * GRAIN, 2 * GRAIN), (5 * GRAIN, GRAIN)]
        assert L.arena_take(h, GRAIN + 1) == 2 * GRAIN  # rounds up to two pages
        assert L.arena_peak(h) == 8 * GRAIN
    finally:
        L.arena_delete(h)
