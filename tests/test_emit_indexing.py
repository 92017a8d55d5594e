"""Host-side check of the index arithmetic that DuplicateWithKeys relies on
(Sec. 3.2, stage 3): the inclusive scan records, per chunk of kDupPairs
pairs, the first Gaussian holding one of its pairs, and each emit workgroup
searches its pairs' Gaussians between that chunk start and the next one.

The model below restates, in numpy, which chunk starts the scan writes and
which window of offsets each workgroup loads, and checks on edge-case
tiles_touched arrays that every write and read stays inside its buffer and
that the window always holds the Gaussians of the workgroup's first and last
pair. No GPU is used."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dup_pairs():
    """The chunk size, read from the library's internal header."""
    with open(os.path.join(ROOT, "paper_2409_08669_amd", "csrc", "adr_internal.h")) as f:
        m = re.search(r"constexpr int kDupPairs = (\d+);", f.read())
    assert m, "kDupPairs not found in adr_internal.h"
    return int(m.group(1))


def check_emit_indexing(touched, K):
    touched = np.asarray(touched, dtype=np.int64)
    assert touched.size > 0 and (touched > 0).all()  # visible Gaussians hold at least one pair
    n_vis = touched.size
    offsets = np.cumsum(touched)  # inclusive
    total = int(offsets[-1])
    grid = (total + K - 1) // K  # duplicate_blocks
    capacity = grid + 1  # words the workspace holds for the chunk starts

    # scan: Gaussian i writes every chunk c with c * K in [before, run)
    dup_first = np.full(capacity, -1, dtype=np.int64)
    writers = np.zeros(capacity, dtype=np.int64)
    before = offsets - touched
    c_lo = (before + K - 1) // K
    c_hi = (offsets + K - 1) // K  # exclusive: c * K < run
    for i in np.nonzero(c_hi > c_lo)[0]:
        assert c_hi[i] <= capacity, "chunk-start write past the buffer"
        dup_first[c_lo[i]:c_hi[i]] = i
        writers[c_lo[i]:c_hi[i]] += 1
    # one writer per chunk (the scan's threads write in no set order), and
    # exactly the chunks the emit reads
    assert (writers[:grid] == 1).all() and (writers[grid:] == 0).all(), "chunk start written twice or not at all"

    # emit: workgroup b covers pairs [b*K, min(b*K + K, total))
    holder = lambda p: int(np.searchsorted(offsets, p, side="right"))  # Gaussian holding pair p
    for b in range(grid):
        p0, p1 = b * K, min(b * K + K, total) - 1
        r_lo = min(int(dup_first[b]), n_vis - 1)
        r_hi = min(int(dup_first[b + 1]), n_vis - 1) if b + 1 < grid else n_vis - 1
        cnt = min(r_hi - r_lo + 1 if r_hi >= r_lo else 1, K + 1)
        assert 0 <= r_lo and r_lo + cnt - 1 <= n_vis - 1, "offsets window outside the visible list"
        assert holder(p0) == r_lo, "window does not start at the Gaussian holding the first pair"
        assert r_lo <= holder(p1) <= r_lo + cnt - 1, "Gaussian holding the last pair outside the window"
    return grid


@pytest.fixture(scope="module")
def K():
    return dup_pairs()


def test_single_gaussians(K):
    for t in (1, K - 1, K, K + 1, 5 * K, 5 * K + 7):
        check_emit_indexing([t], K)


def test_one_pair_each_fills_the_window_exactly(K):
    # every chunk holds K Gaussians, and the next chunk's first one makes K + 1
    for n in (K, 3 * K, 3 * K + 1, 3 * K - 1):
        check_emit_indexing(np.ones(n, dtype=np.int64), K)


def test_chunk_boundaries_on_gaussian_boundaries(K):
    check_emit_indexing([K] * 4, K)
    check_emit_indexing([K // 2] * 8, K)
    check_emit_indexing([K - 1, 1] * 3, K)


def test_heavy_tailed_random_lists(K):
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = int(rng.integers(1, 40_000))
        t = np.minimum(rng.zipf(1.6, size=n), 20 * K).astype(np.int64)
        check_emit_indexing(t, K)


def test_small_random_lists(K):
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(1, 64))
        t = rng.integers(1, 3 * K, size=n)
        check_emit_indexing(t, K)
