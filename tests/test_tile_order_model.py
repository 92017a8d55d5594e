"""CPU model of the tile render order (the first part of Render, Sec. 3.2 stage
6, and the load imbalance of Sec. 4.4): order_count_kernel and
order_scatter_kernel in paper_2409_08669_amd/csrc/render.hip.

The kernels sort the tiles by floor(log2(list length)), longest bucket first
(empty tiles last). One workgroup scans one 16 x 16 superblock of tiles
(superblocks row by row, tiles row-major inside), so ranks inside a bucket
follow that scan. The render's workgroup at position p runs on XCD p mod 8,
and a bucket's ranks are dealt to the XCDs in contiguous runs: the k-th run
takes the bucket's positions p with p mod 8 = k, in increasing order.

The model restates that arithmetic and checks, on grids from one tile to the
73,728 tiles of the largest test frame, that the order is a permutation of
the tiles, that buckets come longest first, that every XCD receives
consecutive ranks of each bucket and at most one more tile of it than any
other XCD, and that the count scratch the library reserves holds every
superblock. CPU only."""
import numpy as np
import pytest

XCDS, SUPER, BUCKETS = 8, 16, 33


def bucket(length):
    return BUCKETS - 1 if length == 0 else (BUCKETS - 2) - (int(length).bit_length() - 1)


def xcd_position(b0, n, r):
    start = 0
    for k in range(XCDS):
        first = b0 + (k + XCDS - b0 % XCDS) % XCDS
        cnt = (b0 + n - first + XCDS - 1) // XCDS if first < b0 + n else 0
        if r < start + cnt:
            return first + XCDS * (r - start)
        start += cnt
    raise AssertionError("rank beyond the bucket")


def superblocks(tx, ty):
    nsx, nsy = -(-tx // SUPER), -(-ty // SUPER)
    for blk in range(nsx * nsy):
        tiles = []
        for th in range(SUPER * SUPER):
            x, y = (blk % nsx) * SUPER + th % SUPER, (blk // nsx) * SUPER + th // SUPER
            if x < tx and y < ty:
                tiles.append(y * tx + x)
        yield tiles


def tile_order(tx, ty, lengths):
    blocks = list(superblocks(tx, ty))
    total = np.zeros(BUCKETS, np.int64)
    for tiles in blocks:
        for t in tiles:
            total[bucket(lengths[t])] += 1
    base = np.concatenate([[0], np.cumsum(total)[:-1]])
    seen = np.zeros(BUCKETS, np.int64)
    order = -np.ones(tx * ty, np.int64)
    rank = {}
    for tiles in blocks:
        for t in tiles:
            b = bucket(lengths[t])
            r = seen[b]
            seen[b] += 1
            p = xcd_position(int(base[b]), int(total[b]), int(r))
            assert order[p] == -1, "two tiles at one position"
            order[p] = t
            rank[t] = r
    return order, base, total, rank, len(blocks)


@pytest.mark.parametrize("tx,ty", [(1, 1), (1, 300), (300, 1), (7, 5), (17, 17), (33, 70), (120, 68),
                                   (240, 135), (384, 192)])
def test_order_is_longest_first_and_xcd_contiguous(tx, ty):
    rng = np.random.default_rng(tx * 1000 + ty)
    n = tx * ty
    lengths = rng.integers(0, 5000, n) * (rng.random(n) < 0.8)
    order, base, total, rank, n_blocks = tile_order(tx, ty, lengths)
    assert sorted(order.tolist()) == list(range(n))
    buckets = np.array([bucket(lengths[t]) for t in order])
    assert (np.diff(buckets) >= 0).all()
    for b in range(BUCKETS):
        per_xcd = []
        for k in range(XCDS):
            ranks = [rank[order[p]] for p in range(base[b], base[b] + total[b]) if p % XCDS == k]
            assert ranks == list(range(ranks[0], ranks[0] + len(ranks))) if ranks else True
            per_xcd.append(len(ranks))
        assert max(per_xcd) - min(per_xcd) <= 1
    # the library reserves 33 words per superblock for n // 256 + n // 16 + 2 superblocks
    assert n_blocks <= n // 256 + n // 16 + 2


def test_position_map_is_a_bijection_for_every_offset():
    for b0 in range(0, 24):
        for n in range(0, 40):
            pos = sorted(xcd_position(b0, n, r) for r in range(n))
            assert pos == list(range(b0, b0 + n))
