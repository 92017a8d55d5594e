"""CPU model of one workgroup of the radix sort's downsweep (SortPairs, Sec. 3.2
stage 4), run with its four waves interleaved in chosen orders.

The kernel (paper_2409_08669_amd/csrc/sort.hip, downsweep_kernel) has three
steps per workgroup:
  1. each wave ranks its keys per digit (stable, per-wave counts in LDS);
  2. thread d turns the four waves' counts of digit d into per-wave offsets and,
     through a workgroup scan, into blk_start[d], the start of digit d's run in
     the workgroup's LDS order;
  3. every lane places its keys and values at blk_start[digit] + wave offset +
     rank, reading blk_start for digits that other waves own; then the scatter
     loop reads back every LDS slot below the workgroup's key count, and the
     last pass of the depth sort gathers gather_src[value].

Thread d belongs to wave d // 64, and blk_start[d] is written after the
scan's last barrier. Without a barrier between step 2's write and step 3, a
wave may place its keys while blk_start still holds what an earlier
workgroup left in LDS. The model shows that such an order (legal on the
hardware without that barrier) leaves LDS slots unwritten, so the scatter reads
stale values, and that stale contents left by the blend kernel's staging
(float bits) send the gather far outside its array; with the barrier every
order gives a permutation. CPU only."""
import numpy as np
import pytest

WAVES, LANES, ITEMS = 4, 64, 8
KEYS = WAVES * LANES * ITEMS  # 2048 keys per workgroup
RADIX = 256


def rank_per_wave(digits):
    """Step 1: per wave, the stable rank of each key among the wave's keys of
    its digit, and the wave's count per digit."""
    d = digits.reshape(WAVES, ITEMS, LANES)  # wave, row, lane (row-major within a wave)
    rank = np.zeros_like(d)
    wcnt = np.zeros((WAVES, RADIX), dtype=np.int64)
    for w in range(WAVES):
        for r in range(ITEMS):
            for lane in range(LANES):
                dig = d[w, r, lane]
                rank[w, r, lane] = wcnt[w, dig]
                wcnt[w, dig] += 1
    return rank, wcnt


def digit_starts(wcnt):
    """Step 2: per-wave offsets of each digit and the workgroup's digit starts."""
    wave_off = np.zeros_like(wcnt)
    wave_off[1:] = np.cumsum(wcnt, axis=0)[:-1]
    tot = wcnt.sum(axis=0)
    blk = np.concatenate([[0], np.cumsum(tot)[:-1]])
    return wave_off, blk


def run_workgroup(digits, values, schedule, stale_blk, stale_lds_vals):
    """Runs steps 2-3 in the given order of (wave, action) events, action
    'write' (the wave's threads store blk_start for their 64 digits) or 'place'
    (the wave's lanes place their keys). Returns the values the scatter loop
    reads from LDS slots [0, KEYS)."""
    rank, wcnt = rank_per_wave(digits)
    wave_off, blk_true = digit_starts(wcnt)
    blk_lds = stale_blk.copy()  # what LDS holds before this workgroup writes it
    svals = stale_lds_vals.copy()
    written = np.zeros(KEYS, dtype=bool)
    d = digits.reshape(WAVES, ITEMS, LANES)
    v = values.reshape(WAVES, ITEMS, LANES)
    for w, action in schedule:
        if action == "write":
            own = np.arange(w * LANES, (w + 1) * LANES)
            blk_lds[own] = blk_true[own]
        else:
            for r in range(ITEMS):
                for lane in range(LANES):
                    dig = d[w, r, lane]
                    pos = blk_lds[dig] + wave_off[w, dig] + rank[w, r, lane]
                    if 0 <= pos < svals.size:
                        svals[pos] = v[w, r, lane]
                        written[pos] = True
    return svals[:KEYS], written[:KEYS]


def _inputs(seed):
    rng = np.random.default_rng(seed)
    digits = rng.integers(0, RADIX, size=KEYS)
    n_gauss = 1_000_000
    values = rng.choice(n_gauss, size=KEYS, replace=False).astype(np.int64)
    # LDS left by an earlier workgroup: digit starts of another workgroup, and
    # the blend kernel's staged records (FP32 bits) where the values go
    stale_blk = np.concatenate([[0], np.cumsum(rng.multinomial(KEYS, np.ones(RADIX) / RADIX))[:-1]])
    stale_vals = rng.uniform(-8.0, 8.0, size=KEYS).astype(np.float32).view(np.uint32).astype(np.int64)
    return digits, values, n_gauss, stale_blk, stale_vals


def barrier_schedule(order):
    """With the barrier: every wave writes before any wave places."""
    return [(w, "write") for w in order] + [(w, "place") for w in order]


def racy_schedule():
    """Without the barrier: wave 0 finishes its scan, writes its 64 digit
    starts and places its keys before waves 1-3 have written theirs."""
    return [(0, "write"), (0, "place"), (1, "write"), (1, "place"), (2, "write"), (2, "place"),
            (3, "write"), (3, "place")]


@pytest.mark.parametrize("order", [(0, 1, 2, 3), (3, 2, 1, 0), (2, 0, 3, 1)])
@pytest.mark.parametrize("seed", [0, 1])
def test_with_the_barrier_every_order_places_a_permutation(order, seed):
    digits, values, _, stale_blk, stale_vals = _inputs(seed)
    svals, written = run_workgroup(digits, values, barrier_schedule(order), stale_blk, stale_vals)
    assert written.all()
    np.testing.assert_array_equal(np.sort(svals), np.sort(values))
    # and the order is the stable order by digit
    expect = values[np.argsort(digits, kind="stable")]
    np.testing.assert_array_equal(svals, expect)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_without_the_barrier_stale_values_reach_the_gather_out_of_bounds(seed):
    digits, values, n_gauss, stale_blk, stale_vals = _inputs(seed)
    svals, written = run_workgroup(digits, values, racy_schedule(), stale_blk, stale_vals)
    assert not written.all()  # slots the scatter loop reads that this workgroup never wrote
    stale_read = svals[~written]
    assert (stale_read >= n_gauss).any()  # gather_src[value] would read past tiles_touched's end
    assert int(stale_read.max()) * 4 > 2 ** 30  # by gigabytes: a GPU memory fault, not a wrong number
