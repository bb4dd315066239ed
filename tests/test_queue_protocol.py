"""Host emulation of the work queues of the persistent batched kernel (CPU).

raycast_batch (csrc/persist.h) keeps resident waves that take work units
from eight queues, one per XCD.  The launch's units are cut into groups of
8 consecutive tiles dealt round-robin to the queues; entry i of queue q is
unit ((i // 8) * 8 + q) * 8 + i % 8.  A wave fetches i = atomicAdd(
counter[q], 1) from the queue of its own XCD, leaves that queue when the
unit of (unsigned)i lies beyond the launch, then does the same with the
other seven in turn (skipping a queue whose counter it reads as already
beyond the launch), and leaves the kernel after the eighth.  batch_reset
writes 0 to all eight counters on the same stream right before every
launch.  The emulation runs the waves in random interleavings with 32-bit
wrap-around counters and checks that

  * the queue entries cover every unit exactly once, each queue in
    increasing order (so the first entry beyond the launch empties it);
  * with the reset, every unit is taken exactly once and every wave leaves
    after at most total + 8 n_waves fetches in all (at most one empty fetch
    per queue per wave);
  * whatever values the counters start from (memory reused from an earlier
    allocation and not cleared), every wave still leaves within
    total + 8 n_waves fetches and no unit outside the launch is rendered: a
    negative start is a huge unsigned index, an empty queue.

The single-counter form of the same loop shows why the comparison is
unsigned: with a signed bound check a stale negative counter would be
fetched total - start times before the last wave left -- about 2^31 for a
value near INT_MIN, which at microseconds per fetch is a kernel that runs
for most of an hour without faulting (checked exactly at a reduced 12-bit
counter width).  That is the one way a queue loop of this form can run on
for minutes without a memory fault."""
import numpy as np
import pytest

INT_MIN = -(1 << 31)
QUEUES, GROUP = 8, 8


def _wrap(v, bits=32):
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >= 1 << (bits - 1) else v


def queue_unit(q, i):
    return ((i // GROUP) * QUEUES + q) * GROUP + i % GROUP


def run_queues(total, n_waves, starts, rng, step_cap=None):
    """Emulate the eight-queue loop; returns (units taken, fetches, waves that left)."""
    counters = [_wrap(s) for s in starts]
    own = rng.integers(0, QUEUES, n_waves)
    stage = [0] * n_waves                       # queues this wave has found empty
    live = list(range(n_waves))
    taken, fetches = [], 0
    while live:
        if step_cap is not None and fetches >= step_cap:
            break
        wv = live[rng.integers(len(live))]
        q = (own[wv] + stage[wv]) % QUEUES
        if stage[wv] > 0 and queue_unit(q, counters[q] & 0xFFFFFFFF) >= total:
            # another XCD's queue read as empty: skipped without a fetch
            stage[wv] += 1
            if stage[wv] == QUEUES:
                live.remove(wv)
            continue
        i = counters[q]
        counters[q] = _wrap(i + 1)
        fetches += 1
        u = queue_unit(q, i & 0xFFFFFFFF)
        if u >= total:
            stage[wv] += 1
            if stage[wv] == QUEUES:
                live.remove(wv)
        else:
            taken.append(u)
    return taken, fetches, n_waves - len(live)


def run_queue(total, n_waves, start, rng, signed=False, bits=32, step_cap=None):
    """The single-counter loop; returns (units taken, fetches, waves that left)."""
    counter = _wrap(start, bits)
    live = list(range(n_waves))
    taken, fetches = [], 0
    while live:
        if step_cap is not None and fetches >= step_cap:
            break
        wv = live[rng.integers(len(live))]
        w = counter
        counter = _wrap(counter + 1, bits)
        fetches += 1
        done = (w >= total) if signed else ((w & ((1 << bits) - 1)) >= total)
        if done:
            live.remove(wv)
        elif 0 <= w < total:
            taken.append(w)
    return taken, fetches, n_waves - len(live)


def test_queue_entries_cover_every_unit_once_in_order():
    n = 5000
    units = []
    for q in range(QUEUES):
        col = [queue_unit(q, i) for i in range(n // QUEUES + GROUP)]
        assert all(b > a for a, b in zip(col, col[1:]))           # increasing in i
        assert all((u // GROUP) % QUEUES == q for u in col)       # the queue's own groups
        units += [u for u in col if u < n]
    assert sorted(units) == list(range(n))
    # a queue entry for any 32-bit index stays a valid (64-bit) unit number
    assert queue_unit(QUEUES - 1, 0xFFFFFFFF) < 1 << 40


@pytest.mark.parametrize("total,n_waves,seed", [(1, 1, 0), (5, 64, 1), (1000, 37, 2),
                                                (4099, 300, 3)])
def test_reset_queues_take_every_unit_once(total, n_waves, seed):
    rng = np.random.default_rng(seed)
    taken, fetches, left = run_queues(total, n_waves, [0] * QUEUES, rng)
    assert sorted(taken) == list(range(total))
    assert left == n_waves and total + n_waves <= fetches <= total + QUEUES * n_waves


@pytest.mark.parametrize("seed", range(6))
def test_unreset_queues_never_keep_a_wave_looping(seed):
    rng = np.random.default_rng(100 + seed)
    total, n_waves = 1000, 48
    pool = [INT_MIN, INT_MIN + 7, -1, -123456, 0, 7, 999, 1000, 1 << 30, (1 << 31) - 1]
    starts = [pool[j] for j in rng.integers(0, len(pool), QUEUES)]
    taken, fetches, left = run_queues(total, n_waves, starts, rng,
                                      step_cap=total + QUEUES * n_waves + 1)
    assert left == n_waves                      # every wave left the loop
    assert fetches <= total + QUEUES * n_waves
    assert len(set(taken)) == len(taken)        # no unit twice
    assert all(0 <= u < total for u in taken)   # no unit outside the launch


@pytest.mark.parametrize("start", [-2048, -1500, -1])
def test_signed_bound_from_a_stale_negative_counter_loops_for_long(start):
    # 12-bit counters: the signed loop takes total - start fetches before the
    # last wave leaves (the 32-bit analogue near INT_MIN is about 2^31)
    rng = np.random.default_rng(-start)
    total, n_waves, bits = 100, 8, 12
    _, fetches, left = run_queue(total, n_waves, start, rng, signed=True, bits=bits)
    assert left == n_waves
    assert fetches == total - start + n_waves
    # the unsigned check from the same start: bounded by total + n_waves,
    # and at once (one fetch per wave) when start <= -n_waves
    _, f_u, _ = run_queue(total, n_waves, start, rng, signed=False, bits=bits)
    assert f_u <= total + n_waves
    if start <= -n_waves:
        assert f_u == n_waves
