"""Host emulation of the work queue of the persistent batched kernel (CPU).

raycast_batch (csrc/persist.h) keeps resident waves that each repeatedly
take w = atomicAdd(counter, 1) and leave the loop when (unsigned)w >= total;
batch_reset writes 0 to the counter on the same stream right before every
launch.  The emulation runs the waves in random interleavings with 32-bit
wrap-around arithmetic and checks that

  * with the reset, every work unit is taken exactly once and every wave
    leaves after total + n_waves fetches in all;
  * whatever value the counter starts from (memory reused from an earlier
    allocation and not cleared), every wave still leaves within
    total + n_waves fetches: a negative start compares as a huge unsigned
    value, so each wave leaves at its first fetch (an incomplete image, not
    a wave that keeps looping);
  * the same loop with a signed bound check would, from a negative start,
    fetch total - start times before the last wave left -- about 2^31 for a
    value near INT_MIN, which at microseconds per fetch is a kernel that
    runs for most of an hour without faulting.  The wrap-around count is
    checked exactly at a reduced 12-bit counter width.

This is the one way a queue loop of this form can run on for minutes
without a memory fault; it is why the counter is compared unsigned and
reset on the launch's own stream."""
import numpy as np
import pytest

INT_MIN, UINT_MASK = -(1 << 31), (1 << 32) - 1


def _wrap(v, bits=32):
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >= 1 << (bits - 1) else v


def run_queue(total, n_waves, start, rng, signed=False, bits=32, step_cap=None):
    """Emulate the loop; returns (units taken, fetches, waves that left)."""
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


@pytest.mark.parametrize("total,n_waves,seed", [(1, 1, 0), (5, 64, 1), (1000, 37, 2),
                                                (4096, 3072, 3)])
def test_reset_counter_takes_every_unit_once(total, n_waves, seed):
    rng = np.random.default_rng(seed)
    taken, fetches, left = run_queue(total, n_waves, 0, rng)
    assert sorted(taken) == list(range(total))
    assert left == n_waves and fetches == total + n_waves


@pytest.mark.parametrize("start", [INT_MIN, INT_MIN + 7, -1, -123456, 7, 999, 1000, 1 << 30,
                                   (1 << 31) - 1])
def test_unreset_counter_never_keeps_a_wave_looping(start):
    rng = np.random.default_rng(abs(start) % 1000)
    total, n_waves = 1000, 48
    taken, fetches, left = run_queue(total, n_waves, start, rng,
                                     step_cap=total + n_waves + 1)
    assert left == n_waves                      # every wave left the loop
    assert fetches <= total + n_waves
    assert all(0 <= w < total for w in taken)   # no out-of-range unit is rendered
    if start <= -n_waves or start >= total:
        # each wave's first fetch ends it; a start between -n_waves and 0
        # ends the first -start waves and lets the rest take every unit
        assert taken == [] and fetches == n_waves


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
