"""The serving loop's admission rule (HBM footprint) on a fake executor: the host-only
simulation runs the same admission code as refeig_server (no GPU needed)."""
import numpy as np
import pytest

MiB = 1 << 20


def _sim(arr, nbytes, dur, lanes, budget):
    from paper_2602_19090_amd import binding as rb
    st, ts, off = rb.host_admission_sim(arr, nbytes, dur, lanes, budget)
    assert st == 0
    return ts, off


def test_budget_below_one_footprint():
    ts, _ = _sim([0.0, 0.0, 1.0], [10 * MiB, 200 * MiB, 10 * MiB], [1.0, 1.0, 1.0], 4, 100 * MiB)
    assert ts[1] == -1.0                  # never fits: never starts
    assert ts[0] == 0.0 and ts[2] == 1.0  # the others run


def test_lanes_bound_concurrency():
    ts, _ = _sim([0, 0, 0], [MiB] * 3, [2.0, 1.0, 1.0], 2, 100 * MiB)
    assert list(ts) == [0.0, 0.0, 1.0]


def test_memory_bounds_concurrency():
    # two 60 MiB requests in 100 MiB: the second starts when the first frees its memory
    ts, off = _sim([0, 0], [60 * MiB, 60 * MiB], [3.0, 1.0], 8, 100 * MiB)
    assert list(ts) == [0.0, 3.0]
    assert list(off) == [0, 0]


def test_small_requests_pass_a_waiting_large_one_at_most_four_times():
    # a 70 MiB request runs; a second 70 MiB one waits for memory; 10 MiB ones behind it
    # start at once, but only four of them: the fifth waits until the large one has started
    arr = [0.0, 0.1] + [0.2 + 0.01 * k for k in range(6)]
    nb = [70 * MiB, 70 * MiB] + [10 * MiB] * 6
    dur = [5.0, 1.0] + [0.05] * 6
    ts, _ = _sim(arr, nb, dur, 8, 110 * MiB)
    assert ts[0] == 0.0 and ts[1] == 5.0
    assert all(ts[2 + k] == arr[2 + k] for k in range(4))
    assert ts[6] >= 5.0 and ts[7] >= 5.0


def test_first_fit_offsets_and_reuse():
    ts, off = _sim([0, 0, 0, 1.5], [30 * MiB, 30 * MiB, 30 * MiB, 50 * MiB], [1.0, 2.0, 3.0, 1.0],
                   4, 100 * MiB)
    assert list(off[:3]) == [0, 30 * MiB, 60 * MiB]
    # at 1.5 s only the first block is free (30 MiB): the 50 MiB request waits for 2.0 s,
    # when 0..60 MiB is one free run again
    assert ts[3] == 2.0 and off[3] == 0


@pytest.mark.parametrize("seed", range(6))
def test_invariants_random_fake_executor(seed):
    rng = np.random.default_rng(seed)
    m = 300
    arr = np.cumsum(rng.exponential(0.01, m))
    nb = (np.exp(rng.uniform(np.log(1), np.log(120), m)) * MiB).astype(np.uint64)
    dur = rng.exponential(0.05, m)
    budget, lanes = 160 * MiB, 4
    ts, off = _sim(arr, nb, dur, lanes, budget)
    nb = (nb + 255) // 256 * 256
    assert np.all((ts == -1.0) == (nb > budget))
    ok = ts >= 0
    assert np.all(ts[ok] >= arr[ok])
    ev = sorted([(ts[i], 1, i) for i in np.nonzero(ok)[0]] +
                [(ts[i] + dur[i], 0, i) for i in np.nonzero(ok)[0]])
    running = set()
    for t, kind, i in ev:
        if kind == 0:
            running.discard(i)
            continue
        running.add(i)
        assert len(running) <= lanes
        spans = sorted((int(off[j]), int(off[j] + nb[j])) for j in running)
        assert spans[-1][1] <= budget
        assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))   # no overlap
