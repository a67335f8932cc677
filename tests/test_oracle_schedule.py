"""Pin of the oracle's measurement schedule.

The contract: after sweep n (n = 0, 1, ...; n + 1 sweeps completed) the
overlap is measured iff measure_every = m > 0, n + 1 > measure_start and
(n + 1 - measure_start) is a multiple of m (the first half of a run
thermalizes, the second half measures: Table I caption).  So after n sweeps
exactly max(0, floor((n - start) / m)) measurements have been taken, they fall
at completed-sweep counts start + m, start + 2m, ..., and each one measures the
state right after its sweep.  Checked here sweep by sweep, under chunk splits,
from the accumulator count and from the recorded plane sums.
"""
import numpy as np
import pytest

from oracle import ea_oracle as O
from paper_1403_4560_amd import workload as W


def tiny_state(m, start, trace_cap=0, seed=1):
    work = W.make_workload([2], 3, (0.5, 2.0), 0.3, seed=seed, measure_every=m, measure_start=start)
    s = 0
    return O.SampleState(work.L[s], work.n_temps[s], work.beta_of(s), work.h[s], work.jkind, work.J_of(s),
                         work.spins0_of(s), work.seed, work.sample_id[s], m, start, O.MODE_MIRROR, trace_cap)


def expected_count(n, m, start):
    return 0 if m <= 0 or n <= start else (n - start) // m


@pytest.mark.parametrize("m,start", [(1, 0), (3, 0), (10, 5), (7, 13), (4, 4), (5, 1), (0, 0)])
def test_measurement_count_sweep_by_sweep(m, start):
    st = tiny_state(m, start)
    for n in range(1, 60):
        st.run(1)
        assert int(st.sweep[0]) == n
        assert np.all(st.acc[:, 0] == expected_count(n, m, start)), (n, st.acc[:, 0])


@pytest.mark.parametrize("m,start,chunks", [(10, 5, [3, 17, 1, 40]), (7, 13, [13, 1, 6, 30]),
                                            (4, 4, [4, 4, 4, 9])])
def test_measurement_count_under_chunk_splits(m, start, chunks):
    split = tiny_state(m, start)
    done = 0
    for c in chunks:
        split.run(c)
        done += c
        assert np.all(split.acc[:, 0] == expected_count(done, m, start))
    whole = tiny_state(m, start).run(done)
    assert np.array_equal(whole.acc, split.acc)
    assert np.array_equal(whole.spins, split.spins)


def test_each_measurement_sees_the_state_after_its_sweep():
    m, start = 3, 4
    st = tiny_state(m, start, trace_cap=64)
    seen = 0
    for n in range(1, 40):
        st.run(1)
        due = n > start and (n - start) % m == 0
        assert int(st.trace_len[0]) == seen + due, n
        if due:
            sp = st.spins_slot_order()
            for t in range(st.n_T):
                _, sums = O.measure_pair(st.L, sp[0, t], sp[1, t])
                assert np.array_equal(st.trace[seen, t], sums), (n, t)
            seen += 1
