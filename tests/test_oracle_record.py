"""Pins of the oracle's event record (the switching-time output of Sec. 4.3's
dwell-time analysis): the record is consistent with the trajectory it logs,
and the gene's dwell times follow the exponential laws of the two-state
promoter (OFF dwell ~ Exp(k_on), ON dwell ~ Exp(k_off))."""
import numpy as np
import pytest
from scipy import stats

from paper_2605_00479_amd import workloads as wl

THREADS = 8


@pytest.mark.parametrize("mode", ["FP64", "MIX_F16_SR", "UNI_BF16_SR_NORM"])
def test_full_record_replays_the_trajectory(orc, mode):
    # every reaction recorded: the log has one entry per event, non-decreasing
    # times ending at t_last, and replaying its reactions from x0 gives the
    # final state
    m = wl.telegraph(0.05, 0.05, 20.0, 1.0)
    x0 = np.array([1, 0, 0], np.int32)
    r = orc.simulate(m, mode, x0, 30.0, [30.0], 3, n_traj=40, record_mask=(1 << m.n_reactions) - 1,
                     record_cap=4000, threads=THREADS)
    nu = np.asarray(m.nu, np.int64).reshape(m.n_reactions, m.n_species)
    for i in range(40):
        n = int(r["n_events"][i])
        assert r["rec_n"][i] == n and n < 4000
        t = r["rec_t"][i, :n]
        assert np.all(np.diff(t) >= 0)
        if n:
            assert t[-1] == r["t_last"][i]
        final = x0 + nu[r["rec_j"][i, :n]].sum(axis=0)
        np.testing.assert_array_equal(final, r["snap"][-1, :, i])


def test_record_keeps_the_prefix_and_counts_all(orc):
    m = wl.telegraph(0.05, 0.05, 20.0, 1.0)
    x0 = np.array([1, 0, 0], np.int32)
    full = orc.simulate(m, "FP64", x0, 200.0, [200.0], 5, n_traj=30, record_mask=0b11, record_cap=100,
                        threads=THREADS)
    cut = orc.simulate(m, "FP64", x0, 200.0, [200.0], 5, n_traj=30, record_mask=0b11, record_cap=3,
                       threads=THREADS)
    np.testing.assert_array_equal(full["rec_n"], cut["rec_n"])
    assert full["rec_n"].max() > 3
    np.testing.assert_array_equal(full["rec_t"][:, :3], cut["rec_t"])
    np.testing.assert_array_equal(full["rec_j"][:, :3], cut["rec_j"])
    # recording changes nothing else
    plain = orc.simulate(m, "FP64", x0, 200.0, [200.0], 5, n_traj=30, threads=THREADS)
    np.testing.assert_array_equal(plain["snap"], full["snap"])
    np.testing.assert_array_equal(plain["n_events"], full["n_events"])


def dwell_times(r, start_before, on_j=0, off_j=1):
    """OFF dwells (an OFF switch to the next ON switch) and ON dwells, pooled,
    counting only dwells that start before `start_before`: a dwell still
    running at the horizon is not in the record, so without this cut long
    dwells would be under-represented."""
    off, on = [], []
    for i in range(r["rec_n"].size):
        n = min(int(r["rec_n"][i]), r["rec_t"].shape[1])
        t, j = r["rec_t"][i, :n], r["rec_j"][i, :n]
        for a in range(1, n):
            if t[a - 1] >= start_before:
                break
            if j[a - 1] == off_j and j[a] == on_j:
                off.append(t[a] - t[a - 1])
            elif j[a - 1] == on_j and j[a] == off_j:
                on.append(t[a] - t[a - 1])
    return np.array(off), np.array(on)


def test_dwell_times_follow_the_exponential_laws(orc):
    # two-state promoter with k_on != k_off; the gene switches alternate, so
    # OFF dwells are Exp(k_on) and ON dwells Exp(k_off) exactly. Dwells that
    # start before T - 300 end before T except with probability e^-15.
    k_on, k_off = 0.05, 0.2
    m = wl.telegraph(k_on, k_off, 20.0, 1.0)
    r = orc.simulate(m, "FP64", np.array([1, 0, 0], np.int32), 600.0, [600.0], 9, n_traj=600,
                     record_mask=0b11, record_cap=300, threads=THREADS)
    assert np.all(r["rec_n"] <= 300)
    # switches alternate: consecutive records are always one ON and one OFF switch
    for i in range(0, 600, 37):
        j = r["rec_j"][i, :r["rec_n"][i]]
        assert np.all(j[1:] != j[:-1]) and (j.size == 0 or j[0] == 0)
    off, on = dwell_times(r, 300.0)
    assert off.size > 5000 and on.size > 5000
    p_off = stats.kstest(off, "expon", args=(0, 1 / k_on)).pvalue
    p_on = stats.kstest(on, "expon", args=(0, 1 / k_off)).pvalue
    assert p_off > 1e-3 and p_on > 1e-3, (p_off, p_on)
    # a wrong rate is rejected at this sample size
    assert stats.kstest(off, "expon", args=(0, 1 / (1.1 * k_on))).pvalue < 1e-3
