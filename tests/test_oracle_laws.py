"""Pins of the oracle's direct method against closed forms and exact laws
(not against itself):

* birth-death: X(t) ~ Poisson(kb/kd (1 - e^{-kd t})) from X0 = 0, and the
  expected number of events kb T + kd int_0^T E[X] dt;
* Schloegl: the truncated chemical master equation (a 1-D birth-death chain)
  solved by a matrix exponential, at several snapshot times;
* telegraph: the Peccoud-Ycart stationary pmf (confluent hypergeometric form),
  mean and Fano factor; the transient mean m(t);
* closed dimer: exact conservation of A + 2D in every precision mode, and the
  detailed-balance stationary law;
* open dimer: the product-form stationary law M ~ Poisson(k1/k2),
  D ~ Poisson(k3 (k1/k2)^2 / (2 k4)) (complex-balanced network);
* self-repressing gene (Hill law): its detailed-balance stationary law;
* statistics the paper prints for its own FP64 runs;
* special cases: absorbing states, FP16 overflow, event caps;
* the reduced modes reduce exactly to FP32 when every 16-bit op is exact.
"""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

from paper_2605_00479_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run(orc, model, mode, x0, t_end, snap_t, n, seed=1, **kw):
    kw.setdefault("threads", 8)
    return orc.simulate(model, mode, np.asarray(x0), t_end, np.asarray(snap_t, float), seed, n_traj=n, **kw)


def chi2_pvalue(sample, pmf, min_expected=10.0):
    """Pearson chi-square of an integer sample against a pmf on 0..len(pmf)-1,
    pooling tail cells until each expected count is >= min_expected."""
    n = sample.size
    counts = np.bincount(sample, minlength=pmf.size)[: pmf.size].astype(float)
    counts[-1] += np.count_nonzero(sample >= pmf.size)
    exp = pmf * n
    obs_c, exp_c = [], []
    o_acc = e_acc = 0.0
    for o, e in zip(counts, exp):
        o_acc += o
        e_acc += e
        if e_acc >= min_expected:
            obs_c.append(o_acc)
            exp_c.append(e_acc)
            o_acc = e_acc = 0.0
    obs_c[-1] += o_acc
    exp_c[-1] += e_acc
    obs_c, exp_c = np.array(obs_c), np.array(exp_c)
    exp_c *= obs_c.sum() / exp_c.sum()
    return stats.chisquare(obs_c, exp_c).pvalue


def golden(key, qty):
    with open(os.path.join(GOLDEN, "paper_fp64_baselines.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == key and parts[1] == qty:
                return float(parts[2]), int(parts[3])
    raise KeyError(key)


# --------------------------------------------------------------------------- birth-death
def test_birth_death_poisson_law_and_event_count(orc):
    W = wl.config_birth_death()
    it = W.items[0]
    r = run(orc, it.model, "FP64", it.x0, W.t_end, W.snap_t, 10_000, seed=W.seed)
    x = r["snap"][0, 0]
    lam = 10.0 / 0.1 * (1 - math.exp(-0.1 * 100.0))
    assert chi2_pvalue(x, stats.poisson.pmf(np.arange(200), lam)) > 1e-3
    assert abs(x.mean() - lam) < 4 * math.sqrt(lam / x.size)
    assert abs(x.var(ddof=1) / lam - 1) < 4 * math.sqrt(2 / x.size)
    # E[events] = kb T + kd * int_0^T lam (1 - e^{-kd t}) dt
    e_events = 10 * 100 + 0.1 * (lam / (1 - math.exp(-10.0))) * (100 - (1 - math.exp(-10.0)) / 0.1)
    ne = r["n_events"].astype(float)
    assert abs(ne.mean() - e_events) < 5 * ne.std() / math.sqrt(ne.size)
    assert np.all(r["status"] == 0)
    assert np.all(r["t_last"] <= 100.0) and np.all(r["t_last"] > 90.0)


def test_birth_death_transient_snapshots(orc):
    """Every snapshot time has its own Poisson law (right-continuous path)."""
    m = wl.birth_death(5.0, 1.0)
    ts = np.array([0.0, 0.05, 0.3, 1.0, 2.5])
    r = run(orc, m, "FP64", [0], 2.5, ts, 40_000, seed=3)
    assert np.all(r["snap"][0, 0] == 0)
    for k, t in enumerate(ts[1:], start=1):
        lam = 5.0 * (1 - math.exp(-t))
        x = r["snap"][k, 0]
        assert chi2_pvalue(x, stats.poisson.pmf(np.arange(40), lam)) > 1e-3, t


def test_paper_birth_death_baseline(orc):
    mean, n_p = golden("birth_death_kb20_kd1", "mean")
    var, _ = golden("birth_death_kb20_kd1", "var")
    r = run(orc, wl.birth_death(20.0, 1.0), "FP64", [0], 30.0, [30.0], 20_000, seed=5)
    x = r["snap"][0, 0]
    se = math.sqrt(20.0 / n_p + 20.0 / x.size)
    assert abs(x.mean() - mean) < 4 * se
    assert abs(x.var(ddof=1) - var) < 4 * 20.0 * math.sqrt(2 / n_p + 2 / x.size)


# --------------------------------------------------------------------------- Schloegl (truncated CME)
def schlogl_cme(ts, x0=250, nmax=1200, c1A=3e-7 * 1e5, c2=1e-4, c3B=1e-3 * 2e5, c4=3.5):
    """Exact law of the Schloegl chain at integer times ts (truncated at nmax,
    far above the upper mode near 560), by repeated application of exp(Q^T)."""
    from scipy.linalg import expm
    x = np.arange(nmax + 1, dtype=float)
    birth = c1A / 2 * x * (x - 1) + c3B
    death = c2 / 6 * x * (x - 1) * (x - 2) + c4 * x
    birth[-1] = 0.0
    Q = np.diag(-(birth + death)) + np.diag(birth[:-1], 1) + np.diag(death[1:], -1)
    step = expm(Q.T)
    p = np.zeros(nmax + 1)
    p[x0] = 1.0
    out, t = {}, 0
    for target in sorted(ts):
        while t < target:
            p = step @ p
            t += 1
        out[target] = np.clip(p, 0, None) / np.clip(p, 0, None).sum()
    return [out[t] for t in ts]


def test_schlogl_matches_truncated_cme(orc):
    W = wl.config_schlogl()
    it = W.items[0]
    ks = [10, 30, 100]
    ts = W.snap_t
    r = run(orc, it.model, "FP64", it.x0, W.t_end, ts, 3000, seed=2)
    assert [ts[k] for k in ks] == [1.0, 3.0, 10.0]
    laws = schlogl_cme([1, 3, 10])
    for k, pmf in zip(ks, laws):
        x = r["snap"][k, 0]
        n = np.arange(pmf.size)
        mean, var = float(n @ pmf), float((n * n) @ pmf - (n @ pmf) ** 2)
        assert abs(x.mean() - mean) < 4 * math.sqrt(var / x.size), (k, x.mean(), mean)
        cdf = np.cumsum(pmf)
        ecdf = np.searchsorted(np.sort(x), n, side="right") / x.size
        d = np.max(np.abs(ecdf - cdf))
        assert d < 1.63 / math.sqrt(x.size) * 1.2, (k, d)   # KS 1% critical value


def test_paper_schlogl_baseline_agrees_with_exact_law():
    """The paper's FP64 Schloegl statistics (N = 10^4, t = 10) agree with the
    exact law of this network reading (reservoirs folded, 1/k! absorbed)."""
    mean_p, n_p = golden("schlogl_t10", "mean")
    var_p, _ = golden("schlogl_t10", "var")
    pmf = schlogl_cme([10])[0]
    n = np.arange(pmf.size)
    mean = float(n @ pmf)
    var = float((n * n) @ pmf) - mean ** 2
    assert abs(mean_p - mean) < 3 * math.sqrt(var / n_p)
    assert abs(var_p / var - 1) < 0.05


# --------------------------------------------------------------------------- telegraph
def telegraph_pmf(k_on, k_off, km, beta, nmax):
    """Peccoud-Ycart stationary mRNA law."""
    a, b, lam = k_on / beta, k_off / beta, km / beta
    n = np.arange(nmax)
    logc = (n * math.log(lam) - special.gammaln(n + 1) + special.gammaln(a + n) + special.gammaln(a + b)
            - special.gammaln(a) - special.gammaln(a + b + n))
    return np.exp(logc) * special.hyp1f1(a + n, a + b + n, -lam)


def test_telegraph_stationary_law(orc):
    W = wl.config_telegraph()
    it = W.items[0]
    r = run(orc, it.model, "FP64", it.x0, W.t_end, W.snap_t, 20_000, seed=4)
    m = r["snap"][-1, 2]
    pmf = telegraph_pmf(0.05, 0.1, 20.0, 1.0, 120)
    assert abs(pmf.sum() - 1) < 1e-9
    assert chi2_pvalue(m, pmf) > 1e-3
    mean = 20.0 * 0.05 / 0.15
    fano = 1 + 20.0 * 0.1 / (0.15 * 1.15)
    assert abs(m.mean() - mean) < 4 * math.sqrt(mean * fano / m.size)
    assert abs(m.var(ddof=1) / m.mean() - fano) < 0.05 * fano
    assert abs(np.mean(m == 0) - pmf[0]) < 4 * math.sqrt(pmf[0] * (1 - pmf[0]) / m.size)
    # gene copies are conserved exactly
    assert np.all(r["snap"][:, 0, :] + r["snap"][:, 1, :] == 1)


def test_telegraph_transient_mean(orc):
    W = wl.config_telegraph()
    it = W.items[0]
    r = run(orc, it.model, "FP64", it.x0, 20.0, np.arange(21.0), 20_000, seed=6)
    kon, koff, km = 0.05, 0.1, 20.0
    kap = kon + koff
    A = km * kon / kap
    for t in (2.0, 5.0, 10.0, 20.0):
        mt = A * (1 - math.exp(-t)) - A * (math.exp(-kap * t) - math.exp(-t)) / (1 - kap)
        x = r["snap"][int(t), 2]
        assert abs(x.mean() - mt) < 4.5 * x.std() / math.sqrt(x.size) + 1e-9, (t, x.mean(), mt)


@pytest.mark.parametrize("key,params", [("telegraph_bimodal", (0.05, 0.05, 20.0, 1.0)),
                                        ("telegraph_stress", (0.01, 0.1, 5.0, 1.0))])
def test_paper_telegraph_baselines(orc, key, params):
    mean_p, n_p = golden(key, "mean")
    kon, koff, km, beta = params
    mean = km / beta * kon / (kon + koff)
    fano = 1 + km / beta * koff / ((kon + koff) * (kon + koff + beta))
    assert abs(mean_p - mean) < 4 * math.sqrt(mean * fano / n_p)
    r = run(orc, wl.telegraph(*params), "FP64", [1, 0, 0], 150.0, [150.0], 20_000, seed=7)
    x = r["snap"][0, 2]
    assert abs(x.mean() - mean_p) < 4 * math.sqrt(mean * fano / n_p + mean * fano / x.size)


# --------------------------------------------------------------------------- dimerisation
def closed_dimer_law(total=100, kf=1e-3, kr=0.1):
    """Detailed balance on D = 0..total/2 with A = total - 2D."""
    dmax = total // 2
    logp = np.zeros(dmax + 1)
    for d in range(dmax):
        A = total - 2 * d
        logp[d + 1] = logp[d] + math.log(kf * A * (A - 1) / 2) - math.log(kr * (d + 1))
    p = np.exp(logp - logp.max())
    return p / p.sum()


@pytest.mark.parametrize("mode", ["FP64", "FP32", "MIX_F16_RTN", "MIX_F16_SR", "MIX_BF16_SR",
                                  "UNI_F16_RTN", "UNI_F16_SR", "UNI_BF16_RTN", "UNI_BF16_SR",
                                  "UNI_BF16_SR_NORM", "UNI_F16_SRA", "UNI_BF16_SRA_NORM"])
def test_closed_dimer_conservation_every_mode(orc, mode):
    m = wl.dimer_closed()
    r = run(orc, m, mode, [100, 0], 20.0, np.arange(21.0), 2000, seed=8, max_events=200_000)
    s = r["snap"]
    assert np.all(s[:, 0, :] + 2 * s[:, 1, :] == 100)
    assert np.all(s >= 0)


def test_closed_dimer_stationary_law_and_paper_values(orc):
    p = closed_dimer_law()
    d = np.arange(p.size)
    meanD = float(d @ p)
    meanA = 100 - 2 * meanD
    for key, qty, val in (("dimer_closed", "meanA", meanA), ("dimer_closed", "meanD", meanD)):
        printed, _ = golden(key, qty)
        assert abs(printed - val) < 0.5      # the paper prints them to the nearest molecule
    r = run(orc, wl.dimer_closed(), "FP64", [100, 0], 100.0, [100.0], 20_000, seed=9)
    assert chi2_pvalue(r["snap"][0, 1], p) > 1e-3


def test_open_dimer_product_form_law(orc):
    m = wl.dimer_open()
    # the total mass M + 2D relaxes on a time scale of tens of time units
    r = run(orc, m, "FP64", [0, 0], 500.0, [500.0], 1000, seed=10)
    M, D = r["snap"][0, 0], r["snap"][0, 1]
    lamM = 50.0 / 0.1
    lamD = 0.001 * lamM ** 2 / (2 * 0.5)
    assert abs(M.mean() - lamM) < 4 * math.sqrt(lamM / M.size)
    assert abs(D.mean() - lamD) < 4 * math.sqrt(lamD / D.size)
    assert abs(M.var(ddof=1) / lamM - 1) < 5 * math.sqrt(2 / M.size)
    assert abs(D.var(ddof=1) / lamD - 1) < 5 * math.sqrt(2 / D.size)
    assert abs(np.corrcoef(M, D)[0, 1]) < 4 / math.sqrt(M.size)


# --------------------------------------------------------------------------- Hill law
def test_self_repressor_detailed_balance(orc):
    b, v, K, h, d = 2.0, 30.0, 10.0, 2, 1.0
    r = run(orc, wl.self_repressor(b, v, K, h, d), "FP64", [0], 30.0, [30.0], 20_000, seed=11)
    x = r["snap"][0, 0]
    nmax = 120
    logp = np.zeros(nmax)
    for n in range(nmax - 1):
        logp[n + 1] = logp[n] + math.log(b + v / (1 + (n / K) ** h)) - math.log(d * (n + 1))
    p = np.exp(logp - logp.max())
    p /= p.sum()
    assert chi2_pvalue(x, p) > 1e-3


def test_paper_repressilator_baseline(orc):
    """Paper parameters: alpha0 = 1, alpha = 216, K = 1 (implicit), h = 2,
    dm = 1, beta = 5, dp = 1, p_A(0) = 5, t_end = 200 (Sec. 4.5)."""
    mean_p, n_p = golden("repressilator_t200", "mean")
    var_p, _ = golden("repressilator_t200", "var")
    m = wl.repressilator(alpha0=1.0, alpha=216.0, K=1.0, h=2, dm=1.0, beta=5.0, dp=1.0)
    r = run(orc, m, "FP64", [0, 0, 0, 5, 0, 0], 200.0, [200.0], 2000, seed=12)
    pA = r["snap"][0, 3].astype(float)
    se = math.sqrt(var_p / n_p + pA.var(ddof=1) / pA.size)
    assert abs(pA.mean() - mean_p) < 4 * se, (pA.mean(), mean_p)
    assert abs(pA.var(ddof=1) / var_p - 1) < 0.25


# --------------------------------------------------------------------------- special cases
def test_pure_decay_absorbs_after_exactly_x0_events(orc):
    m = wl.birth_death(0.0, 1.0)
    for mode in ("FP64", "FP32", "MIX_F16_SR", "UNI_BF16_RTN", "UNI_F16_SR_NORM"):
        r = run(orc, m, mode, [5], 1e6, [1e6], 200, seed=13)
        assert np.all(r["status"] == 1), mode
        assert np.all(r["n_events"] == 5), mode
        assert np.all(r["snap"] == 0), mode


def test_fp16_overflow_freezes_state(orc):
    """A zero-order constant of 1e5 exceeds fp16's largest value 65504
    (Table tab:formats): every 16-bit fp16 mode overflows at event 0 and
    keeps x0, as in the paper's Schloegl FP16 rows (Sec. 4.2)."""
    m = wl.birth_death(1e5, 1.0)
    for mode in ("MIX_F16_RTN", "MIX_F16_SR", "UNI_F16_SR"):
        r = run(orc, m, mode, [250], 10.0, [0.0, 5.0, 10.0], 50, seed=14)
        assert np.all(r["status"] == 2)
        assert np.all(r["n_events"] == 0)
        assert np.all(r["snap"] == 250)
    r = run(orc, m, "MIX_BF16_RTN", [250], 0.001, [0.001], 50, seed=14)
    assert np.all(r["status"] == 0)


def test_paper_original_schlogl_fp16_overflow(orc):
    """With the reservoirs A = 1e5, B = 2e5 as species entering the propensities
    (the paper's original parameterisation), A exceeds fp16's range: every mixed
    FP16 trajectory overflows at its first step and keeps X = 250, giving the
    printed mean 250.0 and variance 0; bf16 has the range and does not overflow."""
    from paper_2605_00479_amd.experiments import schlogl_with_reservoirs
    m = schlogl_with_reservoirs()
    mean_p, _ = golden("schlogl_original_mix_f16", "mean")
    var_p, _ = golden("schlogl_original_mix_f16", "var")
    for mode in ("MIX_F16_RTN", "MIX_F16_SR"):
        r = run(orc, m, mode, [250, 100_000, 200_000], 10.0, [10.0], 500, seed=21)
        x = r["snap"][0, 0]
        assert np.all(r["status"] == 2) and x.mean() == mean_p and x.var() == var_p
    r = run(orc, m, "MIX_BF16_SR", [250, 100_000, 200_000], 1.0, [1.0], 200, seed=21)
    assert np.all(r["status"] == 0)
    # in FP64 the reservoir form is the folded network's law
    a = run(orc, m, "FP64", [250, 100_000, 200_000], 10.0, [10.0], 3000, seed=22)["snap"][0, 0]
    b = run(orc, wl.schlogl(), "FP64", [250], 10.0, [10.0], 3000, seed=23)["snap"][0, 0]
    assert stats.ks_2samp(a, b).pvalue > 1e-3


def test_event_cap(orc):
    m = wl.birth_death(10.0, 0.1)
    r = run(orc, m, "UNI_BF16_RTN", [0], 100.0, [50.0, 100.0], 100, seed=15, max_events=300)
    assert np.all(r["status"] == 3) and np.all(r["n_events"] == 300)
    r2 = run(orc, m, "FP64", [0], 100.0, [100.0], 100, seed=15, max_events=300)
    assert np.all(r2["status"] == 3)


def test_empty_ensemble_and_no_snapshots(orc):
    m = wl.birth_death()
    r = run(orc, m, "FP64", [0], 1.0, [], 0)
    assert r["snap"].shape == (0, 1, 0) and r["n_events"].size == 0
    r = run(orc, m, "FP64", [0], 1.0, [], 10)
    assert r["snap"].shape == (0, 1, 10) and np.all(r["status"] == 0)


# --------------------------------------------------------------------------- invariances
def test_thread_count_and_order_do_not_change_results(orc):
    W = wl.config_schlogl()
    it = W.items[0]
    a = run(orc, it.model, "MIX_F16_SR", it.x0, 2.0, W.snap_t[:21], 300, threads=1)
    b = run(orc, it.model, "MIX_F16_SR", it.x0, 2.0, W.snap_t[:21], 300, threads=8)
    for key in a:
        np.testing.assert_array_equal(a[key], b[key])
    perm = np.random.default_rng(0).permutation(300)
    c = orc.simulate(it.model, "MIX_F16_SR", it.x0, 2.0, W.snap_t[:21], 1, indices=perm, threads=3)
    np.testing.assert_array_equal(c["snap"], a["snap"][:, :, perm])
    np.testing.assert_array_equal(c["n_events"], a["n_events"][perm])


def test_trajectory_id_base_shifts_streams(orc):
    m = wl.birth_death()
    a = run(orc, m, "FP64", [0], 5.0, [5.0], 20)
    b = orc.simulate(m, "FP64", [0], 5.0, [5.0], 1, indices=np.arange(10), traj_id_base=10)
    np.testing.assert_array_equal(b["n_events"], a["n_events"][10:])


@pytest.mark.parametrize("mode", ["MIX_F16_RTN", "MIX_F16_SR", "MIX_BF16_RTN", "MIX_BF16_SR"])
def test_mixed_mode_reduces_to_fp32_when_16bit_ops_are_exact(orc, mode):
    """With power-of-two rate constants and counts inside the 16-bit integer
    range every propensity op is exact, so mixed mode (RTN or SR) must equal
    FP32 mode bit for bit: the paper's mixed RTN and SR rows coincide in
    exactly this situation (Table tab:birth-death)."""
    m = wl.birth_death(16.0, 0.125)      # stationary mean 128 < 256
    ts = wl.snapshot_grid(40.0, 41)
    a = run(orc, m, "FP32", [0], 40.0, ts, 2000, seed=16)
    b = run(orc, m, mode, [0], 40.0, ts, 2000, seed=16)
    assert b["snap"].max() < 256
    for key in a:
        np.testing.assert_array_equal(a[key], b[key])


def test_uniform_sr_is_unbiased_where_rtn_stagnates(orc):
    """Uniform-mode outcomes the paper reports (Table tab:birth-death): BF16 RTN
    loses time and shifts the mean; FP16+SR stays on the FP64 law."""
    m = wl.birth_death(20.0, 1.0)
    ref = run(orc, m, "FP64", [0], 30.0, [30.0], 20_000, seed=17)["snap"][0, 0]
    sr = run(orc, m, "UNI_F16_SR", [0], 30.0, [30.0], 20_000, seed=18)["snap"][0, 0]
    rtn = run(orc, m, "UNI_BF16_RTN", [0], 30.0, [30.0], 20_000, seed=18, max_events=100_000)["snap"][0, 0]
    assert abs(sr.mean() - ref.mean()) < 4 * math.sqrt(40.0 / 20_000)
    assert ref.mean() - rtn.mean() > 6 * math.sqrt(2 * 20.0 / 20_000)
    # SR at the accumulation points alone also removes the clock's stagnation bias
    sra = run(orc, m, "UNI_BF16_SRA", [0], 30.0, [30.0], 20_000, seed=19)["snap"][0, 0]
    assert abs(sra.mean() - ref.mean()) < 0.25 * (ref.mean() - rtn.mean())


def test_selective_sr_draws_only_for_sums_and_clock(orc):
    """With SR at accumulation points only, propensities round to nearest: on a
    network whose uniform-mode ops are all exact except the clock and sums,
    selective SR and full SR see the same propensities; and a mixed-mode
    request for it is rejected (mixed mode accumulates in binary32)."""
    with pytest.raises(ValueError):
        orc.parse_mode("MIX_F16_SRA")
    m = wl.birth_death(16.0, 0.125)
    a = run(orc, m, "UNI_F16_SRA", [0], 5.0, [5.0], 500, seed=20)
    b = run(orc, m, "UNI_F16_SRA", [0], 5.0, [5.0], 500, seed=20, threads=1)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


# --------------------------------------------------------------------------- propensity normalisation
@pytest.mark.parametrize("mode,bd_tol", [("UNI_F16_SR_NORM", None), ("UNI_BF16_SR_NORM", 0.5)])
def test_normalised_uniform_modes_keep_the_laws(orc, mode, bd_tol):
    """Running-max normalisation (abstract; divide every propensity by m, the
    largest propensity seen so far, and the waiting time by m again) leaves
    the law of the process unchanged, so with stochastic rounding the
    normalised uniform modes stay on the exact laws:

    * birth-death kb = 20, kd = 1 from 0: X(30) ~ Poisson(20(1 - e^-30)).
      fp16: mean within 4 standard errors. bf16 uniform SR carries a small
      known bias on this network (the paper's uniform BF16+SR row of Table
      tab:birth-death fails KS), so its mean is held to 20 +- 0.5;
    * telegraph k_on = 0.05, k_off = 0.1, k_m = 20, beta = 1 at T = 200
      (relaxed): stationary mean k_m k_on / (beta (k_on + k_off)) = 20/3 within
      4 standard errors, Fano factor 1 + k_m k_off / ((k_on + k_off)(k_on +
      k_off + beta)) within 8%.

    A waiting time not divided by m stretches time m-fold (birth-death mean
    about 15.5, telegraph about 11.6); summands not divided by m shrink it
    m-fold (telegraph mean about 2.7, not relaxed by T)."""
    bd = run(orc, wl.birth_death(20.0, 1.0), mode, [0], 30.0, [30.0], 20_000, seed=17,
             max_events=100_000)["snap"][0, 0]
    lam = 20.0 * (1 - math.exp(-30.0))
    tol = bd_tol if bd_tol is not None else 4 * math.sqrt(lam / bd.size)
    assert abs(bd.mean() - lam) < tol, (mode, bd.mean())
    W = wl.config_telegraph()
    it = W.items[0]
    m = run(orc, it.model, mode, it.x0, 200.0, [200.0], 20_000, seed=17, max_events=W.max_events)["snap"][0, 2]
    mean = 20.0 * 0.05 / 0.15
    fano = 1 + 20.0 * 0.1 / (0.15 * 1.15)
    assert abs(m.mean() - mean) < 4 * math.sqrt(mean * fano / m.size), (mode, m.mean())
    assert abs(m.var(ddof=1) / m.mean() - fano) < 0.08 * fano, (mode, m.var(ddof=1) / m.mean())
