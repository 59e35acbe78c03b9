"""Pins of the oracle's contingency-table sampler (Section 4) to facts
outside itself: the paper's printed thresholds, exact hypergeometric
quantiles, exact enumeration of small tables, and the paper's p-value."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads
from conftest import read_golden

GEN = O.MRG32K3A


def _golden_table(name):
    return np.array([[int(v) for v in r] for r in read_golden(name)], dtype=np.int32)


def _golden_meta(name, key):
    from conftest import GOLDEN
    import os
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith(f"# {key}:"):
            return line.split(":", 1)[1].split()


@pytest.mark.parametrize("name", ["fisher_month.txt", "fisher_week.txt"])
def test_paper_thresholds(name):
    """Section 4.1 / 4.2: the printed threshold is -sum log(n_ij!) of the
    printed table (Tables 1 and 2), to every printed digit."""
    tab = _golden_table(name)
    val, dec = _golden_meta(name, "threshold")
    assert abs(O.table_stat(tab) - float(val)) <= 0.5 * 10.0 ** (-int(dec))


def _hyper_cdf(Np, K, n):
    lo, hi = max(0, n - (Np - K)), min(n, K)
    tot = math.comb(Np, n)
    cdf, acc = [], Fraction(0)
    for x in range(lo, hi + 1):
        acc += Fraction(math.comb(K, x) * math.comb(Np - K, n - x), tot)
        cdf.append((x, acc))
    return cdf


@pytest.mark.parametrize("Np,K,n", [(10, 4, 3), (30, 12, 17), (200, 5, 150), (400, 180, 200),
                                    (57, 57, 20), (57, 0, 20), (12, 7, 12), (1000, 300, 400),
                                    (1983, 589, 1177)])  # w(mode)/w(lo) > 2^1024
def test_inversion_is_the_hypergeometric_quantile(Np, K, n):
    """The entry sampled from u is the smallest x with u <= F(x), F the exact
    hypergeometric cdf (rational arithmetic), away from the cdf's jumps."""
    cdf = _hyper_cdf(Np, K, n)
    rnd = np.random.default_rng(Np * 7 + K)
    us = list(rnd.uniform(0, 1, size=400)) + [1e-300, 0.5, 1 - 1e-12]
    for u in us:
        want = next(x for x, F in cdf if Fraction(u) <= F)
        if any(abs(float(F) - u) < 1e-9 for _, F in cdf):
            continue
        assert O.hyper_invert(float(u), Np, K, n) == want, (u, Np, K, n)


def test_tables_keep_margins_and_consume_cells():
    I, J, rows, cols = workloads.contingency_margins(300, rng_seed=4)
    seed = workloads.random_seed(6)
    rec = O.create_streams(GEN, seed.copy(), 300)
    work = rec.copy()
    tabs, stats = O.tables(GEN, work, I, J, rows, cols)
    for t in range(300):
        tb = tabs[t, :I[t], :J[t]]
        assert np.all(tb >= 0)
        np.testing.assert_array_equal(tb.sum(axis=1), rows[t, :I[t]])
        np.testing.assert_array_equal(tb.sum(axis=0), cols[t, :J[t]])
        assert np.all(tabs[t, I[t]:, :] == 0) and np.all(tabs[t, :, J[t]:] == 0)
        # exactly (I-1)(J-1) uniforms were drawn
        s = rec[t, :6].copy()
        O.jump(GEN, s, int((I[t] - 1) * (J[t] - 1)))
        np.testing.assert_array_equal(work[t, :6], s)
        assert stats[t] == O.table_stat(tb)


def _enumerate(rows, cols):
    """All tables with the margins, with their exact probabilities under the
    null (multivariate hypergeometric): prod r! prod c! / (N! prod n!)."""
    I, J = len(rows), len(cols)
    N = sum(rows)
    out = []
    for cells in itertools.product(*[range(min(r, c) + 1) for r in rows[:-1] for c in cols[:-1]]):
        t = np.zeros((I, J), dtype=np.int64)
        t[:-1, :-1] = np.array(cells).reshape(I - 1, J - 1)
        t[:-1, -1] = np.array(rows[:-1]) - t[:-1, :-1].sum(axis=1)
        t[-1, :] = np.array(cols) - t[:-1, :].sum(axis=0)
        if (t < 0).any() or t[-1].sum() != rows[-1]:
            continue
        num = math.prod(math.factorial(r) for r in rows) * math.prod(math.factorial(c) for c in cols)
        den = math.factorial(N) * math.prod(math.factorial(int(v)) for v in t.flat)
        out.append((tuple(t.flat), Fraction(num, den)))
    return out


@pytest.mark.parametrize("rows,cols", [([3, 4], [2, 5]), ([3, 2, 4], [4, 2, 3]), ([5, 6], [3, 4, 4])])
def test_table_distribution_matches_exact_enumeration(rows, cols):
    """Sequential sampling by inversion gives Fisher's null distribution:
    chi-square against the exact table probabilities (20000 tables)."""
    probs = _enumerate(rows, cols)
    assert sum(p for _, p in probs) == 1
    B = 20000
    rec = O.create_streams(GEN, workloads.random_seed(11), B)
    counts = {}
    for b in range(B):
        t = O.table_sample(GEN, rec[b, :6].copy(), rows, cols)
        counts[tuple(t.flat)] = counts.get(tuple(t.flat), 0) + 1
    keys = {k for k, _ in probs}
    assert set(counts) <= keys
    chi2 = sum((counts.get(k, 0) - B * float(p)) ** 2 / (B * float(p)) for k, p in probs)
    dof = len(probs) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10, (chi2, dof)


def test_month_pvalue_near_paper():
    """Section 4.1 reports p = 0.403 (and 0.404 from stats::fisher.test) for
    Table 1; 4000 oracle replicates must agree within 4 standard errors."""
    tab = _golden_table("fisher_month.txt")
    B = 4000
    rec = O.create_streams(GEN, workloads.random_seed(12), B)
    cnt, obs = O.fisher_count(GEN, rec, tab)
    p = (1 + cnt) / (B + 1)
    se = math.sqrt(0.403 * 0.597 / B)
    assert abs(p - 0.403) < 4 * se, p


@pytest.mark.parametrize("name", ["fisher_month.txt", "fisher_week.txt"])
def test_cell_moments_on_paper_tables(name):
    """Under the null each cell is hypergeometric: mean r_i c_j / N and
    variance r_i c_j (N - r_i)(N - c_j) / (N^2 (N - 1)).  3000 oracle tables
    with the margins of the paper's tables must agree cell by cell (|z| < 5
    for the mean, variance within 25%).  Overflowing weights put one cell of
    the day-of-week table 9 standard errors off."""
    tab = _golden_table(name).astype(np.int64)
    r, c, N = tab.sum(axis=1), tab.sum(axis=0), int(tab.sum())
    B = 3000
    rec = O.create_streams(GEN, workloads.random_seed(13), B)
    acc = np.zeros(tab.shape)
    acc2 = np.zeros(tab.shape)
    for b in range(B):
        t = O.table_sample(GEN, rec[b, :6].copy(), r.astype(np.int32), c.astype(np.int32)).astype(np.float64)
        acc += t
        acc2 += t * t
    mean = acc / B
    var = acc2 / B - mean ** 2
    E = np.outer(r, c) / N
    V = np.outer(r, c) * np.outer(N - r, N - c) / (N ** 2 * (N - 1))
    z = (mean - E) / np.sqrt(V / B)
    assert np.abs(z).max() < 5, np.unravel_index(np.abs(z).argmax(), z.shape)
    assert np.all(np.abs(var / V - 1) < 0.25)


def test_week_pvalue_near_paper():
    """Section 4.2 reports p = 0.000125 (1255 of 10027008) for Table 2, and
    0.000127 from stats::fisher.test; 160000 oracle replicates (8 threads)
    must count 20 +- 4 sqrt(20)."""
    import threading
    tab = _golden_table("fisher_week.txt")
    B, T = 160000, 8
    rec = O.create_streams(GEN, workloads.random_seed(14), B)
    counts = []

    def work(lo, hi):
        cnt, _ = O.fisher_count(GEN, rec[lo:hi].copy(), tab)
        counts.append(cnt)

    ts = [threading.Thread(target=work, args=(k * B // T, (k + 1) * B // T)) for k in range(T)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    expect = 0.000125 * B
    assert abs(sum(counts) - expect) < 4 * math.sqrt(expect), sum(counts)


# ------------------------------------------------------------- the count rule
def _exact_count(tables, observed):
    """Replicates whose statistic is at most the observed one, decided exactly:
    -sum log(n_ij!) <= -sum log(o_ij!)  <=>  prod n_ij! >= prod o_ij!, in
    Python integers (no rounding anywhere)."""
    def prod_fact(t):
        p = 1
        for v in np.asarray(t).ravel():
            p *= math.factorial(int(v))
        return p
    want = prod_fact(observed)
    return sum(1 for t in tables if prod_fact(t) >= want)


def _replicates(streams, observed):
    obs = np.asarray(observed, dtype=np.int32)
    rows, cols = obs.sum(axis=1), obs.sum(axis=0)
    return [O.table_sample(GEN, streams[b, 0:6].copy(), rows, cols) for b in range(streams.shape[0])]


@pytest.mark.parametrize("observed", [[[3, 0, 7, 1]], [[4], [0], [9]], [[17]]])
def test_determined_tables_count_every_replicate(observed):
    """Section 4's count is of replicates at most as probable as the observed
    table.  With one row or one column the margins fix the table, so every
    replicate equals the observed table and must count: count = B."""
    B = 300
    st = O.create_streams(GEN, workloads.random_seed(71), B)
    cnt, obs_stat = O.fisher_count(GEN, st, np.array(observed, dtype=np.int32))
    assert cnt == B
    assert obs_stat == O.table_stat(np.array(observed, dtype=np.int32))


def test_ties_count_whatever_the_rounding():
    """Section 4 counts replicates whose statistic is at most the observed one
    ("less or equal", as stats::fisher.test to which it compares).  Observed
    [[2,4],[4,2]]: the replicate [[4,2],[2,4]] has the same statistic
    mathematically, but its row-major double sum rounds 8.9e-16 above the
    observed one, so a rule without the near-tie allowance would miss it (and
    an allowance in the wrong direction would miss the observed table too).
    With the allowance, '<' and '<=' differ only for a statistic equal to the
    threshold bit for bit.  The oracle's count must equal the exact count from
    integer factorials."""
    obs = np.array([[2, 4], [4, 2]], dtype=np.int32)
    per = np.array([[4, 2], [2, 4]], dtype=np.int32)
    assert O.table_stat(per) > O.table_stat(obs)  # the case the allowance exists for
    B = 4000
    st = O.create_streams(GEN, workloads.random_seed(72), B)
    tabs = _replicates(st.copy(), obs)
    assert sum(1 for t in tabs if np.array_equal(t, per)) > 500
    assert sum(1 for t in tabs if np.array_equal(t, obs)) > 500
    cnt, _ = O.fisher_count(GEN, st.copy(), obs)
    assert cnt == _exact_count(tabs, obs)
    assert cnt < B  # [[3,3],[3,3]] is more probable and must not count


@pytest.mark.parametrize("observed", [[[1, 2, 3], [3, 2, 1]], [[2, 1, 1], [1, 2, 1], [1, 1, 2]],
                                      [[5, 0], [0, 5]]])
def test_count_equals_exact_factorial_comparison(observed):
    """Small tables with many equal-statistic replicates (permutations of the
    observed entries): the oracle's count equals the exact integer count."""
    obs = np.array(observed, dtype=np.int32)
    B = 2500
    st = O.create_streams(GEN, workloads.random_seed(73 + obs.size), B)
    tabs = _replicates(st.copy(), obs)
    cnt, _ = O.fisher_count(GEN, st.copy(), obs)
    assert cnt == _exact_count(tabs, obs)
