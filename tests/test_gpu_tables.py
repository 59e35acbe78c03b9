"""GPU parity of the contingency-table consumer (Section 4) against the
oracle: tables bit-exact (integer work), advanced stream states bit-exact,
statistics within the lgamma tolerance, Fisher counts exact; edge cases
(determined tables, zero margins, invalid margins, ragged counts, the
largest shapes)."""
import numpy as np
import pytest

import oracle as O
import workloads
from conftest import read_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_06604_amd as P  # noqa: E402

GEN = O.MRG32K3A
# log(n!) on both sides is lgammal(n+1) rounded to double (the library
# uploads a host-built table), summed row-major without contraction: the
# statistics are compared bit for bit.


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _device(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _records(seed, n):
    return O.create_streams(GEN, np.array(seed, dtype=np.uint32), n)


def _run_tables(rec, I, J, rows, cols):
    d = _device(rec.view(np.int32).copy())
    tabs, stats = P.mrg_tables_sample(d, _device(I), _device(J), _device(rows), _device(cols), stats=True)
    torch.cuda.synchronize()
    n = I.shape[0]
    return (tabs[:n].cpu().numpy(), stats[:n].cpu().numpy(), d.cpu().numpy().view(np.uint32))


def _check_stats(got, want):
    bad = got != want
    assert not bad.any(), (np.flatnonzero(bad)[:5], got[bad][:5], want[bad][:5])


@pytest.mark.parametrize("n,seed_id", [(1, 1), (255, 2), (4097, 3), (65536 + 77, 4)])
def test_tables_match_oracle(n, seed_id):
    I, J, rows, cols = workloads.contingency_margins(n, rng_seed=seed_id)
    rec = _records(workloads.random_seed(seed_id), n)
    tabs, stats, after = _run_tables(rec, I, J, rows, cols)
    work = rec.copy()
    wtabs, wstats = O.tables(GEN, work, I, J, rows, cols)
    np.testing.assert_array_equal(tabs, wtabs)
    np.testing.assert_array_equal(after, work)
    _check_stats(stats, wstats)


def test_tables_full_workload_bit_exact():
    """The full simulation workload: 1e6 tables, 2x2..5x5, totals 5..200,
    every table compared with the oracle's."""
    n = 1_000_000
    I, J, rows, cols = workloads.contingency_margins(n)
    rec = _records(workloads.random_seed(), n)
    tabs, stats, after = _run_tables(rec, I, J, rows, cols)
    work = rec.copy()
    wtabs, wstats = O.tables(GEN, work, I, J, rows, cols)
    np.testing.assert_array_equal(tabs, wtabs)
    np.testing.assert_array_equal(after, work)
    _check_stats(stats, wstats)


def test_tables_degenerate_cases():
    """1 x J and I x 1 tables use no draws; zero margins; margins in the
    thousands (entries spanning hundreds of values)."""
    I = np.array([1, 5, 2, 3, 5, 2], dtype=np.int32)
    J = np.array([5, 1, 2, 3, 5, 5], dtype=np.int32)
    rows = np.zeros((6, 5), dtype=np.int32)
    cols = np.zeros((6, 5), dtype=np.int32)
    rows[0, :1], cols[0, :5] = [15], [1, 2, 3, 4, 5]
    rows[1, :5], cols[1, :1] = [1, 2, 3, 4, 5], [15]
    rows[2, :2], cols[2, :2] = [0, 0], [0, 0]
    rows[3, :3], cols[3, :3] = [0, 7, 0], [3, 0, 4]
    rows[4, :5], cols[4, :5] = [1500, 1, 0, 400, 3], [800, 700, 4, 0, 400]
    rows[5, :2], cols[5, :5] = [1, 1], [0, 1, 0, 1, 0]
    rec = _records(workloads.random_seed(21), 6)
    tabs, stats, after = _run_tables(rec, I, J, rows, cols)
    work = rec.copy()
    wtabs, wstats = O.tables(GEN, work, I, J, rows, cols)
    np.testing.assert_array_equal(tabs, wtabs)
    np.testing.assert_array_equal(after, work)
    _check_stats(stats, wstats)
    np.testing.assert_array_equal(after[:2], rec[:2])  # no draws


def test_tables_at_the_total_bound():
    """Tables whose grand total is the largest accepted, 2^20: the ratio of
    consecutive hypergeometric weights multiplies factors up to 2^20, the
    largest products the kernel forms in fp64 (below 2^42, exact), and the
    searches span hundreds of thousands of values.  Sixteen tables of random
    shapes and margins, bit-exact with the oracle."""
    rng = np.random.default_rng(2201066)
    n, total = 16, 1 << 20
    I = rng.integers(2, 6, size=n).astype(np.int32)
    J = rng.integers(2, 6, size=n).astype(np.int32)
    rows = np.zeros((n, 5), dtype=np.int32)
    cols = np.zeros((n, 5), dtype=np.int32)

    def composition(k):  # k positive parts summing to total
        cuts = np.sort(rng.choice(np.arange(1, total), size=k - 1, replace=False))
        return np.diff(np.concatenate(([0], cuts, [total])))

    for t in range(n):
        rows[t, :I[t]] = composition(I[t])
        cols[t, :J[t]] = composition(J[t])
    rec = _records(workloads.random_seed(23), n)
    tabs, stats, after = _run_tables(rec, I, J, rows, cols)
    work = rec.copy()
    wtabs, wstats = O.tables(GEN, work, I, J, rows, cols)
    np.testing.assert_array_equal(tabs, wtabs)
    np.testing.assert_array_equal(after, work)
    _check_stats(stats, wstats)
    assert (tabs.reshape(n, -1).sum(axis=1) == total).all()


def test_tables_invalid_margins_leave_stream():
    """Unequal sums, a negative margin, a shape out of range or a total above
    2^20 give zeros, a NaN statistic and an untouched stream; valid tables in
    the same launch are unaffected."""
    I = np.array([2, 2, 6, 2, 3, 2], dtype=np.int32)
    J = np.array([2, 2, 2, 0, 3, 3], dtype=np.int32)
    rows = np.zeros((6, 5), dtype=np.int32)
    cols = np.zeros((6, 5), dtype=np.int32)
    rows[0, :2], cols[0, :2] = [3, 4], [2, 4]
    rows[1, :2], cols[1, :2] = [-1, 4], [1, 2]
    rows[2, :5], cols[2, :2] = [1, 1, 1, 1, 1], [2, 3]
    rows[3, :2] = [1, 1]
    rows[4, :3], cols[4, :3] = [1 << 20, 1, 0], [1, 1 << 20, 0]
    rows[5, :2], cols[5, :3] = [30, 40], [20, 25, 25]  # valid
    rec = _records(workloads.random_seed(22), 6)
    tabs, stats, after = _run_tables(rec, I, J, rows, cols)
    assert np.all(tabs[:5] == 0) and np.all(np.isnan(stats[:5]))
    np.testing.assert_array_equal(after[:5], rec[:5])
    work = rec[5:].copy()
    wtabs, wstats = O.tables(GEN, work, I[5:], J[5:], rows[5:], cols[5:])
    np.testing.assert_array_equal(tabs[5:], wtabs)
    np.testing.assert_array_equal(after[5:], work)
    _check_stats(stats[5:], wstats)


def test_tables_states_continue():
    """Two launches in a row on the same streams equal the oracle's two calls
    (the state written back is where the next draw starts)."""
    n = 3000
    I, J, rows, cols = workloads.contingency_margins(n, rng_seed=31)
    rec = _records(workloads.random_seed(31), n)
    d = _device(rec.view(np.int32).copy())
    dI, dJ, dr, dc = _device(I), _device(J), _device(rows), _device(cols)
    P.mrg_tables_sample(d, dI, dJ, dr, dc)
    t2, _ = P.mrg_tables_sample(d, dI, dJ, dr, dc)
    work = rec.copy()
    O.tables(GEN, work, I, J, rows, cols)
    w2, _ = O.tables(GEN, work, I, J, rows, cols)
    np.testing.assert_array_equal(t2.cpu().numpy(), w2)
    np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), work)


def _golden_table(name):
    return np.array([[int(v) for v in r] for r in read_golden(name)], dtype=np.int32)


@pytest.mark.parametrize("name,B", [("fisher_month.txt", 20000 + 13), ("fisher_week.txt", 8192)])
def test_fisher_count_matches_oracle(name, B):
    tab = _golden_table(name)
    rec = _records(workloads.random_seed(41), B)
    d = _device(rec.view(np.int32).copy())
    cnt, obs, stats = P.mrg_fisher_sim(d, tab, stats=True)
    torch.cuda.synchronize()
    work = rec.copy()
    wcnt, wobs = O.fisher_count(GEN, work, tab)
    assert int(cnt.item()) == wcnt
    assert obs == wobs
    np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), work)
    # each replicate's statistic against the oracle's table for that stream
    r, c = tab.sum(axis=1).astype(np.int32), tab.sum(axis=0).astype(np.int32)
    got = stats[:B].cpu().numpy()
    for b in range(0, B, 997):
        t = O.table_sample(GEN, rec[b, :6].copy(), r, c)
        want = O.table_stat(t)
        assert got[b] == want, b


def test_fisher_month_full_size_count():
    """Table 1 (12 x 12) at the benchmarked B = 2^20: the count equals the
    oracle's (its replicates split over 16 host threads) and every stream
    advances as the oracle's does."""
    from concurrent.futures import ThreadPoolExecutor
    tab = _golden_table("fisher_month.txt")
    B = 1 << 20
    rec = _records(workloads.random_seed(43), B)
    d = _device(rec.view(np.int32).copy())
    cnt, obs, _ = P.mrg_fisher_sim(d, tab)
    torch.cuda.synchronize()
    work = rec.copy()
    bounds = np.linspace(0, B, 17).astype(int)
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda k: O.fisher_count(GEN, work[bounds[k]:bounds[k + 1]], tab), range(16)))
    assert int(cnt.item()) == sum(p[0] for p in parts)
    assert obs == parts[0][1]
    np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), work)


def test_fisher_edge_cases():
    rec = _records(workloads.random_seed(42), 300)
    d = _device(rec.view(np.int32).copy())
    cnt, _, _ = P.mrg_fisher_sim(d, [[3, 4, 5]], B=300)   # one row: every replicate is the table
    assert int(cnt.item()) == 300
    cnt, _, _ = P.mrg_fisher_sim(d, [[3, 4], [5, 6]], B=0)
    assert int(cnt.item()) == 0
    # 32 x 32, the largest shape, small totals
    rng = np.random.default_rng(5)
    big = rng.integers(0, 4, size=(32, 32)).astype(np.int32)
    B = 193
    rec = _records(workloads.random_seed(43), B)
    d = _device(rec.view(np.int32).copy())
    cnt, obs, stats = P.mrg_fisher_sim(d, big, stats=True)
    work = rec.copy()
    wcnt, wobs = O.fisher_count(GEN, work, big)
    assert int(cnt.item()) == wcnt
    np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), work)


def test_fisher_month_pvalue_near_paper():
    """Section 4.1 prints p = 0.403 for Table 1 (1048576 replicates); 2^20
    GPU replicates must land within 4 standard errors."""
    tab = _golden_table("fisher_month.txt")
    B = 1 << 20
    c = P.mrg_creator_init(list(workloads.random_seed(44)))
    d = P.new_streams_tensor(B)
    P.mrg_streams_create_device(c, B, out=d)
    cnt, _, _ = P.mrg_fisher_sim(d, tab)
    p = P.mrg_fisher_pvalue(int(cnt.item()), B)
    se = np.sqrt(0.403 * 0.597 / B)
    assert abs(p - 0.403) < 4 * se, p


def test_fisher_week_pvalue_near_paper():
    """Section 4.2 prints p = 0.000125 (1255 of 10027008 replicates) for
    Table 2; the same number of GPU replicates must count 1255 +- 4 sqrt(1255)."""
    tab = _golden_table("fisher_week.txt")
    B = 10027008
    c = P.mrg_creator_init(list(workloads.random_seed(45)))
    d = P.new_streams_tensor(B)
    P.mrg_streams_create_device(c, B, out=d)
    cnt, _, _ = P.mrg_fisher_sim(d, tab)
    k = int(cnt.item())
    assert abs(k - 1255) < 4 * np.sqrt(1255), k


def test_tables_and_fisher_replayed_from_a_graph():
    """Both calls captured in one HIP graph (after a first eager call on the
    device) and replayed three times with eager work in between: every replay
    equals the oracle's next call on the same streams."""
    tab = _golden_table("fisher_month.txt")
    B, n = 3000, 2000
    I, J, rows, cols = workloads.contingency_margins(n, rng_seed=51)
    rec_f = _records(workloads.random_seed(52), B)
    rec_t = _records(workloads.random_seed(53), n)
    df, dt = _device(rec_f.view(np.int32).copy()), _device(rec_t.view(np.int32).copy())
    dI, dJ, dr, dc = _device(I), _device(J), _device(rows), _device(cols)
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    tabs = torch.empty((n, 5, 5), dtype=torch.int32, device="cuda")
    stats = torch.empty(n, dtype=torch.float64, device="cuda")
    warm = _device(rec_f[:8].view(np.int32).copy())
    P.mrg_fisher_sim(warm, tab, B=8)  # first call on the device: table upload
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.mrg_fisher_sim(df, tab, count=count)
        P.mrg_tables_sample(dt, dI, dJ, dr, dc, tables=tabs, stats=stats)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(df), rec_f)  # capture ran nothing
    wf, wt = rec_f.copy(), rec_t.copy()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        wcnt, _ = O.fisher_count(GEN, wf, tab)
        wtabs, wstats = O.tables(GEN, wt, I, J, rows, cols)
        assert int(count.item()) == wcnt, rep
        np.testing.assert_array_equal(tabs.cpu().numpy(), wtabs)
        _check_stats(stats.cpu().numpy(), wstats)
        np.testing.assert_array_equal(P.as_u32(df), wf)
        np.testing.assert_array_equal(P.as_u32(dt), wt)
        torch.ones(1 << 20, device="cuda").sum().item()  # eager work between replays
    del g
