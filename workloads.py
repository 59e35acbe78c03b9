"""Seeded synthetic inputs shared by the tests, the oracle legs and bench.py.

This module holds no arithmetic of the method: it only draws seeds, sizes,
request mixes and table margins from numpy's seeded generators.  Both the
oracle side and the GPU side receive what it returns.
"""
import numpy as np

DEFAULT_RNG_SEED = 220106604

# Upper bounds (exclusive) of the two seed triples, per generator id
# (1 = MRG32k3a, 2 = MRG31k3p): the component moduli.
SEED_BOUNDS = {1: (4294967087, 4294944443), 2: (2147483647, 2147462579)}

PAPER_SEED = [12345] * 6


def random_seed(rng_seed: int = DEFAULT_RNG_SEED, gen: int = 1) -> np.ndarray:
    """A valid 6-word seed: words 0-2 uniform below m1, words 3-5 below m2,
    each triple redrawn until not all zero."""
    rng = np.random.default_rng(rng_seed)
    b1, b2 = SEED_BOUNDS[gen]
    out = []
    for bound in (b1, b2):
        while True:
            t = rng.integers(0, bound, size=3, dtype=np.uint64)
            if t.any():
                break
        out.extend(int(v) for v in t)
    return np.array(out, dtype=np.uint32)


def random_states(n: int, rng_seed: int, gen: int = 1) -> np.ndarray:
    """n arbitrary valid 6-word states (not stream starts), for tests of the
    recurrence away from stream boundaries."""
    rng = np.random.default_rng(rng_seed)
    b1, b2 = SEED_BOUNDS[gen]
    a = np.empty((n, 6), dtype=np.uint32)
    a[:, :3] = rng.integers(1, b1, size=(n, 3), dtype=np.uint64)
    a[:, 3:] = rng.integers(1, b2, size=(n, 3), dtype=np.uint64)
    return a


def batch_requests(n_req: int = 4096, rng_seed: int = DEFAULT_RNG_SEED,
                   len_lo: float = 1e3, len_hi: float = 1e7,
                   s_lo: int = 64, s_hi: int = 1024):
    """A mix of generation requests: length floor(10^U(log10 lo, log10 hi)),
    stream count uniform in [s_lo, s_hi], distribution uniform in
    {uniform, normal, exponential(rate 1)}, dtype uniform in {f32, f64}.
    Returns a list of dicts; request r takes the next n_streams streams of one
    creator in order."""
    rng = np.random.default_rng(rng_seed)
    lens = np.floor(10.0 ** rng.uniform(np.log10(len_lo), np.log10(len_hi), size=n_req)).astype(np.int64)
    ss = rng.integers(s_lo, s_hi + 1, size=n_req)
    dists = rng.integers(0, 3, size=n_req)           # 0 uniform, 1 normal, 2 exponential
    dtypes = rng.integers(0, 2, size=n_req)          # 0 f64, 1 f32
    reqs = []
    first = 0
    for r in range(n_req):
        reqs.append(dict(n=int(lens[r]), n_streams=int(ss[r]), first_stream=first,
                         dist=int(dists[r]), dtype=int(dtypes[r]), param=1.0))
        first += int(ss[r])
    return reqs


def contingency_margins(n_tables: int, rng_seed: int = DEFAULT_RNG_SEED,
                        dim_lo: int = 2, dim_hi: int = 5, tot_lo: int = 5, tot_hi: int = 200):
    """Random table shapes I x J (uniform in [dim_lo, dim_hi]) and margins:
    row totals uniform in [tot_lo, tot_hi]; column totals uniform in the same
    range for the first J-1 columns, the last one making the sums equal; a
    table whose last column total falls outside [tot_lo, tot_hi] has all its
    totals redrawn.  Returns (I, J, rows[n,5], cols[n,5]) with zero padding."""
    rng = np.random.default_rng(rng_seed)
    I = rng.integers(dim_lo, dim_hi + 1, size=n_tables)
    J = rng.integers(dim_lo, dim_hi + 1, size=n_tables)
    rows = np.zeros((n_tables, 5), dtype=np.int64)
    cols = np.zeros((n_tables, 5), dtype=np.int64)
    k = np.arange(5)
    todo = np.arange(n_tables)
    while todo.size:
        r = rng.integers(tot_lo, tot_hi + 1, size=(todo.size, 5))
        c = rng.integers(tot_lo, tot_hi + 1, size=(todo.size, 5))
        r[k[None, :] >= I[todo, None]] = 0
        c[k[None, :] >= J[todo, None] - 1] = 0
        last = r.sum(axis=1) - c.sum(axis=1)
        ok = (last >= tot_lo) & (last <= tot_hi)
        sel = todo[ok]
        rows[sel] = r[ok]
        c[ok.nonzero()[0], J[sel] - 1] = last[ok]
        cols[sel] = c[ok]
        todo = todo[~ok]
    return I.astype(np.int32), J.astype(np.int32), rows.astype(np.int32), cols.astype(np.int32)


def poisson_arrivals(rate_per_s: float, duration_s: float, n_sessions: int = 256,
                     rng_seed: int = DEFAULT_RNG_SEED, len_lo: float = 1e2, len_hi: float = 1e6):
    """Open-loop Poisson arrivals: times (s), session ids, lengths
    floor(10^U(log10 lo, log10 hi))."""
    rng = np.random.default_rng(rng_seed)
    n_exp = int(rate_per_s * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_per_s, size=n_exp)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    n = t.shape[0]
    sess = rng.integers(0, n_sessions, size=n)
    lens = np.floor(10.0 ** rng.uniform(np.log10(len_lo), np.log10(len_hi), size=n)).astype(np.int64)
    return t, sess, lens
