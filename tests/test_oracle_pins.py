"""Pins of the CPU oracle to facts outside itself (no GPU needed).

Each test names what fixes the expected value: a value printed in the paper,
a closed-form property of the generator, brute-force stepping, or an
independent implementation (rocRAND's open-source MRG32k3a header).
"""
import math
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from conftest import ROOT, read_golden
import workloads

M1, M2 = 4294967087, 4294944443          # MRG32k3a moduli
P1, P2 = 2147483647, 2147462579          # MRG31k3p moduli
MODULI = {O.MRG32K3A: (M1, M2), O.MRG31K3P: (P1, P2)}
I3 = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]


# ----------------------------------------------------------- paper's values
def _paper_streams():
    c = np.array(workloads.PAPER_SEED, dtype=np.uint32)
    return O.create_streams(O.MRG31K3P, c, 4)


def test_paper_stream_table_exact():
    """Section 2.1: the 4 streams created from 12345 x 6 (24 printed words).
    Pins the generic 3x3 jump-ahead, Z = 2^134, stream 1 = the seed, and the
    newest-first word order of the printed table."""
    want = np.array([[int(v) for v in row] for row in read_golden("mrg31k3p_stream_table.txt")],
                    dtype=np.uint32)
    got = _paper_streams()
    np.testing.assert_array_equal(got[:, 0:6], want)      # current
    np.testing.assert_array_equal(got[:, 6:12], want)     # initial
    np.testing.assert_array_equal(got[:, 12:18], want)    # substream start


def test_paper_runif_example():
    """Section 2.2: 8 printed uniforms (3 decimals) = draws 1..4 of streams 1
    and 3, interleaved.  Pins step-then-output and the 1/(m1+1) scaling."""
    rows = read_golden("mrg31k3p_runif_example.txt")
    want = [float(v) for v in rows[0]]
    S = _paper_streams()
    d1 = O.stream_draws(O.MRG31K3P, S[0, :6].copy(), 4)
    d3 = O.stream_draws(O.MRG31K3P, S[2, :6].copy(), 4)
    got = np.empty(8)
    got[0::2], got[1::2] = d1, d3
    assert np.all(np.abs(got - np.array(want)) <= 0.5e-3 + 1e-12), (got, want)


def test_paper_rexp_example():
    """Section 3.2: the printed 2 x 4 exponential matrix equals -log(u) of
    draws 5 and 6 of the four streams, to every printed digit."""
    S = _paper_streams()
    draws = [O.stream_draws(O.MRG31K3P, S[s, :6].copy(), 6, O.EXPONENTIAL, O.F64, 1.0)
             for s in range(4)]
    for r, c, val, dec in read_golden("mrg31k3p_rexp_example.txt"):
        r, c, dec = int(r), int(c), int(dec)
        got = draws[2 * r + c % 2][4 + c // 2]
        assert abs(got - float(val)) <= 0.5 * 10.0 ** (-dec) + 1e-12, (r, c, got, val)


# ------------------------------------------------ closed-form generator facts
def _is_prime(n):
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:   # deterministic below 3.3e24
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _pollard(n):
    if n % 2 == 0:
        return 2
    rnd = random.Random(n)
    while True:
        c = rnd.randrange(1, n)
        f = lambda x: (x * x + c) % n
        x = y = rnd.randrange(2, n)
        d = 1
        while d == 1:
            x, y = f(x), f(f(y))
            d = math.gcd(abs(x - y), n)
        if d != n:
            return d


def _factor(n, out=None):
    out = {} if out is None else out
    for p in range(2, 1000):
        while n % p == 0:
            out[p] = out.get(p, 0) + 1
            n //= p
    if n == 1:
        return out
    if _is_prime(n):
        out[n] = out.get(n, 0) + 1
        return out
    d = _pollard(n)
    _factor(d, out)
    _factor(n // d, out)
    return out


@pytest.mark.parametrize("gen", [O.MRG32K3A, O.MRG31K3P])
@pytest.mark.parametrize("comp", [0, 1])
def test_component_has_full_period(gen, comp):
    """Each component's one-step matrix has order exactly m^3 - 1 (its
    characteristic polynomial is primitive), the defining property of the
    published parameters.  A mistyped multiplier or sign breaks it."""
    m = MODULI[gen][comp]
    order = m ** 3 - 1
    assert O.matpow(gen, comp, order) == I3
    for q in _factor(order):
        assert O.matpow(gen, comp, order // q) != I3, q


@pytest.mark.parametrize("gen", [O.MRG32K3A, O.MRG31K3P])
def test_jump_equals_stepping(gen):
    """A^k s equals k single steps, for small k, a few larger k and random
    k < 2^24 (brute force)."""
    states = workloads.random_states(6, rng_seed=7 + gen, gen=gen)
    rnd = np.random.default_rng(11)
    ks = [0, 1, 2, 3, 4, 5, 7, 64, 1000, 65537] + [int(k) for k in rnd.integers(0, 2**24, size=3)]
    for st in states:
        for k in ks:
            a = st.copy()
            O.jump(gen, a, k)
            b = st.copy()
            if k:
                O.stream_draws(gen, b, k, O.RAW, O.U32)
            np.testing.assert_array_equal(a, b, err_msg=f"k={k}")


def test_jump_one_million_steps():
    st = np.array(workloads.random_seed(), dtype=np.uint32)
    a, b = st.copy(), st.copy()
    O.jump(O.MRG32K3A, a, 10**6)
    O.stream_draws(O.MRG32K3A, b, 10**6, O.RAW, O.U32)
    np.testing.assert_array_equal(a, b)


def _matmul(A, B, m):
    return [[sum(A[r][k] * B[k][c] for k in range(3)) % m for c in range(3)] for r in range(3)]


@pytest.mark.parametrize("comp", [0, 1])
def test_stream_and_substream_spacing(comp):
    """(A^(2^76))^(2^51) = A^(2^127), A^a A^b = A^(a+b)."""
    m = MODULI[O.MRG32K3A][comp]
    K = O.matpow(O.MRG32K3A, comp, 2**76)
    J = O.matpow(O.MRG32K3A, comp, 2**127)
    P = K
    for _ in range(51):
        P = _matmul(P, P, m)
    assert P == J
    a, b = 2**100 + 12345, 2**127 + 987654321
    assert _matmul(O.matpow(O.MRG32K3A, comp, a), O.matpow(O.MRG32K3A, comp, b), m) == \
        O.matpow(O.MRG32K3A, comp, a + b)


def test_creation_is_repeated_jump():
    """Stream i starts at the seed advanced i * 2^127 steps; the creator ends
    advanced n * 2^127 steps."""
    seed = workloads.random_seed()
    c = seed.copy()
    S = O.create_streams(O.MRG32K3A, c, 5)
    for i in range(5):
        s = seed.copy()
        O.jump(O.MRG32K3A, s, i * 2**127)
        np.testing.assert_array_equal(S[i, :6], s)
    s = seed.copy()
    O.jump(O.MRG32K3A, s, 5 * 2**127)
    np.testing.assert_array_equal(c, s)


def test_worked_example_first_output():
    """Hand arithmetic from the published recurrence, seed 12345 x 6:
    x1 = (1403580 - 810728) * 12345 mod m1 = 3023790853,
    x2 = (527612 - 1370589) * 12345 mod m2 = 2478282264,
    z = x1 - x2 = 545508589, u = z / (m1 + 1) = 0.12701112204657714."""
    st = np.array([12345] * 6, dtype=np.uint32)
    z = O.step(O.MRG32K3A, st)
    assert z == 545508589
    np.testing.assert_array_equal(st, [12345, 12345, 3023790853, 12345, 12345, 2478282264])
    assert O.uniform_f64(O.MRG32K3A, z) == 545508589 * (1.0 / 4294967088.0)
    assert abs(O.uniform_f64(O.MRG32K3A, z) - 0.12701112204657714) < 1e-16


# ------------------------------------------- independent implementation
def _xcheck_binary(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = "/opt/rocm/include/rocrand/rocrand_mrg32k3a.h"
    if not (os.path.exists(hipcc) and os.path.exists(hdr)):
        pytest.skip("rocRAND header or hipcc not available")
    out = str(tmp_path_factory.mktemp("xcheck") / "xcheck")
    src = os.path.join(ROOT, "tests", "xcheck", "rocrand_mrg32k3a_xcheck.cpp")
    subprocess.run([hipcc, "-O1", "-std=c++17", src, "-o", out], check=True, cwd="/tmp",
                   capture_output=True)
    return out


def test_rocrand_crosscheck(tmp_path_factory):
    """rocRAND's MRG32k3a (oldest-first words, 2^76 substreams, 2^127
    sequences) agrees with the oracle on outputs and on jumped states."""
    exe = _xcheck_binary(tmp_path_factory)
    states = [np.array([12345] * 6, dtype=np.uint32)] + list(workloads.random_states(4, 99))
    lines, expect = [], []
    for st in states:
        w = " ".join(str(int(v)) for v in st)
        lines.append(f"{w} step 20")
        a = st.copy()
        zs = [O.step(O.MRG32K3A, a) for _ in range(20)]
        expect.append(" ".join(map(str, zs)))
        expect.append(" ".join(str(int(v)) for v in a))
        for op, k, e in (("skip", 123456789, 123456789), ("sub", 3, 3 * 2**76),
                         ("seq", 5, 5 * 2**127)):
            lines.append(f"{w} {op} {k}")
            a = st.copy()
            O.jump(O.MRG32K3A, a, e)
            expect.append(" ".join(str(int(v)) for v in a))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True)
    got = [ln.strip() for ln in res.stdout.strip().splitlines()]
    assert got == expect


# ------------------------------------------------------------ output range
def test_output_range_extremes():
    """z in [1, m1]; u in [1/(m1+1), m1/(m1+1)] strictly inside (0,1)."""
    g = O.MRG32K3A
    assert O.output(g, 5, 5) == M1                 # x1 == x2 -> m1
    assert O.output(g, M1 - 1, 0) == M1 - 1
    assert O.output(g, 1, 0) == 1
    assert O.output(g, 0, M2 - 1) == M1 - M2 + 1
    assert O.output(g, 0, 0) == M1
    u_lo, u_hi = O.uniform_f64(g, 1), O.uniform_f64(g, M1)
    assert 0.0 < u_lo and u_hi < 1.0
    assert u_hi == M1 * O.norm(g)
    assert O.norm(g) == 1.0 / (M1 + 1)


def test_f32_round_toward_zero():
    """f32 uniform = largest float <= u.  At the top: RZ gives 1 - 2^-24,
    while round-to-nearest would give exactly 1.0."""
    u_hi = O.uniform_f64(O.MRG32K3A, M1)
    assert np.float32(u_hi) == np.float32(1.0)
    assert O.f32_rz(u_hi) == np.float32(1.0 - 2.0**-24)
    rnd = np.random.default_rng(5)
    us = [O.uniform_f64(O.MRG32K3A, int(z)) for z in rnd.integers(1, M1 + 1, size=2000)]
    us += [O.uniform_f64(O.MRG32K3A, 1)]
    for u in us:
        f = O.f32_rz(u)
        assert float(f) <= u < float(np.nextafter(f, np.float32(2.0)))


# --------------------------------------------------------------- transforms
def test_box_muller_identities():
    """Algorithm 1: X^2 + Y^2 = -2 log U1 and atan2(Y, X) = 2 pi U2 (mod 2 pi);
    U2 = 0 gives (R, 0), U2 = 1/4 gives (0, R)."""
    rnd = np.random.default_rng(3)
    for _ in range(500):
        u1, u2 = rnd.uniform(1e-9, 1.0), rnd.uniform(0.0, 1.0)
        x, y = O.box_muller(u1, u2)
        r2 = -2.0 * math.log(u1)
        assert abs(x * x + y * y - r2) <= 1e-13 * max(r2, 1.0)
        th = math.atan2(y, x) % (2 * math.pi)
        d = abs(th - 2 * math.pi * u2)
        assert min(d, 2 * math.pi - d) < 1e-9
    x, y = O.box_muller(0.5, 0.0)
    assert x == math.sqrt(-2 * math.log(0.5)) and y == 0.0
    x, y = O.box_muller(0.5, 0.25)
    assert abs(x) < 1e-18 and abs(y - math.sqrt(2 * math.log(2))) < 1e-15


def test_exponential_identities():
    """Section 3.2: F(x) = 1 - exp(-rate x); our reading E = -log(u)/rate.
    exp(-rate E) = u; rate * E_rate = E_1; E(1/2) = log 2."""
    assert abs(O.exponential(0.5) - math.log(2.0)) < 1e-16
    rnd = np.random.default_rng(4)
    for u in rnd.uniform(1e-10, 1.0, size=300):
        for rate in (0.25, 1.0, 3.0):
            e = O.exponential(float(u), rate)
            assert e > 0
            assert abs(math.exp(-rate * e) - u) <= 1e-14 * u
            assert abs(rate * e - O.exponential(float(u), 1.0)) <= 1e-15 * max(1.0, rate * e)


def test_normal_moments_and_exponential_mean():
    """Loose distribution checks on 2^18 oracle draws."""
    seed = workloads.random_seed()
    S = O.create_streams(O.MRG32K3A, seed.copy(), 64)
    z = O.generate(O.MRG32K3A, S.copy(), 1 << 18, O.NORMAL, O.F64)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    e = O.generate(O.MRG32K3A, S.copy(), 1 << 18, O.EXPONENTIAL, O.F64, 2.0)
    assert abs(e.mean() - 0.5) < 0.005
    u = O.generate(O.MRG32K3A, S.copy(), 1 << 18, O.UNIFORM, O.F64)
    assert abs(u.mean() - 0.5) < 0.003 and u.min() > 0.0 and u.max() < 1.0


# --------------------------------------------------------------- seed rules
def test_seed_rules():
    g = O.MRG32K3A
    assert O.seed_valid(g, [12345] * 6)
    assert O.seed_valid(g, [M1 - 1, 0, 0, 0, 0, M2 - 1])
    assert not O.seed_valid(g, [M1, 1, 1, 1, 1, 1])
    assert not O.seed_valid(g, [1, 1, 1, M2, 1, 1])
    assert not O.seed_valid(g, [0, 0, 0, 1, 1, 1])
    assert not O.seed_valid(g, [1, 1, 1, 0, 0, 0])
    assert O.seed_valid(g, workloads.random_seed())


# -------------------------------------------------- placement and counting
@pytest.mark.parametrize("dist,dtype", [(O.UNIFORM, O.F64), (O.UNIFORM, O.F32), (O.RAW, O.U32),
                                        (O.NORMAL, O.F64), (O.EXPONENTIAL, O.F32)])
@pytest.mark.parametrize("S,n", [(7, 0), (7, 5), (7, 7), (7, 52), (1, 9), (16, 16 * 9 + 3)])
def test_placement_rule(dist, dtype, S, n):
    """out[k*S + s] is draw k of stream s; stream s makes floor(n/S) + (s < n%S)
    draws and consumes as many steps (normals: twice the pairs)."""
    seed = workloads.random_seed(1)
    streams = O.create_streams(O.MRG32K3A, seed.copy(), S)
    work = streams.copy()
    out = O.generate(O.MRG32K3A, work, n, dist, dtype, 1.0)
    for s in range(S):
        cnt = n // S + (1 if s < n % S else 0)
        cur = streams[s, :6].copy()
        d = O.stream_draws(O.MRG32K3A, cur, cnt, dist, dtype, 1.0)
        np.testing.assert_array_equal(out[s::S][:cnt], d)
        steps = 2 * ((cnt + 1) // 2) if dist == O.NORMAL else cnt
        ref = streams[s, :6].copy()
        O.jump(O.MRG32K3A, ref, steps)
        np.testing.assert_array_equal(work[s, :6], ref)
        np.testing.assert_array_equal(work[s, 6:], streams[s, 6:])


@pytest.mark.parametrize("dist", [O.NORMAL, O.EXPONENTIAL])
def test_f32_transforms_are_the_f64_values_rounded_to_nearest(dist):
    """Our reading for fp32 normals and exponentials: the fp64 value of the
    same draw rounded to the nearest float (numpy's conversion, ties to even),
    unlike fp32 uniforms, which round toward zero so as never to reach 1.
    A truncating or toward-zero narrowing would differ on about half of the
    draws."""
    seed = workloads.random_seed(9)
    st = O.create_streams(O.MRG32K3A, seed.copy(), 8)
    n = 8 * 4001
    f64 = O.generate(O.MRG32K3A, st.copy(), n, dist, O.F64, 1.5)
    f32 = O.generate(O.MRG32K3A, st.copy(), n, dist, O.F32, 1.5)
    assert f32.dtype == np.float32
    np.testing.assert_array_equal(f32, f64.astype(np.float32))
    rz = np.where(np.abs(f64.astype(np.float32).astype(np.float64)) > np.abs(f64),
                  np.nextafter(f64.astype(np.float32), np.float32(0)), f64.astype(np.float32))
    assert (rz != f32).mean() > 0.3  # the two rules are told apart on this sample


def test_normal_pairs_come_from_one_stream():
    """Draws 2p, 2p+1 of a stream are X, Y of Algorithm 1 fed by that stream's
    steps 2p, 2p+1 (our reading of the pairing)."""
    st = workloads.random_seed(2)
    d = O.stream_draws(O.MRG32K3A, st.copy(), 6, O.NORMAL)
    u = O.stream_draws(O.MRG32K3A, st.copy(), 6, O.UNIFORM)
    for p in range(3):
        x, y = O.box_muller(float(u[2 * p]), float(u[2 * p + 1]))
        assert d[2 * p] == x and d[2 * p + 1] == y


# ------------------------------------------------------------- substreams
def test_substreams():
    seed = workloads.random_seed(3)
    S = O.create_streams(O.MRG32K3A, seed.copy(), 3)
    T = S.copy()
    O.next_substream(O.MRG32K3A, T)
    for i in range(3):
        s = S[i, 12:18].copy()
        O.jump(O.MRG32K3A, s, 2**76)
        np.testing.assert_array_equal(T[i, 12:18], s)
        np.testing.assert_array_equal(T[i, 0:6], s)
        np.testing.assert_array_equal(T[i, 6:12], S[i, 6:12])
    O.advance(O.MRG32K3A, T, 1000)
    U = T.copy()
    O.reset_substream(U)
    np.testing.assert_array_equal(U[:, 0:6], T[:, 12:18])
    O.reset_stream(U)
    np.testing.assert_array_equal(U[:, 0:6], S[:, 6:12])
    np.testing.assert_array_equal(U[:, 12:18], S[:, 6:12])


@pytest.mark.parametrize("comp", [0, 1])
def test_mrg31k3p_substream_spacing(comp):
    """MRG31k3p substreams (2^72 apart, the clRNG spacing) tile its streams
    exactly: (A^(2^72))^(2^62) = A^(2^134), the stream spacing that the
    stream table printed in Section 2.1 pins; and next_substream is a jump of
    2^72 steps."""
    m = MODULI[O.MRG31K3P][comp]
    K = O.matpow(O.MRG31K3P, comp, 2**72)
    P = K
    for _ in range(62):
        P = _matmul(P, P, m)
    assert P == O.matpow(O.MRG31K3P, comp, 2**134)
    assert K != O.matpow(O.MRG31K3P, comp, 2**71) and K != O.matpow(O.MRG31K3P, comp, 2**73)


def test_mrg31k3p_next_substream_is_a_2_72_jump():
    seed = workloads.random_seed(4, gen=O.MRG31K3P)
    S = O.create_streams(O.MRG31K3P, seed.copy(), 3)
    T = S.copy()
    O.next_substream(O.MRG31K3P, T)
    for i in range(3):
        s = S[i, 12:18].copy()
        O.jump(O.MRG31K3P, s, 2**72)
        np.testing.assert_array_equal(T[i, 12:18], s)
        np.testing.assert_array_equal(T[i, 0:6], s)
