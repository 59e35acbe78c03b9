"""GPU parity of the normal (Algorithm 1, Section 3.1) and exponential
(Section 3.2) transforms at their edge inputs, and an exhaustive check of the
library's own log / sqrt / sin(pi t) / cos(pi t) over every generator output.

Edge inputs come from crafted states (tests/crafted.py) whose next outputs are
chosen integers z: the smallest and largest uniforms (z = 1, 2, 3 and m1 - 2,
m1 - 1, m1: u near 2^-32 gives the largest radius and exponential, u near 1
the smallest), and the angles where the library's quadrant reduction changes
branch -- 2u2 near k/4 for k = 1..7 (z near k (m1+1)/8, including the
quadrant boundaries 2u2 near 1/2, 1, 3/2, where sin or cos is zero or nearly
so).  Each value is compared with the oracle under |gpu - ref| <=
tol * max(|ref|, 1), tol = 1e-15 (f64) / 1e-6 (f32).
"""
import numpy as np
import pytest

import crafted as C
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_06604_amd as P  # noqa: E402

TOL = {P.MRG_F64: 1e-15, P.MRG_F32: 1e-6}
ODT = {P.MRG_F64: O.F64, P.MRG_F32: O.F32}
ODIST = {P.MRG_NORMAL: O.NORMAL, P.MRG_EXPONENTIAL: O.EXPONENTIAL}
GENS = [P.MRG_GEN_MRG32K3A, P.MRG_GEN_MRG31K3P]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def extremes(gen):
    m1 = C.modulus1(gen)
    return [1, 2, 3, m1 - 2, m1 - 1, m1]


def angle_points(gen):
    """z with 2 z/(m1+1) within a few steps of k/4, k = 1..7."""
    m1 = C.modulus1(gen)
    q8 = (m1 + 1) // 8  # exact for both generators: m1 + 1 is 2^4 * 268435443 or 2^31
    return [k * q8 + d for k in range(1, 8) for d in (-2, -1, 0, 1, 2)]


def crafted_records(gen, triples, seed):
    rng = np.random.default_rng(seed)
    states = [C.state_with_outputs(gen, list(t), rng) for t in triples]
    rec = C.records(states)
    for st, t in zip(states, triples):  # the crafting itself, checked by the oracle
        s = st.copy()
        assert [O.step(gen, s) for _ in t] == list(t)
    return rec


def check(got, want, dtype, ctx):
    g = got.astype(np.float64)
    w = want.astype(np.float64)
    assert np.all(np.isfinite(g)), ctx
    err = np.abs(g - w) / np.maximum(np.abs(w), 1.0)
    assert err.max() <= TOL[dtype], f"{ctx}: max err {err.max():.3e} at {err.argmax()}: {g[err.argmax()]} vs {w[err.argmax()]}"


def run(gen, rec, n, dist, dtype, param, cfg=None):
    d = torch.from_numpy(rec.view(np.int32).copy()).cuda()
    out = P.mrg_generate(d, n, dist, dtype, param, cfg=cfg, gen=gen)
    torch.cuda.synchronize()
    work = rec.copy()
    want = O.generate(gen, work, n, ODIST[dist], ODT[dtype], param)
    check(out.cpu().numpy()[:n], want, dtype, f"gen={gen} dist={dist} dtype={dtype} cfg={cfg}")
    np.testing.assert_array_equal(P.as_u32(d), work)


def normal_triples(gen, rng):
    """(u1, u2, third) output triples: every edge value as u1 and as u2, the
    two extreme radii against every angle point, random fill elsewhere."""
    m1 = C.modulus1(gen)
    r = lambda: int(rng.integers(1, m1 + 1))  # noqa: E731
    targets = extremes(gen) + angle_points(gen)
    out = [(t, r(), r()) for t in targets] + [(r(), t, r()) for t in targets]
    out += [(e, a, r()) for e in (1, m1) for a in angle_points(gen)]
    if len(out) % 2:
        out.append((r(), r(), r()))
    return out


CFGS = [None, dict(streams_per_lane=2), dict(streams_per_lane=1, chunk=1), dict(arith=1)]


@pytest.mark.parametrize("cfg", CFGS, ids=str)
@pytest.mark.parametrize("dtype", [P.MRG_F64, P.MRG_F32])
@pytest.mark.parametrize("gen", GENS)
def test_normal_edge_inputs(gen, dtype, cfg):
    """Box-Muller pairs with u1 and u2 at the edges (three draws per stream:
    one whole pair, then an X whose Y is dropped)."""
    rng = np.random.default_rng(100 + gen)
    triples = normal_triples(gen, rng)
    rec = crafted_records(gen, triples, 200 + gen)
    run(gen, rec, 3 * len(triples), P.MRG_NORMAL, dtype, 1.0, cfg)


@pytest.mark.parametrize("rate", [1.0, 0.75])
@pytest.mark.parametrize("dtype", [P.MRG_F64, P.MRG_F32])
@pytest.mark.parametrize("gen", GENS)
def test_exponential_edge_inputs(gen, dtype, rate):
    """-log(u)/rate at the smallest and largest uniforms and at the angle
    points (no branch there, but a spread of exponents)."""
    rng = np.random.default_rng(300 + gen)
    m1 = C.modulus1(gen)
    targets = extremes(gen) + angle_points(gen)
    triples = [(t, int(rng.integers(1, m1 + 1)), t) for t in targets]
    rec = crafted_records(gen, triples, 400 + gen)
    for cfg in (None, dict(streams_per_lane=1, chunk=1)):
        run(gen, rec, 3 * len(triples), P.MRG_EXPONENTIAL, dtype, rate, cfg)


# ---------------------------------------------------- every generator output
FNS = {P.MRG_CHECK_LOG: "log", P.MRG_CHECK_SQRT: "sqrt", P.MRG_CHECK_SINPI: "sinpi",
       P.MRG_CHECK_COSPI: "cospi"}


@pytest.mark.parametrize("fn", list(FNS), ids=lambda f: FNS[f])
@pytest.mark.parametrize("gen", GENS)
def test_transcendentals_every_output(gen, fn):
    """Over every z in [1, m1] (2^32 - 209 values for MRG32k3a, 2^31 - 1 for
    MRG31k3p) the library's own function stays within 2 ulp of the HIP device
    math library (the square root of the radius argument is bit-identical),
    and at the input where the two differ most the transforms still match the
    oracle's long-double values within the tolerance."""
    m1 = C.modulus1(gen)
    r = P.mrg_transform_accuracy(fn, gen=gen)
    print(f"gen={gen} {FNS[fn]}: ulp histogram {r['hist']}, max {r['max_ulp']} at z={r['z_at_max']}")
    assert sum(r["hist"]) == m1
    assert r["hist"][3] == 0 and r["hist"][4] == 0, r
    if fn == P.MRG_CHECK_SQRT:
        assert r["hist"][0] == m1, r
    z = r["z_at_max"]
    assert 1 <= z <= m1
    rng = np.random.default_rng(z % 1000003)
    other = lambda: int(rng.integers(1, m1 + 1))  # noqa: E731
    if fn in (P.MRG_CHECK_LOG, P.MRG_CHECK_SQRT):
        triples = [(z, other(), z), (z, z, other())]
        for dtype in (P.MRG_F64, P.MRG_F32):
            rec = crafted_records(gen, triples, z)
            run(gen, rec, 3 * len(triples), P.MRG_NORMAL, dtype, 1.0)
            run(gen, rec, 3 * len(triples), P.MRG_EXPONENTIAL, dtype, 1.0)
    else:
        triples = [(other(), z, other()), (1, z, other()), (m1, z, other())]
        triples.append((other(), other(), other()))
        for dtype in (P.MRG_F64, P.MRG_F32):
            rec = crafted_records(gen, triples, z)
            run(gen, rec, 3 * len(triples), P.MRG_NORMAL, dtype, 1.0)


FNS32 = {P.MRG_CHECK_LOG_F32OUT: "log", P.MRG_CHECK_SQRT_F32OUT: "sqrt", P.MRG_CHECK_SINPI_F32OUT: "sinpi",
         P.MRG_CHECK_COSPI_F32OUT: "cospi"}


@pytest.mark.parametrize("fn", list(FNS32), ids=lambda f: FNS32[f] + "_f32out")
@pytest.mark.parametrize("gen", GENS)
def test_f32out_transcendentals_every_output(gen, fn):
    """The shorter evaluations that fp32 normals and exponentials use stay
    within 2e-7 relative of the HIP device math library over every z in
    [1, m1]: d doubles apart is at most d * 2^-52 relative.  Rounded to
    float (2^-24 relative) the stored value is then within 3e-7 of the exact
    one, against the 1e-6 fp32 tolerance; at the worst input the fp32
    transforms match the oracle within that tolerance."""
    m1 = C.modulus1(gen)
    r = P.mrg_transform_accuracy(fn, gen=gen)
    rel = r["max_ulp"] * 2.0 ** -52
    print(f"gen={gen} {FNS32[fn]} f32out: max {r['max_ulp']} doubles apart (<= {rel:.3e} relative) "
          f"at z={r['z_at_max']}")
    assert sum(r["hist"]) == m1
    assert rel <= 2e-7, r
    z = r["z_at_max"]
    assert 1 <= z <= m1
    rng = np.random.default_rng(z % 1000003)
    other = lambda: int(rng.integers(1, m1 + 1))  # noqa: E731
    if fn in (P.MRG_CHECK_LOG_F32OUT, P.MRG_CHECK_SQRT_F32OUT):
        triples = [(z, other(), z), (z, z, other())]
        rec = crafted_records(gen, triples, z)
        run(gen, rec, 3 * len(triples), P.MRG_NORMAL, P.MRG_F32, 1.0)
        run(gen, rec, 3 * len(triples), P.MRG_EXPONENTIAL, P.MRG_F32, 1.0)
    else:
        triples = [(other(), z, other()), (1, z, other()), (m1, z, other())]
        rec = crafted_records(gen, triples, z)
        run(gen, rec, 3 * len(triples), P.MRG_NORMAL, P.MRG_F32, 1.0)


def test_transform_accuracy_partial_range_and_errors():
    """A sub-range counts exactly its inputs; bad ranges are refused."""
    r = P.mrg_transform_accuracy(P.MRG_CHECK_LOG, 1000, 1000 + 12345)
    assert sum(r["hist"]) == 12345 and 1000 <= r["z_at_max"] < 1000 + 12345
    r = P.mrg_transform_accuracy(P.MRG_CHECK_COSPI, 5, 5)
    assert sum(r["hist"]) == 0
    for lo, hi in ((0, 10), (10, 5), (1, 4294967087 + 2)):
        with pytest.raises(P.MrgError):
            P.mrg_transform_accuracy(P.MRG_CHECK_LOG, lo, hi)
    with pytest.raises(P.MrgError):
        P.mrg_transform_accuracy(8, 1, 10)
