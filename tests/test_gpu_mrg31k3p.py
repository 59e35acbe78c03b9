"""GPU parity of the paper's own generator, MRG31k3p (generator id 2), with
the oracle and with the values the paper prints: the Section 2.1 stream
table from device creation, the Section 2.2 uniforms and the Section 3.2
exponentials from the GPU kernels; every distribution, dtype and launch
shape against the oracle (states and uniforms bit-exact, transforms to
1e-15 / 1e-6); substreams 2^72 apart, jumps, save/restore, tables and the
Fisher count."""
import numpy as np
import pytest

import oracle as O
import workloads
from conftest import read_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_06604_amd as P  # noqa: E402

GEN = O.MRG31K3P
G = P.MRG_GEN_MRG31K3P
P1, P2 = 2147483647, 2147462579
TOL = {P.MRG_F64: 1e-15, P.MRG_F32: 1e-6}
ODIST = {P.MRG_UNIFORM: O.UNIFORM, P.MRG_NORMAL: O.NORMAL, P.MRG_EXPONENTIAL: O.EXPONENTIAL,
         P.MRG_RAW: O.RAW}
ODT = {P.MRG_F64: O.F64, P.MRG_F32: O.F32, P.MRG_U32: O.U32}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(rec):
    return torch.from_numpy(rec.view(np.int32).copy()).cuda()


def host(t, dtype):
    a = t.cpu().numpy()
    return a.view(np.uint32) if dtype == P.MRG_U32 else a


def records(seed, n):
    return O.create_streams(GEN, np.array(seed, dtype=np.uint32), n)


def check(got, want, dist, dtype, ctx):
    if dist in (P.MRG_UNIFORM, P.MRG_RAW):
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, f"{ctx}: {bad.size} mismatches at {bad[:5]}"
        return
    g, w = got.astype(np.float64), want.astype(np.float64)
    assert np.all(np.isfinite(g)), ctx
    err = np.abs(g - w) / np.maximum(np.abs(w), 1.0)
    assert err.size == 0 or err.max() <= TOL[dtype], f"{ctx}: {err.max():.3e}"


def run(rec, n, dist, dtype, param=1.0, cfg=None):
    d = dev(rec)
    out = P.mrg_generate(d, n, dist, dtype, param, cfg=cfg, gen=G)
    torch.cuda.synchronize()
    work = rec.copy()
    want = O.generate(GEN, work, n, ODIST[dist], ODT[dtype], param, threads=8)
    check(host(out, dtype)[:n], want, dist, dtype, f"S={rec.shape[0]} n={n} {dist}/{dtype} {cfg}")
    np.testing.assert_array_equal(P.as_u32(d), work)


def paper_streams_device():
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=G)
    return P.mrg_streams_create_device(c, 4, gen=G), c


def test_device_creation_is_the_papers_table():
    """Section 2.1: createStreamsGpu from 12345 x 6, all 24 printed words."""
    want = np.array([[int(v) for v in r] for r in read_golden("mrg31k3p_stream_table.txt")], dtype=np.uint32)
    d, c = paper_streams_device()
    got = P.as_u32(d)
    for k in range(3):
        np.testing.assert_array_equal(got[:, 6 * k:6 * k + 6], want)
    oc = np.array(workloads.PAPER_SEED, dtype=np.uint32)
    O.create_streams(GEN, oc, 4)
    np.testing.assert_array_equal(P.creator_words(c), oc)


def test_device_creation_large_equals_oracle():
    seed = workloads.random_seed(71) % np.uint32(P2)
    c = P.mrg_creator_init(seed, gen=G)
    d = P.mrg_streams_create_device(c, 50001, gen=G)
    oc = np.array(seed, dtype=np.uint32)
    want = O.create_streams(GEN, oc, 50001)
    np.testing.assert_array_equal(P.as_u32(d), want)
    np.testing.assert_array_equal(P.creator_words(c), oc)


def test_paper_runif_example_on_gpu():
    """Section 2.2: the 8 printed uniforms interleave draws 1..4 of streams 1
    and 3; the GPU kernel on those two streams prints the same to 3 decimals
    and equals the oracle bit for bit."""
    d, _ = paper_streams_device()
    two = d[[0, 2]].contiguous()
    out = P.mrg_generate(two, 8, P.MRG_UNIFORM, P.MRG_F64, gen=G).cpu().numpy()[:8]
    want = np.array([float(v) for v in read_golden("mrg31k3p_runif_example.txt")[0]])
    assert np.all(np.abs(out - want) <= 0.5e-3 + 1e-12), (out, want)
    rec = records(workloads.PAPER_SEED, 4)[[0, 2]].copy()
    assert np.array_equal(out, O.generate(GEN, rec, 8))


def test_paper_rexp_example_on_gpu():
    """Section 3.2: the printed 2 x 4 exponential matrix, element (r, c) =
    draw 4 + c//2 of stream 2r + c%2, from the GPU kernel."""
    d, _ = paper_streams_device()
    out = P.mrg_generate(d, 24, P.MRG_EXPONENTIAL, P.MRG_F64, 1.0, gen=G).cpu().numpy()
    for r, c, val, dec in read_golden("mrg31k3p_rexp_example.txt"):
        r, c, dec = int(r), int(c), int(dec)
        got = out[(4 + c // 2) * 4 + 2 * r + c % 2]
        assert abs(got - float(val)) <= 0.5 * 10.0 ** (-dec) + 1e-12, (r, c, got, val)


CASES = [(P.MRG_UNIFORM, P.MRG_F64), (P.MRG_UNIFORM, P.MRG_F32), (P.MRG_RAW, P.MRG_U32),
         (P.MRG_NORMAL, P.MRG_F64), (P.MRG_NORMAL, P.MRG_F32), (P.MRG_EXPONENTIAL, P.MRG_F64),
         (P.MRG_EXPONENTIAL, P.MRG_F32)]


@pytest.mark.parametrize("dist,dtype", CASES)
@pytest.mark.parametrize("S,n", [(1, 1001), (77, 77 * 21 + 5), (130, 130 * 9 + 129), (512, 512 * 40),
                                 (4099, 4099 * 3 + 7)])
def test_distributions_match_oracle(dist, dtype, S, n):
    run(records(workloads.random_seed(S) % np.uint32(P2), S), n, dist, dtype, 2.5)


@pytest.mark.parametrize("cfg", [dict(chunk=1, block=64), dict(chunk=7, block=512), dict(streams_per_lane=2),
                                 dict(streams_per_lane=4, chunk=3, xcd_remap=1), dict(arith=1, chunk=5),
                                 dict(nontemporal=1, block=1024, chunk=100000)], ids=str)
def test_launch_shapes(cfg):
    rec = records(workloads.random_seed(33) % np.uint32(P2), 300)
    run(rec, 300 * 37 + 123, P.MRG_UNIFORM, P.MRG_F64, cfg=cfg)
    run(rec, 300 * 37 + 123, P.MRG_UNIFORM, P.MRG_F32, cfg=cfg)
    run(rec, 300 * 11 + 5, P.MRG_NORMAL, P.MRG_F64, cfg=cfg)


@pytest.mark.parametrize("S,n", [(65536, 65536 * 1100), (100003, 100003 * 700 + 77)])
def test_default_plan_lockstep_at_scale(S, n):
    """fp64 uniforms in the automatic full-size shape (lockstep blocks) at
    these stream counts (several chunks per stream; an odd stream count with
    spare waves)."""
    plan = P.mrg_generate_plan(S, 1 << 30, gen=G)
    assert plan["lockstep"] == 1, plan
    cfg = {k: v for k, v in plan.items() if k != "chunk"}
    run(records(workloads.random_seed(S) % np.uint32(P2), S), n, P.MRG_UNIFORM, P.MRG_F64, cfg=cfg)


def test_extreme_states():
    """Words at the top of their ranges and x1 == x2 (z = p1)."""
    st = np.array([[P1 - 1, P1 - 1, P1 - 1, P2 - 1, P2 - 1, P2 - 1],
                   [1, 0, 0, 1, 0, 0],
                   [0, 0, 1, 0, 0, 1],
                   [P1 - 1, 0, P1 - 1, 0, P2 - 1, 0],
                   [5, 5, 5, 5, 5, 5],
                   [0x7fffff00, 0x40000000, 0x3fffffff, P2 - 2, 0x40000000, 1]], dtype=np.uint32)
    rec = np.concatenate([st, st, st], axis=1)
    run(rec, 6 * 60, P.MRG_RAW, P.MRG_U32)
    run(rec, 6 * 60, P.MRG_UNIFORM, P.MRG_F32)
    run(rec, 6 * 60 + 1, P.MRG_UNIFORM, P.MRG_F64, cfg=dict(chunk=4))


def test_many_chunks_one_stream():
    rec = records(workloads.random_seed(4) % np.uint32(P2), 1)
    run(rec, 200003, P.MRG_UNIFORM, P.MRG_F64, cfg=dict(chunk=777))
    run(rec, 200003, P.MRG_NORMAL, P.MRG_F64, cfg=dict(chunk=333))


def test_substreams_and_advance():
    rec = records(workloads.random_seed(12) % np.uint32(P2), 129)
    d = dev(rec)
    work = rec.copy()
    P.mrg_streams_advance(d, 123456789012345, gen=G)
    O.advance(GEN, work, 123456789012345)
    P.mrg_streams_reset(d, P.MRG_NEXT_SUBSTREAM, gen=G)
    O.next_substream(GEN, work)
    P.mrg_streams_advance(d, 2**64 - 1, gen=G)
    O.advance(GEN, work, 2**64 - 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)
    P.mrg_streams_reset(d, P.MRG_RESET_SUBSTREAM, gen=G)
    O.reset_substream(work)
    P.mrg_streams_reset(d, P.MRG_NEXT_SUBSTREAM, gen=G)
    O.next_substream(GEN, work)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)
    P.mrg_streams_reset(d, P.MRG_RESET_STREAM, gen=G)
    O.reset_stream(work)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)


# as in the MRG32k3a tests: base-64 digits 1 and 63 at every position
ADVANCE_COUNTS = [c for d in range(11) for v in (1, 63) for c in [v << (6 * d)] if c < 2**64] + \
    [2**64 - 1, 0x0123456789ABCDEF, 3]


def test_advance_every_digit():
    """Each advance against the oracle's, state by state."""
    rec = records(workloads.random_seed(13) % np.uint32(P2), 67)
    d = dev(rec)
    work = rec.copy()
    for c in ADVANCE_COUNTS:
        P.mrg_streams_advance(d, c, gen=G)
        O.advance(GEN, work, c)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(P.as_u32(d), work, err_msg=f"count {c:#x}")



def test_export_import_roundtrip():
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=G)
    d = P.mrg_streams_create_device(c, 300, gen=G)
    P.mrg_generate(d, 300 * 5 + 1, P.MRG_NORMAL, P.MRG_F64, gen=G)
    blob = P.mrg_streams_export(d, creator=c, gen=G)
    d2 = P.new_streams_tensor(300)
    c2 = P.mrg_creator()
    assert P.mrg_streams_import(blob, d2, creator=c2, gen=G) == 300
    with pytest.raises(P.MrgError):  # saved as MRG31k3p, not MRG32k3a
        P.mrg_streams_import(blob, d2)
    a = P.mrg_generate(d, 3000, gen=G)
    b = P.mrg_generate(d2, 3000, gen=G)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    np.testing.assert_array_equal(P.creator_words(c), P.creator_words(c2))


def test_tables_and_fisher_with_mrg31k3p():
    """Section 4 ran fisher.sim on MRG31k3p streams: tables bit-exact and
    the count exact against the oracle on the same generator."""
    n = 5000
    I, J, rows, cols = workloads.contingency_margins(n, rng_seed=8)
    rec = records(workloads.PAPER_SEED, n)
    d = dev(rec)
    tabs, stats = P.mrg_tables_sample(d, *(torch.from_numpy(a).cuda() for a in (I, J, rows, cols)),
                                      stats=True, gen=G)
    work = rec.copy()
    wtabs, wstats = O.tables(GEN, work, I, J, rows, cols)
    np.testing.assert_array_equal(tabs[:n].cpu().numpy(), wtabs)
    np.testing.assert_array_equal(P.as_u32(d), work)
    tab = np.array([[int(v) for v in r] for r in read_golden("fisher_month.txt")], dtype=np.int32)
    B = 4096
    rec = records(workloads.PAPER_SEED, B)
    d = dev(rec)
    cnt, _, _ = P.mrg_fisher_sim(d, tab, gen=G)
    wcnt, _ = O.fisher_count(GEN, rec.copy(), tab)
    assert int(cnt.item()) == wcnt


def test_throughput_size_every_number():
    """The benchmarked MRG31k3p launch: 262,144 streams created on the device
    from the paper's seed, 4,096 fp64 uniforms each in the automatic shape;
    all 2^30 numbers bit-exact against the oracle in blocks of 16,384 streams,
    and every final state."""
    S, per, blk = 262144, 4096, 16384
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=G)
    d = P.mrg_streams_create_device(c, S, gen=G)
    rec = O.create_streams(GEN, np.array(workloads.PAPER_SEED, dtype=np.uint32), S)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), rec)
    out = P.mrg_generate(d, S * per, P.MRG_UNIFORM, P.MRG_F64, gen=G)
    torch.cuda.synchronize()
    fin = rec[:, 0:6].copy()
    O.jump_many(GEN, fin, per)
    np.testing.assert_array_equal(P.as_u32(d)[:, 0:6], fin)
    mat = out.view(per, S)
    for s0 in range(0, S, blk):
        got = mat[:, s0:s0 + blk].cpu().numpy()
        want = O.generate(GEN, rec[s0:s0 + blk].copy(), per * blk, O.UNIFORM, O.F64, threads=16).reshape(per, blk)
        assert np.array_equal(got, want), f"streams {s0}..{s0 + blk - 1}"
    del out
