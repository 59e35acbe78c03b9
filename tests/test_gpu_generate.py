"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

States, uniforms (f64, f32 round-toward-zero) and raw integers must match
bit for bit.  Normals and exponentials must satisfy
|gpu - ref| <= tol * max(|ref|, 1) with tol = 1e-15 (f64) and 1e-6 (f32).
"""
import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_06604_amd as P  # noqa: E402

GEN = O.MRG32K3A
TOL = {P.MRG_F64: 1e-15, P.MRG_F32: 1e-6}
ODIST = {P.MRG_UNIFORM: O.UNIFORM, P.MRG_NORMAL: O.NORMAL, P.MRG_EXPONENTIAL: O.EXPONENTIAL,
         P.MRG_RAW: O.RAW}
ODT = {P.MRG_F64: O.F64, P.MRG_F32: O.F32, P.MRG_U32: O.U32}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def dev_streams(host_records):
    t = torch.from_numpy(host_records.view(np.int32).copy()).cuda()
    return t


def host_out(t, dtype):
    a = t.cpu().numpy()
    return a.view(np.uint32) if dtype == P.MRG_U32 else a


def check_values(got, want, dist, dtype, ctx=""):
    if dist in (P.MRG_UNIFORM, P.MRG_RAW):
        if not np.array_equal(got, want):
            bad = np.nonzero(got != want)[0]
            raise AssertionError(f"{ctx}: {bad.size} mismatches, first at {bad[:5]}: "
                                 f"{got[bad[:5]]} vs {want[bad[:5]]}")
        return
    if got.size == 0:
        assert want.size == 0, ctx
        return
    g = got.astype(np.float64)
    w = want.astype(np.float64)
    err = np.abs(g - w) / np.maximum(np.abs(w), 1.0)
    assert np.all(np.isfinite(g)), ctx
    assert err.max() <= TOL[dtype], f"{ctx}: max rel err {err.max():.3e} at {err.argmax()}"


def run_case(records, n, dist, dtype, param=1.0, cfg=None):
    """Generate on the GPU and with the oracle; compare outputs and states."""
    S = records.shape[0]
    d = dev_streams(records)
    out = P.mrg_generate(d, n, dist, dtype, param, cfg=cfg)
    torch.cuda.synchronize()
    work = records.copy()
    want = O.generate(GEN, work, n, ODIST[dist], ODT[dtype], param, threads=8)
    got = host_out(out, dtype)[:n]
    check_values(got, want, dist, dtype, ctx=f"S={S} n={n} dist={dist} dtype={dtype} cfg={cfg}")
    np.testing.assert_array_equal(P.as_u32(d), work, err_msg=f"states S={S} n={n} cfg={cfg}")


# --------------------------------------------------------------- the paper's small config
def test_plain_small_1024_streams_bit_exact():
    """Seed 12345 x 6; 1024 streams by 2^127 jumps (device and host creation);
    1024 fp64 uniforms each: every value and every final state bit-exact."""
    c_dev = P.mrg_creator_init(workloads.PAPER_SEED)
    c_host = P.mrg_creator_init(workloads.PAPER_SEED)
    d = P.mrg_streams_create_device(c_dev, 1024)
    h = P.mrg_streams_create_host(c_host, 1024)
    oc = np.array(workloads.PAPER_SEED, dtype=np.uint32)
    want_rec = O.create_streams(GEN, oc, 1024)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), want_rec)
    np.testing.assert_array_equal(h, want_rec)
    np.testing.assert_array_equal(P.creator_words(c_dev), oc)
    np.testing.assert_array_equal(P.creator_words(c_host), oc)
    out = P.mrg_generate(d, 1 << 20, P.MRG_UNIFORM, P.MRG_F64)
    torch.cuda.synchronize()
    work = want_rec.copy()
    want = O.generate(GEN, work, 1 << 20, O.UNIFORM, O.F64)
    got = out.cpu().numpy()
    assert np.array_equal(got, want)
    assert got.min() > 0.0 and got.max() < 1.0
    np.testing.assert_array_equal(P.as_u32(d), work)
    # the first value is the worked example's u
    assert got[0] == 545508589 * (1.0 / 4294967088.0)


# ------------------------------------------------------ launch shapes and arithmetic
CFGS = [None,
        dict(arith=1), dict(arith=2),
        dict(block=64, chunk=1, arith=1), dict(block=64, chunk=1, arith=2),
        dict(block=128, chunk=2, arith=1), dict(block=1024, chunk=5, arith=2, nontemporal=1),
        dict(block=256, chunk=64, arith=1, nontemporal=1), dict(block=512, chunk=7, arith=2),
        dict(block=256, chunk=100000, arith=1),
        dict(streams_per_lane=1, arith=2), dict(streams_per_lane=2, arith=1, chunk=9),
        dict(streams_per_lane=2, arith=2, xcd_remap=1, nontemporal=1),
        dict(streams_per_lane=2, arith=2, xcd_remap=1, block=64, chunk=3)]


@pytest.mark.parametrize("cfg", CFGS, ids=lambda c: str(c))
def test_schedule_invariance_uniform(cfg):
    """Every launch shape and both arithmetic forms give the oracle's bits."""
    rec = O.create_streams(GEN, workloads.random_seed(21), 300)
    run_case(rec, 300 * 37 + 123, P.MRG_UNIFORM, P.MRG_F64, cfg=cfg)


@pytest.mark.parametrize("cfg", [dict(arith=1, chunk=4), dict(arith=2, chunk=3), dict(arith=2, chunk=0),
                                 dict(arith=1, chunk=5, streams_per_lane=4, xcd_remap=1),
                                 dict(arith=2, chunk=2, streams_per_lane=2, nontemporal=1)],
                         ids=str)
@pytest.mark.parametrize("dist,dtype", [(P.MRG_UNIFORM, P.MRG_F32), (P.MRG_RAW, P.MRG_U32),
                                        (P.MRG_NORMAL, P.MRG_F64), (P.MRG_NORMAL, P.MRG_F32),
                                        (P.MRG_EXPONENTIAL, P.MRG_F64),
                                        (P.MRG_EXPONENTIAL, P.MRG_F32)])
@pytest.mark.parametrize("S,n", [(77, 77 * 20), (77, 77 * 21 + 5), (130, 130 * 9 + 129), (1, 1001),
                                 (256, 256 * 13 + 255), (260, 260 * 7 + 1)])
def test_distributions(cfg, dist, dtype, S, n):
    rec = O.create_streams(GEN, workloads.random_seed(S + n), S)
    run_case(rec, n, dist, dtype, 1.0, cfg)


LOCK_CFGS = [dict(block=512, streams_per_lane=2, lockstep=1, nontemporal=1, xcd_remap=1),
             dict(block=512, streams_per_lane=2, lockstep=1, chunk=7),
             dict(block=256, streams_per_lane=4, lockstep=1, chunk=5, nontemporal=1),
             dict(block=1024, streams_per_lane=1, lockstep=1, chunk=4),
             dict(block=1024, streams_per_lane=2, lockstep=1, chunk=16, arith=1)]


@pytest.mark.parametrize("cfg", LOCK_CFGS, ids=str)
@pytest.mark.parametrize("dist,dtype", [(P.MRG_UNIFORM, P.MRG_F64), (P.MRG_UNIFORM, P.MRG_F32),
                                        (P.MRG_RAW, P.MRG_U32), (P.MRG_NORMAL, P.MRG_F64),
                                        (P.MRG_EXPONENTIAL, P.MRG_F32)])
@pytest.mark.parametrize("S,n", [(2048, 2048 * 37 + 1001), (4096, 4096 * 9), (1000, 1000 * 11 + 7)])
def test_lockstep_blocks(cfg, dist, dtype, S, n):
    """Blocks whose waves pass a barrier per row (every wave full: S a
    multiple of the block's streams; otherwise the option is ignored) give
    the oracle's values, ragged tail and chunk boundaries included."""
    rec = O.create_streams(GEN, workloads.random_seed(S + 3 * n), S)
    run_case(rec, n, dist, dtype, 1.0, cfg)


@pytest.mark.parametrize("S,n", [(100003, 100003 * 700 + 77), (100000, 100000 * 700 + 99999), (65536, 65536 * 1100)])
def test_default_plan_lockstep_at_scale(S, n):
    """The automatic full-size shape (lockstep blocks) at these stream counts,
    over fewer draws per stream: ragged stream counts (the last block's spare
    waves only pass the barriers), odd S (one stream per lane, rows off
    128-byte lines, ordinary stores) and a ragged tail; every value and state
    against the oracle."""
    plan = P.mrg_generate_plan(S, 1 << 30)
    assert plan["lockstep"] == 1, plan
    cfg = {k: v for k, v in plan.items() if k != "chunk"}
    rec = O.create_streams(GEN, workloads.random_seed(S), S)
    run_case(rec, n, P.MRG_UNIFORM, P.MRG_F64, 1.0, cfg)


@pytest.mark.parametrize("rate", [0.5, 3.0])
def test_exponential_rate(rate):
    rec = O.create_streams(GEN, workloads.random_seed(5), 64)
    run_case(rec, 64 * 50 + 3, P.MRG_EXPONENTIAL, P.MRG_F64, rate)


@pytest.mark.parametrize("S,n", [(5, 0), (100, 7), (100, 99), (64, 64), (65, 1), (1, 3)])
def test_edges(S, n):
    """Empty calls, fewer numbers than streams, single streams."""
    rec = O.create_streams(GEN, workloads.random_seed(9), S)
    for dist, dtype in [(P.MRG_UNIFORM, P.MRG_F64), (P.MRG_NORMAL, P.MRG_F64)]:
        run_case(rec, n, dist, dtype)


def test_arbitrary_states_not_stream_starts():
    """States far from stream starts (random valid words)."""
    st = workloads.random_states(200, 77)
    rec = np.zeros((200, 18), dtype=np.uint32)
    rec[:, 0:6] = st
    rec[:, 6:12] = st
    rec[:, 12:18] = st
    run_case(rec, 200 * 33 + 17, P.MRG_UNIFORM, P.MRG_F64, cfg=dict(arith=1, chunk=8))
    run_case(rec, 200 * 33 + 17, P.MRG_UNIFORM, P.MRG_F64, cfg=dict(arith=2, chunk=8))
    run_case(rec, 200 * 33 + 17, P.MRG_RAW, P.MRG_U32, cfg=dict(arith=2))


def test_extreme_states():
    """Words at the top of their ranges, and the z = m1 output (x1 == x2)."""
    M1, M2 = 4294967087, 4294944443
    st = np.array([[M1 - 1, M1 - 1, M1 - 1, M2 - 1, M2 - 1, M2 - 1],
                   [1, 0, 0, 1, 0, 0],
                   [0, 0, 1, 0, 0, 1],
                   [M1 - 1, 0, M1 - 1, 0, M2 - 1, 0],
                   [5, 5, 5, 5, 5, 5]], dtype=np.uint32)
    rec = np.concatenate([st, st, st], axis=1)
    for cfg in (dict(arith=1), dict(arith=2)):
        run_case(rec, 5 * 40, P.MRG_RAW, P.MRG_U32, cfg=cfg)
        run_case(rec, 5 * 40, P.MRG_UNIFORM, P.MRG_F32, cfg=cfg)


@pytest.mark.parametrize("spl", [1, 2, 4])
def test_misaligned_output_and_odd_stream_counts(spl):
    """Outputs offset by one element and stream counts not divisible by the
    requested streams per lane fall back to narrower stores, same bits."""
    for S in (130, 131, 388):
        rec = O.create_streams(GEN, workloads.random_seed(S), S)
        n = S * 10 + 3
        d = dev_streams(rec)
        buf = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
        view = buf[1:]
        P.mrg_generate(d, n, P.MRG_UNIFORM, P.MRG_F32, out=view, cfg=dict(streams_per_lane=spl))
        torch.cuda.synchronize()
        work = rec.copy()
        want = O.generate(GEN, work, n, O.UNIFORM, O.F32)
        assert np.array_equal(view.cpu().numpy(), want)
        assert buf[0].item() == 0.0
        np.testing.assert_array_equal(P.as_u32(d), work)


def test_many_chunks_one_stream():
    """One long stream split over many work-items (chunk jumps of many bits)."""
    rec = O.create_streams(GEN, workloads.random_seed(4), 1)
    run_case(rec, 200003, P.MRG_UNIFORM, P.MRG_F64, cfg=dict(chunk=777, arith=1))
    run_case(rec, 200003, P.MRG_NORMAL, P.MRG_F64, cfg=dict(chunk=333, arith=2))


# ------------------------------------------------------------ streams API
def test_device_creation_equals_host_creation_large():
    seed = workloads.random_seed()
    c1, c2 = P.mrg_creator_init(seed), P.mrg_creator_init(seed)
    d = P.mrg_streams_create_device(c1, 70001)
    h = P.mrg_streams_create_host(c2, 70001)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), h)
    np.testing.assert_array_equal(P.creator_words(c1), P.creator_words(c2))
    oc = seed.copy()
    want = O.create_streams(GEN, oc, 70001)
    np.testing.assert_array_equal(h, want)
    np.testing.assert_array_equal(P.creator_words(c1), oc)


def test_substreams_and_advance():
    seed = workloads.random_seed(12)
    rec = O.create_streams(GEN, seed.copy(), 129)
    d = dev_streams(rec)
    work = rec.copy()
    P.mrg_streams_advance(d, 123456789012345)
    O.advance(GEN, work, 123456789012345)
    P.mrg_streams_reset(d, P.MRG_NEXT_SUBSTREAM)
    O.next_substream(GEN, work)
    P.mrg_streams_advance(d, 2**64 - 1)
    O.advance(GEN, work, 2**64 - 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)
    P.mrg_streams_reset(d, P.MRG_RESET_SUBSTREAM)
    O.reset_substream(work)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)
    P.mrg_streams_reset(d, P.MRG_NEXT_SUBSTREAM)
    P.mrg_streams_reset(d, P.MRG_NEXT_SUBSTREAM)
    O.next_substream(GEN, work)
    O.next_substream(GEN, work)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)
    P.mrg_streams_reset(d, P.MRG_RESET_STREAM)
    O.reset_stream(work)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), work)

# Counts whose base-64 digits are 1 and 63 at every position, the largest
# count, and a mixed one: the device jump takes one table product per digit.
ADVANCE_COUNTS = [c for d in range(11) for v in (1, 63) for c in [v << (6 * d)] if c < 2**64] + \
    [2**64 - 1, 0x0123456789ABCDEF, 3]


def test_advance_every_digit():
    """Each advance against the oracle's, state by state."""
    rec = O.create_streams(GEN, workloads.random_seed(13), 67)
    d = dev_streams(rec)
    work = rec.copy()
    for c in ADVANCE_COUNTS:
        P.mrg_streams_advance(d, c)
        O.advance(GEN, work, c)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(P.as_u32(d), work, err_msg=f"count {c:#x}")



def test_export_import_roundtrip_continues_identically():
    """Save/restore (saveRDS/readRDS example): generation continued from a
    restored copy equals uninterrupted generation."""
    c = P.mrg_creator_init(workloads.random_seed(31))
    d = P.mrg_streams_create_device(c, 500)
    P.mrg_generate(d, 500 * 11 + 7, P.MRG_NORMAL, P.MRG_F64)
    blob = P.mrg_streams_export(d, creator=c)
    d2 = P.new_streams_tensor(500)
    c2 = P.mrg_creator()
    assert P.mrg_streams_import(blob, d2, creator=c2) == 500
    np.testing.assert_array_equal(P.creator_words(c2), P.creator_words(c))
    a = P.mrg_generate(d, 500 * 20, P.MRG_UNIFORM, P.MRG_F64)
    b = P.mrg_generate(d2, 500 * 20, P.MRG_UNIFORM, P.MRG_F64)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    np.testing.assert_array_equal(P.as_u32(d), P.as_u32(d2))
    # new streams from the restored creator continue the same sequence
    e1 = P.mrg_streams_create_device(c, 3)
    e2 = P.mrg_streams_create_device(c2, 3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(e1), P.as_u32(e2))


def test_reproducible_by_creation_order():
    """Same creator seed and creation order give identical numbers (Section 2.2
    reproducibility loop)."""
    def program():
        c = P.mrg_creator_init([11, 22, 33, 44, 55, 66])
        rows = []
        for i in range(1, 11):
            if i % 2 == 0:
                s = P.mrg_streams_create_device(c, 4)
                rows.append(P.mrg_generate(s, 6, P.MRG_NORMAL, P.MRG_F64).cpu().numpy()[:6])
            elif i == 3:
                s = P.mrg_streams_create_device(c, 4)
                rows.append(P.mrg_generate(s, 6, P.MRG_UNIFORM, P.MRG_F64).cpu().numpy()[:6])
            else:
                s = P.mrg_streams_create_device(c, 8)
                rows.append(P.mrg_generate(s, 6, P.MRG_EXPONENTIAL, P.MRG_F64).cpu().numpy()[:6])
        return np.array(rows)
    a, b = program(), program()
    assert np.array_equal(a, b)


# ------------------------------------------------------------ full size
FULL_VARIANTS = [(P.MRG_UNIFORM, P.MRG_F64), (P.MRG_UNIFORM, P.MRG_F32), (P.MRG_RAW, P.MRG_U32),
                 (P.MRG_NORMAL, P.MRG_F64), (P.MRG_EXPONENTIAL, P.MRG_F64), (P.MRG_NORMAL, P.MRG_F32),
                 (P.MRG_EXPONENTIAL, P.MRG_F32)]


@pytest.mark.parametrize("S", [262144, 65536])
@pytest.mark.parametrize("dist,dtype", FULL_VARIANTS, ids=lambda v: str(v))
def test_throughput_config_full_size_sampled(dist, dtype, S):
    """S streams x 4,096 draws of every output kind in the automatic launch
    shape: 2^30 draws (the shapes the benchmark times) and 2^28 (the next
    size class's tuned shapes).  Every final state, 4,096 random streams in
    full, and the first 16 draws of every stream (uniforms and raw words
    bit-exact, transforms within the tolerance)."""
    per = 4096
    seed = workloads.random_seed()
    c = P.mrg_creator_init(seed)
    d = P.mrg_streams_create_device(c, S)
    oc = seed.copy()
    rec = O.create_streams(GEN, oc, S)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), rec)
    out = P.mrg_generate(d, S * per, dist, dtype)
    torch.cuda.synchronize()
    fin = rec[:, 0:6].copy()
    O.jump_many(GEN, fin, per)  # 4,096 draws consume 4,096 steps (an even count for normals)
    np.testing.assert_array_equal(P.as_u32(d)[:, 0:6], fin)
    np.testing.assert_array_equal(P.as_u32(d)[:, 6:18], rec[:, 6:18])
    mat = out.view(per, S)
    u32 = (lambda a: a.view(np.uint32)) if dtype == P.MRG_U32 else (lambda a: a)
    head = u32(mat[:16].cpu().numpy())
    want_head = O.generate(GEN, rec.copy(), 16 * S, ODIST[dist], ODT[dtype], threads=8).reshape(16, S)
    check_values(head.ravel(), want_head.ravel(), dist, dtype, ctx="first 16 draws of every stream")
    rnd = np.random.default_rng(3)
    idx = np.sort(rnd.choice(S, size=4096, replace=False))
    cols = u32(mat[:, torch.from_numpy(idx).cuda()].cpu().numpy())
    sub = rec[idx].copy()
    want_cols = O.generate(GEN, sub, per * 4096, ODIST[dist], ODT[dtype], threads=8).reshape(per, 4096)
    check_values(cols.ravel(), want_cols.ravel(), dist, dtype, ctx="4096 whole streams")
    del out


@pytest.mark.parametrize("dist,dtype", FULL_VARIANTS, ids=lambda v: str(v))
def test_throughput_config_every_number(dist, dtype):
    """All 2^30 numbers of the throughput configuration, for every output kind
    the benchmark times, in the launch it times, compared with the oracle in
    blocks of 16,384 streams (columns of the k*S + s layout): uniforms and raw
    words bit-exact, transforms within the tolerance (1-8 s per kind with 16
    host threads)."""
    S, per, blk = 262144, 4096, 16384
    seed = workloads.random_seed()
    c = P.mrg_creator_init(seed)
    d = P.mrg_streams_create_device(c, S)
    rec = O.create_streams(GEN, seed.copy(), S)
    out = P.mrg_generate(d, S * per, dist, dtype)
    torch.cuda.synchronize()
    mat = out.view(per, S)
    for s0 in range(0, S, blk):
        got = mat[:, s0:s0 + blk].cpu().numpy()
        if dtype == P.MRG_U32:
            got = got.view(np.uint32)
        want = O.generate(GEN, rec[s0:s0 + blk].copy(), per * blk, ODIST[dist], ODT[dtype],
                          threads=16).reshape(per, blk)
        check_values(got.ravel(), want.ravel(), dist, dtype, ctx=f"streams {s0}..{s0 + blk - 1}")
    del out


@pytest.mark.parametrize("dist,dtype", [(P.MRG_NORMAL, P.MRG_F64), (P.MRG_EXPONENTIAL, P.MRG_F64),
                                        (P.MRG_NORMAL, P.MRG_F32), (P.MRG_EXPONENTIAL, P.MRG_F32)])
def test_transforms_large_sample(dist, dtype):
    """2^22 transformed draws (8,192 streams x 512) in the default launch
    shape against the oracle's long-double transforms: the library's own log
    and sin/cos(pi t) stay inside the tolerance over a large sample."""
    rec = O.create_streams(GEN, workloads.random_seed(61), 8192)
    run_case(rec, 8192 * 512, dist, dtype, param=1.0 if dist == P.MRG_NORMAL else 0.75)


def test_short_buffers_are_rejected_before_launch():
    """The binding refuses buffers that cannot hold the result (the C ABI
    cannot see device buffer sizes): nothing is launched, nothing moves."""
    rec = O.create_streams(GEN, workloads.random_seed(62), 100)
    d = dev_streams(rec)
    short = torch.empty(99, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        P.mrg_generate(d, 100, out=short)
    with pytest.raises(ValueError):  # wrong element size for f64
        P.mrg_generate(d, 10, out=torch.empty(10, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):  # 100 records claimed, 50 given
        P.mrg_generate(d[:50], 100, n_streams=100)
    with pytest.raises(ValueError):
        P.mrg_streams_advance(d[:10], 5, n=11)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), rec)


@pytest.mark.parametrize("S,rows,dtype", [(262144, 16, P.MRG_F64), (262144, 24, P.MRG_F32), (1000, 30, P.MRG_F64),
                                          (131, 7, P.MRG_F32), (64, 3, P.MRG_F64)])
def test_store_ceiling_writes_exactly_the_output(S, rows, dtype):
    """The store-only ceiling kernel writes every one of the n elements and
    nothing past them, in the launch shape mrg_generate would use."""
    n = S * rows
    tdt = torch.float64 if dtype == P.MRG_F64 else torch.float32
    buf = torch.full((n + 64,), -1.0, dtype=tdt, device="cuda")
    P.mrg_store_ceiling(S, n, dtype, out=buf[:n])
    torch.cuda.synchronize()
    assert bool((buf[:n] == 0.5).all())
    assert bool((buf[n:] == -1.0).all())
    with pytest.raises(P.MrgError):
        P.mrg_store_ceiling(S, n + 1, dtype, out=buf)
