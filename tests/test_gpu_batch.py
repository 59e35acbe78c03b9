"""GPU parity of the batched persistent launch: every request of a batch gives
the same bits (outputs and final states) as its own mrg_generate call and as
the oracle, for any tile shape, in graph replays, and after autotuning."""
import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_06604_amd as P  # noqa: E402

GEN = O.MRG32K3A
ODIST = {P.MRG_UNIFORM: O.UNIFORM, P.MRG_NORMAL: O.NORMAL, P.MRG_EXPONENTIAL: O.EXPONENTIAL,
         P.MRG_RAW: O.RAW}
ODT = {P.MRG_F64: O.F64, P.MRG_F32: O.F32, P.MRG_U32: O.U32}
TDT = {P.MRG_F64: torch.float64, P.MRG_F32: torch.float32, P.MRG_U32: torch.int32}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (n_streams, n, dist, dtype, rate): ragged counts, odd normals, n < S, n = 0,
# stream counts that do and do not allow wide stores, long streams (chunks).
MIX = [
    (64, 64 * 100, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (130, 130 * 37 + 11, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (131, 131 * 5 + 130, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (256, 256 * 21 + 3, P.MRG_UNIFORM, P.MRG_F32, 1.0),
    (77, 77 * 9 + 5, P.MRG_UNIFORM, P.MRG_F32, 1.0),
    (100, 7, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (12, 0, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (192, 192 * 15 + 1, P.MRG_RAW, P.MRG_U32, 1.0),
    (65, 65 * 31 + 64, P.MRG_NORMAL, P.MRG_F64, 1.0),
    (64, 64 * 20, P.MRG_NORMAL, P.MRG_F32, 1.0),
    (70, 70 * 13 + 9, P.MRG_EXPONENTIAL, P.MRG_F64, 2.5),
    (33, 33 * 17 + 2, P.MRG_EXPONENTIAL, P.MRG_F32, 1.0),
    (2, 2 * 9000 + 1, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (4, 4 * 7001, P.MRG_NORMAL, P.MRG_F64, 1.0),
    (1, 12345, P.MRG_UNIFORM, P.MRG_F32, 1.0),
    # uniform/raw requests over several workgroup tiles per chunk: spare waves
    # in the last group, odd S (one stream per lane), rows off 128-byte lines
    (1100, 1100 * 23 + 77, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (1031, 1031 * 11 + 3, P.MRG_UNIFORM, P.MRG_F32, 1.0),
    (520, 520 * 40, P.MRG_RAW, P.MRG_U32, 1.0),
    # transforms over even stream counts of at least 128: two streams per lane
    (130, 130 * 21 + 5, P.MRG_NORMAL, P.MRG_F64, 1.0),
    (256, 256 * 9 + 3, P.MRG_EXPONENTIAL, P.MRG_F32, 1.5),
    (200, 200 * 40 + 1, P.MRG_NORMAL, P.MRG_F32, 1.0),
    (1024, 1024 * 7, P.MRG_EXPONENTIAL, P.MRG_F64, 1.0),
]


class Mix:
    """Device streams and outputs for a request mix; request r takes the next
    S_r streams of one creator, in order."""

    def __init__(self, mix, seed_id=0):
        self.mix = mix
        total = sum(m[0] for m in mix)
        seed = workloads.random_seed(100 + seed_id)
        self.records = O.create_streams(GEN, seed.copy(), total)
        self.reset()

    def reset(self):
        self.streams, self.outs, self.host_rec = [], [], []
        first = 0
        for S, n, dist, dtype, rate in self.mix:
            rec = self.records[first:first + S].copy()
            first += S
            self.host_rec.append(rec)
            self.streams.append(torch.from_numpy(rec.view(np.int32).copy()).cuda())
            self.outs.append(torch.full((max(n, 1),), 7, dtype=TDT[dtype], device="cuda"))

    def requests(self):
        return [P.make_request(st, n, dist, dtype, rate, out)
                for st, out, (S, n, dist, dtype, rate) in zip(self.streams, self.outs, self.mix)]

    def plain(self):
        outs = []
        for st, (S, n, dist, dtype, rate) in zip(self.streams, self.mix):
            outs.append(P.mrg_generate(st, n, dist, dtype, rate) if n else None)
        return outs


def _equal(a, b, n):
    return torch.equal(a[:n], b[:n])


def test_batch_equals_plain_equals_oracle():
    A, B = Mix(MIX), Mix(MIX)
    plan = P.BatchPlan(A.requests())
    plan.upload()
    plan.launch()
    want = B.plain()
    torch.cuda.synchronize()
    for i, (S, n, dist, dtype, rate) in enumerate(MIX):
        if n:
            assert _equal(A.outs[i], want[i], n), f"request {i}"
        assert torch.equal(A.streams[i], B.streams[i]), f"states of request {i}"
        # against the oracle too
        work = A.host_rec[i].copy()
        ref = O.generate(GEN, work, n, ODIST[dist], ODT[dtype], rate)
        got = A.outs[i].cpu().numpy()[:n]
        if dtype == P.MRG_U32:
            got = got.view(np.uint32)
        if dist in (P.MRG_UNIFORM, P.MRG_RAW):
            assert np.array_equal(got, ref), f"request {i}"
        elif n:
            tol = 1e-15 if dtype == P.MRG_F64 else 1e-6
            err = np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), 1.0)
            assert err.max() <= tol, f"request {i}: {err.max()}"
        np.testing.assert_array_equal(P.as_u32(A.streams[i]), work)
    times = plan.request_times()
    assert times[0] > 0
    for i, (S, n, *_ ) in enumerate(MIX):
        if n:
            assert times[1 + i] >= times[0], i
        else:
            assert times[1 + i] == 0


@pytest.mark.parametrize("cfg", [dict(tile_units=1), dict(tile_units=7, waves_per_simd=1),
                                 dict(tile_units=64, wide_stores=1), dict(tile_units=100000),
                                 dict(waves_per_simd=16), dict(tile_units=333, waves_per_simd=2),
                                 dict(gang_waves=4), dict(gang_waves=2, tile_units=7),
                                 dict(gang_waves=8, tile_units=333, waves_per_simd=2),
                                 dict(gang_waves=4, tile_units=1, waves_per_simd=1),
                                 dict(gang_waves=8, tile_units=64, wide_stores=1),
                                 dict(gang_waves=2, tile_units=100000, waves_per_simd=16),
                                 dict(gang_waves=4, wide_stores=1, waves_per_simd=6),
                                 dict(gang_waves=8, wide_stores=1, tile_units=7, waves_per_simd=3),
                                 dict(gang_waves=4, wide_stores=2), dict(gang_waves=8, wide_stores=2, tile_units=64),
                                 dict(wide_stores=2, tile_units=300)],
                         ids=str)
def test_batch_shape_invariance(cfg):
    A, B = Mix(MIX, 1), Mix(MIX, 1)
    plan = P.BatchPlan(A.requests(), cfg)
    plan.upload()
    plan.launch()
    want = B.plain()
    torch.cuda.synchronize()
    for i, (S, n, *_ ) in enumerate(MIX):
        if n:
            assert _equal(A.outs[i], want[i], n), f"request {i} cfg {cfg}"
        assert torch.equal(A.streams[i], B.streams[i]), f"states {i} cfg {cfg}"


def test_batch_relaunch_continues_streams():
    """Launching the same plan twice continues every request's streams, like
    two mrg_generate calls."""
    A, B = Mix(MIX, 2), Mix(MIX, 2)
    plan = P.BatchPlan(A.requests(), dict(tile_units=50))
    plan.upload()
    plan.launch()
    plan.launch()
    B.plain()
    want = B.plain()
    torch.cuda.synchronize()
    for i, (S, n, *_ ) in enumerate(MIX):
        if n:
            assert _equal(A.outs[i], want[i], n), f"request {i}"
        assert torch.equal(A.streams[i], B.streams[i])


# Requests whose last stream block is small (1, 16, 20, 32 or 36 streams of
# 64), a normal request with an odd count, a single stream: over gangs, tiny
# and odd chunks and a single chunk.
SMALL_TAIL_MIX = [
    (65, 65 * 400 + 3, P.MRG_UNIFORM, P.MRG_F64, 1.0),
    (96, 96 * 300 + 50, P.MRG_NORMAL, P.MRG_F64, 1.0),
    (100, 100 * 257, P.MRG_NORMAL, P.MRG_F32, 1.0),
    (80, 80 * 513 + 79, P.MRG_EXPONENTIAL, P.MRG_F32, 0.5),
    (20, 20 * 700, P.MRG_RAW, P.MRG_U32, 1.0),
    (1, 5000, P.MRG_UNIFORM, P.MRG_F32, 1.0),
    (130, 130 * 1001 + 7, P.MRG_EXPONENTIAL, P.MRG_F64, 1.0),
    (40, 40 * 301, P.MRG_NORMAL, P.MRG_F64, 1.0),
    (144, 144 * 222 + 100, P.MRG_UNIFORM, P.MRG_F64, 1.0),
]


@pytest.mark.parametrize("cfg", [dict(gang_waves=8, tile_units=64, wide_stores=1),
                                 dict(gang_waves=4, tile_units=200, waves_per_simd=2, wide_stores=1),
                                 dict(gang_waves=8, wide_stores=2),
                                 dict(gang_waves=2, tile_units=6, wide_stores=1),
                                 dict(gang_waves=8, tile_units=2, wide_stores=1),
                                 dict(gang_waves=4, tile_units=63, wide_stores=1),
                                 dict(gang_waves=4, tile_units=100000, wide_stores=1),
                                 None], ids=str)
def test_batch_small_last_blocks(cfg):
    """The plain launch's values and states, and the oracle's."""
    A, B = Mix(SMALL_TAIL_MIX, 2), Mix(SMALL_TAIL_MIX, 2)
    plan = P.BatchPlan(A.requests(), cfg)
    plan.upload()
    plan.launch()
    want = B.plain()
    torch.cuda.synchronize()
    for i, (S, n, dist, dtype, rate) in enumerate(SMALL_TAIL_MIX):
        assert _equal(A.outs[i], want[i], n), f"request {i} cfg {cfg}"
        assert torch.equal(A.streams[i], B.streams[i]), f"states {i} cfg {cfg}"
        work = A.host_rec[i].copy()
        ref = O.generate(GEN, work, n, ODIST[dist], ODT[dtype], rate)
        got = A.outs[i].cpu().numpy()[:n]
        if dtype == P.MRG_U32:
            got = got.view(np.uint32)
        if dist in (P.MRG_UNIFORM, P.MRG_RAW):
            assert np.array_equal(got, ref), f"request {i} cfg {cfg}"
        else:
            tol = 1e-15 if dtype == P.MRG_F64 else 1e-6
            err = np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), 1.0)
            assert err.max() <= tol, f"request {i} cfg {cfg}: {err.max()}"
        np.testing.assert_array_equal(P.as_u32(A.streams[i]), work)


@pytest.mark.parametrize("cfg", [dict(tile_units=200, gang_waves=1), dict(tile_units=200, gang_waves=4),
                                 dict(tile_units=200, gang_waves=4, wide_stores=2, waves_per_simd=6)], ids=str)
def test_batch_graph_replay_matches_eager(cfg):
    """Capture one launch in a HIP graph, replay it three times with eager
    work in between; each replay must equal the matching eager launch."""
    A, B = Mix(MIX, 3), Mix(MIX, 3)
    planA = P.BatchPlan(A.requests(), cfg)
    planA.upload()
    planB = P.BatchPlan(B.requests(), dict(tile_units=200))
    planB.upload()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        # warm the stream; the capture itself runs nothing
        pass
    with torch.cuda.graph(g, stream=s):
        planA.launch(stream=s.cuda_stream)
    torch.cuda.synchronize()
    junk = torch.empty(1 << 20, device="cuda")
    for rep in range(3):
        g.replay()
        junk.uniform_()  # eager work between replays
        torch.cuda.synchronize()
        planB.launch()
        torch.cuda.synchronize()
        for i, (S, n, *_ ) in enumerate(MIX):
            if n:
                assert _equal(A.outs[i], B.outs[i], n), f"replay {rep} request {i}"
            assert torch.equal(A.streams[i], B.streams[i]), f"replay {rep} states {i}"


def test_batch_autotune_leaves_streams_and_stays_exact():
    A, B = Mix(MIX, 4), Mix(MIX, 4)
    small = P.BatchPlan(A.requests(), dict(tile_units=512))
    plan = P.BatchPlan(A.requests())
    assert plan.autotune_workspace_size() >= small.workspace_size()
    plan.alloc_workspace()  # the default cut's size: autotune grows it where a trial cut needs more
    plan.upload()
    before = [t.clone() for t in A.streams]
    best, ms = plan.autotune()
    assert plan.workspace_size() <= plan._ws_bytes
    assert best["tile_units"] in (192, 256, 512, 1024, 2048, 4096, 8192) and best["waves_per_simd"] in (2, 3, 4, 5, 6)
    assert best["gang_waves"] in (1, 4, 8) and best["wide_stores"] in (1, 2)
    assert ms > 0
    for a, b in zip(A.streams, before):
        assert torch.equal(a, b)
    plan.launch()
    want = B.plain()
    torch.cuda.synchronize()
    for i, (S, n, *_ ) in enumerate(MIX):
        if n:
            assert _equal(A.outs[i], want[i], n), f"request {i}"
        assert torch.equal(A.streams[i], B.streams[i])


@pytest.mark.parametrize("cfg", [None, dict(tile_units=1024, waves_per_simd=2, gang_waves=4),
                                 dict(tile_units=512, waves_per_simd=4, gang_waves=4, wide_stores=2)], ids=str)
def test_batched_config_full_size(cfg):
    """4096 requests, lengths log-uniform in [1e3, 1e7], 64-1024 streams each,
    random mix of f32/f64 and uniform/normal/exponential: the batch equals
    4096 plain launches bit for bit (outputs and states); sampled requests
    also equal the oracle."""
    reqs = workloads.batch_requests()
    total_S = sum(r["n_streams"] for r in reqs)
    seed = workloads.random_seed()
    c = P.mrg_creator_init(seed)
    allA = P.mrg_streams_create_device(c, total_S)
    allB = allA.clone()
    dmap = {0: P.MRG_UNIFORM, 1: P.MRG_NORMAL, 2: P.MRG_EXPONENTIAL}
    tmap = {0: P.MRG_F64, 1: P.MRG_F32}
    creqs, outsA, outsB, meta = [], [], [], []
    for r in reqs:
        dist, dtype = dmap[r["dist"]], tmap[r["dtype"]]
        sA = allA[r["first_stream"]:r["first_stream"] + r["n_streams"]]
        oA = torch.empty(r["n"], dtype=TDT[dtype], device="cuda")
        outsA.append(oA)
        creqs.append(P.make_request(sA, r["n"], dist, dtype, 1.0, oA))
        meta.append((r, dist, dtype))
    print(f"full-size batch, cfg {cfg}", flush=True)
    plan = P.BatchPlan(creqs, cfg)
    plan.upload()
    plan.launch()
    torch.cuda.synchronize()
    for r, dist, dtype in meta:
        sB = allB[r["first_stream"]:r["first_stream"] + r["n_streams"]]
        outsB.append(P.mrg_generate(sB, r["n"], dist, dtype, 1.0))
    torch.cuda.synchronize()
    bad = [i for i in range(len(meta)) if not torch.equal(outsA[i], outsB[i])]
    assert not bad, f"{len(bad)} requests differ, first {bad[:5]}"
    assert torch.equal(allA, allB)
    times = plan.request_times()
    assert np.all(times[1:] >= times[0]) and np.all(times[1:] > 0)
    # oracle on a few requests of each kind (first 2048 draws of each)
    rec = O.create_streams(GEN, seed.copy(), total_S)
    seen = set()
    for i, (r, dist, dtype) in enumerate(meta):
        if (dist, dtype) in seen:
            continue
        seen.add((dist, dtype))
        S = r["n_streams"]
        sub = rec[r["first_stream"]:r["first_stream"] + S].copy()
        k = min(r["n"], S * 8)
        ref = O.generate(GEN, sub, k, ODIST[dist], ODT[dtype], 1.0)
        got = outsA[i][:k].cpu().numpy()
        if dist == P.MRG_UNIFORM:
            assert np.array_equal(got, ref), i
        else:
            tol = 1e-15 if dtype == P.MRG_F64 else 1e-6
            assert (np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), 1.0)).max() <= tol


def test_batched_config_every_number():
    """The 4,096-request mix in the default plan: every number of every
    request (4.4e9 in all; uniforms bit-exact, transforms within 1e-15 fp64 /
    1e-6 fp32) and every stream record against the oracle."""
    reqs = workloads.batch_requests()
    total_S = sum(r["n_streams"] for r in reqs)
    seed = workloads.random_seed(5)
    c = P.mrg_creator_init(seed)
    allA = P.mrg_streams_create_device(c, total_S)
    dmap = {0: P.MRG_UNIFORM, 1: P.MRG_NORMAL, 2: P.MRG_EXPONENTIAL}
    tmap = {0: P.MRG_F64, 1: P.MRG_F32}
    creqs, outs, meta = [], [], []
    for r in reqs:
        dist, dtype = dmap[r["dist"]], tmap[r["dtype"]]
        sA = allA[r["first_stream"]:r["first_stream"] + r["n_streams"]]
        o = torch.empty(r["n"], dtype=TDT[dtype], device="cuda")
        outs.append(o)
        creqs.append(P.make_request(sA, r["n"], dist, dtype, 1.0, o))
        meta.append((r, dist, dtype))
    plan = P.BatchPlan(creqs)
    plan.upload()
    plan.launch()
    torch.cuda.synchronize()
    rec = O.create_streams(GEN, seed.copy(), total_S)
    for i, (r, dist, dtype) in enumerate(meta):
        sub = rec[r["first_stream"]:r["first_stream"] + r["n_streams"]]
        want = O.generate(GEN, sub, r["n"], ODIST[dist], ODT[dtype], 1.0, threads=16)
        got = outs[i].cpu().numpy()
        if dist == P.MRG_UNIFORM:
            assert np.array_equal(got, want), f"request {i}"
        else:
            tol = 1e-15 if dtype == P.MRG_F64 else 1e-6
            err = np.abs(got.astype(np.float64) - want) / np.maximum(np.abs(want), 1.0)
            assert err.max() <= tol, f"request {i}: {err.max()}"
        outs[i] = None
    np.testing.assert_array_equal(P.as_u32(allA), rec)
