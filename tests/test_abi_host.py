"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side logic (seed rule, creator, host stream
creation, argument validation, saved-state validation) is right.  Calls that
would launch a kernel are only made with arguments that fail validation, so
they return before touching HIP."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads
from conftest import ROOT

import paper_2201_06604_amd as P

M1, M2 = 4294967087, 4294944443
P1, P2 = 2147483647, 2147462579
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(mrg_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = P.lib()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(P.EXPORTED) == declared
    assert P.mrg_abi_version() == 3


def test_status_strings():
    L = P.lib()
    for code in P.STATUS:
        assert L.mrg_status_string(code)


def test_seed_rule_matches_oracle():
    cases = [[12345] * 6, [0, 0, 1, 0, 0, 1], [M1 - 1] * 3 + [M2 - 1] * 3, [M1, 1, 1, 1, 1, 1],
             [1, 1, 1, M2, 1, 1], [0, 0, 0, 5, 5, 5], [5, 5, 5, 0, 0, 0], [2**32 - 1] * 6]
    rnd = np.random.default_rng(8)
    cases += [list(rnd.integers(0, 2**32, size=6)) for _ in range(50)]
    for c in cases:
        ok = P.mrg_seed_check(c) == 0
        assert ok == O.seed_valid(O.MRG32K3A, c), c
        if not ok:
            assert P.mrg_seed_check(c) == -2


def test_creator_init_rejects_invalid_seed():
    with pytest.raises(P.MrgError) as e:
        P.mrg_creator_init([0, 0, 0, 1, 1, 1])
    assert e.value.status == -2
    with pytest.raises(P.MrgError) as e:
        P.mrg_creator_init([1] * 6, gen=7)
    assert e.value.status == -1
    with pytest.raises(P.MrgError) as e:  # word 0 = p1 is not below MRG31k3p's m1
        P.mrg_creator_init([2147483647, 1, 1, 1, 1, 1], gen=P.MRG_GEN_MRG31K3P)
    assert e.value.status == -2


@pytest.mark.parametrize("seed", [workloads.PAPER_SEED, list(workloads.random_seed())])
def test_host_creation_matches_oracle(seed):
    """createStreamsCpu: records and creator equal the oracle's sequential
    creation, bit for bit."""
    c = P.mrg_creator_init(seed)
    got = P.mrg_streams_create_host(c, 100)
    oc = np.array(seed, dtype=np.uint32)
    want = O.create_streams(O.MRG32K3A, oc, 100)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(P.creator_words(c), oc)
    # creation continues from the advanced creator
    got2 = P.mrg_streams_create_host(c, 3)
    want2 = O.create_streams(O.MRG32K3A, oc, 3)
    np.testing.assert_array_equal(got2, want2)


def test_host_creation_zero_is_noop():
    c = P.mrg_creator_init([12345] * 6)
    before = P.creator_words(c).copy()
    P.mrg_streams_create_host(c, 0)
    np.testing.assert_array_equal(P.creator_words(c), before)


def test_generate_argument_validation_no_side_effects():
    """Validation failures return before any HIP call (this host has no GPU)."""
    f = P.mrg_generate_status
    E = -1
    # dist/dtype mismatches
    assert f(256, 4, 10, P.MRG_RAW, P.MRG_F64, 1.0, 256) == E
    assert f(256, 4, 10, P.MRG_UNIFORM, P.MRG_U32, 1.0, 256) == E
    assert f(256, 4, 10, P.MRG_NORMAL, P.MRG_U32, 1.0, 256) == E
    # bad enum values
    assert f(256, 4, 10, 9, P.MRG_F64, 1.0, 256) == E
    assert f(256, 4, 10, P.MRG_UNIFORM, 9, 1.0, 256) == E
    # exponential rate
    for rate in (0.0, -1.0, float("inf"), float("nan")):
        assert f(256, 4, 10, P.MRG_EXPONENTIAL, P.MRG_F64, rate, 256) == E
    # zero streams with n > 0, null pointers, misaligned output
    assert f(256, 0, 10, P.MRG_UNIFORM, P.MRG_F64, 1.0, 256) == E
    assert f(0, 4, 10, P.MRG_UNIFORM, P.MRG_F64, 1.0, 256) == E
    assert f(256, 4, 10, P.MRG_UNIFORM, P.MRG_F64, 1.0, 0) == E
    assert f(256, 4, 10, P.MRG_UNIFORM, P.MRG_F64, 1.0, 260) == E
    assert f(256, 4, 10, P.MRG_UNIFORM, P.MRG_F32, 1.0, 258) == E
    assert f(256, 2**31 + 1, 10, P.MRG_UNIFORM, P.MRG_F64, 1.0, 256) == E
    # n = 0 is a no-op, even with null pointers
    assert f(0, 0, 0, P.MRG_UNIFORM, P.MRG_F64, 1.0, 0) == 0
    # unknown generator
    L = P.lib()
    assert L.mrg_generate(7, ctypes.c_void_p(256), 4, 10, 0, 0, 1.0, ctypes.c_void_p(256), None) == -1


def test_launch_cfg_validation():
    L = P.lib()
    for cfg in [(100, 0, 0, 0, 0, 0), (256, 0, 2, 0, 0, 0), (256, 0, 0, 3, 0, 0),
                (256, 0, 0, 0, 3, 0), (256, 0, 0, 0, 8, 0), (256, 0, 0, 0, 0, 2),
                (256, 0, 0, 0, 0, 0, 2)]:
        c = P.mrg_launch_cfg(*cfg)
        st = L.mrg_generate_ex(1, ctypes.c_void_p(256), 4, 10, 0, 0, 1.0, ctypes.c_void_p(256),
                               ctypes.byref(c), None)
        assert st == -1, cfg


def test_generate_plan_resolves_the_launch():
    """The host-side plan: the automatic shape at 2^30 draws over 262,144
    streams (fp64 uniforms in lockstep blocks of 8 waves, one chunk per
    stream), free-running waves for the VALU-bound kinds, explicit shapes
    kept, and the same argument checks as mrg_generate_ex."""
    S, n = 262144, 262144 * 4096
    assert P.mrg_generate_plan(S, n) == dict(block=512, chunk=4096, nontemporal=1, arith=2,
                                             streams_per_lane=2, xcd_remap=1, lockstep=1)
    for dist, dtype in [(P.MRG_UNIFORM, P.MRG_F32), (P.MRG_RAW, P.MRG_U32), (P.MRG_NORMAL, P.MRG_F64),
                        (P.MRG_EXPONENTIAL, P.MRG_F64), (P.MRG_EXPONENTIAL, P.MRG_F32)]:
        p = P.mrg_generate_plan(S, n, dist, dtype)
        assert p["lockstep"] == 0 and p["nontemporal"] == 1, (dist, dtype, p)
        units = 4096 // 2 if dist == P.MRG_NORMAL else 4096
        assert p["chunk"] * -(-units // p["chunk"]) >= units
    # full-size calls (2^29 draws and up) keep lockstep at ragged stream
    # counts (idle waves pass the barriers); small, latency-bound grids run free
    for S2, n2 in [(100000, 10 ** 9), (300000, 300000 * 4096 + 17), (131072, 131072 * 4096)]:
        p = P.mrg_generate_plan(S2, n2)
        assert p["lockstep"] == 1 and p["block"] == 512 and S2 % p["streams_per_lane"] == 0, (S2, p)
    for S2, n2 in [(1024, 1024 * 1024), (1000, 1000 * 37 + 5), (1, 1001)]:
        p = P.mrg_generate_plan(S2, n2)
        assert p["lockstep"] == 0, (S2, p)
    cfg = dict(block=1024, chunk=7, streams_per_lane=4, lockstep=1, nontemporal=0, xcd_remap=0, arith=1)
    assert P.mrg_generate_plan(1000, 50000, P.MRG_UNIFORM, P.MRG_F32, cfg=cfg) == cfg
    assert P.mrg_generate_plan(S, n, gen=P.MRG_GEN_MRG31K3P)["arith"] == 0
    assert set(P.mrg_generate_plan(S, 0).values()) == {0}
    for args, kw in [((S, n, P.MRG_RAW, P.MRG_F64), {}), ((S, n, P.MRG_EXPONENTIAL, P.MRG_F64, 0.0), {}),
                     ((0, n), {}), ((S, n), dict(cfg=dict(lockstep=2))), ((1, 1 << 46), {}),
                     ((S, n), dict(gen=9))]:
        with pytest.raises(P.MrgError):
            P.mrg_generate_plan(*args, **kw)


def _saved(n, flags=0, gen=1, version=1, magic=b"MRG3", records=None, creator=None, extra=b""):
    import struct
    head = magic + struct.pack("<IIIQ", version, gen, flags, n)
    body = b"" if records is None else np.ascontiguousarray(records, dtype=np.uint32).tobytes()
    tail = b"" if creator is None else np.asarray(creator, dtype=np.uint32).tobytes()
    return head + body + tail + extra


def _import_status(data, n_room=8):
    L = P.lib()
    buf = ctypes.create_string_buffer(data, len(data))
    cnt = ctypes.c_size_t()
    cr = P.mrg_creator()
    # device pointer 256 is never touched: every case below fails validation
    return L.mrg_streams_import(1, buf, len(data), ctypes.c_void_p(256), n_room, ctypes.byref(cnt),
                                ctypes.byref(cr), None)


def test_import_rejects_corrupt_buffers():
    c = P.mrg_creator_init(workloads.random_seed())
    recs = P.mrg_streams_create_host(c, 3)
    cre = P.creator_words(c)
    C = -6
    assert _import_status(_saved(3, records=recs)[:10]) == C                      # short
    assert _import_status(_saved(3, records=recs, magic=b"XRG3")) == C            # magic
    assert _import_status(_saved(3, records=recs, version=2)) == C                # version
    assert _import_status(_saved(3, records=recs, gen=2)) == C                    # generator
    assert _import_status(_saved(3, records=recs, flags=4)) == C                  # flags
    assert _import_status(_saved(3, records=recs, extra=b"\0")) == C              # length
    assert _import_status(_saved(4, records=recs)) == C                           # count
    assert _import_status(_saved(3, flags=1, records=recs)) == C                  # missing creator
    bad = recs.copy()
    bad[1, 7] = M1                                                                # start word >= m1
    assert _import_status(_saved(3, records=bad)) == C
    bad = recs.copy()
    bad[2, 15:18] = 0                                                             # zero sub triple
    assert _import_status(_saved(3, records=bad)) == C
    assert _import_status(_saved(3, flags=1, records=recs, creator=[0, 0, 0, 1, 1, 1])) == C
    # too little room is reported as such, after validation
    assert _import_status(_saved(3, flags=1, records=recs, creator=cre), n_room=2) == -5


def test_export_size():
    sz = ctypes.c_size_t()
    assert P.lib().mrg_streams_export_size(10, 1, ctypes.byref(sz)) == 0
    assert sz.value == 24 + 10 * 72 + 24


# ------------------------------------------------------------------ batching
def _req(streams, S, n, dist=0, dtype=0, rate=1.0, out=4096):
    return P.mrg_request(streams, S, n, dist, dtype, rate, out)


def _plan_status(reqs, cfg=None):
    arr = (P.mrg_request * max(len(reqs), 1))(*reqs)
    plan = ctypes.c_void_p()
    c = None if cfg is None else ctypes.byref(P.mrg_batch_cfg(*cfg))
    st = P.lib().mrg_batch_plan_create(1, arr, len(reqs), c, ctypes.byref(plan))
    return st, plan


def test_batch_plan_validation():
    """Plans are built on the host; invalid requests are refused before any
    device work.  Pointers are never dereferenced here."""
    base = 1 << 20
    ok = [_req(base, 64, 64 * 10, out=1 << 30), _req(base + 64 * 72, 64, 640, out=(1 << 30) + 640 * 8)]
    st, plan = _plan_status(ok)
    assert st == 0
    sz, nt = ctypes.c_size_t(), ctypes.c_size_t()
    assert P.lib().mrg_batch_workspace_size(plan, ctypes.byref(sz)) == 0 and sz.value % 256 == 0
    assert P.lib().mrg_batch_tile_count(plan, ctypes.byref(nt)) == 0
    # 64 streams x 10 draws each: one wave tile per request (one stream per
    # lane, the automatic width in gang mode), in one gang of 8 waves
    assert nt.value == 8
    most = ctypes.c_size_t()
    assert P.lib().mrg_batch_autotune_workspace_size(plan, ctypes.byref(most)) == 0
    assert most.value >= sz.value and most.value % 256 == 0
    P.lib().mrg_batch_plan_destroy(plan)
    # a long request: smaller trial tiles need a larger workspace than a 4096-unit cut
    st, plan = _plan_status([_req(base, 1024, 1024 * 200000, out=1 << 32)], (4096, 0, 0, 1))
    assert st == 0
    assert P.lib().mrg_batch_workspace_size(plan, ctypes.byref(sz)) == 0
    assert P.lib().mrg_batch_autotune_workspace_size(plan, ctypes.byref(most)) == 0
    assert most.value > sz.value
    P.lib().mrg_batch_plan_destroy(plan)
    bad_cases = [
        [_req(base, 64, 640, out=1 << 30), _req(base + 63 * 72, 64, 640, out=(1 << 31))],  # shared streams
        [_req(base, 64, 640, out=1 << 30), _req(base + 64 * 72, 64, 640, out=(1 << 30) + 8)],  # shared out
        [_req(base, 64, 640, dist=3, dtype=0)],   # raw needs u32
        [_req(base, 64, 640, dist=2, rate=0.0)],  # bad rate
        [_req(base, 0, 640)],                     # no streams
        [_req(0, 64, 640)],                       # NULL streams
        [_req(base, 64, 640, out=4097)],          # misaligned output
    ]
    for reqs in bad_cases:
        st, _ = _plan_status(reqs)
        assert st == -1, reqs
    st, _ = _plan_status(ok, (0, 17, 0))
    assert st == -1  # waves_per_simd above 16
    st, _ = _plan_status(ok, (0, 0, 3))
    assert st == -1  # wide_stores above 2
    arr = (P.mrg_request * 1)(*ok[:1])
    plan = ctypes.c_void_p()
    assert P.lib().mrg_batch_plan_create(2, arr, 1, None, ctypes.byref(plan)) == -3


def test_batch_tiles_cover_requests():
    """Tile counts follow the cut: ceil(S / (64*SPL)) stream blocks times
    ceil(units / tile_units) chunks, summed over requests.  SPL is the widest
    store the request allows unless a narrower one leaves fewer lane slots
    idle (S = 130: two streams per lane would cover 256, one covers 192)."""
    base = 1 << 20
    S1, n1 = 130, 130 * 1000 + 7          # f64 uniform: 1 stream/lane, 3 blocks
    S2, n2 = 77, 77 * 301                 # normal, 1 stream/lane, pairs = 151
    S3, n3 = 256, 256 * 250               # f64 uniform: 2 streams/lane, 2 blocks
    reqs = [_req(base, S1, n1, out=1 << 32),
            _req(base + S1 * 72, S2, n2, dist=1, out=(1 << 33)),
            _req(base + (S1 + S2) * 72, S3, n3, out=(1 << 34))]
    nt = ctypes.c_size_t()
    want = 3 * ((1001 + 99) // 100) + 2 * ((151 + 99) // 100) + 2 * ((250 + 99) // 100)   # 43
    narrow = 3 * 11 + 2 * 2 + 4 * 3                                                       # 49
    # (tile_units, waves, wide_stores, gang): automatic width outside gang mode
    # is the widest fitting one; in gang mode it is one stream per lane.  Gang
    # plans pad each class (here uniform and normal) to whole gangs.
    cases = {(100, 0, 0, 1): want, (100, 0, 2, 1): want, (100, 0, 1, 1): narrow,
             (100, 0, 2, 4): 40 + 4, (100, 0, 0, 8): 48 + 8, (100, 0, 1, 8): 48 + 8}
    for cfg, n in cases.items():
        st, plan = _plan_status(reqs, cfg)
        assert st == 0
        P.lib().mrg_batch_tile_count(plan, ctypes.byref(nt))
        assert nt.value == n, (cfg, nt.value)
        P.lib().mrg_batch_plan_destroy(plan)


# ------------------------------------------------------------------ serving
def test_server_create_validation():
    """Server configuration errors are refused before any device work."""
    L = P.lib()
    srv = ctypes.c_void_p()
    assert L.mrg_server_create(None, ctypes.byref(srv)) == -1

    def cfg(**kw):
        c = P.mrg_server_cfg()
        c.n_sessions = kw.get("n_sessions", 4)
        for i in range(6):
            c.seed[i] = kw.get("seed", [12345] * 6)[i]
        c.pool = kw.get("pool", 1 << 20)
        c.pool_bytes = kw.get("pool_bytes", 1 << 20)
        c.mode = kw.get("mode", 0)
        c.lanes = kw.get("lanes", 0)
        c.streams_per_session = kw.get("sps", 0)
        c.workspace = kw.get("workspace", 1 << 32)  # never touched: every case fails validation
        c.workspace_bytes = 1 << 30
        return c
    for bad in [dict(n_sessions=0), dict(pool=0), dict(pool_bytes=16), dict(pool=(1 << 20) + 8),
                dict(mode=2), dict(lanes=65), dict(sps=70000)]:
        assert L.mrg_server_create(ctypes.byref(cfg(**bad)), ctypes.byref(srv)) == -1, bad
    assert L.mrg_server_create(ctypes.byref(cfg(seed=[0, 0, 0, 1, 1, 1])), ctypes.byref(srv)) == -2


def _fisher_status(obs, B=10, dev_count=64, dev_streams=4096):
    obs = np.ascontiguousarray(np.asarray(obs, dtype=np.int32))
    return P.lib().mrg_fisher_sim(P.MRG_GEN_MRG32K3A, ctypes.c_void_p(dev_streams), B, obs.shape[0],
                                  obs.shape[1], obs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  ctypes.c_void_p(dev_count), None, None, None)


def test_fisher_sim_validation():
    """Shape, entries, total, pointers and B are checked before any launch."""
    assert _fisher_status(np.ones((33, 2))) == -1
    assert _fisher_status(np.ones((2, 33))) == -1
    assert _fisher_status([[1, -1], [2, 3]]) == -1
    assert _fisher_status([[1 << 19, 1 << 19], [1, 0]]) == -1  # total above 2^20
    assert _fisher_status([[1, 2], [3, 4]], dev_count=0) == -1
    assert _fisher_status([[1, 2], [3, 4]], dev_count=12) == -1  # misaligned count
    assert _fisher_status([[1, 2], [3, 4]], dev_streams=0) == -1
    assert _fisher_status([[1, 2], [3, 4]], B=(1 << 31) + 1) == -1
    assert P.mrg_fisher_pvalue(0, 999) == pytest.approx(1e-3)


def test_tables_sample_validation():
    L = P.lib()
    v = ctypes.c_void_p(4096)
    assert L.mrg_tables_sample(P.MRG_GEN_MRG32K3A, v, 0, None, None, None, None, None, None, None) == 0
    assert L.mrg_tables_sample(P.MRG_GEN_MRG32K3A, v, 5, v, None, v, v, v, None, None) == -1
    assert L.mrg_tables_sample(P.MRG_GEN_MRG32K3A, v, 5, v, v, v, v, ctypes.c_void_p(4098), None, None) == -1
    assert L.mrg_tables_sample(P.MRG_GEN_MRG32K3A, v, 5, v, v, v, v, v, ctypes.c_void_p(4100), None) == -1
    assert L.mrg_tables_sample(9, v, 5, v, v, v, v, v, None, None) == -1


# ------------------------------------------------------------ MRG31k3p
def test_mrg31k3p_host_creation_is_the_papers_table():
    """Section 2.1: createStreamsCpu(4) from 12345 x 6 with MRG31k3p gives the
    printed table (24 words), through the C ABI's host creation; the creator
    then continues where the oracle's does."""
    from conftest import read_golden
    want = np.array([[int(v) for v in r] for r in read_golden("mrg31k3p_stream_table.txt")], dtype=np.uint32)
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=P.MRG_GEN_MRG31K3P)
    got = P.mrg_streams_create_host(c, 4, gen=P.MRG_GEN_MRG31K3P)
    for k in range(3):
        np.testing.assert_array_equal(got[:, 6 * k:6 * k + 6], want)
    oc = np.array(workloads.PAPER_SEED, dtype=np.uint32)
    O.create_streams(O.MRG31K3P, oc, 4)
    np.testing.assert_array_equal(P.creator_words(c), oc)
    more = P.mrg_streams_create_host(c, 50, gen=P.MRG_GEN_MRG31K3P)
    np.testing.assert_array_equal(more, O.create_streams(O.MRG31K3P, oc, 50))


def test_mrg31k3p_seed_rule_matches_oracle():
    cases = [[12345] * 6, [P1 - 1] * 3 + [P2 - 1] * 3, [P1, 1, 1, 1, 1, 1], [1, 1, 1, P2, 1, 1],
             [0, 0, 0, 5, 5, 5], [5, 5, 5, 0, 0, 0], [M1 - 1] * 6]
    rnd = np.random.default_rng(9)
    cases += [list(rnd.integers(0, 2**31, size=6)) for _ in range(50)]
    for cse in cases:
        ok = P.mrg_seed_check(cse, gen=P.MRG_GEN_MRG31K3P) == 0
        assert ok == O.seed_valid(O.MRG31K3P, cse), cse


def test_mrg31k3p_import_checks_its_moduli():
    """A saved MRG31k3p state with a word in [p1, m1) is corrupt for MRG31k3p
    (valid for MRG32k3a); a saved MRG32k3a buffer is refused as MRG31k3p."""
    rec = np.full((1, 18), 7, dtype=np.uint32)
    rec[0, 0] = P1
    buf = _saved(1, gen=2, records=rec)
    st = P.lib().mrg_streams_import(2, buf, len(buf), ctypes.c_void_p(4096), 1, None, None, None)
    assert st == -6
    buf = _saved(1, gen=1, records=np.full((1, 18), 7, dtype=np.uint32))
    st = P.lib().mrg_streams_import(2, buf, len(buf), ctypes.c_void_p(4096), 1, None, None, None)
    assert st == -6


def test_batch_rejects_mrg31k3p():
    req = (P.mrg_request * 1)()
    plan = ctypes.c_void_p()
    assert P.lib().mrg_batch_plan_create(2, req, 1, None, ctypes.byref(plan)) == -3


def test_generate_paper_validation():
    """Lattice, stream count, padding, pairing and size checks come before
    any launch."""
    L = P.lib()
    v = ctypes.c_void_p(4096)

    def st(n_streams, nrow, ncol, npad, G0, G1, dist=0, dtype=0, param=1.0, out=v, gen=1):
        return L.mrg_generate_paper(gen, v, n_streams, nrow, ncol, npad, G0, G1, dist, dtype, param, out, None)

    assert st(4, 2, 4, 4, 0, 2) == -1           # empty lattice
    assert st(4, 2, 4, 4, 3, 2) == -1           # 6 work-items, 4 streams
    assert st(4, 2, 4, 3, 2, 2) == -1           # npad < ncol
    assert st(4, 2, 3, 4, 1, 2, dist=1) == -1   # normals: odd ncol
    assert st(4, 2, 4, 4, 1, 3, dist=1) == -1   # normals: odd G1
    assert st(4, 2, 4, 4, 2, 2, dist=3, dtype=0) == -1
    assert st(4, 2, 4, 4, 2, 2, dist=2, param=0.0) == -1
    assert st(4, 1 << 31, 4, 4, 2, 2) == -1
    assert st(4, 2, 4, 4, 2, 2, out=ctypes.c_void_p(4100)) == -1
    assert st(4, 2, 4, 4, 2, 2, gen=5) == -1
    assert st(4, 0, 4, 4, 2, 2, out=None) == 0  # empty block: no-op


def test_device_creation_size_limit():
    c = P.mrg_creator_init([12345] * 6)
    before = P.creator_words(c).copy()
    st = P.lib().mrg_streams_create_device(1, ctypes.byref(c), (1 << 36) + 1, ctypes.c_void_p(4096), None)
    assert st == -1
    np.testing.assert_array_equal(P.creator_words(c), before)


def test_generate_rejects_more_than_2_46_draws_per_stream():
    assert P.mrg_generate_status(256, 1, 1 << 46, P.MRG_UNIFORM, P.MRG_F64, 1.0, 256) == -1
    assert P.mrg_generate_status(256, 4, (1 << 48), P.MRG_UNIFORM, P.MRG_F64, 1.0, 256) == -1


def _server_cfg(**kw):
    cfg = P.mrg_server_cfg()
    cfg.n_sessions = kw.get("n_sessions", 256)
    cfg.streams_per_session = kw.get("streams_per_session", 0)
    for i, v in enumerate(workloads.PAPER_SEED):
        cfg.seed[i] = v
    cfg.pool = kw.get("pool", 1 << 40)
    cfg.pool_bytes = kw.get("pool_bytes", 1 << 30)
    cfg.lanes, cfg.max_batch, cfg.mode = kw.get("lanes", 0), kw.get("max_batch", 0), kw.get("mode", 0)
    cfg.workspace = kw.get("workspace", None)
    cfg.workspace_bytes = kw.get("workspace_bytes", 0)
    return cfg


def test_server_workspace_is_the_callers():
    """The server's device memory (session streams, lane workspaces) is a
    caller buffer of mrg_server_workspace_size bytes; a missing, misaligned,
    short or overlapping one is refused before any HIP call."""
    L = P.lib()
    need = ctypes.c_size_t()
    cfg = _server_cfg()
    assert L.mrg_server_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == 0
    streams = 256 * 64 * 72
    assert need.value >= streams + 4 * 256 * 16  # records + four lane workspaces
    plain = _server_cfg(mode=1)
    n1 = ctypes.c_size_t()
    assert L.mrg_server_workspace_size(ctypes.byref(plain), ctypes.byref(n1)) == 0
    assert n1.value == -(-streams // 256) * 256  # mode 1 has no lanes
    srv = ctypes.c_void_p()
    for bad, status in [(dict(workspace=None), -1), (dict(workspace=(1 << 41) + 8, workspace_bytes=need.value), -1),
                        (dict(workspace=1 << 41, workspace_bytes=need.value - 1), -5),
                        (dict(workspace=(1 << 40) + 4096, workspace_bytes=need.value), -1),
                        (dict(workspace=1 << 41, workspace_bytes=need.value, n_sessions=0), -1),
                        (dict(workspace=1 << 41, workspace_bytes=need.value, mode=2), -1)]:
        c = _server_cfg(**bad)
        assert L.mrg_server_create(ctypes.byref(c), ctypes.byref(srv)) == status, bad
        assert not srv.value


def test_fisher_rejects_huge_entries_before_summing():
    """Observed entries whose sum passes 2^31 are refused (grand total above
    2^20) without overflowing the margin sums first."""
    L = P.lib()
    obs = np.array([[2**31 - 1, 2**31 - 1], [5, 5]], dtype=np.int32)
    cnt = ctypes.c_void_p(256)
    st = L.mrg_fisher_sim(1, ctypes.c_void_p(256), 10, 2, 2, obs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          cnt, None, None, None)
    assert st == -1
    assert "2^20" in L.mrg_last_error().decode()



def test_static_batch_rejects_a_plan_above_its_workspace():
    """mrg_batch_launch_static refuses, before touching HIP, a plan whose
    workspace exceeds the library's static array (2^20 one-unit tiles need
    more than 16 MiB); the pointers are never dereferenced."""
    req = P.mrg_request(1 << 40, 64, 64 << 20, P.MRG_UNIFORM, P.MRG_F64, 1.0, 1 << 44)
    plan = P.BatchPlan([req], cfg=dict(tile_units=1))
    assert plan.workspace_size() > P.MRG_BATCH_STATIC_WORKSPACE_BYTES
    with pytest.raises(P.MrgError) as e:
        plan.launch_static(stream=0)
    assert e.value.status == -5
    assert "static workspace" in str(e.value)


def test_batch_gang_plans():
    """Gang plans (blocks of 2, 4 or 8 waves taking neighbouring tiles
    together) hold a whole number of gangs; other gang sizes are refused."""
    base = 1 << 20
    reqs = [_req(base, 131, 131 * 5000, out=1 << 30), _req(base + 131 * 72, 64, 64 * 7, dist=1, out=1 << 31),
            _req(base + 195 * 72, 1000, 1000 * 3001, dtype=1, out=1 << 32)]
    for g in (2, 4, 8):
        st, plan = _plan_status(reqs, (512, 0, 0, g))
        assert st == 0
        n = ctypes.c_size_t()
        assert P.lib().mrg_batch_tile_count(plan, ctypes.byref(n)) == 0
        assert n.value % g == 0 and n.value > 0
        P.lib().mrg_batch_plan_destroy(plan)
    for g in (3, 5, 16):
        st, _ = _plan_status(reqs, (512, 0, 0, g))
        assert st == -1


def test_tuned_table_resolution_matches_the_library():
    """The tuner works out the launch shape each candidate table entry gives
    (tune_plain.resolve); for the committed table that must be the shape the
    library's automatic plan reports, at every kind's representative sizes
    and at a few others of each size class."""
    from paper_2201_06604_amd import tune_plain as T
    table = T.read_table()
    others = [(100, 7), (3, 1000001), (131071, 33), (1 << 20, 64), (65, 100000), (4096, 1 << 16), (77, 5000)]
    for k, (name, dist, dtype) in enumerate(T.KINDS):
        for S, per in T.CLASSES + others:
            for extra in (0, 3):
                n = S * per + extra
                c = 0 if n < 1 << 18 else 1 if n < 1 << 22 else 2 if n < 1 << 26 else 3 if n < 1 << 29 else 4
                want = T.resolve(table[k][c], S, n, dist, dtype)
                got = P.mrg_generate_plan(S, n, dist, dtype)
                assert got == want, (name, S, n, got, want)
