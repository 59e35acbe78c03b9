"""GPU parity of the paper-geometry entry point (mrg_generate_paper: the
work-item lattice of Listing 1 and Listing 2) with the oracle: the printed
runifGpu / rexpGpu values on MRG31k3p, random lattices and blocks for every
distribution and both generators (values, padding and every stream state),
several row blocks per work-item, and the paper's 10000 x 10000 rnormGpu
example with Nglobal = 512 x 128, sampled work-item by work-item."""
import numpy as np
import pytest

import oracle as O
import workloads
from conftest import read_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_06604_amd as P  # noqa: E402

TOL = {P.MRG_F64: 1e-15, P.MRG_F32: 1e-6}
ODIST = {P.MRG_UNIFORM: O.UNIFORM, P.MRG_NORMAL: O.NORMAL, P.MRG_EXPONENTIAL: O.EXPONENTIAL,
         P.MRG_RAW: O.RAW}
ODT = {P.MRG_F64: O.F64, P.MRG_F32: O.F32, P.MRG_U32: O.U32}
OGEN = {P.MRG_GEN_MRG32K3A: O.MRG32K3A, P.MRG_GEN_MRG31K3P: O.MRG31K3P}
TDT = {P.MRG_F64: torch.float64, P.MRG_F32: torch.float32, P.MRG_U32: torch.int32}
SENTINEL = 12345


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(rec):
    return torch.from_numpy(rec.view(np.int32).copy()).cuda()


def run(gen, rec, nrow, ncol, npad, G0, G1, dist, dtype, param=1.0):
    d = dev(rec)
    out = torch.full((nrow, npad), SENTINEL, dtype=TDT[dtype], device="cuda")
    P.mrg_generate_paper(d, nrow, ncol, G0, G1, dist, dtype, param, out=out, npad=npad, gen=gen)
    torch.cuda.synchronize()
    work = rec.copy()
    want = O.generate_paper(OGEN[gen], work, nrow, ncol, G0, G1, ODIST[dist], ODT[dtype], param, npad=npad,
                            fill=SENTINEL)
    got = out.cpu().numpy()
    if dtype == P.MRG_U32:
        got = got.view(np.uint32)
    ctx = f"gen={gen} {nrow}x{ncol}/{npad} G={G0}x{G1} dist={dist} dtype={dtype}"
    if dist in (P.MRG_UNIFORM, P.MRG_RAW):
        assert np.array_equal(got, want), ctx
    else:
        assert np.array_equal(got[:, ncol:], want[:, ncol:]), ctx
        g, w = got[:, :ncol].astype(np.float64), want[:, :ncol].astype(np.float64)
        err = np.abs(g - w) / np.maximum(np.abs(w), 1.0)
        assert err.size == 0 or err.max() <= TOL[dtype], (ctx, err.max())
    np.testing.assert_array_equal(P.as_u32(d), work, err_msg=ctx)


def paper_streams(gen=P.MRG_GEN_MRG31K3P):
    return O.create_streams(OGEN[gen], np.array(workloads.PAPER_SEED, dtype=np.uint32), 4)


def test_runif_printout_on_gpu():
    rec = paper_streams()
    d = dev(rec)
    out = P.mrg_generate_paper(d, 1, 8, 2, 2, gen=P.MRG_GEN_MRG31K3P).cpu().numpy()[0]
    want = np.array([float(v) for v in read_golden("mrg31k3p_runif_example.txt")[0]])
    assert np.all(np.abs(out - want) <= 0.5e-3 + 1e-12), out
    run(P.MRG_GEN_MRG31K3P, rec, 1, 8, 8, 2, 2, P.MRG_UNIFORM, P.MRG_F64)


def test_rexp_printout_on_gpu():
    rec = paper_streams()
    O.advance(O.MRG31K3P, rec, 4)
    d = dev(rec)
    out = P.mrg_generate_paper(d, 2, 4, 2, 2, P.MRG_EXPONENTIAL, P.MRG_F64, 1.0,
                               gen=P.MRG_GEN_MRG31K3P).cpu().numpy()
    for r, c, val, dec in read_golden("mrg31k3p_rexp_example.txt"):
        r, c, dec = int(r), int(c), int(dec)
        assert abs(out[r, c] - float(val)) <= 0.5 * 10.0 ** (-dec) + 1e-12, (r, c)
    run(P.MRG_GEN_MRG31K3P, rec, 2, 4, 4, 2, 2, P.MRG_EXPONENTIAL, P.MRG_F64)


CASES = [(P.MRG_UNIFORM, P.MRG_F64), (P.MRG_UNIFORM, P.MRG_F32), (P.MRG_RAW, P.MRG_U32),
         (P.MRG_NORMAL, P.MRG_F64), (P.MRG_NORMAL, P.MRG_F32), (P.MRG_EXPONENTIAL, P.MRG_F64),
         (P.MRG_EXPONENTIAL, P.MRG_F32)]
# (nrow, ncol, npad, G0, G1): one row block; many row blocks (finalize path);
# cells fewer than work-items; ragged lattices; padding
SHAPES = [(1, 8, 8, 2, 2), (7, 6, 9, 3, 2), (50, 14, 16, 2, 4), (3, 4, 4, 5, 6), (301, 130, 131, 16, 8),
          (2048, 2048, 2048, 1024, 1024)]


@pytest.mark.parametrize("gen", [P.MRG_GEN_MRG32K3A, P.MRG_GEN_MRG31K3P])
@pytest.mark.parametrize("dist,dtype", CASES)
@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_geometry_matches_oracle(gen, dist, dtype, shape):
    nrow, ncol, npad, G0, G1 = shape
    if dist == P.MRG_NORMAL and (ncol % 2 or G1 % 2):
        pytest.skip("normals need an even G1 and ncol")
    seed = workloads.random_seed(nrow + 7 * ncol) % np.uint32(2147462579)
    rec = O.create_streams(OGEN[gen], seed, G0 * G1 + 5)
    run(gen, rec, nrow, ncol, npad, G0, G1, dist, dtype, 1.5)


def test_rejects_unpaired_normals_and_short_streams():
    rec = paper_streams()
    d = dev(rec)
    with pytest.raises(P.MrgError):
        P.mrg_generate_paper(d, 2, 3, 1, 2, P.MRG_NORMAL)
    with pytest.raises(P.MrgError):
        P.mrg_generate_paper(d, 2, 4, 1, 3, P.MRG_NORMAL)
    with pytest.raises(P.MrgError):
        P.mrg_generate_paper(d, 4, 4, 3, 2)  # 6 work-items, 4 streams
    before = P.as_u32(d).copy()
    P.mrg_generate_paper(d, 0, 5, 2, 2)  # empty: nothing moves
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.as_u32(d), before)


def test_paper_rnorm_example_sampled():
    """Section 3.1: rnormGpu(c(10000, 10000)) with Nglobal = c(512, 128) on
    65536 MRG31k3p streams (1e8 normals).  Twelve pairs of work-items are
    recomputed from their two streams: every cell they own, within 1e-15."""
    gen = P.MRG_GEN_MRG31K3P
    n_s, G0, G1, N = 65536, 512, 128, 10000
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=gen)
    d = P.mrg_streams_create_device(c, n_s, gen=gen)
    rec = P.as_u32(d).copy()
    out = P.mrg_generate_paper(d, N, N, G0, G1, P.MRG_NORMAL, gen=gen)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    picks = [(0, 0), (G0 - 1, G1 - 2), (271, 14), (272, 16)] + \
        [(int(a), 2 * int(b)) for a, b in zip(rng.integers(0, G0, 8), rng.integers(0, G1 // 2, 8))]
    after = P.as_u32(d)
    for g0, g1 in picks:
        sa, sb = g0 * G1 + g1, g0 * G1 + g1 + 1
        rows = np.arange(g0, N, G0)
        cols = np.arange(g1, N, G1)
        k = rows.size * cols.size
        ua = O.stream_draws(O.MRG31K3P, rec[sa, :6].copy(), k)
        ub = O.stream_draws(O.MRG31K3P, rec[sb, :6].copy(), k)
        X = np.empty(k)
        Y = np.empty(k)
        for t in range(k):
            X[t], Y[t] = O.box_muller(ua[t], ub[t])
        sub = out[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy().ravel()
        sub2 = out[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols + 1).cuda()].cpu().numpy().ravel()
        for got, want in ((sub, X), (sub2, Y)):
            err = np.abs(got - want) / np.maximum(np.abs(want), 1.0)
            assert err.max() <= 1e-15, (g0, g1, err.max())
        for s in (sa, sb):
            st = rec[s, :6].copy()
            O.jump(O.MRG31K3P, st, k)
            np.testing.assert_array_equal(after[s, :6], st)


def test_paper_rnorm_example_every_number():
    """Section 3.1's rnormGpu(c(10000, 10000)) on a 512 x 128 lattice of
    65,536 MRG31k3p streams: all 10^8 normals against the oracle's
    paper-geometry generator, within 1e-15, and every stream record after."""
    gen = P.MRG_GEN_MRG31K3P
    n_s, G0, G1, N = 65536, 512, 128, 10000
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=gen)
    d = P.mrg_streams_create_device(c, n_s, gen=gen)
    work = P.as_u32(d).copy()
    out = P.mrg_generate_paper(d, N, N, G0, G1, P.MRG_NORMAL, gen=gen)
    torch.cuda.synchronize()
    want = O.generate_paper(O.MRG31K3P, work, N, N, G0, G1, O.NORMAL, O.F64)
    for r0 in range(0, N, 1000):
        got = out[r0:r0 + 1000].cpu().numpy()
        w = want[r0:r0 + 1000]
        err = np.abs(got - w) / np.maximum(np.abs(w), 1.0)
        assert err.max() <= 1e-15, (r0, err.max())
    np.testing.assert_array_equal(P.as_u32(d), work)
