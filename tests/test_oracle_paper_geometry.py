"""Pins of the oracle's paper-geometry generation (the work-item lattice of
Listing 1, Section 2.2, and Listing 2, Section 3.1) to facts outside it: the
values the paper prints for runifGpu and rexpGpu, a closed-form statement of
the placement (cell -> work-item, visit number -> draw), stream advances,
and the Box-Muller identities across the two streams of a pair."""
import math

import numpy as np
import pytest

import oracle as O
import workloads
from conftest import read_golden

GEN = O.MRG31K3P


def _paper_streams():
    return O.create_streams(GEN, np.array(workloads.PAPER_SEED, dtype=np.uint32), 4)


def test_runif_printout():
    """Section 2.2: runifGpu(n = 8, Nglobal = c(2,2)) on the four fresh
    streams prints these 8 values (3 decimals); a vector is one row."""
    want = np.array([float(v) for v in read_golden("mrg31k3p_runif_example.txt")[0]])
    S = _paper_streams()
    got = O.generate_paper(GEN, S, 1, 8, 2, 2)[0]
    assert np.all(np.abs(got - want) <= 0.5e-3 + 1e-12), got
    # only the work-items (0,0) and (0,1) own cells: streams 1 and 3
    # (1-based) advanced 4 steps, streams 2 and 4 did not move
    ref = _paper_streams()
    for s, k in enumerate([4, 0, 4, 0]):
        st = ref[s, :6].copy()
        O.jump(GEN, st, k)
        np.testing.assert_array_equal(S[s, :6], st)


def test_rexp_printout():
    """Section 3.2: rexpGpu(c(2,4), rate = 1, Nglobal = c(2,2)) prints this
    2 x 4 matrix; the streams had made 4 draws each before it."""
    S = _paper_streams()
    O.advance(GEN, S, 4)
    got = O.generate_paper(GEN, S, 2, 4, 2, 2, O.EXPONENTIAL, O.F64, 1.0)
    for r, c, val, dec in read_golden("mrg31k3p_rexp_example.txt"):
        r, c, dec = int(r), int(c), int(dec)
        assert abs(got[r, c] - float(val)) <= 0.5 * 10.0 ** (-dec) + 1e-12, (r, c, got[r, c], val)


def _closed_form(gen, rec, nrow, ncol, G0, G1, dist, dtype, param, npad):
    """Cell (r, c) belongs to work-item (r mod G0, c mod G1); it is that
    work-item's visit number ((r - g0)/G0) * nc + (c - g1)/G1 with nc its
    number of columns; the value is the stream's draw of that number."""
    out = np.full((nrow, npad), 12345, dtype=np.float64 if dtype == O.F64 else
                  (np.float32 if dtype == O.F32 else np.uint32))
    for g0 in range(G0):
        for g1 in range(G1):
            s = g0 + G0 * g1 if dist in (O.UNIFORM, O.RAW) else g0 * G1 + g1
            nr = len(range(g0, nrow, G0))
            nc = len(range(g1, ncol, G1))
            draws = O.stream_draws(gen, rec[s, :6].copy(), nr * nc, dist, dtype, param)
            for r in range(g0, nrow, G0):
                for c in range(g1, ncol, G1):
                    out[r, c] = draws[((r - g0) // G0) * nc + (c - g1) // G1]
    return out


@pytest.mark.parametrize("gen", [O.MRG31K3P, O.MRG32K3A])
@pytest.mark.parametrize("dist,dtype", [(O.UNIFORM, O.F64), (O.UNIFORM, O.F32), (O.RAW, O.U32),
                                        (O.EXPONENTIAL, O.F64)])
@pytest.mark.parametrize("nrow,ncol,npad,G0,G1", [(1, 8, 8, 2, 2), (7, 5, 9, 3, 2), (10, 13, 13, 4, 5),
                                                  (3, 3, 4, 5, 7), (16, 1, 2, 2, 3)])
def test_placement_closed_form(gen, dist, dtype, nrow, ncol, npad, G0, G1):
    rec = O.create_streams(gen, workloads.random_seed(nrow * 31 + ncol) % np.uint32(2147462579), G0 * G1 + 3)
    a = rec.copy()
    got = O.generate_paper(gen, a, nrow, ncol, G0, G1, dist, dtype, 0.7, npad=npad, fill=12345)
    want = _closed_form(gen, rec, nrow, ncol, G0, G1, dist, dtype, 0.7, npad)
    np.testing.assert_array_equal(got, want)
    # streams advance by their visit counts; the extra ones do not move
    for s in range(G0 * G1 + 3):
        if s < G0 * G1:
            if dist in (O.UNIFORM, O.RAW):
                g0, g1 = s % G0, s // G0
            else:
                g0, g1 = s // G1, s % G1
            k = len(range(g0, nrow, G0)) * len(range(g1, ncol, G1))
        else:
            k = 0
        st = rec[s, :6].copy()
        O.jump(gen, st, k)
        np.testing.assert_array_equal(a[s, :6], st, err_msg=str(s))


def test_normal_pairs_use_two_streams():
    """Listing 2: X and Y of a pair come from U1 of the even work-item's
    stream and U2 of the odd one's: X^2 + Y^2 = -2 log U1 and
    atan2(Y, X) = 2 pi U2 (mod 2 pi), cell by cell."""
    nrow, ncol, G0, G1 = 5, 8, 2, 4
    rec = O.create_streams(GEN, workloads.random_seed(3) % np.uint32(2147462579), G0 * G1)
    out = O.generate_paper(GEN, rec.copy(), nrow, ncol, G0, G1, O.NORMAL)
    for g0 in range(G0):
        for p in range(G1 // 2):
            sa, sb = g0 * G1 + 2 * p, g0 * G1 + 2 * p + 1
            nr, nc = len(range(g0, nrow, G0)), len(range(2 * p, ncol, G1))
            ua = O.stream_draws(GEN, rec[sa, :6].copy(), nr * nc)
            ub = O.stream_draws(GEN, rec[sb, :6].copy(), nr * nc)
            t = 0
            for r in range(g0, nrow, G0):
                for c in range(2 * p, ncol, G1):
                    X, Y = out[r, c], out[r, c + 1]
                    assert abs(X * X + Y * Y + 2 * math.log(ua[t])) < 1e-12 * max(1.0, X * X + Y * Y)
                    ang = math.atan2(Y, X) % (2 * math.pi)
                    d = abs(ang - 2 * math.pi * ub[t])
                    assert min(d, 2 * math.pi - d) < 1e-12, (r, c)
                    t += 1


@pytest.mark.parametrize("args", [(3, 5, 2, 2), (3, 6, 2, 3), (0, 0, 0, 1), (2, 2, 1, 0)])
def test_invalid_geometry(args):
    nrow, ncol, G0, G1 = args
    rec = O.create_streams(GEN, np.array(workloads.PAPER_SEED, dtype=np.uint32), 8)
    with pytest.raises(ValueError):
        O.generate_paper(GEN, rec, nrow, ncol, G0, G1, O.NORMAL)
    with pytest.raises(ValueError):  # too few streams for the lattice
        O.generate_paper(GEN, rec, 4, 4, 3, 3)
