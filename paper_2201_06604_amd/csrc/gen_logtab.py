"""Write mrg_logtab.h: the 512-entry table of log_unit (mrg_engine.h).

    python paper_2201_06604_amd/csrc/gen_logtab.py

A uniform u = m 2^k (m in [1/2, 1)) falls in interval j = floor(1024 (m - 1/2))
of width 1/1024 (the top 9 fraction bits of m).  Entry j holds R_j, the
multiple of 2^-9 nearest 1/c_j (c_j the interval's midpoint; R_511 = 1, so
that t = m - 1 near u = 1), and -log(R_j) split as hi + lo, hi a multiple of
2^-40.  Then |t| = |m R_j - 1| < 2^-9 (checked below for every interval), and
t is exact in one FMA: m is a multiple of 2^-53 and R_j of 2^-9, so t is a
multiple of 2^-62 of magnitude below 2^-9, at most 53 significant bits.
log(u) = k ln2 + hi + lo + log1p(t).  Logarithms come from Python's decimal
module at 60 significant digits, each rounded once to double.
"""
import os
from decimal import Decimal, getcontext

getcontext().prec = 60
HERE = os.path.dirname(os.path.abspath(__file__))
N = 512


def to_double(d: Decimal) -> float:
    """Round a Decimal to the nearest double."""
    return float(d)  # Decimal -> float rounds correctly (via the exact decimal string)


def entries():
    out = []
    for j in range(N):
        if j == N - 1:
            r = Decimal(1)
        else:
            c = Decimal(1) / 2 + (Decimal(j) + Decimal(1) / 2) / 1024
            r = (Decimal(512) / c).to_integral_value() / 512
        t = -r.ln()
        hi = (t * (Decimal(2) ** 40)).to_integral_value() / (Decimal(2) ** 40)
        lo = t - hi
        out.append((float(r), float(hi), to_double(lo)))
        assert Decimal(out[-1][0]) == r and Decimal(out[-1][1]) == hi
        # |t| < 2^-9 over the interval
        m_lo = Decimal(1) / 2 + Decimal(j) / 1024
        m_hi = m_lo + Decimal(1) / 1024
        assert max(abs(m_lo * r - 1), abs(m_hi * r - 1)) < Decimal(2) ** -9, j
    return out


def main():
    rows = [f"    {{{r.hex()}, {hi.hex()}, {lo.hex()}}},  // j = {j}" for j, (r, hi, lo) in enumerate(entries())]
    text = """// mrg_logtab.h -- table of log_unit (mrg_engine.h): for interval j of the
// mantissa m in [1/2, 1) (m in [1/2 + j/1024, 1/2 + (j+1)/1024)), the multiple R
// of 2^-9 nearest the reciprocal of the interval's midpoint (R = 1 for the last one)
// and -log(R) as hi + lo (hi a multiple of 2^-40).  Written by gen_logtab.py
// (Python decimal arithmetic at 60 digits, each value rounded once); do not
// edit.
#pragma once

namespace mrg355 {

constexpr int kLogTabN = %d;
struct LogTable {
    double e[kLogTabN][3];  // (R, hi, lo) of each interval
};
constexpr LogTable kLogTable = {{
%s
}};

}  // namespace mrg355
""" % (N, "\n".join(rows))
    with open(os.path.join(HERE, "mrg_logtab.h"), "w") as f:
        f.write(text)


if __name__ == "__main__":
    main()
