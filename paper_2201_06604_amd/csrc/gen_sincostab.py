"""Write mrg_sincostab.h: the 129-entry table of sincospi_unit (mrg_engine.h).

    python paper_2201_06604_amd/csrc/gen_sincostab.py

The Box-Muller angle argument t = 2 u2 lies in (0, 2).  Entry j (0 <= j <= 128)
holds sin(pi j/64) and cos(pi j/64), each as hi + lo (hi the double nearest
the value, lo the double nearest the remainder); at j = 0, 32, 64, 96, 128 the
values are exactly 0 or +-1 and lo is 0.  sincospi_unit takes j = rint(64 t)
and d = t - j/64 (exact, |d| <= 1/128) and combines the entry with sin(pi d)
and cos(pi d) - 1 by the angle-sum formulas.  pi comes from Machin's formula
and sin/cos from their Taylor series, all in Python's decimal arithmetic at 60
significant digits; each stored value is rounded once.
"""
import os
from decimal import Decimal, getcontext

getcontext().prec = 60
HERE = os.path.dirname(os.path.abspath(__file__))
N = 128  # entries j = 0 .. N


def atan_inv(x: int) -> Decimal:
    """atan(1/x) by its series."""
    x2 = x * x
    term = Decimal(1) / x
    total, k = term, 1
    while True:
        term /= -x2
        nxt = total + term / (2 * k + 1)
        if nxt == total:
            return total
        total, k = nxt, k + 1


PI = 16 * atan_inv(5) - 4 * atan_inv(239)


def sin_cos(x: Decimal):
    s, c = Decimal(0), Decimal(0)
    term, n = Decimal(1), 0  # x^n / n!
    while True:
        if n % 4 == 0:
            c += term
        elif n % 4 == 1:
            s += term
        elif n % 4 == 2:
            c -= term
        else:
            s -= term
        n += 1
        term = term * x / n
        if abs(term) < Decimal(10) ** -70:
            return s, c


def split(v: Decimal):
    hi = float(v)
    lo = float(v - Decimal(hi))
    return hi, lo


def entries():
    out = []
    for j in range(N + 1):
        if j % 32 == 0:  # the axes: exact values
            q = j // 32
            s = [0.0, 1.0, 0.0, -1.0, 0.0][q]
            c = [1.0, 0.0, -1.0, 0.0, 1.0][q]
            out.append((s, 0.0, c, 0.0))
            continue
        sv, cv = sin_cos(PI * j / 64)
        out.append(split(sv) + split(cv))
    return out


def main():
    rows = [f"    {{{a.hex()}, {b.hex()}, {c.hex()}, {d.hex()}}},  // j = {j}"
            for j, (a, b, c, d) in enumerate(entries())]
    text = """// mrg_sincostab.h -- table of sincospi_unit (mrg_engine.h): for j = 0..128,
// sin(pi j/64) and cos(pi j/64), each as hi + lo (exact 0 or +-1 on the axes).
// Written by gen_sincostab.py (Python decimal arithmetic at 60 digits, each
// value rounded once); do not edit.
#pragma once

namespace mrg355 {

constexpr int kSinCosTabN = %d;
struct SinCosTable {
    double e[kSinCosTabN][4];  // (sin hi, sin lo, cos hi, cos lo) of each entry
};
constexpr SinCosTable kSinCosTable = {{
%s
}};

}  // namespace mrg355
""" % (N + 1, "\n".join(rows))
    with open(os.path.join(HERE, "mrg_sincostab.h"), "w") as f:
        f.write(text)


if __name__ == "__main__":
    main()
