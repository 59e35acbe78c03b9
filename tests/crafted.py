"""Crafted generator states for edge-input tests (test infrastructure).

A state is built backwards: choose the state after k steps so that those k
steps output chosen integers z (k <= 3), then undo the k steps one at a time.
Undoing a step solves the recurrence for its oldest term:

    x[n] = a1 x[n-1] + a2 x[n-2] + a3 x[n-3]  (mod m)
    =>  x[n-3] = (x[n] - a1 x[n-1] - a2 x[n-2]) * a3^(-1)  (mod m)

which needs only Python integers and a modular inverse.  The combined output
of a step is z = x1 - x2 if x1 > x2, else x1 - x2 + m1 (an integer in
[1, m1]); to make a step output z, its new component-1 value is set to
(x2 + z) mod m1, which gives back z for every z in [1, m1] because x2 < m1.

The multipliers below are the published parameters of the two generators
(MRG32k3a: L'Ecuyer 1999; MRG31k3p: L'Ecuyer and Touzin 2000, the paper's
Section 2).  Tests check every crafted state with the oracle (its outputs are
the chosen ones) before using it, so a slip here cannot pass silently.
"""
import numpy as np

MRG32K3A, MRG31K3P = 1, 2

# per generator: moduli, (a1, a2, a3) per component, word order of the
# external 6-word state (False = oldest-first, True = newest-first)
PARAMS = {
    MRG32K3A: ((4294967087, 4294944443), ((0, 1403580, -810728), (527612, 0, -1370589)), False),
    MRG31K3P: ((2147483647, 2147462579), ((0, 1 << 22, (1 << 7) + 1), (1 << 15, 0, (1 << 15) + 1)), True),
}


def modulus1(gen):
    return PARAMS[gen][0][0]


def _to_external(gen, c1, c2):
    """Oldest-first component triples -> the generator's 6-word order."""
    newest_first = PARAMS[gen][2]
    if newest_first:
        return [c1[2], c1[1], c1[0], c2[2], c2[1], c2[0]]
    return list(c1) + list(c2)


def _undo(c, a, m):
    """(x[n-2], x[n-1], x[n]) -> (x[n-3], x[n-2], x[n-1]) for one component."""
    a1, a2, a3 = a
    xn2, xn1, xn = c
    xn3 = (xn - a1 * xn1 - a2 * xn2) * pow(a3 % m, -1, m) % m
    return (xn3, xn2, xn1)


def state_with_outputs(gen, zs, rng):
    """A valid 6-word state (uint32) whose next len(zs) outputs are zs
    (1 <= len(zs) <= 3, each in [1, m1]); the other words are drawn from
    `rng` (numpy Generator)."""
    (m1, m2), (a_1, a_2), _ = PARAMS[gen]
    k = len(zs)
    assert 1 <= k <= 3 and all(1 <= z <= m1 for z in zs)
    while True:
        # the state after k steps, oldest-first: its last k words are the
        # values the k steps produced
        c2 = [int(v) for v in rng.integers(0, m2, size=3)]
        c1 = [int(v) for v in rng.integers(0, m1, size=3)]
        for i, z in enumerate(zs):
            pos = 3 - k + i
            c1[pos] = (c2[pos] + z) % m1
        s1, s2 = tuple(c1), tuple(c2)
        for _ in range(k):
            s1 = _undo(s1, a_1, m1)
            s2 = _undo(s2, a_2, m2)
        if any(s1) and any(s2) and any(c1) and any(c2):
            return np.array(_to_external(gen, s1, s2), dtype=np.uint32)


def records(states):
    """Stream records (n x 18: current, initial, substream start) whose three
    states are all the given ones."""
    st = np.asarray(states, dtype=np.uint32).reshape(-1, 6)
    return np.ascontiguousarray(np.concatenate([st, st, st], axis=1))
