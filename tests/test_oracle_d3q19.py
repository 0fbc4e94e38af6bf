"""Pins for the oracle's D3Q19 constants: the defining moment identities of
the velocity set and weights, checked in exact rational arithmetic."""
from fractions import Fraction
from itertools import product

import numpy as np

from oracle.d3q19 import C, W, OPP, Q

WF = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12


def test_velocity_set_is_d3q19():
    assert Q == 19 and C.shape == (19, 3)
    vs = {tuple(int(v) for v in c) for c in C}
    expect = {c for c in product((-1, 0, 1), repeat=3) if sum(map(abs, c)) <= 2}
    assert vs == expect  # rest + 6 faces + 12 edges of the unit cube
    assert tuple(C[0]) == (0, 0, 0)


def test_weights_are_the_rounded_rationals():
    for q in range(Q):
        assert W[q] == float(WF[q])
        # weight depends only on |c|^2
        assert WF[q] == {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}[int((C[q] ** 2).sum())]


def test_isotropy_exact():
    d = lambda a, b: 1 if a == b else 0
    assert sum(WF) == 1
    for a in range(3):
        assert sum(WF[q] * int(C[q, a]) for q in range(Q)) == 0
    for a, b in product(range(3), repeat=2):
        assert sum(WF[q] * int(C[q, a]) * int(C[q, b]) for q in range(Q)) == Fraction(d(a, b), 3)
    for a, b, c in product(range(3), repeat=3):
        assert sum(WF[q] * int(C[q, a] * C[q, b] * C[q, c]) for q in range(Q)) == 0
    for a, b, c, e in product(range(3), repeat=4):
        lhs = sum(WF[q] * int(C[q, a] * C[q, b] * C[q, c] * C[q, e]) for q in range(Q))
        rhs = Fraction(d(a, b) * d(c, e) + d(a, c) * d(b, e) + d(a, e) * d(b, c), 9)
        assert lhs == rhs


def test_opposites():
    for q in range(Q):
        assert np.all(C[OPP[q]] == -C[q])
        assert OPP[OPP[q]] == q
    assert OPP[0] == 0
