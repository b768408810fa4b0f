"""Finite-difference weights from the moment conditions, in exact rationals.

TEST INFRASTRUCTURE (part of the oracle).  The worked examples of the paper
ask for an 8th-order, 9-point second derivative (Sec. 4.1) and a second-order
central difference (Sec. 4.2); the discretisation of Sec. 5.1 prints the
second-order second and fourth derivatives.  Rather than recalling tables,
the weights w_a on the integer offsets a are the unique solution of the
moment (Vandermonde) system

    sum_a w_a * a**q / q!  =  [q == m],     q = 0 .. K-1,

for K offsets and derivative order m: the stencil is then exact on every
polynomial of degree below K (the Taylor expansion of u(x + a h) about x).
Solved by Gauss-Jordan elimination over fractions.Fraction.
"""
from fractions import Fraction
from math import factorial
from typing import List, Sequence


def fd_weights(m: int, offsets: Sequence[int]) -> List[Fraction]:
    """Weights (per unit spacing; divide by h**m) of the m-th derivative on
    the integer offsets given."""
    offs = [int(a) for a in offsets]
    K = len(offs)
    if len(set(offs)) != K or not 0 <= m < K:
        raise ValueError("need distinct offsets and 0 <= m < len(offsets)")
    rows = [[Fraction(a) ** q / factorial(q) for a in offs]
            + [Fraction(1 if q == m else 0)] for q in range(K)]
    for col in range(K):
        piv = next(r for r in range(col, K) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        p = rows[col][col]
        rows[col] = [v / p for v in rows[col]]
        for r in range(K):
            if r != col and rows[r][col] != 0:
                f = rows[r][col]
                rows[r] = [v - f * u for v, u in zip(rows[r], rows[col])]
    return [rows[k][K] for k in range(K)]


def central_weights(m: int, half_width: int) -> List[Fraction]:
    """Central stencil on offsets -half_width .. half_width."""
    return fd_weights(m, range(-half_width, half_width + 1))


def as_floats(ws: Sequence[Fraction], h: float = 1.0, m: int = 0) -> List[float]:
    """Float weights divided by h**m."""
    return [float(w) / h ** m for w in ws]
