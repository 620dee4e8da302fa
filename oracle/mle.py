"""Multilinear extensions and the identity polynomial (GKR section; Section 3.2.2).

Convention: a table of 2^k values is indexed by b in [0, 2^k); variable 1 is the
most significant bit of b and variable k the least significant one. So for a
data-parallel layer with index g = z * 2^n + c the local (sub-circuit) bits are
the first variables and the copy bits the last ones, which is where the
distributed sumcheck of Section 3.2.1 places the worker index.

eq(a, b) is the paper's identity polynomial beta~(a, b) = prod_k ((1-a_k)(1-b_k) + a_k b_k).
The multilinear extension of V is V~(r) = sum_b V[b] eq(r, bits(b)).
"""
from typing import List, Sequence

from .field import P


def bits_msb_first(b: int, k: int) -> List[int]:
    return [(b >> (k - 1 - j)) & 1 for j in range(k)]


def eq(a: Sequence[int], b: Sequence[int]) -> int:
    """The identity polynomial beta~(a, b) evaluated at two points of the same length."""
    if len(a) != len(b):
        raise ValueError("points of different length")
    acc = 1
    for ak, bk in zip(a, b):
        acc = acc * ((1 - ak) * (1 - bk) + ak * bk) % P
    return acc


def eq_table(r: Sequence[int]) -> List[int]:
    """[eq(r, bits(b)) for b in 0 .. 2^len(r) - 1].

    Built one variable at a time: appending variable r_k as the new least
    significant bit splits every entry t into (t * (1 - r_k), t * r_k).
    """
    table = [1]
    for rk in r:
        nk = (1 - rk) % P
        table = [v for t in table for v in (t * nk % P, t * rk % P)]
    return table


def fold(table: Sequence[int], r: int) -> List[int]:
    """Bind the most significant variable to r: X'[b] = X[b] + r (X[b + M/2] - X[b])."""
    h = len(table) // 2
    lo, hi = table[:h], table[h:]
    return [(a + r * (b - a)) % P for a, b in zip(lo, hi)]


def evaluate_by_folding(table: Sequence[int], r: Sequence[int]) -> int:
    """V~(r) by binding variables 1, 2, ... in order."""
    if len(table) != 1 << len(r):
        raise ValueError("table size does not match the point")
    x = list(table)
    for rj in r:
        x = fold(x, rj)
    return x[0]


def evaluate_by_eq(table: Sequence[int], r: Sequence[int]) -> int:
    """V~(r) = sum_b V[b] eq(r, bits(b)), straight from the definition."""
    if len(table) != 1 << len(r):
        raise ValueError("table size does not match the point")
    return sum(v * e for v, e in zip(table, eq_table(r))) % P


evaluate = evaluate_by_folding
