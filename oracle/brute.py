"""Pure-Python brute force for tiny causal sets.

TEST INFRASTRUCTURE ONLY (used by ``tests/``).  Shares nothing with the C oracle
or the GPU library: relations are given as Python sets and every interval is
enumerated element by element, following the definition of the inclusive order
intervals (Cunningham 2018, Sec. 4.2, eq. IOIs): for a related pair (i, j) the
Alexandroff set A_ij = {k : i ≺ k ≺ j}; N_n counts related pairs with |A_ij| = n.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import permutations


def order_from_dominance(u, v):
    """2D order: i ≺ j iff u_i < u_j and v_i < v_j.  Returns the set of pairs."""
    n = len(u)
    return {(i, j) for i in range(n) for j in range(n) if u[i] < u[j] and v[i] < v[j]}


def abundances(n, rel):
    """N_m for m = 0..n-2 by enumerating each Alexandroff set."""
    hist = [0] * max(n - 1, 1)
    for (i, j) in rel:
        inside = [k for k in range(n) if (i, k) in rel and (k, j) in rel]
        hist[len(inside)] += 1
    return hist


def all_2d_orders(n):
    """Every labelled 2D order on n elements as (u ranks, v ranks), u = identity."""
    base = list(range(n))
    for perm in permutations(base):
        yield base, list(perm)


def smear_exact(dim, m, eps: Fraction) -> Fraction:
    """The thesis's smearing function f_d(m, eps), evaluated exactly in rationals
    in its printed (direct) form; requires eps < 1."""
    one = Fraction(1)
    q = one - eps
    if dim == 2:
        br = one - Fraction(2 * m) * eps / q + Fraction(m * (m - 1)) * eps ** 2 / (2 * q ** 2)
    elif dim == 3:
        br = (one - Fraction(27 * m) * eps / (8 * q)
              + Fraction(9 * m * (m - 1)) * eps ** 2 / (8 * q ** 2))
    elif dim == 4:
        br = (one - Fraction(9 * m) * eps / q + Fraction(8 * m * (m - 1)) * eps ** 2 / q ** 2
              - Fraction(4 * m * (m - 1) * (m - 2)) * eps ** 3 / (3 * q ** 3))
    else:
        raise ValueError(dim)
    return q ** m * br


def smeared_bracket_exact(hist, n, dim, eps: Fraction) -> Fraction:
    """The bracket [N - c eps sum_m N_m f(m, eps)] of the smeared action, exactly
    (c = 2 in 1+1, c = 1 in 2+1 and 3+1)."""
    c = 2 if dim == 2 else 1
    s = sum(Fraction(int(h)) * smear_exact(dim, m, eps) for m, h in enumerate(hist) if h)
    return Fraction(n) - c * eps * s


def local_integer(hist, n, dim):
    """The combination inside the local BD action (a rational in 2+1)."""
    h = [int(x) for x in hist] + [0, 0, 0, 0]
    if dim == 2:
        return n - 2 * h[0] + 4 * h[1] - 2 * h[2]
    if dim == 3:
        return Fraction(n - h[0]) + Fraction(27, 8) * h[1] - Fraction(9, 4) * h[2]
    return n - h[0] + 9 * h[1] - 16 * h[2] + 8 * h[3]


def dalembertian_2d_exact(n, rel, phi, ell2: Fraction):
    """B^(1+1) phi(j) = (2 / ell^2) [-phi(j) + 2 (sum_{L1} - 2 sum_{L2} + sum_{L3})] in exact
    rationals, with L_m(j) found by enumerating each Alexandroff set (Sec. 4.1)."""
    coef = {0: 2, 1: -4, 2: 2}
    out = []
    for j in range(n):
        acc = -Fraction(phi[j])
        for i in range(n):
            if (i, j) not in rel:
                continue
            inside = sum(1 for k in range(n) if (i, k) in rel and (k, j) in rel)
            if inside in coef:
                acc += coef[inside] * Fraction(phi[i])
        out.append(2 * acc / ell2)
    return out
