"""Lower bounds on the number of colours and the tile policy (arXiv:2106.01275).

TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle/__init__.py).

Everything here is plain Python over explicit point sets:
  * clique_C / clique_T / clique_S build the sets of Thm. evenC (eq. cond:1)
    and Thm. oddC (eqs. cond:2, cond:3) on Z^d, by enumeration;
  * col_lower_bound is eq. (pBounds) (Sec. 3.2), with |C(d, alpha, beta)|
    counted from the set definition (not from the recursive listing, whose
    d == 1 branch omits the 2p term and gives 9 instead of 37 for (2, 4));
  * p0_lower_bound is eq. (7) for p = 0;
  * tile_shape is the tile policy of Sec. 3.5.
"""
from __future__ import annotations

import itertools
import math


def l1_ball(d: int, r: int):
    """Points of Z^d with L1 norm <= r (N^d(0, 0, r) plus the centre)."""
    if r < 0:
        return []
    return [x for x in itertools.product(range(-r, r + 1), repeat=d)
            if sum(abs(t) for t in x) <= r]


def clique_C(d: int, alpha: int, beta: int):
    """C(d, alpha, beta) = {x : |x|_1 <= alpha and sum_{i>=2} |x_i| <= beta} (eq. cond:1)."""
    return [x for x in l1_ball(d, alpha) if sum(abs(t) for t in x[1:]) <= beta]


def clique_T(d: int, p: int, beta: int):
    """T of Thm. oddC (eq. cond:2): -(p-1) <= x1 <= p, 1 <= x2 <= beta+1,
    sum_{i>=2} |x_i| = beta + 1.  The printed strict bound x2 < beta+1 is
    read as <=: only then does |S| + |T| = |C(d-1, alpha, beta)| hold as the
    paper states (with < the set T is empty whenever beta = 0)."""
    if d < 2:
        return []
    out = []
    for x1 in range(-(p - 1), p + 1):
        for rest in itertools.product(range(-(beta + 1), beta + 2), repeat=d - 1):
            if 1 <= rest[0] <= beta + 1 and sum(abs(t) for t in rest) == beta + 1:
                out.append((x1,) + rest)
    return out


def clique_S(d: int, p: int, alpha: int, beta: int):
    """S of Thm. oddC (eq. cond:3): p+1 <= x1 <= alpha+1, |x2| <= beta,
    |x|_1 = alpha + 1."""
    out = []
    for x1 in range(p + 1, alpha + 2):
        for rest in itertools.product(range(-(alpha + 1), alpha + 2), repeat=d - 1):
            if d >= 2 and abs(rest[0]) > beta:
                continue
            if abs(x1) + sum(abs(t) for t in rest) == alpha + 1:
                out.append((x1,) + rest)
    return out


def size_C(d: int, alpha: int, beta: int) -> int:
    if d == 0:
        return 1
    return len(clique_C(d, alpha, beta))


def p0_lower_bound(d: int, k: int) -> int:
    """eq. (7): |N^d(0,0,k/2)| (k even), |N^d(0,0,k//2)| + |N^{d-1}(0,0,k//2)| (k odd)."""
    h = k // 2
    n = len(l1_ball(d, h))
    if k % 2:
        n += len(l1_ball(d - 1, h)) if d > 1 else 1
    return n


def col_lower_bound(d: int, p: int, k: int) -> int:
    """eq. (pBounds) (Sec. 3.2): lower bound on col(Z^d_inf, p, k)."""
    if k == p:
        return 2 * k + 1
    if k < p:
        return math.ceil(2 * p / (p - k))
    alpha, beta = (k + p) // 2, (k - p) // 2
    if (k + p) % 2 == 0:
        return size_C(d, alpha, beta)
    return size_C(d, alpha, beta) + size_C(d - 1, alpha, beta)


def _next_pow2(n: int) -> int:
    t = 1
    while t < n:
        t *= 2
    return t


def tile_shape(dims, p: int, k: int):
    """Tile policy of Sec. 3.5 (displacement along dimension 0): each side at
    least 2k+1 (2(p+k)+1 along the displacement), rounded up to a power of
    two and capped at the lattice extent.  Where that power of two does not
    divide the extent, the smallest divisor of the extent that is at least
    the minimum length is taken (our reading; the paper's lattices are powers
    of two)."""
    out = []
    for i, D in enumerate(dims):
        need = 2 * (p + k) + 1 if i == 0 else 2 * k + 1
        t = _next_pow2(need)
        if t >= D:
            t = D
        elif D % t:
            t = next(c for c in range(need, D + 1) if D % c == 0)
        out.append(t)
    return tuple(out)
