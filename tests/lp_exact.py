"""Exact-rational brute force for triangle-pair intersection (test helper).

Two closed triangles P (corners P0..P2) and Q (Q0..Q2) share a point exactly
when the linear program
    lam >= 0, sum(lam) = 1, mu >= 0, sum(mu) = 1, sum lam_i P_i = sum mu_j Q_j
is feasible.  With s shared vertex ids the pair is a self-intersection (the
exact reading of Sec. 5.2 / Appendix 3 of the paper) when
    s = 0: the program is feasible;
    s = 1, 2: some common point has positive barycentric weight on a corner of
              P that is not shared, i.e. max sum(lam_i, i not shared) > 0;
    s = 3: always.
Everything is computed with ``fractions.Fraction`` by a two-phase simplex with
Bland's rule, so there is no rounding anywhere.  This uses no orientation
predicate at all, which makes it independent of the oracle under test.
"""
from __future__ import annotations

from fractions import Fraction as Fr


def _simplex_max(A, b, c):
    """max c.x s.t. A x = b, x >= 0 (exact).  Returns None if infeasible."""
    m, n = len(A), len(A[0])
    A = [[Fr(x) for x in row] for row in A]
    b = [Fr(x) for x in b]
    for i in range(m):
        if b[i] < 0:
            A[i] = [-x for x in A[i]]
            b[i] = -b[i]
    # tableau with artificials n..n+m-1
    T = [A[i] + [Fr(1) if j == i else Fr(0) for j in range(m)] + [b[i]] for i in range(m)]
    basis = [n + i for i in range(m)]
    N = n + m

    def pivot(r, col):
        pv = T[r][col]
        T[r] = [x / pv for x in T[r]]
        for i in range(m):
            if i != r and T[i][col] != 0:
                f = T[i][col]
                T[i] = [x - f * y for x, y in zip(T[i], T[r])]
        basis[r] = col

    def optimize(cost, allowed):
        # maximize cost.x over current tableau; Bland's rule
        while True:
            # reduced costs: r_j = cost_j - sum_i cost_{basis_i} T[i][j]
            enter = None
            for j in range(N):
                if j not in allowed or j in basis:
                    continue
                rj = cost[j] - sum(cost[basis[i]] * T[i][j] for i in range(m))
                if rj > 0:
                    enter = j
                    break
            if enter is None:
                return
            best = None
            for i in range(m):
                if T[i][enter] > 0:
                    ratio = T[i][-1] / T[i][enter]
                    if best is None or ratio < best[0] or (ratio == best[0] and basis[i] < basis[best[1]]):
                        best = (ratio, i)
            if best is None:
                raise RuntimeError("unbounded")
            pivot(best[1], enter)

    # phase 1: maximize -sum(artificials)
    c1 = [Fr(0)] * n + [Fr(-1)] * m
    optimize(c1, set(range(N)))
    if sum(T[i][-1] for i in range(m) if basis[i] >= n) != 0:
        return None
    # drive artificials out of the basis where possible
    for i in range(m):
        if basis[i] >= n:
            for j in range(n):
                if T[i][j] != 0:
                    pivot(i, j)
                    break
    c2 = [Fr(x) for x in c] + [Fr(0)] * m
    optimize(c2, set(range(n)) | {basis[i] for i in range(m) if basis[i] >= n})
    x = [Fr(0)] * N
    for i in range(m):
        x[basis[i]] = T[i][-1]
    return sum(c2[j] * x[j] for j in range(N))


def tri_pair_exact(P, ip, Q, iq) -> bool:
    P = [[Fr(float(v)) for v in p] for p in P]
    Q = [[Fr(float(v)) for v in q] for q in Q]
    ip = [int(x) for x in ip]
    iq = [int(x) for x in iq]
    shared = [i for i in range(3) if ip[i] in iq]
    s = len(shared)
    if s == 3:
        return True
    # rows: sum lam = 1, sum mu = 1, 3 coordinate equalities
    A = [[1, 1, 1, 0, 0, 0], [0, 0, 0, 1, 1, 1]]
    b = [1, 1]
    for k in range(3):
        A.append([P[0][k], P[1][k], P[2][k], -Q[0][k], -Q[1][k], -Q[2][k]])
        b.append(0)
    c = [0] * 6
    for i in range(3):
        if i not in shared:
            c[i] = 1
    best = _simplex_max(A, b, c)
    if best is None:
        return False
    if s == 0:
        return True
    return best > 0
