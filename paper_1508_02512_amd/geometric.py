"""Geometric sector decomposition of one primary sector (Section II, the
strategy the paper adopts, after Kaneko and Ueda).

A primary sector is the unit cube in d variables t with polynomials U(t)
and F(t).  Let P = Newt(U) + Newt(F) + R^d_{>=0}: the Newton polytope of
U F plus the positive orthant.  Under t -> -ln t the cube becomes the
positive orthant, and the normal fan of P covers it.  Each vertex v of P
has a normal cone C_v spanned by the inward normals of the facets through
v; for every direction in C_v the terms u* of U and f* of F with
u* + f* = v have the smallest weight, so on that part of the cube they
dominate.

A simplicial cone with primitive integer rays r_1..r_d maps s in (0, 1]^d
onto its part of the cube by t_j = prod_k s_k^{r_k[j]}.  The map is linear
in the logarithms, so it is one-to-one even when |det V| > 1 (V holds the
rays as columns); its Jacobian is |det V| prod_k s_k^{|r_k|_1 - 1}, and a
monomial t^e becomes prod_k s_k^{<r_k, e>}.  Every ray lies in C_v, so
<r_k, e> is smallest at e = u* for all k at once: U = prod_k s_k^{<r_k, u*>}
(c_{u*} + terms that vanish at s = 0), and likewise F.  The exponent map
e -> V^T e is injective, so no two terms merge.

Choices the paper leaves open, fixed here:
  * a normal cone with more than d rays is triangulated by pulling: its
    lexicographically smallest ray r0 is joined to the simplicial cones of
    every facet of the cone that does not contain r0, the facets being
    triangulated by the same rule;
  * the rays of a simplicial cone become s_1..s_d in lexicographic order.

Facets of P come from Qhull on Newt(U F) + conv{0, e_1, .., e_d} (whose
facets with non-negative normals are exactly those of P) and are then
recomputed and checked in exact integer arithmetic.
"""

from __future__ import annotations

import itertools
from fractions import Fraction
from math import gcd

import numpy as np


# --------------------------------------------------------- exact linear algebra

def _rank(rows):
    """Rank of a list of integer vectors (exact)."""
    M = [[Fraction(x) for x in r] for r in rows]
    rank, ncol = 0, len(M[0]) if M else 0
    for c in range(ncol):
        p = next((i for i in range(rank, len(M)) if M[i][c] != 0), None)
        if p is None:
            continue
        M[rank], M[p] = M[p], M[rank]
        for i in range(rank + 1, len(M)):
            if M[i][c] != 0:
                f = M[i][c] / M[rank][c]
                M[i] = [x - f * y for x, y in zip(M[i], M[rank])]
        rank += 1
        if rank == len(M):
            break
    return rank


def _det(M):
    """Determinant of a square integer matrix (Bareiss, exact)."""
    A = [list(map(int, r)) for r in M]
    n = len(A)
    if n == 0:
        return 1
    sign, prev = 1, 1
    for k in range(n - 1):
        if A[k][k] == 0:
            p = next((i for i in range(k + 1, n) if A[i][k] != 0), None)
            if p is None:
                return 0
            A[k], A[p] = A[p], A[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                A[i][j] = (A[i][j] * A[k][k] - A[i][k] * A[k][j]) // prev
        prev = A[k][k]
    return sign * A[n - 1][n - 1]


def _primitive(v):
    g = 0
    for x in v:
        g = gcd(g, int(x))
    return tuple(int(x) // g for x in v) if g else tuple(int(x) for x in v)


def _normal(rows):
    """Integer normal of r - 1 vectors in Z^r (generalised cross product)."""
    r = len(rows) + 1
    return [(-1) ** i * _det([[row[c] for c in range(r) if c != i] for row in rows])
            for i in range(r)]


# ------------------------------------------------------------ polytope facets

def facets(E):
    """Facets of Newt(E) + R^d_{>=0} as {primitive inward normal: offset}.

    E is an integer array [n_points][d]; the offset is min_e <normal, e>."""
    from scipy.spatial import ConvexHull

    E = np.unique(np.asarray(E, dtype=np.int64), axis=0)
    d = E.shape[1]
    if d == 1:
        return {(1,): int(E[:, 0].min())}
    pts = np.unique(np.concatenate([E] + [E + np.eye(d, dtype=np.int64)[j]
                                          for j in range(d)]), axis=0)
    try:
        hull = ConvexHull(pts.astype(np.float64))
    except Exception:               # nearly degenerate input: joggled hull
        hull = ConvexHull(pts.astype(np.float64), qhull_options="QJ")
    scale = float(np.abs(pts).max()) + 1.0
    out = {}
    for eq in np.unique(np.round(hull.equations, 9), axis=0):
        inward = -eq[:-1]
        if np.any(inward < -1e-9):
            continue
        on = np.flatnonzero(np.abs(pts @ eq[:-1] + eq[-1]) < 1e-7 * scale)
        diffs = (pts[on[1:]] - pts[on[0]]).tolist()
        # exact normal: the cross product of d - 1 independent differences
        basis = []
        for row in diffs:
            if _rank(basis + [row]) > len(basis):
                basis.append(row)
            if len(basis) == d - 1:
                break
        if len(basis) != d - 1:
            raise RuntimeError("degenerate facet in the Newton polytope")
        n = np.array(_primitive(_normal(basis)), dtype=np.int64)
        if np.dot(n, inward) < 0:
            n = -n
        vals = pts @ n
        h = int(vals.min())
        if np.any(n < 0) or np.any(vals[on] != h):
            raise RuntimeError("inexact facet of the Newton polytope")
        out[tuple(int(x) for x in n)] = h
    return out


def vertex_cones(E, F):
    """[(vertex, sorted rays of its normal cone)] for every vertex of P."""
    E = np.unique(np.asarray(E, dtype=np.int64), axis=0)
    d = E.shape[1]
    normals = sorted(F)
    Nm = np.array(normals, dtype=np.int64).reshape(-1, d)
    H = np.array([F[n] for n in normals], dtype=np.int64)
    out = []
    for e in E:
        tight = np.flatnonzero(Nm @ e == H)
        rays = [normals[i] for i in tight]
        if len(rays) >= d and _rank(rays) == d:
            out.append((tuple(int(x) for x in e), rays))
    return out


# ------------------------------------------------------------- triangulation

def _cone_facets(rays, r):
    """Facets (as sorted ray tuples) of the cone spanned by `rays`, rank r."""
    # project onto r coordinates on which the span maps one-to-one
    d = len(rays[0])
    cols = None
    for c in itertools.combinations(range(d), r):
        if _rank([[x[i] for i in c] for x in rays]) == r:
            cols = c
            break
    P = [[x[i] for i in cols] for x in rays]
    found = {}
    for S in itertools.combinations(range(len(rays)), r - 1):
        rows = [P[i] for i in S]
        f = _normal(rows)
        if not any(f):
            continue
        dots = [sum(a * b for a, b in zip(f, x)) for x in P]
        if all(v >= 0 for v in dots) or all(v <= 0 for v in dots):
            G = tuple(rays[i] for i in range(len(rays)) if dots[i] == 0)
            found[G] = True
    return sorted(found)


def triangulate(rays):
    """Pulling triangulation of a pointed cone into simplicial cones."""
    rays = sorted(set(tuple(x) for x in rays))
    r = _rank(rays)
    if len(rays) == r:
        return [tuple(rays)]
    r0 = rays[0]
    out = []
    for G in _cone_facets(rays, r):
        if r0 in G:
            continue
        for tau in triangulate(G):
            out.append(tuple(sorted((r0,) + tau)))
    return out


# --------------------------------------------------------------- the sectors

def decompose_primary(EU, EF):
    """Simplicial cones of one primary sector: list of (V, |det V|) with V
    an integer array [d][d] whose column k is the ray of s_k."""
    EU = np.asarray(EU, dtype=np.int64)
    EF = np.asarray(EF, dtype=np.int64)
    E = (EU[:, None, :] + EF[None, :, :]).reshape(-1, EU.shape[1])
    F = facets(E)
    out = []
    for _, rays in vertex_cones(E, F):
        for cone in triangulate(rays):
            V = np.array(cone, dtype=np.int64).T
            out.append((V, abs(_det(V.tolist()))))
    return out
