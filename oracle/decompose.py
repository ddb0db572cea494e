r"""Oracle: sector decomposition (Section II, Eqs. 3-9).  TEST INFRASTRUCTURE.

Primary sectors (Eqs. 3-6): in sector l the largest Feynman parameter is
x_l; x_j = x_l t_j for the others, and the delta constraint is used to set
x_l = 1 (Cheng-Wu, exact by projective invariance), which leaves the
(N-1)-cube with monomial prefactor prod t_j^{nu_j - 1} (the exponent of the
x that t_j stands for).

Iterated decomposition (Eqs. 7-8): a sector is split again until both U
and F are a monomial times a polynomial with a non-vanishing constant term.
The paper does not fix the splitting rule, so this uses a deterministic
one that provably terminates ("closest-pair" rule):

  1. factor the largest common monomial out of U, then out of F, moving
     its exponents (times the powers of U and F) into the prefactor;
  2. if both remainders have a constant term (coefficient a non-zero
     linear form of the invariants, decided exactly) the sector is final;
  3. otherwise take the first remainder without a constant term (U before
     F) and its minimal exponent vectors (those not dominated
     componentwise by another exponent of the same polynomial; there are
     at least two).  Among all pairs v < w (lexicographic) of minimal
     vectors take the one with the smallest |v - w|_1, ties broken by the
     lexicographically smallest (v, w).  Let i be the first index with
     v_i != w_i and j the first index where v - w has the opposite sign;
     S = {i, j};
  4. split into |S| children, k in S in increasing order: t_j -> t_k t_j
     for j in S\{k}; t_k collects the Jacobian t_k^{|S|-1} and the old
     prefactor exponents of those t_j;
  5. depth is capped at 64.

The substitution of step 4 is a non-negative, invertible linear map on
exponent vectors, so domination is preserved and the number of minimal
vectors never grows; in each child either that number drops or the
chosen pair stays minimal with |v - w|_1 strictly smaller (one of its
coordinates becomes v_i - w_i + v_j - w_j).  Hence the recursion ends.

Each final sector is the form of Eq. 9 with D_la = 1 (the constants C, C'
are kept inside the remainders, so no kinematics-dependent normalisation
enters D).  Polynomials are dicts {exponent tuple: {invariant: Fraction}}.
"""

from __future__ import annotations

from fractions import Fraction
from .feynman import exponents, symanzik

MAX_DEPTH = 64


def _add_form(acc, form):
    for k, v in form.items():
        acc[k] = acc.get(k, Fraction(0)) + v
        if acc[k] == 0:
            del acc[k]


def _primary(poly, l):
    """Set x_l = 1 and rename the other x's t_0..t_{N-2} in index order."""
    out = {}
    for e, form in poly.items():
        key = tuple(e[:l]) + tuple(e[l + 1:])
        acc = out.setdefault(key, {})
        _add_form(acc, form)
        if not acc:
            del out[key]
    return out


def _common_monomial(poly, d):
    return [min(e[j] for e in poly) for j in range(d)]


def _divide(poly, m):
    return {tuple(e[j] - m[j] for j in range(len(m))): f for e, f in poly.items()}


def _vanishes(poly, S):
    return all(any(e[j] > 0 for j in S) for e in poly)


def _minimal(poly):
    exps = list(poly)
    return sorted(e for e in exps
                  if not any(f != e and all(fj <= ej for fj, ej in zip(f, e))
                             for f in exps))


def _closest_pair_split(poly):
    mins = _minimal(poly)
    assert len(mins) >= 2
    best = None
    for x in range(len(mins)):
        for y in range(x + 1, len(mins)):
            v, w = mins[x], mins[y]
            dist = sum(abs(p - q) for p, q in zip(v, w))
            if best is None or (dist, v, w) < best:
                best = (dist, v, w)
    _, v, w = best
    delta = [p - q for p, q in zip(v, w)]
    i = next(k for k, x in enumerate(delta) if x != 0)
    j = next(k for k, x in enumerate(delta) if x * delta[i] < 0)
    return tuple(sorted((i, j)))


def _substitute(poly, S, k):
    """t_j -> t_k t_j for j in S\\{k}: exponent of t_k grows by sum e_j."""
    out = {}
    for e, f in poly.items():
        e = list(e)
        e[k] += sum(e[j] for j in S if j != k)
        out[tuple(e)] = f
    assert len(out) == len(poly)       # the map is injective on monomials
    return out


def _iterate(sec, ex, depth, out):
    if depth > MAX_DEPTH:
        raise RuntimeError("iterated decomposition exceeded the depth cap")
    u0, u1, f0, f1 = ex
    d = len(sec["a"])
    a, b = list(sec["a"]), list(sec["b"])
    U, F = sec["U"], sec["F"]
    mu = _common_monomial(U, d)
    U = _divide(U, mu)
    mf = _common_monomial(F, d)
    F = _divide(F, mf)
    for j in range(d):
        a[j] += mu[j] * u0 + mf[j] * f0
        b[j] += mu[j] * u1 + mf[j] * f1
    zero = (0,) * d
    if zero in U and zero in F:
        out.append({"a": a, "b": b, "U": U, "F": F})
        return
    P = U if zero not in U else F
    chosen = _closest_pair_split(P)
    S = chosen
    for k in S:
        na, nb = list(a), list(b)
        na[k] += sum(a[j] for j in S if j != k) + (len(S) - 1)
        nb[k] += sum(b[j] for j in S if j != k)
        child = {"a": na, "b": nb, "U": _substitute(U, S, k),
                 "F": _substitute(F, S, k)}
        _iterate(child, ex, depth + 1, out)


def decompose(problem):
    """All final sectors of a problem, primary sector by primary sector.

    Returns (sectors, info) where each sector is a dict with keys
    a, b (exponents of t_j^{a_j + b_j eps}), U, F (remainder polynomials),
    and info holds u0, u1, f0, f1, the Gamma argument and N_nu.
    """
    U, F, _ = symanzik(problem)
    u0, u1, f0, f1, gam, Nnu = exponents(problem)
    N = len(problem.props)
    nus = [p.power for p in problem.props]
    sectors = []
    for l in range(N):
        others = [j for j in range(N) if j != l]
        sec = {"a": [Fraction(nus[j] - 1) for j in others],
               "b": [Fraction(0) for _ in others],
               "U": _primary(U, l), "F": _primary(F, l)}
        _iterate(sec, (u0, u1, f0, f1), 0, sectors)
    info = {"u0": u0, "u1": u1, "f0": f0, "f1": f1, "gamma": gam, "Nnu": Nnu,
            "nus": nus, "invariants": list(problem.invariants),
            "dim": N - 1}
    return sectors, info
