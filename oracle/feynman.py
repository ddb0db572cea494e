"""Oracle: Feynman parametrisation (Section II, Eq. 2).  TEST INFRASTRUCTURE.

Only tests, the smoke check and the CPU baseline of the benchmark may use
anything under ``oracle/``; the GPU path never does.

For propagators 1/(-q_j^2 + m_j^2 - i0)^nu_j write

    sum_j x_j (-q_j^2 + m_j^2) = -k^T M k + 2 k.Q + J .

Completing the square, Wick-rotating and integrating the loop momenta with
measure d^D k/(i pi^{D/2}) gives Eq. 2 (without the (-1)^{N_nu} of the
q^2 - m^2 convention) with

    U = det M,        F = det M (Q^T M^{-1} Q + J)      (F carries the -i0),

the exponents  U^{N_nu - (L+1) D/2}  and  F^{-(N_nu - L D/2)}  and the
prefactor Gamma(N_nu - L D/2) / prod_j Gamma(nu_j), D = 4 - 2 eps.

This module does the linear algebra with sympy (exact rationals) and
returns U and F as dicts  {exponent tuple: {invariant: Fraction}} , i.e.
polynomials in x whose coefficients are linear forms in the invariants
(key "1" for the constant part).
"""

from __future__ import annotations

from fractions import Fraction

import sympy as sp


def _form_to_dict(expr, inv_syms):
    """Linear form in the invariants -> {name: Fraction} (no zero entries)."""
    expr = sp.expand(expr)
    out = {}
    const = expr
    for name, sym in inv_syms.items():
        c = expr.coeff(sym)
        if c != 0:
            out[name] = Fraction(str(sp.nsimplify(c)))
        const = const - c * sym
    const = sp.nsimplify(sp.expand(const))
    if const != 0:
        out["1"] = Fraction(str(const))
    if inv_syms:
        # a coefficient must be linear in the invariants
        assert expr.as_poly(*inv_syms.values()).total_degree() <= 1
    return out


def symanzik(problem):
    """Return (U, F, xs) for a problem from ``seeded_inputs.problems``.

    U and F are dicts {exps (tuple of N ints): {invariant: Fraction}}.
    """
    N = len(problem.props)
    L = problem.loops
    xs = sp.symbols(f"x1:{N + 1}")
    inv = {name: sp.Symbol(name) for name in problem.invariants}
    ext = list(problem.externals)

    def sp_ext(a, b):
        key = (a, b) if (a, b) in problem.sp else (b, a)
        form = problem.sp[key]
        return sum((sp.Rational(v) * (1 if k == "1" else inv[k])
                    for k, v in form.items()), sp.Integer(0))

    def dot(u, v):
        """Minkowski product of two external combinations {e: coef}."""
        return sum((cu * cv * sp_ext(eu, ev)
                    for eu, cu in u.items() for ev, cv in v.items()),
                   sp.Integer(0))

    M = sp.zeros(L, L)
    Qpoly = [dict() for _ in range(L)]
    J = sp.Integer(0)
    for x, prop in zip(xs, problem.props):
        al = prop.loop
        P = {e: c for e, c in prop.ext.items() if c != 0}
        for a in range(L):
            for b in range(L):
                M[a, b] += x * al[a] * al[b]
        # -q^2 contains -2 alpha_a k_a.P  =  2 k_a . (-alpha_a x P)
        for a in range(L):
            if al[a] != 0:
                for e, c in P.items():
                    Qpoly[a][e] = Qpoly[a].get(e, 0) - x * al[a] * c
        m2 = inv[prop.mass] if prop.mass else 0
        J += x * (-dot(P, P) + m2)
        assert prop.power >= 1
    U = sp.expand(M.det())
    adj = M.adjugate()                   # M^{-1} = adj / det
    quad = sp.Integer(0)
    for a in range(L):
        for b in range(L):
            quad += adj[a, b] * sum((ca * cb * sp_ext(ea, eb)
                                     for ea, ca in Qpoly[a].items()
                                     for eb, cb in Qpoly[b].items()),
                                    sp.Integer(0))
    F = sp.expand(quad + U * J)
    return _poly_dict(U, xs, inv), _poly_dict(F, xs, inv), xs


def _poly_dict(expr, xs, inv):
    poly = sp.Poly(expr, *xs)
    out = {}
    for monom, coeff in poly.terms():
        form = _form_to_dict(coeff, inv)
        if form:
            out[tuple(int(e) for e in monom)] = form
    return out


def exponents(problem):
    """(u0, u1, f0, f1, prefactor Gamma argument (g0, g1), N_nu).

    U^{u0 + u1 eps}, F^{f0 + f1 eps}, prefactor Gamma(g0 + g1 eps)/prod Gamma(nu).
    """
    L = problem.loops
    Nnu = sum(p.power for p in problem.props)
    # N_nu - (L+1) D/2 with D = 4 - 2 eps
    u0, u1 = Nnu - 2 * (L + 1), (L + 1)
    # -(N_nu - L D/2)
    f0, f1 = -(Nnu - 2 * L), -L
    return (Fraction(u0), Fraction(u1), Fraction(f0), Fraction(f1),
            (Fraction(Nnu - 2 * L), Fraction(L)), Nnu)
