r"""Oracle: integration by parts in the sector variables (Section II, Eq. 13).
TEST INFRASTRUCTURE: only tests, the smoke check and the CPU baseline of the
benchmark use this module.

A sector variable t with exponent alpha + beta eps, alpha < -1, makes the
integral diverge at t = 0 faster than the subtraction of Eq. 11 with one
term (alpha = -1) can handle; this happens for propagators raised to
powers nu > 1 (dotted propagators).  Eq. 13 trades the singular power for
the derivative of the rest of the integrand:

    int_0^1 t^(alpha+beta eps) f(t) dt
        = f(1)/(alpha+1+beta eps) - 1/(alpha+1+beta eps) int_0^1 t^(alpha+1+beta eps) df/dt dt,

and it is applied again while the power stays below -1.  When it reaches
-1 exactly the remaining pole is the one Eq. 11 subtracts; a power between
-2 and -1 ends above -1 and needs nothing more.  Applied also at -1 (the
paper's alternative to the subtraction), 1/(alpha + 1 + beta eps) becomes
1/(beta eps) and the sector comes out without a pole, its coefficient
series starting at eps^-1.

Here f = C(eps) * P_1 ... P_r * U^(u0 + u1 eps) * F^(f0 + f1 eps) times the
monomials of the other variables, with numerator factors P_i (polynomials
in the sector variables, any sign) and a Laurent coefficient C(eps) per
sector.  The product rule gives

    df/dt = sum_i C P_1 .. (dP_i/dt) .. P_r U^u F^f
            + C (u0 + u1 eps) P_1 .. P_r (dU/dt) U^(u-1) F^f
            + C (f0 + f1 eps) P_1 .. P_r (dF/dt) U^u F^(f-1),

so every term is again of the same form: the derivative of a numerator
factor replaces that factor, the derivative of U or F is appended as a new
factor and lowers the power of U or F by one.  Terms whose new factor is
the zero polynomial are dropped.  The boundary term f(1) is the same form
with t set to 1: one variable fewer.  A sector left with no variable keeps
one dummy variable (power 0, absent from every polynomial), so that it is
still an integral over [0,1].

The order of the resulting sectors is fixed: variables in increasing
index; for each application of Eq. 13, the boundary term first, then the
derivative terms (numerator factors in order, then U, then F), each
expanded completely (depth first) before the next.

Polynomials are dicts {exponent tuple: {invariant: Fraction}} as in the
decomposition; C(eps) is an exact power series {order: Fraction}.
"""

from __future__ import annotations

from fractions import Fraction

NSER = 12          # orders of eps kept in a sector's coefficient series


def _form_add(acc, form, scale=Fraction(1)):
    for k, v in form.items():
        acc[k] = acc.get(k, Fraction(0)) + scale * v
        if acc[k] == 0:
            del acc[k]


def _poly_clean(poly):
    return {e: f for e, f in poly.items() if f}


def _deriv(poly, j):
    """d/dt_j of a polynomial."""
    out = {}
    for e, form in poly.items():
        if e[j] == 0:
            continue
        ne = list(e)
        ne[j] -= 1
        acc = out.setdefault(tuple(ne), {})
        _form_add(acc, form, Fraction(e[j]))
    return _poly_clean(out)


def _at_one(poly, j):
    """The polynomial with t_j = 1 (exponent j set to 0, equal terms merged)."""
    out = {}
    for e, form in poly.items():
        ne = list(e)
        ne[j] = 0
        acc = out.setdefault(tuple(ne), {})
        _form_add(acc, form)
    return _poly_clean(out)


def _ser_mul(x, y):
    """Product of two Laurent series, orders below NSER kept."""
    out = {}
    for p, a in x.items():
        for q, b in y.items():
            if p + q < NSER:
                out[p + q] = out.get(p + q, Fraction(0)) + a * b
    return {k: v for k, v in out.items() if v != 0}


def _ser_inv_linear(c0, c1):
    """1/(c0 + c1 eps) as a Laurent series: a power series for c0 != 0,
    1/(c1 eps) for c0 = 0 (an exponent -1 taken by Eq. 13)."""
    if c0 == 0:
        return {-1: 1 / c1}
    r = -c1 / c0
    return {k: (r ** k) / c0 for k in range(NSER) if r ** k != 0 or k == 0}


def _copy(sec):
    out = dict(sec)
    out["a"] = list(sec["a"])
    out["b"] = list(sec["b"])
    out["P"] = list(sec["P"])
    out["fixed"] = set(sec["fixed"])
    return out


def _step(sec, j):
    """One application of Eq. 13 in variable j, in the fixed order."""
    alpha, beta = sec["a"][j], sec["b"][j]
    inv = _ser_inv_linear(alpha + 1, beta)
    out = []
    # boundary term: f(1)/(alpha + 1 + beta eps)
    bnd = _copy(sec)
    bnd["fixed"].add(j)
    bnd["U"] = _at_one(sec["U"], j)
    bnd["F"] = _at_one(sec["F"], j)
    bnd["P"] = [_at_one(p, j) for p in sec["P"]]
    bnd["C"] = _ser_mul(sec["C"], inv)
    if all(bnd["P"]) and bnd["C"]:
        out.append(bnd)
    # derivative terms: -1/(alpha + 1 + beta eps) t^(alpha+1+beta eps) df/dt
    minus_inv = {k: -v for k, v in inv.items()}
    base = _copy(sec)
    base["a"][j] = alpha + 1
    base["C"] = _ser_mul(sec["C"], minus_inv)
    for i, p in enumerate(sec["P"]):
        dp = _deriv(p, j)
        if dp:
            t = _copy(base)
            t["P"][i] = dp
            out.append(t)
    for which, key in (("U", "u"), ("F", "f")):
        dq = _deriv(sec[which], j)
        e0, e1 = sec[key]
        if not dq or (e0 == 0 and e1 == 0):
            continue
        t = _copy(base)
        t["P"].append(dq)
        t[key] = (e0 - 1, e1)
        t["C"] = _ser_mul(base["C"], {k: v for k, v in ((0, e0), (1, e1)) if v != 0})
        if t["C"]:
            out.append(t)
    return out


def _expand_var(sec, j, poles):
    """Eq. 13 in variable j while its power is below -1, or (poles) while
    it is -1 or below."""
    a = sec["a"][j]
    if j in sec["fixed"] or a > -1 or (a == -1 and not poles):
        return [sec]
    if a == -1 and sec["b"][j] == 0:
        raise ValueError("a = -1 with b = 0: the pole is not regulated")
    out = []
    for t in _step(sec, j):
        out.extend(_expand_var(t, j, poles))
    return out


def _compact(sec, origin):
    keep = [j for j in range(len(sec["a"])) if j not in sec["fixed"]]
    dummy = not keep

    def sel(poly):
        if dummy:
            return {(0,): f for e, f in poly.items()}
        return {tuple(e[j] for j in keep): f for e, f in poly.items()}

    for which in ("U", "F"):
        zero = tuple(0 for _ in range(len(sec["a"])))
        if zero not in sec[which]:
            raise ValueError(f"{which} lost its constant term at t = 1 (sector {origin})")
    return {"a": [sec["a"][j] for j in keep] or [Fraction(0)],
            "b": [sec["b"][j] for j in keep] or [Fraction(0)],
            "U": sel(sec["U"]), "F": sel(sec["F"]), "P": [sel(p) for p in sec["P"]],
            "u": sec["u"], "f": sec["f"], "C": sec["C"], "origin": origin}


def needs_ibp(sectors, poles=False):
    return any(a < -1 or (poles and a == -1) for s in sectors for a in s["a"])


def expand(sectors, info, poles=False):
    """Every sector with some a_j < -1 replaced by its Eq. 13 expansion;
    with poles=True also every a_j = -1 (Eq. 13 as the alternative to the
    subtraction of Eq. 11: the sectors come out without poles, and their
    coefficient series C start at eps^-p, p the number of poles taken).

    Each output sector carries its own powers u = (u0, u1), f = (f0, f1),
    numerator factors P, coefficient series C (a Laurent series, times the
    input sector's D) and the index of the input sector it came from."""
    out = []
    for idx, s in enumerate(sectors):
        d = len(s["a"])
        sec = {"a": list(s["a"]), "b": list(s["b"]), "U": s["U"], "F": s["F"], "P": [],
               "u": (Fraction(info["u0"]), Fraction(info["u1"])),
               "f": (Fraction(info["f0"]), Fraction(info["f1"])),
               "C": {0: Fraction(s.get("D", 1))}, "fixed": set()}
        secs = [sec]
        for j in range(d):
            nxt = []
            for t in secs:
                nxt.extend(_expand_var(t, j, poles))
            secs = nxt
        out.extend(_compact(t, idx) for t in secs)
    return out
