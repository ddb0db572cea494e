"""Pins of the oracle's integration by parts (Section II, Eq. 13) for sector
exponents a_j < -1, as dotted propagators produce them.

- Closed forms: the massless one-loop bubble with powers (nu1, nu2) and the
  massless two-loop sunset with powers (nu1, nu2, nu3), products of Gamma
  functions exact in eps, through the oracle's whole pipeline
  (decomposition, Eq. 13, Eq. 11, lattice sums, Eqs. 19-20).
- The Taylor subtraction of Eq. 11 with p > 0 on a one-variable problem
  with kinematics-dependent numerators, evaluated by adaptive quadrature at
  complex eps (an independent route to the same Laurent coefficients).
- A non-integer power a = -3/2 against its hypergeometric closed form.
- The expansion of the dotted bubble worked by hand.
CPU only.
"""

from fractions import Fraction

import mpmath as mp
import pytest

from oracle import ibp, qmc
from oracle.decompose import decompose
from oracle.geometric import decompose as geometric
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import PROBLEMS
from seeded_inputs.rng import shift_table

mp.mp.dps = 30


def _G(a, b, D):
    """One-loop massless propagator integral with powers a, b (momentum q):
    (-q^2)^(D/2 - a - b) times this."""
    return (mp.gamma(a + b - D / 2) * mp.gamma(D / 2 - a) * mp.gamma(D / 2 - b)
            / (mp.gamma(a) * mp.gamma(b) * mp.gamma(D - a - b)))


def _laurent(f, lo, hi, npts=48, radius=0.1):
    """Laurent coefficients lo..hi at eps = 0 from the Cauchy integrals of
    f(eps) eps^-(p+1) on the circle |eps| = radius, by the trapezoidal rule
    (geometrically convergent for a function analytic on an annulus around
    the circle; every f here has its next singularity at |eps| >= 1/2).
    f is never evaluated at the pole."""
    vals = []
    for j in range(npts):
        z = radius * mp.expjpi(mp.mpf(2 * j) / npts)
        vals.append((z, f(z)))
    out = {}
    for p in range(lo, hi + 1):
        out[p] = complex(sum(v * z ** (-p) for z, v in vals) / npts)
    return out


def _bubble(nu1, nu2, s):
    L = mp.log(-s)
    return lambda e: mp.exp((2 - e - nu1 - nu2) * L) * _G(nu1, nu2, 4 - 2 * e)


def _sunset(n1, n2, n3, s):
    # loop by loop: the (1, 3) pair first, then the remaining bubble
    L = mp.log(-s)
    return lambda e: (mp.exp((4 - 2 * e - n1 - n2 - n3) * L) * _G(n1, n3, 4 - 2 * e)
                      * _G(n2, n1 + n3 - (2 - e), 4 - 2 * e))


def _check(res, exact, sigmas=6.0, floor=1e-12):
    for p, want in exact.items():
        i = res["orders"].index(p)
        got = res["mean"][i]
        tol = sigmas * res["err_re"][i] + floor * max(1.0, abs(want))
        assert abs(got.real - want.real) <= tol, (p, got, want, res["err_re"][i])
        assert abs(got.imag - want.imag) <= sigmas * res["err_im"][i] + floor, (p, got, want)


def _run(name, kin, n=100003, m=8, eps_hi=1):
    return qmc.integrate(PROBLEMS[name], kin, n, lattice(n), shift_table(0, m, 8), eps_hi=eps_hi)


@pytest.mark.parametrize("name,nus", [("bubble_dot", (1, 3)), ("bubble_dot23", (2, 3)),
                                      ("bubble_dot14", (1, 4))])
@pytest.mark.parametrize("s", [-3.0, -0.4])
def test_dotted_bubble_closed_form(name, nus, s):
    secs, _ = decompose(PROBLEMS[name])
    assert min(a for sec in secs for a in sec["a"]) <= -2
    res = _run(name, {"s": s})
    _check(res, _laurent(_bubble(*nus, s), -1, 1))


@pytest.mark.parametrize("name,nus", [("sunset_dot", (1, 1, 3)), ("sunset_dot114", (1, 1, 4)),
                                      ("sunset_dot123", (1, 2, 3))])
def test_dotted_sunset_closed_form(name, nus):
    res = _run(name, {"s": -2.0}, n=10007)
    _check(res, _laurent(_sunset(*nus, -2.0), -2, 1))


def test_sunset_114_differentiates_numerator_factors():
    """a = -3 in two-variable sectors: the second application of Eq. 13
    meets a numerator factor that depends on the variable."""
    secs, info = decompose(PROBLEMS["sunset_dot114"])
    out = ibp.expand(secs, info)
    assert max(len(s["P"]) for s in out) == 3
    # some factor is a second derivative of U or F (degree drops by two)
    assert any(any(sum(e) == 0 for e in p) and len(p) >= 1 for s in out for p in s["P"])


def _taylor_subtracted_1d(a, b, g, order_lo, order_hi):
    """int_0^1 t^(a + b eps) g(t, eps) dt by Eq. 11 with p = 0 .. |a| - 1:
    sum_p g^(p)(0)/(p! (a + p + 1 + b eps)) + int t^(a+b eps) (g - Taylor) dt,
    by adaptive quadrature at complex eps; Laurent coefficients by Cauchy
    integrals.  The remainder is integrated by quadrature on [delta, 1];
    on [0, delta] it is the next two Taylor terms, integrated exactly (the
    neglected part is O(delta^3)), which keeps the subtraction's
    cancellation away from t -> 0."""
    P = int(-a)
    delta = mp.mpf("1e-8")

    def f(e):
        c = mp.taylor(lambda t: g(t, e), 0, P + 1)
        x = a + b * e
        tot = sum(c[p] / (x + p + 1) for p in range(P))
        tot += sum(c[p] * delta ** (x + p + 1) / (x + p + 1) for p in (P, P + 1))

        def rem(t):
            return t ** x * (g(t, e) - sum(c[p] * t ** p for p in range(P)))
        return tot + mp.quad(rem, [delta, mp.mpf("1e-4"), mp.mpf("0.01"), 1])
    return _laurent(f, order_lo, order_hi)


def test_massive_dotted_bubble_against_taylor_subtraction():
    """One massive propagator, one massless cubed: the a = -2 sector has
    F = (msq - s) + msq t, so Eq. 13 brings in the numerator msq.  Both
    primary sectors are one-variable integrals; the sum of their Taylor-
    subtracted forms (Eq. 11 with p > 0) at complex eps is the reference."""
    s, msq = -2.0, 1.5
    secs, info = decompose(PROBLEMS["bubble_massive_dot"])
    u0, u1, f0, f1 = (float(info[k]) for k in ("u0", "u1", "f0", "f1"))
    g0, g1 = (float(x) for x in info["gamma"])

    def val(form):
        return sum(float(v) * (1.0 if k == "1" else {"s": s, "msq": msq}[k])
                   for k, v in form.items())

    def poly(P, t):
        return sum(val(f) * t ** e[0] for e, f in P.items())

    total = {p: 0j for p in range(-1, 2)}
    for sec in secs:
        a, b = float(sec["a"][0]), float(sec["b"][0])
        U, F = sec["U"], sec["F"]

        def g(t, e, U=U, F=F):
            return poly(U, t) ** (u0 + u1 * e) * poly(F, t) ** (f0 + f1 * e)
        if a <= -1:
            part = _taylor_subtracted_1d(a, b, g, -1, 1)
        else:
            part = _laurent(lambda e: mp.quad(lambda t: t ** (a + b * e) * g(t, e), [0, 1]),
                            -1, 1)
        for p in total:
            total[p] += part[p]
    # times Gamma(g0 + g1 eps) / prod Gamma(nu) (here 1/Gamma(3) = 1/2)
    pref = _laurent(lambda e: mp.gamma(g0 + g1 * e) / 2, 0, 2)
    want = {p: sum(pref.get(p - q, 0) * total[q] for q in total if p - q >= 0)
            for p in range(-1, 2)}
    res = _run("bubble_massive_dot", {"s": s, "msq": msq})
    _check(res, want, floor=1e-10)


def test_non_integer_power_below_minus_one():
    """int_0^1 t^(-3/2 + eps) (1 + t)^(1/3 + eps) dt: one application of
    Eq. 13 ends at -1/2.  Closed form (1/c) 2F1(-u, c; c + 1; -1),
    c = -1/2 + eps, u = 1/3 + eps (continued analytically in c)."""
    one = {"1": Fraction(1)}
    sec = {"a": [Fraction(-3, 2)], "b": [Fraction(1)],
           "U": {(0,): one, (1,): one}, "F": {(0,): one}}
    info = {"u0": Fraction(1, 3), "u1": Fraction(1), "f0": Fraction(0), "f1": Fraction(0),
            "gamma": (Fraction(1), Fraction(0)), "nus": [1], "Nnu": 1}
    out = ibp.expand([sec], info)
    assert [s["a"] for s in out] == [[Fraction(0)], [Fraction(-1, 2)]]
    n = 100003
    res = qmc.integrate(None, {}, n, lattice(n), shift_table(0, 8, 8), eps_hi=2,
                        sectors=([sec], info))

    def f(e):
        c = mp.mpf(-0.5) + e
        return mp.hyp2f1(-(mp.mpf(1) / 3 + e), c, c + 1, -1) / c
    _check(res, _laurent(f, 0, 2))


def test_dotted_bubble_expansion_by_hand():
    """Sector x2 = 1 of the bubble with powers (1, 3):
    t^(-2 - eps) (1 + t)^(2 eps) (-s)^(-2 - eps).  Eq. 13 gives
      f(1)/(-1 - eps)                        (no variable left: dummy)
      + 2 eps/(1 + eps) t^(-1 - eps) (1 + t)^(2 eps - 1) (-s)^(-2 - eps)."""
    secs, info = decompose(PROBLEMS["bubble_dot"])
    out = ibp.expand(secs, info)
    assert len(out) == 3
    first, bnd, der = out
    assert first["origin"] == 0 and first["P"] == [] and first["C"] == {0: 1}
    assert bnd["origin"] == 1 and bnd["a"] == [0] and bnd["b"] == [0] and bnd["P"] == []
    # 1/(-1 - eps) = -1 + eps - eps^2 + ...
    assert all(bnd["C"][k] == (-1) ** (k + 1) for k in range(ibp.NSER))
    # U and F at t = 1 moved to the dummy variable's constant term
    assert bnd["U"] == {(0,): {"1": Fraction(2)}} and bnd["F"] == {(0,): {"s": Fraction(-1)}}
    assert der["a"] == [-1] and der["b"] == [-1]
    assert der["u"] == (Fraction(-1), Fraction(2)) and der["f"] == (Fraction(-2), Fraction(-1))
    assert der["P"] == [{(0,): {"1": Fraction(1)}}]
    # 2 eps/(1 + eps) = 2 eps - 2 eps^2 + ...
    assert der["C"].get(0, 0) == 0
    assert all(der["C"][k] == 2 * (-1) ** (k + 1) for k in range(1, ibp.NSER))


def test_geometric_sectors_with_integration_by_parts():
    """The geometric decomposition also leaves powers below -1 (here -2 in
    the sunset with powers (1, 2, 3)); Eq. 13 on its sectors reproduces the
    closed form as well."""
    secs, info = geometric(PROBLEMS["sunset_dot123"])
    assert min(a for s in secs for a in s["a"]) == -2
    n = 10007
    res = qmc.integrate(None, {"s": -2.0}, n, lattice(n), shift_table(0, 8, 8), eps_hi=1,
                        sectors=(secs, info))
    _check(res, _laurent(_sunset(1, 2, 3, -2.0), -2, 1))
