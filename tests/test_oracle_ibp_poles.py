"""Pins of the oracle's integration by parts taken at the poles as well
(Section II, Eq. 13 as the alternative to the subtraction of Eq. 11): every
variable with a_j = -1 is integrated by parts once more, 1/(a_j+1+b_j eps)
becomes 1/(b_j eps), and the sectors come out without poles, their
coefficient series starting at eps^-p.

- Closed forms through the whole oracle pipeline: the massless one-loop box
  (two poles per sector), the dotted bubble and the dotted sunset (Eq. 13
  below -1 and at -1 in one sector).
- A one-variable integral with its hypergeometric closed form.
- The expansion of one pole worked by hand.
- The same integrals by both pole methods (Eq. 11 and Eq. 13 share no
  arithmetic after the decomposition): the dotted box and sunset.
- The Eq. 20 error of the pole method's assembly, calibrated over 40 shift
  seeds against the box closed form.
CPU only.
"""

from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import ibp, qmc
from oracle.decompose import decompose
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import PROBLEMS
from seeded_inputs.rng import shift_table
from test_oracle_ibp import _bubble, _check, _laurent, _sunset
from test_oracle_pins import _box_exact

mp.mp.dps = 30


def _run(name, kin, n, eps_hi=0, m=8, poles="ibp", sectors=None):
    return qmc.integrate(PROBLEMS[name] if name else None, kin, n, lattice(n),
                         shift_table(0, m, 8), eps_hi=eps_hi, poles=poles, sectors=sectors)


def test_box_closed_form():
    secs, info = decompose(PROBLEMS["box"])
    out = ibp.expand(secs, info, poles=True)
    assert all(a != -1 for s in out for a in s["a"])
    assert min(min(s["C"]) for s in out) == -2
    _check(_run("box", {"s": -3.0, "t": -2.0}, 10007), _box_exact(-3.0, -2.0))


@pytest.mark.parametrize("name,exact,eps_hi", [
    ("bubble_dot14", lambda: _laurent(_bubble(1, 4, -3.0), -1, 1), 1),
    ("sunset_dot123", lambda: _laurent(_sunset(1, 2, 3, -2.0), -2, 0), 0)])
def test_dotted_closed_forms(name, exact, eps_hi):
    """The leading pole of both vanishes (eps^-1 of the bubble, eps^-2 of
    the sunset); after Eq. 13 at the poles no sector's series reaches it,
    so the result starts one order later."""
    kin = {"s": -3.0} if name.startswith("bubble") else {"s": -2.0}
    res = _run(name, kin, 100003, eps_hi)
    want = exact()
    lo = min(want)
    assert lo not in res["orders"] and abs(want[lo]) < 1e-30
    _check(res, {p: v for p, v in want.items() if p > lo})


def _one_var():
    one = {"1": Fraction(1)}
    sec = {"a": [Fraction(-1)], "b": [Fraction(1)],
           "U": {(0,): one, (1,): one}, "F": {(0,): one}}
    info = {"u0": Fraction(1, 3), "u1": Fraction(1), "f0": Fraction(0), "f1": Fraction(0),
            "gamma": (Fraction(1), Fraction(0)), "nus": [1], "Nnu": 1}
    return sec, info


def test_one_pole_expansion_by_hand():
    """int_0^1 t^(-1 + eps) (1 + t)^(1/3 + eps) dt by Eq. 13 at a = -1:
      f(1)/eps                                        (dummy variable, C = 1/eps)
      - (1/3 + eps)/eps int_0^1 t^eps * 1 * (1 + t)^(-2/3 + eps) dt."""
    sec, info = _one_var()
    bnd, der = ibp.expand([sec], info, poles=True)
    assert bnd["a"] == [0] and bnd["P"] == [] and bnd["C"] == {-1: 1}
    assert bnd["U"] == {(0,): {"1": Fraction(2)}}
    assert der["a"] == [0] and der["b"] == [1]
    assert der["P"] == [{(0,): {"1": Fraction(1)}}]
    assert der["u"] == (Fraction(-2, 3), Fraction(1))
    assert der["C"] == {-1: Fraction(-1, 3), 0: Fraction(-1)}
    # without the pole mode the sector is left to the subtraction
    assert ibp.expand([sec], info)[0]["C"] == {0: 1}


@pytest.mark.parametrize("poles", ["ibp", "subtract"])
def test_one_variable_closed_form(poles):
    """The same integral = (1/c) 2F1(-u, c; c + 1; -1), c = eps, u = 1/3 + eps,
    by either pole method."""
    sec, info = _one_var()
    res = _run(None, {}, 100003, eps_hi=2, poles=poles, sectors=([sec], info))

    def f(e):
        return mp.hyp2f1(-(mp.mpf(1) / 3 + e), e, e + 1, -1) / e
    _check(res, _laurent(f, -1, 2))


@pytest.mark.parametrize("name,kin", [("box_dot", {"s": -3.0, "t": -2.0}),
                                      ("sunset_dot", {"s": -2.0})])
def test_both_pole_methods_agree(name, kin):
    """Integrals with no closed form here, each with poles (two per sector in
    the dotted box): Eq. 11 and Eq. 13 agree within their combined errors."""
    a = _run(name, kin, 10007, poles="subtract")
    b = _run(name, kin, 10007, poles="ibp")
    for i, p in enumerate(b["orders"]):
        j = a["orders"].index(p)
        d = a["mean"][j] - b["mean"][i]
        assert abs(d.real) <= 6 * np.hypot(a["err_re"][j], b["err_re"][i]) + 1e-12, \
            (p, a["mean"][j], b["mean"][i])
    # orders only the subtraction carries vanish there
    for j, p in enumerate(a["orders"]):
        if p not in b["orders"]:
            assert abs(a["mean"][j]) <= 6 * a["err_re"][j] + 1e-12


def test_unregulated_pole_is_refused():
    sec, info = _one_var()
    sec = dict(sec, b=[Fraction(0)])
    with pytest.raises(ValueError, match="not regulated"):
        ibp.expand([sec], info, poles=True)
    with pytest.raises(ValueError, match="pole method"):
        _run(None, {}, 1009, poles="taylor", sectors=([dict(_one_var()[0])], info))


def test_error_estimate_is_calibrated():
    """Eq. 20 on the pole method's Laurent assembly: the box over 40
    independent shift seeds (n = 1009, m = 10), |Qbar - exact| <= 3 err in
    at least 38 of 40 seeds for every order, and the mean squared deviation
    within a factor 2.5 of the mean err^2."""
    exact = _box_exact(-3.0, -2.0)
    secs = decompose(PROBLEMS["box"])
    n, m = 1009, 10
    dev = {p: [] for p in exact}
    var = {p: [] for p in exact}
    for seed in range(100, 140):
        res = qmc.integrate(PROBLEMS["box"], {"s": -3.0, "t": -2.0}, n, lattice(n),
                            shift_table(seed, m, 8), sectors=secs, poles="ibp")
        for p, want in exact.items():
            i = res["orders"].index(p)
            dev[p].append(res["mean"][i].real - want.real)
            var[p].append(res["err_re"][i] ** 2)
    for p in exact:
        d, v = np.array(dev[p]), np.array(var[p])
        assert np.sqrt(v.mean()) > 1e-12
        inside = np.sum(np.abs(d) <= 3 * np.sqrt(v))
        assert inside >= 38, (p, inside)
        ratio = np.mean(d ** 2) / np.mean(v)
        assert 0.4 <= ratio <= 2.5, (p, ratio)
