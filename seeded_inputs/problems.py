"""Feynman integrals used as workloads, written as plain data.

Each problem is the momentum representation of Section II, Eq. 1, with the
propagator convention 1/(-q_j^2 + m_j^2 - i0)^nu_j and measure
d^D k / (i pi^{D/2}) per loop (the examples of Section IV with the causal
sign of the i0).  A propagator is

    (loop coefficients, {external: coefficient}, mass-squared symbol or None, nu)

so that q_j = sum_a loop[a] k_a + sum_e ext[e] p_e.  ``sp`` gives every
scalar product p_e . p_f of the independent external momenta as a linear
form over the problem's kinematic invariants (a dict invariant -> rational
written as a string).  The constant invariant "1" is implicit.

No arithmetic of the method lives here: turning these into U, F and
sectors is done separately by the oracle and by the GPU path's front end.
"""

from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Propagator:
    loop: tuple
    ext: dict
    mass: str | None = None
    power: int = 1


@dataclass(frozen=True)
class Problem:
    name: str
    loops: int
    externals: tuple
    invariants: tuple
    sp: dict
    props: tuple
    note: str = ""
    extra: dict = field(default_factory=dict)


def _P(loop, ext=None, mass=None, power=1):
    return Propagator(tuple(loop), dict(ext or {}), mass, power)


# --- one loop ---------------------------------------------------------------

BUBBLE = Problem(
    "bubble", 1, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1]), _P([1], {"p": 1})),
    note="massless two-point function, p^2 = s")

BUBBLE_MASSIVE = Problem(
    "bubble_massive", 1, ("p",), ("s", "msq"),
    {("p", "p"): {"s": "1"}},
    (_P([1], mass="msq"), _P([1], {"p": 1}, mass="msq")),
    note="equal-mass two-point function, threshold at s = 4 msq")

# dotted propagators (powers nu > 1): their sectors carry t^(a + b eps) with
# a < -1, which the integration by parts of Eq. 13 reduces
BUBBLE_DOT = Problem(
    "bubble_dot", 1, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1]), _P([1], {"p": 1}, power=3)),
    note="massless two-point function with powers (1, 3)")

BUBBLE_DOT23 = Problem(
    "bubble_dot23", 1, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1], power=2), _P([1], {"p": 1}, power=3)),
    note="massless two-point function with powers (2, 3)")

BUBBLE_DOT14 = Problem(
    "bubble_dot14", 1, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1]), _P([1], {"p": 1}, power=4)),
    note="massless two-point function with powers (1, 4)")

BUBBLE_MASSIVE_DOT = Problem(
    "bubble_massive_dot", 1, ("p",), ("s", "msq"),
    {("p", "p"): {"s": "1"}},
    (_P([1], mass="msq"), _P([1], {"p": 1}, power=3)),
    note="two-point function, one massive propagator and one massless cubed")

SUNSET_DOT = Problem(
    "sunset_dot", 2, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1, 0]), _P([0, 1]), _P([1, 1], {"p": -1}, power=3)),
    note="massless two-loop sunset with powers (1, 1, 3)")

SUNSET_DOT114 = Problem(
    "sunset_dot114", 2, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1, 0]), _P([0, 1]), _P([1, 1], {"p": -1}, power=4)),
    note="massless two-loop sunset with powers (1, 1, 4)")

SUNSET_DOT123 = Problem(
    "sunset_dot123", 2, ("p",), ("s",),
    {("p", "p"): {"s": "1"}},
    (_P([1, 0]), _P([0, 1], power=2), _P([1, 1], {"p": -1}, power=3)),
    note="massless two-loop sunset with powers (1, 2, 3)")

# all momenta incoming, p4 = -p1-p2-p3, s = (p1+p2)^2, t = (p2+p3)^2
_SP_MASSLESS_4PT = {
    ("p1", "p1"): {}, ("p2", "p2"): {}, ("p3", "p3"): {},
    ("p1", "p2"): {"s": "1/2"},
    ("p2", "p3"): {"t": "1/2"},
    ("p1", "p3"): {"s": "-1/2", "t": "-1/2"},     # u = -s - t
}

BOX = Problem(
    "box", 1, ("p1", "p2", "p3"), ("s", "t"), _SP_MASSLESS_4PT,
    (_P([1]), _P([1], {"p1": 1}), _P([1], {"p1": 1, "p2": 1}),
     _P([1], {"p1": 1, "p2": 1, "p3": 1})),
    note="massless on-shell scalar box")

# massless triangle with three off-shell legs (finite in D = 4):
# momenta incoming, p3 = -p1-p2, p1.p2 = (p3sq - p1sq - p2sq)/2
TRIANGLE_OFFSHELL = Problem(
    "triangle_offshell", 1, ("p1", "p2"), ("p1sq", "p2sq", "p3sq"),
    {("p1", "p1"): {"p1sq": "1"}, ("p2", "p2"): {"p2sq": "1"},
     ("p1", "p2"): {"p3sq": "1/2", "p1sq": "-1/2", "p2sq": "-1/2"}},
    (_P([1]), _P([1], {"p1": 1}), _P([1], {"p1": 1, "p2": 1})),
    note="one-loop massless triangle, three off-shell legs")

BOX_DOT = Problem(
    "box_dot", 1, ("p1", "p2", "p3"), ("s", "t"), _SP_MASSLESS_4PT,
    (_P([1], power=2), _P([1], {"p1": 1}), _P([1], {"p1": 1, "p2": 1}),
     _P([1], {"p1": 1, "p2": 1, "p3": 1})),
    note="massless on-shell box with the first propagator squared")

TRIANGLE_OFFSHELL_DOT = Problem(
    "triangle_offshell_dot", 1, ("p1", "p2"), ("p1sq", "p2sq", "p3sq"),
    {("p1", "p1"): {"p1sq": "1"}, ("p2", "p2"): {"p2sq": "1"},
     ("p1", "p2"): {"p3sq": "1/2", "p1sq": "-1/2", "p2sq": "-1/2"}},
    (_P([1], power=3), _P([1], {"p1": 1}), _P([1], {"p1": 1, "p2": 1})),
    note="off-shell massless triangle, first propagator cubed")

# --- two loops ----------------------------------------------------------------

# Planar double box with the momentum routing of Section IV.B (I_B):
# k1^2, (k1-p1)^2, (k1+p2)^2, (k1-k2-p1)^2, k2^2, (k1+p2-k2+p3)^2, (k1-k2+p2)^2
_DB_PROPS = (
    _P([1, 0]), _P([1, 0], {"p1": -1}), _P([1, 0], {"p2": 1}),
    _P([1, -1], {"p1": -1}), _P([0, 1]),
    _P([1, -1], {"p2": 1, "p3": 1}), _P([1, -1], {"p2": 1}))

_SP_OFFSHELL_4PT = {
    ("p1", "p1"): {"p1sq": "1"}, ("p2", "p2"): {"p2sq": "1"},
    ("p3", "p3"): {"p3sq": "1"},
    ("p1", "p2"): {"s": "1/2", "p1sq": "-1/2", "p2sq": "-1/2"},
    ("p2", "p3"): {"t": "1/2", "p2sq": "-1/2", "p3sq": "-1/2"},
    # u = p1sq+p2sq+p3sq+p4sq-s-t,  p1.p3 = (u - p1sq - p3sq)/2
    ("p1", "p3"): {"p2sq": "1/2", "p4sq": "1/2", "s": "-1/2", "t": "-1/2"},
}

DOUBLEBOX = Problem(
    "doublebox", 2, ("p1", "p2", "p3"), ("s", "t"), _SP_MASSLESS_4PT, _DB_PROPS,
    note="massless on-shell planar double box (7 propagators, 6 dims)")

DOUBLEBOX_OFFSHELL = Problem(
    "doublebox_offshell", 2, ("p1", "p2", "p3"),
    ("s", "t", "p1sq", "p2sq", "p3sq", "p4sq"), _SP_OFFSHELL_4PT, _DB_PROPS,
    note="planar double box with off-shell legs (Section IV.B, Table 1)")

# Non-planar two-loop vertex: graph K_{2,3} between internal vertices X, Y
# and external vertices A (p1 in), B (p2 in), C (p1+p2 out).  The four
# lines X-A, A-Y, X-B, B-Y form a closed massive loop; the two lines at C
# are massless.  p1^2 = p2^2 = 0, (p1+p2)^2 = s.
_SP_VERTEX = {("p1", "p1"): {}, ("p2", "p2"): {}, ("p1", "p2"): {"s": "1/2"}}

NP_VERTEX = Problem(
    "np_vertex", 2, ("p1", "p2"), ("s", "msq"), _SP_VERTEX,
    (_P([1, 0], mass="msq"), _P([1, 0], {"p1": 1}, mass="msq"),
     _P([0, 1], mass="msq"), _P([0, 1], {"p2": 1}, mass="msq"),
     _P([1, 1], {"p1": 1, "p2": 1}), _P([1, 1])),
    note="non-planar two-loop vertex with a massive internal loop")

# Planar two-loop vertex (ladder triangle), all six lines of mass^2 = msq:
# A-B: k1, X-A: k1-p1, B-Y: k1+p2, X-Y: k2, C-X: k1+k2-p1, Y-C: k1+k2+p2.
TRIANGLE2L = Problem(
    "triangle2l", 2, ("p1", "p2"), ("s", "msq"), _SP_VERTEX,
    (_P([1, 0], mass="msq"), _P([1, 0], {"p1": -1}, mass="msq"),
     _P([1, 0], {"p2": 1}, mass="msq"), _P([0, 1], mass="msq"),
     _P([1, 1], {"p1": -1}, mass="msq"), _P([1, 1], {"p2": 1}, mass="msq")),
    note="planar two-loop vertex, all lines massive; threshold at s = 4 msq")



def _offshell_sp(legs):
    """Scalar products for the four-point kinematics with only ``legs``
    (subset of 1..4) off-shell; the others have p_i^2 = 0 identically."""
    def keep(form):
        return {k: v for k, v in form.items()
                if not (k.startswith("p") and int(k[1]) not in legs)}
    return {key: keep(form) for key, form in _SP_OFFSHELL_4PT.items()}


def _doublebox_legs(legs):
    tag = "".join(str(i) for i in legs)
    return Problem(
        f"doublebox_off{tag}", 2, ("p1", "p2", "p3"),
        ("s", "t") + tuple(f"p{i}sq" for i in legs), _offshell_sp(legs),
        _DB_PROPS,
        note=f"planar double box, legs {legs} off-shell (Section IV.B, Table 1)")


# The three columns of Table 1: (p1^2, p2^2, p3^2, p4^2) = (-1,0,0,-1),
# (0,-1,0,-1), (0,0,-1,-1) with s = t = u = -2/3.
DOUBLEBOX_OFF14 = _doublebox_legs((1, 4))
DOUBLEBOX_OFF24 = _doublebox_legs((2, 4))
DOUBLEBOX_OFF34 = _doublebox_legs((3, 4))

# Higgs-pair kinematics of Section IV.C-D: incoming gluons p1, p2
# (p1^2 = p2^2 = 0), outgoing Higgs bosons p3, p4 (p^2 = mhsq),
# p4 = p1 + p2 - p3, s = (p1+p2)^2, t = (p2-p3)^2, so
# p2.p3 = (mhsq - t)/2 and p1.p3 = (s + t - mhsq)/2.
_SP_HH = {
    ("p1", "p1"): {}, ("p2", "p2"): {}, ("p3", "p3"): {"mhsq": "1"},
    ("p1", "p2"): {"s": "1/2"},
    ("p2", "p3"): {"mhsq": "1/2", "t": "-1/2"},
    ("p1", "p3"): {"s": "1/2", "t": "1/2", "mhsq": "-1/2"},
}

# I_A (Section IV.A): one-loop box for gg -> HH with four top-quark lines,
# k^2-mt^2, (k+p1)^2-mt^2, (k-p2)^2-mt^2, (k+p1-p4)^2-mt^2 = (k-p2+p3)^2-mt^2.
# The paper's measure there is d^D k / (2 pi)^D, i pi^(D/2) / (2 pi)^D times
# the measure used here.
HH_BOX = Problem(
    "hh_box", 1, ("p1", "p2", "p3"), ("s", "t", "mtsq", "mhsq"), _SP_HH,
    (_P([1], mass="mtsq"), _P([1], {"p1": 1}, mass="mtsq"),
     _P([1], {"p2": -1}, mass="mtsq"), _P([1], {"p2": -1, "p3": 1}, mass="mtsq")),
    note="one-loop box for gg -> HH (Section IV.A, threshold at s = 4 mt^2)")

# I_C (Section IV.C): planar double box with four top-quark lines,
# k1^2, (k1-p1)^2, (k1+p2)^2, (k1-k2-p1)^2-mt^2, k2^2-mt^2,
# (k1+p2-k2-p3)^2-mt^2, (k1-k2+p2)^2-mt^2.
HH_PLANAR = Problem(
    "hh_planar", 2, ("p1", "p2", "p3"), ("s", "t", "mtsq", "mhsq"), _SP_HH,
    (_P([1, 0]), _P([1, 0], {"p1": -1}), _P([1, 0], {"p2": 1}),
     _P([1, -1], {"p1": -1}, mass="mtsq"), _P([0, 1], mass="mtsq"),
     _P([1, -1], {"p2": 1, "p3": -1}, mass="mtsq"),
     _P([1, -1], {"p2": 1}, mass="mtsq")),
    note="planar two-loop double box for gg -> HH (Section IV.C, Table 2)")

# I_D (Section IV.D): non-planar double box with four top-quark lines,
# k1^2, (k1+p1)^2, (k1-p2)^2, (k1+p1-k2)^2-mt^2, k2^2-mt^2,
# (k2-p4)^2-mt^2, (k1+p1-k2-p3)^2-mt^2.
HH_NONPLANAR = Problem(
    "hh_nonplanar", 2, ("p1", "p2", "p3"), ("s", "t", "mtsq", "mhsq"), _SP_HH,
    (_P([1, 0]), _P([1, 0], {"p1": 1}), _P([1, 0], {"p2": -1}),
     _P([1, -1], {"p1": 1}, mass="mtsq"), _P([0, 1], mass="mtsq"),
     _P([0, 1], {"p1": -1, "p2": -1, "p3": 1}, mass="mtsq"),
     _P([1, -1], {"p1": 1, "p3": -1}, mass="mtsq")),
    note="non-planar two-loop double box for gg -> HH (Section IV.D, Table 3)")

# The kinematic point of Tables 2 and 3 (GeV^2): s = 160000, t = -6000,
# M_t = 172, M_H = 125 (Section IV).
HH_POINT = {"s": 160000.0, "t": -6000.0, "mtsq": 172.0 ** 2, "mhsq": 125.0 ** 2}

PROBLEMS = {p.name: p for p in (BUBBLE, BUBBLE_MASSIVE, BOX, TRIANGLE_OFFSHELL,
                                BUBBLE_DOT, BUBBLE_DOT23, BUBBLE_DOT14, BUBBLE_MASSIVE_DOT,
                                SUNSET_DOT, SUNSET_DOT114, SUNSET_DOT123, BOX_DOT,
                                TRIANGLE_OFFSHELL_DOT,
                                DOUBLEBOX,
                                DOUBLEBOX_OFFSHELL, DOUBLEBOX_OFF14,
                                DOUBLEBOX_OFF24, DOUBLEBOX_OFF34,
                                NP_VERTEX, TRIANGLE2L, HH_BOX, HH_PLANAR,
                                HH_NONPLANAR)}
