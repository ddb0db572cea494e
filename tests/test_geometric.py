"""Geometric sector decomposition (Section II, the strategy the paper adopts).

Pins that do not depend on either implementation:
  * a two-variable fan worked out by hand;
  * the sectors of every primary sector tile the unit cube: the volumes
    |det V| prod_k 1/|n_k|_1 add up to exactly 1, and random points of the
    cube (in logarithmic coordinates) fall into exactly one sector;
  * in every sector U and F keep a non-vanishing constant term;
  * the integral does not depend on the strategy: the oracle's estimate
    over geometric sectors reproduces the closed forms and the printed
    Table 1 values that the iterated sectors reproduce.
The product front end and the oracle implement the same rule independently;
their sector lists must agree exactly, in order.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import geometric as og
from oracle import qmc
from oracle.decompose import _primary
from oracle.decompose import decompose as iterated
from oracle.feynman import symanzik
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import geometric as pg
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import PROBLEMS
from seeded_inputs.rng import shift_table

ALL = ["bubble", "bubble_massive", "triangle_offshell", "box", "np_vertex", "triangle2l",
       "hh_box", "hh_planar", "hh_nonplanar",
       "doublebox", "doublebox_off14"]


def _primaries(name):
    U, F, _ = symanzik(PROBLEMS[name])
    N = len(PROBLEMS[name].props)
    return [(_primary(U, l), _primary(F, l)) for l in range(N)]


def _oracle_cones(U, F):
    d = len(next(iter(U)))
    pts = og.newton_points(U, F)
    cones = []
    for _, rays in og.normal_cones(pts, og.polyhedron_facets(pts, d), d):
        cones += og.pulling(rays)
    return cones


def test_two_variable_fan_by_hand():
    """U = t1 + t2, F = 1: the fan of the orthant plus the segment has the
    rays (1,0), (1,1), (0,1) and two cones, giving the textbook split:
    t1 = s2, t2 = s1 s2 (and mirrored), U = s2 (1 + s1), Jacobian s2."""
    one = {"1": Fraction(1)}
    sec = {"a": [Fraction(0)] * 2, "b": [Fraction(0)] * 2,
           "U": {(1, 0): one, (0, 1): one}, "F": {(0, 0): one}}
    out = og.sectors_of_primary(sec, (Fraction(1), Fraction(0), Fraction(0), Fraction(0)))
    assert len(out) == 2
    for s in out:
        assert s["D"] == 1
        assert sorted(s["U"]) == [(0, 0), (1, 0)]          # 1 + s1
        assert s["F"] == {(0, 0): one}
        # s2 carries the Jacobian s2^1 and U's factor s2^(1 * u0) with u0 = 1
        assert s["a"] == [0, 2] and s["b"] == [0, 0]
    cones = _oracle_cones(sec["U"], sec["F"])
    assert sorted(cones) == [((0, 1), (1, 1)), ((1, 0), (1, 1))]
    got = sorted(tuple(map(tuple, V.T.tolist()))
                 for V, _ in pg.decompose_primary(np.array([[1, 0], [0, 1]]), np.array([[0, 0]])))
    assert got == sorted(cones)


@pytest.mark.parametrize("name", ALL)
def test_sectors_tile_the_cube(name):
    """Exact volumes add up to 1 in every primary sector; each random
    direction w > 0 (w = -ln t) lies in exactly one cone."""
    rng = np.random.default_rng(7)
    for U, F in _primaries(name):
        cones = _oracle_cones(U, F)
        d = len(cones[0])
        vol = Fraction(0)
        for cone in cones:
            V = np.array(cone, dtype=np.int64).T
            piece = Fraction(abs(int(round(np.linalg.det(V)))))
            for k in range(d):
                piece /= int(V[:, k].sum())
            vol += piece
        assert vol == 1
        W = rng.exponential(size=(400, d))
        inv = [np.linalg.inv(np.array(c, dtype=float).T) for c in cones]
        hits = np.zeros(len(W), dtype=int)
        for Vi in inv:
            hits += np.all(W @ Vi.T >= 0, axis=1)
        assert np.all(hits == 1)


@pytest.mark.parametrize("name", ALL)
def test_every_sector_keeps_constant_terms(name):
    secs, _ = og.decompose(PROBLEMS[name])
    for s in secs:
        d = len(s["a"])
        assert (0,) * d in s["U"] and (0,) * d in s["F"]
        assert all(min(e) >= 0 for e in list(s["U"]) + list(s["F"]))
        # regulated: every non-integrable power carries an eps part
        assert all(a > -1 or b != 0 for a, b in zip(s["a"], s["b"]))


def _canon_product(s, inv):
    def poly(E, C):
        return sorted((tuple(int(x) for x in e),
                       tuple((inv[i], v) for i, v in enumerate(c) if v != 0))
                      for e, c in zip(E, C))
    return (list(s["a"]), list(s["b"]), poly(s["EU"], s["CU"]), poly(s["EF"], s["CF"]),
            int(s["D"]))


def _canon_oracle(s, inv):
    order = {k: i for i, k in enumerate(inv)}

    def poly(P):
        return sorted((e, tuple(sorted(f.items(), key=lambda kv: order[kv[0]])))
                      for e, f in P.items())
    return (list(s["a"]), list(s["b"]), poly(s["U"]), poly(s["F"]), s["D"])


@pytest.mark.parametrize("name", ALL)
def test_front_end_matches_oracle(name):
    psecs, pinfo = fe.decompose(PROBLEMS[name], "geometric")
    osecs, _ = og.decompose(PROBLEMS[name])
    inv = pinfo["invariants"]
    assert [_canon_product(s, inv) for s in psecs] == [_canon_oracle(s, inv) for s in osecs]


def test_fewer_sectors_than_iterated():
    counts = {}
    for name in ALL:
        counts[name] = (len(fe.decompose(PROBLEMS[name], "geometric")[0]),
                        len(fe.decompose(PROBLEMS[name])[0]))
        assert counts[name][0] <= counts[name][1]
    assert counts["doublebox"] == (266, 882)


# --- strategy independence of the integral ------------------------------------

def _run(name, kin, n, m=8, lam=0.0, eps_hi=0):
    return qmc.integrate(PROBLEMS[name], kin, n, lattice(n), shift_table(0, m, 8),
                         lam=lam, eps_hi=eps_hi, sectors=og.decompose(PROBLEMS[name]))


def test_oracle_geometric_box_closed_form():
    from test_oracle_pins import _box_exact, _check
    _check(_run("box", {"s": -3.0, "t": -2.0}, 10007), _box_exact(-3.0, -2.0))


def test_oracle_geometric_np_vertex_matches_iterated():
    kin = {"s": 4.5, "msq": 1.0}
    g = _run("np_vertex", kin, 4099, lam=0.5)
    it = qmc.integrate(PROBLEMS["np_vertex"], kin, 4099, lattice(4099), shift_table(0, 8, 8),
                       lam=0.5, sectors=iterated(PROBLEMS["np_vertex"]))
    i = g["orders"].index(0)
    j = it["orders"].index(0)
    diff = g["mean"][i] - it["mean"][j]
    assert abs(diff.real) <= 5 * np.hypot(g["err_re"][i], it["err_re"][j])
    assert abs(diff.imag) <= 5 * np.hypot(g["err_im"][i], it["err_im"][j])


def test_oracle_geometric_table1_column():
    from paper_norm import GOLDEN, check_against, p_coefficients
    col = GOLDEN["table1"]["columns"]["14"]
    kin = {"s": -2 / 3, "t": -2 / 3, **col["offshell"]}
    res = _run("doublebox_off14", kin, 1009)
    P = p_coefficients(list(res["orders"]), res["mean"], res["err_re"], res["err_im"], -2 / 3)
    check_against(P, col["qmc"], nsig=5.0, extra=1e-9)
