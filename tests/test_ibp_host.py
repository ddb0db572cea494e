"""The planner's host-side integration by parts (Section II, Eq. 13;
csrc/qmc_ibp.cpp) against the oracle's own expansion (oracle/ibp.py), on
the CPU: for every planned sector, the input sector it comes from, its
dimension, exponents, numerator-factor count, powers of U and F, the
coefficient series C(eps), and U, F and every numerator factor evaluated
at one point, for powers below -1 and for the pole method (Eq. 13 at
a_j = -1 as well), including the double box's 48798 sectors.  The wrapper
is compiled into a temporary library with hipcc (host code only)."""

import ctypes as C
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import ibp
from oracle.decompose import decompose as odec
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import qmc
from seeded_inputs.problems import PROBLEMS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
P = C.POINTER


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("ibp") / "libibp_probe.so")
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-fPIC", "-shared",
                    os.path.join(ROOT, "tests", "ibp_host_probe.cpp"),
                    os.path.join(ROOT, "paper_1508_02512_amd", "csrc", "qmc_ibp.cpp"),
                    "-o", out], check=True, capture_output=True)
    lib = C.CDLL(out)
    lib.ibp_host_expand.restype = C.c_int
    return lib


def _problem(name):
    secs, info = fe.decompose(PROBLEMS[name])
    arrs = fe.sector_arrays(secs, info)
    keep = []
    arr = (qmc.qmc_sector * len(arrs))()
    for i, s in enumerate(arrs):
        r = arr[i]
        r.dim = s["dim"]
        keep += [s[k] for k in ("a", "b", "EU", "CU", "EF", "CF")]
        r.mono_a, r.mono_b = qmc._dptr(s["a"]), qmc._dptr(s["b"])
        for nm, E, Cm in (("U", s["EU"], s["CU"]), ("F", s["EF"], s["CF"])):
            poly = getattr(r, nm)
            poly.n_terms = E.shape[0]
            poly.exps = E.ctypes.data_as(P(C.c_uint8))
            poly.coef = qmc._dptr(Cm)
        r.u_exp[0], r.u_exp[1] = s["u"]
        r.f_exp[0], r.f_exp[1] = s["f"]
        r.coef_re, r.coef_im = float(s["D"]), 0.0
    prob = qmc.qmc_problem()
    prob.n_sectors = len(arrs)
    prob.sectors = arr
    prob.n_inv = len(info["invariants"])
    return prob, info, (arr, keep)


def _expand(lib, name, poles, kin):
    prob, info, keep = _problem(name)
    kv = fe.kin_vector(info, kin)
    mx = 1 << 16
    n = C.c_int()
    meta = np.zeros((mx, 6), np.int32)
    expo = np.zeros((mx, 4))
    ab = np.zeros((mx, 2, 8))
    coef = np.zeros((mx, 8, 2))
    vals = np.zeros((mx, 6))
    err = C.create_string_buffer(256)
    ip = lambda x: x.ctypes.data_as(P(C.c_int))
    rc = lib.ibp_host_expand(C.byref(prob), int(poles), qmc._dptr(kv), mx, C.byref(n), ip(meta),
                             qmc._dptr(expo), qmc._dptr(ab), qmc._dptr(coef), qmc._dptr(vals),
                             err, 256)
    return rc, err.value.decode(), n.value, meta, expo, ab, coef, vals


def _poly_at(poly, kin, t):
    s = 0.0
    for e, form in poly.items():
        cf = sum(float(v) * (1.0 if k == "1" else kin[k]) for k, v in form.items())
        m = 1.0
        for v, p in enumerate(e):
            m *= t[v] ** p
        s += cf * m
    return s


CASES = [("bubble_dot", {"s": -3.0}), ("bubble_dot14", {"s": -3.0}),
         ("bubble_massive_dot", {"s": -2.0, "msq": 1.5}), ("sunset_dot114", {"s": -2.0}),
         ("sunset_dot123", {"s": -2.0}), ("box_dot", {"s": -3.0, "t": -2.0}),
         ("triangle_offshell_dot", {"p1sq": -1.0, "p2sq": -2.0, "p3sq": -3.0}),
         ("box", {"s": -3.0, "t": -2.0})]


@pytest.mark.parametrize("poles", [False, True])
@pytest.mark.parametrize("name,kin", CASES)
def test_expansion_matches_oracle(probe, name, kin, poles):
    osecs, oinfo = odec(PROBLEMS[name])
    if not ibp.needs_ibp(osecs, poles):
        osecs = [dict(s, origin=i, P=[], C={0: Fraction(s.get("D", 1))},
                      u=(oinfo["u0"], oinfo["u1"]), f=(oinfo["f0"], oinfo["f1"]))
                 for i, s in enumerate(osecs)]
    else:
        osecs = ibp.expand(osecs, oinfo, poles)
    rc, msg, n, meta, expo, ab, coef, vals = _expand(probe, name, poles, kin)
    assert rc == 0, msg
    assert n == len(osecs)
    t = [0.3 + 0.1 * v for v in range(8)]
    for s, o in enumerate(osecs):
        d = len(o["a"])
        clo = meta[s, 3]
        assert clo == (-qmc.QMC_MAX_POLES if poles else 0)
        assert (meta[s, 0], meta[s, 1], meta[s, 2]) == (o["origin"], d, len(o["P"])), s
        assert np.array_equal(ab[s, 0, :d], [float(x) for x in o["a"]]), s
        assert np.array_equal(ab[s, 1, :d], [float(x) for x in o["b"]]), s
        assert np.array_equal(expo[s], [float(x) for x in (*o["u"], *o["f"])]), s
        want = np.array([float(o["C"].get(k + clo, 0)) for k in range(8)])
        assert np.allclose(coef[s, :, 0], want, rtol=1e-14, atol=1e-15), (s, coef[s, :, 0], want)
        assert np.all(coef[s, :, 1] == 0.0)
        # the wrapper reports 4 factors (the planner refuses more; the
        # expansion itself has no limit: the dotted sunset's pole method
        # reaches 5)
        polys = ([o["U"], o["F"]] + list(o["P"]))[:6]
        for i, poly in enumerate(polys):
            w = _poly_at(poly, kin, t)
            assert abs(vals[s, i] - w) <= 1e-12 * max(1.0, abs(w)), (s, i, vals[s, i], w)


def test_double_box_pole_method(probe):
    """882 sectors with up to 4 poles: 48798 planned sectors, every one
    compared (metadata, C(eps), polynomials at one point)."""
    kin = {"s": -3.0, "t": -1.0}
    osecs, oinfo = odec(PROBLEMS["doublebox"])
    osecs = ibp.expand(osecs, oinfo, True)
    rc, msg, n, meta, expo, ab, coef, vals = _expand(probe, "doublebox", True, kin)
    assert rc == 0, msg
    assert n == len(osecs) == 48798
    t = [0.3 + 0.1 * v for v in range(8)]
    for s, o in enumerate(osecs):
        assert (meta[s, 0], meta[s, 1], meta[s, 2]) == (o["origin"], len(o["a"]), len(o["P"]))
        want = np.array([float(o["C"].get(k - qmc.QMC_MAX_POLES, 0)) for k in range(8)])
        assert np.allclose(coef[s, :, 0], want, rtol=1e-14, atol=1e-15), s
        for i, poly in enumerate(([o["U"], o["F"]] + list(o["P"]))[:6]):
            w = _poly_at(poly, kin, t)
            assert abs(vals[s, i] - w) <= 1e-12 * max(1.0, abs(w)), (s, i)


def test_refusals(probe):
    # the pole method divides by b eps: b = 0 at a = -1 is refused
    prob, info, keep = _problem("box")
    arr = keep[0]
    b = np.ctypeslib.as_array(arr[0].mono_b, shape=(arr[0].dim,))
    a = np.ctypeslib.as_array(arr[0].mono_a, shape=(arr[0].dim,))
    b[a == -1.0] = 0.0
    n = C.c_int()
    z = np.zeros(1 << 10)
    err = C.create_string_buffer(256)
    rc = probe.ibp_host_expand(C.byref(prob), 1, qmc._dptr(np.ones(3)), 0, C.byref(n),
                               z.ctypes.data_as(P(C.c_int)), qmc._dptr(z), qmc._dptr(z),
                               qmc._dptr(z), qmc._dptr(z), err, 256)
    assert rc == qmc.QMC_EUNREGULATED and b"not regulated" in err.value
