"""GPU path of the integration by parts taken at the poles as well (Section
II, Eq. 13 as the alternative to the subtraction of Eq. 11; pole method
QMC_POLES_IBP): the planner's expansion against the oracle's, sector sums
per (sector, shift, order) against the oracle at 1e-12 of sum |w g| (the
pole-free sectors carry up to 7 orders: the wide kernel builds), the
assembled result and Eq. 20 errors against the oracle's, whole results
against closed forms in FP64 and FP32, both pole methods on the double box,
several kinematic points with uneven lattices and graph replay, serving,
and the refusals."""

import numpy as np
import pytest

from gpu_util import (assert_assembly_matches, compare_sectors, ctx, gpu_plan,
                      oracle_assembled, oracle_sectors)
from oracle import qmc as oq
from oracle.decompose import decompose as odec
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import qmc
from seeded_inputs.lattice import embedded_lattice, lattice
from seeded_inputs.problems import PROBLEMS
from seeded_inputs.rng import shift_table
from test_oracle_ibp import _laurent, _sunset
from test_oracle_pins import _box_exact

pytestmark = pytest.mark.gpu

# (problem, kinematic point, eps_hi)
POLES = [
    ("box", {"s": -3.0, "t": -2.0}, 0),
    ("box_dot", {"s": -3.0, "t": -2.0}, 0),
    ("bubble_massive_dot", {"s": -2.0, "msq": 1.5}, 1),
    ("sunset_dot123", {"s": -2.0}, 0),
    ("triangle_offshell_dot", {"p1sq": -1.0, "p2sq": -2.0, "p3sq": -3.0}, 0),
    ("sunset_dot", {"s": -2.0}, 0),
    ("bubble_dot23", {"s": -0.4}, 1),
]
DB_KIN = {"s": -3.0, "t": -1.0}


def _check_plan(name, eps_hi, every=1):
    plan, _ = gpu_plan(name, eps_hi, poles=True)
    osecs, _ = oracle_sectors(name, poles=True)
    assert plan.n_input_sectors == len(odec(PROBLEMS[name])[0])
    assert plan.n_sectors == len(osecs)
    assert plan.info.max_poles == 0
    for s in range(0, len(osecs), every):
        o = osecs[s]
        si = plan.sector_info(s)
        assert si["origin"] == o["origin"], s
        assert si["dim"] == len(o["a"]), s
        assert si["poles"] == 0 and all(a != -1 for a in o["a"]), s
        assert si["factors"] == len(o["P"]), s
        assert si["u"] == tuple(float(x) for x in o["u"]), s
        assert si["f"] == tuple(float(x) for x in o["f"]), s
        assert si["C_lo"] == -qmc.QMC_MAX_POLES
        want = np.array([float(o["C"].get(k + si["C_lo"], 0))
                         for k in range(qmc.QMC_MAX_ORDERS)])
        assert np.allclose(si["C"].real, want, rtol=1e-14, atol=1e-14), (s, si["C"], want)
        assert np.all(si["C"].imag == 0.0)
    plan.close()


@pytest.mark.parametrize("name,kin,eps_hi", POLES)
def test_planned_sectors_match_oracle_expansion(name, kin, eps_hi):
    print(f"ibp poles plan: {name}", flush=True)
    _check_plan(name, eps_hi)


def test_double_box_plan_matches_oracle_expansion():
    """882 sectors with up to 4 poles become 48798 pole-free ones; every
    97th is compared."""
    print("ibp poles plan: doublebox", flush=True)
    _check_plan("doublebox", 0, every=97)


@pytest.mark.parametrize("name,kin,eps_hi", POLES)
def test_sector_sums_match_oracle(name, kin, eps_hi):
    """Every planned sector against the oracle on the same lattice and
    shifts: 3 shifts, n = 10007 (ragged last tile)."""
    print(f"ibp poles parity: {name}", flush=True)
    compare_sectors(name, kin, 10007, 3, eps_hi=eps_hi, poles=True)


@pytest.mark.parametrize("precision", [qmc.QMC_FP64, qmc.QMC_FP32_EVAL])
def test_double_box_sector_sums_match_oracle(precision):
    """Sampled sectors of the double box (5 orders per sector in the wide
    builds) against the oracle; FP32 evaluation at its own bar."""
    print(f"ibp poles parity: doublebox precision {precision}", flush=True)
    osecs, _ = oracle_sectors("doublebox", poles=True)
    sample = list(range(0, len(osecs), 997)) + [len(osecs) - 1]
    tol = 1e-12 if precision == qmc.QMC_FP64 else 1e-5
    compare_sectors("doublebox", DB_KIN, 10007, 2, sectors=sample, poles=True,
                    precision=precision, tol=tol)


@pytest.mark.parametrize("name,kin", [("box", {"s": -3.0, "t": -2.0}),
                                      ("sunset_dot123", {"s": -2.0})])
def test_geometric_sectors_match_oracle(name, kin):
    print(f"ibp poles parity: {name}, geometric sectors", flush=True)
    compare_sectors(name, kin, 10007, 3, strategy="geometric", poles=True)


def test_sector_sums_many_tiles_and_persistent_points_per_lane():
    print("ibp poles parity: box_dot, ppl 3", flush=True)
    compare_sectors("box_dot", {"s": -3.0, "t": -2.0}, 100003, 2, ppl=3, poles=True)


@pytest.mark.parametrize("name,kin,eps_hi", [POLES[0], POLES[2], POLES[3]])
def test_assembly_and_errors_match_oracle(name, kin, eps_hi):
    """Laurent assembly with coefficient series starting below eps^0, and
    the Eq. 20 errors, against the oracle's."""
    print(f"ibp poles assembly: {name}", flush=True)
    plan, info = gpu_plan(name, eps_hi, poles=True)
    n, m = 4099, 5
    z = lattice(n)
    shifts = shift_table(3, m, 8)
    res = plan.integrate(fe.kin_vector(info, kin), (n, z), shifts)
    ora = oracle_assembled(name, kin, n, z, shifts, eps_hi=eps_hi, poles=True)
    lo = ora["orders"][0]
    k = list(res["orders"]).index(lo)
    gpu = {key: (np.asarray(res[key])[:, k:] if key != "orders" else list(res["orders"])[k:])
           for key in ("mean", "err_re", "err_im", "orders")}
    # orders below the oracle's lowest (a bound taken before Eq. 13) are 0
    assert np.all(np.asarray(res["mean"])[:, :k] == 0)
    assert_assembly_matches(gpu, ora)
    plan.close()


@pytest.mark.parametrize("precision", [qmc.QMC_FP64, qmc.QMC_FP32_EVAL])
def test_whole_results_against_closed_forms(precision):
    """Whole GPU results within 6 standard errors of the closed forms (FP32
    evaluation: also within 1e-5 relative); the vanishing eps^-2 of the
    dotted sunset comes out exactly 0."""
    cases = [("box", {"s": -3.0, "t": -2.0}, 0, _box_exact(-3.0, -2.0)),
             ("sunset_dot123", {"s": -2.0}, 0, _laurent(_sunset(1, 2, 3, -2.0), -1, 0))]
    n, m = 100003, 8
    for name, kin, eps_hi, exact in cases:
        print(f"ibp poles closed form: {name} precision {precision}", flush=True)
        plan, info = gpu_plan(name, eps_hi, precision=precision, poles=True)
        res = plan.integrate(fe.kin_vector(info, kin), (n, lattice(n)), shift_table(0, m, 8))
        for p, want in exact.items():
            i = list(res["orders"]).index(p)
            got, err = res["mean"][0][i], res["err_re"][0][i]
            tol = 6 * err + 1e-12 * max(1.0, abs(want))
            if precision == qmc.QMC_FP32_EVAL:
                tol += 1e-5 * max(1.0, abs(want))
            assert abs(got.real - want.real) <= tol, (name, p, got, want, err)
        if name == "sunset_dot123":
            assert res["mean"][0][list(res["orders"]).index(-2)] == 0
        plan.close()


def test_double_box_both_pole_methods_agree():
    """The double box by Eq. 11 and by Eq. 13 on the same lattice: equal
    within their combined errors at every order."""
    print("ibp poles: doublebox both methods", flush=True)
    n, m = 100003, 8
    out = []
    for poles in (False, True):
        plan, info = gpu_plan("doublebox", 0, poles=poles)
        out.append(plan.integrate(fe.kin_vector(info, DB_KIN), (n, lattice(n)),
                                  shift_table(0, m, 8)))
        plan.close()
    a, b = out
    assert list(a["orders"]) == list(b["orders"])
    for i, p in enumerate(a["orders"]):
        d = a["mean"][0][i] - b["mean"][0][i]
        sig = np.hypot(a["err_re"][0][i], b["err_re"][0][i])
        assert abs(d.real) <= 6 * sig + 1e-12 * abs(a["mean"][0][i]), \
            (p, a["mean"][0][i], b["mean"][0][i], sig)


def test_batch_points_uneven_lattices_and_graph():
    """Pole-method plan of the dotted box at 6 Euclidean points with uneven
    per-sector lattices in one bind: graph replays give the eager bits, and
    sampled (point, sector) sums match the oracle at 1e-12."""
    print("ibp poles batch: box_dot 6 points, uneven lattices", flush=True)
    plan, info = gpu_plan("box_dot", poles=True)
    pts = [{"s": -0.5 - 0.7 * i, "t": -2.5 + 0.3 * i} for i in range(6)]
    kin = np.stack([fe.kin_vector(info, k) for k in pts])
    sizes = [1009, 4099, 10007]
    lats = [(n, lattice(n)) for n in (sizes[i % 3] for i in range(plan.n_sectors))]
    sh = shift_table(6, 3, 8)
    eager = plan.integrate(kin, None, sh, lat_per_sector=lats, sector_sums=True)
    job = plan.bind(kin, None, sh, lat_per_sector=lats)
    job.use_graph(True)
    for rep in range(3):
        job.run()
        got = job.fetch(sector_sums=True)
        np.testing.assert_array_equal(got["sector_sums"], eager["sector_sums"])
        plan.integrate(kin[:2], None, sh, lat_per_sector=lats)
    job.close()
    osecs, oinfo = oracle_sectors("box_dot", poles=True)
    rng = np.random.default_rng(2)
    for p in rng.choice(len(pts), size=3, replace=False):
        for s in rng.choice(len(osecs), size=6, replace=False):
            ns = oq.NumericSector(osecs[s], oinfo, pts[p])
            n, z = lats[s]
            sums, abss, _ = oq.sector_sums(ns, n, z, sh, 2, 0.0, eager["sec_lo"],
                                           plan.info.sec_orders)
            scale = abss[..., 0] + abss[..., 1]
            err = np.abs(eager["sector_sums"][p, s] - sums)
            assert np.all(err <= 1e-12 * np.maximum(scale, 1e-300)), (p, s)
    plan.close()


def test_served_request():
    """A served request on a plan expanded at the poles: converges, and its
    result equals one pass of qmc_integrate over the same 2^k points."""
    print("ibp poles serve: box", flush=True)
    plan, info = gpu_plan("box", poles=True)
    kin = fe.kin_vector(info, {"s": -3.0, "t": -2.0})
    z = embedded_lattice()
    r = qmc.submit(plan, kin, 1e-7, 1 << 10, 1 << 20, 8, 5, z).wait(120)
    assert r["rc"] == 0
    ref = plan.integrate(kin, (r["n_final"], z), shift_table(5, 8, 8))
    assert np.allclose(r["mean"], ref["mean"], rtol=1e-12, atol=1e-14)
    for p, want in _box_exact(-3.0, -2.0).items():
        i = list(r["orders"]).index(p)
        assert abs(r["mean"][0][i].real - want.real) <= 6 * r["err_re"][0][i] + 1e-12
    plan.close()


def test_refusals():
    # Eq. 13 with contour deformation is not supported
    with pytest.raises(qmc.QMCError) as e:
        gpu_plan("box", lam=0.5, poles=True)
    assert e.value.code == qmc.QMC_EUNSUPPORTED and "pole method" in str(e.value)
    secs, info = fe.decompose(PROBLEMS["box"])
    arrs = fe.sector_arrays(secs, info)
    # an unknown pole method
    with pytest.raises(qmc.QMCError) as e:
        ctx().plan(arrs, info, 0, fe.prefactor_series(info, 12), pole_method=7)
    assert e.value.code == qmc.QMC_EINVAL
    # a pole without regulator
    arrs[0] = dict(arrs[0], b=np.where(arrs[0]["a"] == -1.0, 0.0, arrs[0]["b"]))
    with pytest.raises(qmc.QMCError) as e:
        ctx().plan(arrs, info, 0, fe.prefactor_series(info, 12),
                   pole_method=qmc.QMC_POLES_IBP)
    assert e.value.code == qmc.QMC_EUNREGULATED
