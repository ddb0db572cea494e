"""Geometric sectors (the strategy Section II adopts) through the GPU path:
parity with the oracle on its own, independently built sector lists, and
the same integrals as the iterated sectors and the printed tables."""

import numpy as np
import pytest

from gpu_util import compare_sectors, gpu_plan, sample_sectors
from paper_1508_02512_amd import frontend as fe
from paper_norm import GOLDEN, check_against, p_coefficients
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import HH_POINT
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu


def test_double_box_geometric_sectors():
    print("doublebox geometric n=1009 m=2", flush=True)
    compare_sectors("doublebox", {"s": -3.0, "t": -1.0}, 1009, 2, strategy="geometric",
                    sectors=sample_sectors("doublebox", strategy="geometric"))


def test_hh_planar_geometric_sectors_deformed():
    print("hh_planar geometric n=1009 m=2 lambda=1", flush=True)
    res, _ = compare_sectors("hh_planar", HH_POINT, 1009, 2, lam=1.0, strategy="geometric",
                             sectors=sample_sectors("hh_planar", per_class=6,
                                                    strategy="geometric"))
    assert res["violations"] == 0


def test_double_box_same_integral_both_strategies():
    """266 geometric against 882 iterated sectors: every Laurent order of
    the massless double box agrees within the combined errors."""
    print("doublebox both strategies n=1000003 m=16", flush=True)
    kin = {"s": -3.0, "t": -1.0}
    n = 1000003
    out = []
    for strategy in ("iterated", "geometric"):
        plan, info = gpu_plan("doublebox", strategy=strategy)
        out.append(plan.integrate(fe.kin_vector(info, kin), (n, lattice(n)),
                                  shift_table(0, 16, 8)))
        plan.close()
    it, ge = out
    err = np.hypot(np.hypot(it["err_re"], it["err_im"]), np.hypot(ge["err_re"], ge["err_im"]))
    assert np.all(np.abs(it["mean"] - ge["mean"]) <= 5 * err)
    assert np.all(np.isfinite(ge["mean"]))


def test_table1_column_geometric():
    print("Table 1 column 14 geometric n=1000003 m=16", flush=True)
    col = GOLDEN["table1"]["columns"]["14"]
    kin = {"s": -2 / 3, "t": -2 / 3, **col["offshell"]}
    plan, info = gpu_plan("doublebox_off14", strategy="geometric")
    n = 1000003
    res = plan.integrate(fe.kin_vector(info, kin), (n, lattice(n)), shift_table(0, 16, 8))
    P = p_coefficients(plan.orders, res["mean"][0], res["err_re"][0], res["err_im"][0], -2 / 3)
    check_against(P, col["qmc"], nsig=5.0, extra=1e-9)
    plan.close()


def test_table2_geometric():
    print("Table 2 geometric n=1000003 m=16 lambda=1", flush=True)
    tab = GOLDEN["table2"]
    plan, info = gpu_plan(tab["problem"], lam=1.0, strategy="geometric")
    n = 1000003
    res = plan.integrate(fe.kin_vector(info, HH_POINT), (n, lattice(n)), shift_table(0, 16, 8))
    assert res["violations"] == 0
    P = p_coefficients(plan.orders, res["mean"][0], res["err_re"][0], res["err_im"][0],
                       HH_POINT["s"])
    check_against(P, tab["qmc"], nsig=5.0)
    plan.close()
