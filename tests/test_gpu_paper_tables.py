"""End-to-end results of the GPU path against the values printed in
Section IV (tests/golden/paper_tables.json): the Euclidean off-shell double
box of Table 1 and the physical gg -> HH double boxes of Tables 2-3."""

import pytest

from gpu_util import gpu_plan
from paper_1508_02512_amd import frontend as fe
from paper_norm import GOLDEN, check_against, p_coefficients
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import HH_POINT
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu

N = 1000003


@pytest.mark.parametrize("legs", ["14", "24", "34"])
def test_table1_double_box_columns(legs):
    print(f"Table 1 column {legs}: n={N} m=16", flush=True)
    col = GOLDEN["table1"]["columns"][legs]
    kin = {"s": -2 / 3, "t": -2 / 3, **col["offshell"]}
    plan, info = gpu_plan(f"doublebox_off{legs}")
    res = plan.integrate(fe.kin_vector(info, kin), (N, lattice(N)), shift_table(0, 16, 8))
    P = p_coefficients(plan.orders, res["mean"][0], res["err_re"][0], res["err_im"][0], -2 / 3)
    check_against(P, col["qmc"], nsig=5.0, extra=1e-9)
    plan.close()


@pytest.mark.parametrize("table,lam", [("table2", 1.0), ("table3", 0.5)])
def test_tables2_3_physical_double_boxes(table, lam):
    print(f"{table}: n={N} m=16 lambda={lam}", flush=True)
    tab = GOLDEN[table]
    plan, info = gpu_plan(tab["problem"], lam=lam)
    res = plan.integrate(fe.kin_vector(info, HH_POINT), (N, lattice(N)), shift_table(0, 16, 8))
    assert res["violations"] == 0
    P = p_coefficients(plan.orders, res["mean"][0], res["err_re"][0], res["err_im"][0],
                       HH_POINT["s"])
    check_against(P, tab["qmc"], nsig=5.0)
    plan.close()
