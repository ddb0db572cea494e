"""Serving: continuous batching with embedded-lattice doubling."""

import numpy as np
import pytest

from gpu_util import assert_assembly_matches, ctx, gpu_plan, oracle_assembled
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import qmc
from seeded_inputs.lattice import embedded_lattice
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu

Z = embedded_lattice()        # odd vector of the embedded rule, used for every n = 2^k


def _box_kin(info, s=-3.0, t=-2.0):
    return fe.kin_vector(info, {"s": s, "t": t})


def test_single_request_converges_and_matches_integrate():
    print("serve: one box request", flush=True)
    plan, info = gpu_plan("box")
    kin = _box_kin(info)
    # the box reaches 1e-6 on the first 2^12 points; a tighter target makes
    # the request double its lattice several times before it retires
    r = qmc.submit(plan, kin, 1e-10, 1 << 10, 1 << 22, 8, 7, Z).wait(120)
    assert r["rc"] == 0 and r["steps"] >= 3
    assert r["n_final"] == (1 << 10) << (r["steps"] - 1)
    # the doubled lattice reproduces one pass over the same 2^k points
    ref = plan.integrate(kin, (r["n_final"], Z), shift_table(7, 8, 8))
    assert np.allclose(r["mean"], ref["mean"], rtol=1e-12, atol=1e-14)
    assert np.allclose(r["err_re"], ref["err_re"], rtol=1e-8, atol=1e-16)
    want = np.array([0.666666666666667, -0.982063599677040, -1.48360889993076])
    assert np.all(np.abs(r["mean"][0].real - want) <= 6 * r["err_re"][0] + 1e-12)
    plan.close()


@pytest.mark.parametrize("name,kin,lam,m", [
    ("box", {"s": -3.0, "t": -2.0}, 0.0, 8),
    ("np_vertex", {"s": 4.5, "msq": 1.0}, 0.5, 4),
])
def test_served_doubling_matches_oracle(name, kin, lam, m):
    """A request that doubles n = 2^10 -> 2^11 -> 2^12 (the last two steps
    over the odd indices of the embedded lattice only) and then stops at
    n_max: its mean and Eq. 20 errors equal the oracle's on all 2^12 points
    of the same lattice and shifts, within 1e-12 of the rounding scale.
    The non-planar vertex takes the deformed kernel."""
    print(f"serve vs oracle: {name}", flush=True)
    plan, info = gpu_plan(name, lam=lam)
    seed = 21
    r = qmc.submit(plan, fe.kin_vector(info, kin), 1e-15, 1 << 10, 1 << 12, m, seed,
                   Z).wait(120)
    assert r["rc"] == -7 and r["n_final"] == 1 << 12 and r["steps"] == 3
    ora = oracle_assembled(name, kin, 1 << 12, Z, shift_table(seed, m, 8), lam=lam)
    assert_assembly_matches(r, ora)
    plan.close()


def test_same_result_alone_and_in_mix():
    print("serve: alone vs mix", flush=True)
    box, binfo = gpu_plan("box")
    bub, uinfo = gpu_plan("bubble_massive", lam=0.5)
    np_, ninfo = gpu_plan("np_vertex", lam=0.5)
    kin = _box_kin(binfo, -2.5, -1.5)
    alone = qmc.submit(box, kin, 1e-5, 1 << 12, 1 << 20, 8, 11, Z).wait(120)
    others = []
    rng = np.random.default_rng(0)
    for i in range(12):
        if i % 3 == 0:
            k = fe.kin_vector(uinfo, {"s": float(rng.uniform(4.2, 8.0)), "msq": 1.0})
            others.append(qmc.submit(bub, k, 1e-4, 1 << 10, 1 << 20, 8, 100 + i, Z))
        elif i % 3 == 1:
            k = fe.kin_vector(ninfo, {"s": float(rng.uniform(4.2, 6.0)), "msq": 1.0})
            others.append(qmc.submit(np_, k, 3e-3, 1 << 12, 1 << 18, 8, 100 + i, Z))
        else:
            k = _box_kin(binfo, float(rng.uniform(-5, -1)), float(rng.uniform(-5, -1)))
            others.append(qmc.submit(box, k, 1e-4, 1 << 10, 1 << 20, 8, 100 + i, Z))
    mixed = qmc.submit(box, kin, 1e-5, 1 << 12, 1 << 20, 8, 11, Z)
    res = [o.wait(300) for o in others]
    again = mixed.wait(300)
    assert all(x is not None and x["rc"] in (0, -7) for x in res)
    assert again["rc"] == 0 and alone["rc"] == 0
    assert np.array_equal(alone["mean"], again["mean"])
    assert np.array_equal(alone["err_re"], again["err_re"])
    for p in (box, bub, np_):
        p.close()


def test_not_converged_and_cancel():
    print("serve: n_max and cancel", flush=True)
    plan, info = gpu_plan("box")
    kin = _box_kin(info)
    r = qmc.submit(plan, kin, 1e-14, 1 << 10, 1 << 12, 4, 1, Z).wait(60)
    assert r["rc"] == -7 and r["n_final"] == 1 << 12
    slow = qmc.submit(plan, kin, 1e-15, 1 << 20, 1 << 30, 4, 2, Z)
    slow.cancel()
    assert slow.wait(60)["rc"] == -9
    plan.close()


def test_budget_too_small():
    print("serve: budget", flush=True)
    small = qmc.Context(0, hbm_budget=8 << 20)
    secs, info = fe.decompose(__import__("seeded_inputs.problems", fromlist=["x"]).PROBLEMS["doublebox"])
    plan = small.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 12))
    r = qmc.submit(plan, fe.kin_vector(info, {"s": -3.0, "t": -1.0}), 1e-3, 1 << 16, 1 << 20,
                   16, 1, Z).wait(60)
    assert r["rc"] == -5
    plan.close()
    small.close()


def test_large_request_runs_in_bounded_steps_beside_small_ones():
    """A request that doubles to n = 2^25 (past 2^24, where a level needs
    more work items than one step takes) shares a context with a tight
    budget (64 MiB) with small requests submitted after it: each step takes
    only a bounded window of the large request's items, so the small ones
    are admitted and finish first, and the large one ends at n_max
    (QMC_ENOTCONVERGED), neither refused nor failing the others."""
    print("serve: bounded steps, one large and six small requests", flush=True)
    small_ctx = qmc.Context(0, hbm_budget=64 << 20)
    secs, info = fe.decompose(__import__("seeded_inputs.problems", fromlist=["x"]).PROBLEMS["box"])
    plan = small_ctx.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 8))
    big = qmc.submit(plan, _box_kin(info), 1e-300, 1 << 10, 1 << 25, 4, 5, Z)
    smalls = [qmc.submit(plan, _box_kin(info, -2.0 - 0.1 * i, -1.5), 1e-4, 1 << 10, 1 << 16,
                         4, 40 + i, Z) for i in range(6)]
    rs = [x.wait(300) for x in smalls]
    rb = big.wait(300)
    assert rb["rc"] == -7 and rb["n_final"] == 1 << 25, rb["rc"]
    assert all(r["rc"] == 0 for r in rs)
    assert max(r["latency_ms"] for r in rs) < rb["latency_ms"]
    plan.close()
    small_ctx.close()


def test_deformation_violation_reported():
    print("serve: lambda too large", flush=True)
    plan, info = gpu_plan("np_vertex", lam=1.0)
    r = qmc.submit(plan, fe.kin_vector(info, {"s": 4.5, "msq": 1.0}), 1e-3, 1 << 10, 1 << 16,
                   4, 1, Z).wait(60)
    assert r["rc"] == -6 and r["violations"] > 0
    plan.close()


def test_lambda_backoff_recovers():
    """lambda = 1 violates the sign conditions for the non-planar vertex at
    s = 4.5 (the plain request retires with QMC_EDEFORM); with back-offs the
    violating sectors run at lambda/2^k, the request converges, and its
    result agrees with the one at a safe lambda within the errors."""
    print("serve: lambda back-off", flush=True)
    plan, info = gpu_plan("np_vertex", lam=1.0)
    safe, _ = gpu_plan("np_vertex", lam=0.25)
    kin = fe.kin_vector(info, {"s": 4.5, "msq": 1.0})
    plain = qmc.submit(plan, kin, 1e-3, 1 << 12, 1 << 20, 8, 3, Z).wait(120)
    assert plain["rc"] == -6 and plain["lambda_halvings"] == 0
    r = qmc.submit(plan, kin, 1e-3, 1 << 12, 1 << 20, 8, 3, Z, lambda_halvings=4).wait(120)
    assert r["rc"] == 0 and 1 <= r["lambda_halvings"] <= 4 and r["violations"] == 0
    ref = qmc.submit(safe, kin, 1e-3, 1 << 12, 1 << 23, 8, 3, Z).wait(120)
    assert ref["rc"] == 0
    err = np.hypot(r["err_re"], r["err_im"]) + np.hypot(ref["err_re"], ref["err_im"])
    assert np.all(np.abs(r["mean"] - ref["mean"]) <= 5 * err + 1e-12)
    with pytest.raises(qmc.QMCError):
        qmc.submit(plan, kin, 1e-3, 1 << 12, 1 << 20, 8, 3, Z, lambda_halvings=17)
    plan.close()
    safe.close()


def test_geometric_sectors_serve_the_table2_integral():
    """I_C at the Table 2 point served from its 46 geometric sectors: the
    request meets 1e-3 on every order without a lambda back-off, and its
    result equals one pass of qmc_integrate over the same 2^k points."""
    from seeded_inputs.problems import HH_POINT
    print("serve: I_C geometric sectors", flush=True)
    plan, info = gpu_plan("hh_planar", lam=1.0, strategy="geometric")
    kin = fe.kin_vector(info, HH_POINT)
    r = qmc.submit(plan, kin, 1e-3, 1 << 14, 1 << 22, 8, 3, Z, lambda_halvings=2).wait(300)
    assert r["rc"] == 0 and r["lambda_halvings"] == 0
    ref = plan.integrate(kin, (r["n_final"], Z), shift_table(3, 8, 8))
    assert np.allclose(r["mean"], ref["mean"], rtol=1e-12, atol=1e-14)
    rel = np.hypot(r["err_re"], r["err_im"]) / np.abs(r["mean"])
    assert np.all(rel <= 1e-3)
    plan.close()
