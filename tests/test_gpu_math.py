"""Error bounds of the elementary functions inside the integrand kernels,
against the host's extended-precision (80-bit) library on wide samples."""

import numpy as np
import pytest
import torch

from gpu_util import ctx
from paper_1508_02512_amd import qmc

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -53


def _samples(fn, rng, n=1 << 20):
    u = rng.uniform
    if fn == qmc.QMC_MATH_LN:
        parts = [10.0 ** u(-307, 307, n), 1.0 + u(-1e-3, 1e-3, n), u(0.0, 1.0, n),
                 1.0 + 10.0 ** u(-16, -1, n) * rng.choice([-1, 1], n),
                 np.sqrt(0.5) * (1.0 + u(-1e-6, 1e-6, n)), 2.0 ** rng.integers(-1000, 1000, n)]
    elif fn == qmc.QMC_MATH_LN1P:
        parts = [-1.0 + 10.0 ** u(-15, 0, n), 10.0 ** u(-300, 0, n) * rng.choice([-1, 1], n),
                 10.0 ** u(0, 12, n), u(-0.5, 1.0, n)]
    elif fn == qmc.QMC_MATH_EXP:
        parts = [u(-700, 700, n), u(-1, 1, n), 10.0 ** u(-300, 0, n) * rng.choice([-1, 1], n),
                 np.log(2.0) / 2 * (1.0 + u(-1e-9, 1e-9, n)) * rng.choice([-1, 1], n)]
    elif fn == qmc.QMC_MATH_RCP:
        parts = [10.0 ** u(-300, 300, n) * rng.choice([-1, 1], n), u(0.5, 2.0, n),
                 1.0 + u(-1e-12, 1e-12, n), u(1.0, 3.0, n)]
    else:
        parts = [u(-40, 40, n), 10.0 ** u(-300, 0, n) * rng.choice([-1, 1], n),
                 np.log(2.0) / 2 * (1.0 + u(-1e-9, 1e-9, n)) * rng.choice([-1, 1], n),
                 u(-0.5, 0.5, n)]
    x = np.concatenate(parts)
    return x[np.isfinite(x) & (x != 0.0) if fn == qmc.QMC_MATH_LN else np.isfinite(x)]


def _reference(fn, x):
    xl = x.astype(np.longdouble)
    return {qmc.QMC_MATH_LN: np.log, qmc.QMC_MATH_LN1P: np.log1p,
            qmc.QMC_MATH_EXP: np.exp, qmc.QMC_MATH_EXPM1: np.expm1,
            qmc.QMC_MATH_RCP: lambda v: 1 / v}[fn](xl)


@pytest.mark.parametrize("fn,bound_ulp", [(qmc.QMC_MATH_LN, 2.0), (qmc.QMC_MATH_LN1P, 3.0),
                                          (qmc.QMC_MATH_EXP, 2.0), (qmc.QMC_MATH_EXPM1, 3.0),
                                          (qmc.QMC_MATH_RCP, 2.0)])
def test_relative_error(fn, bound_ulp):
    print(f"math: fn {fn}", flush=True)
    rng = np.random.default_rng(fn)
    x = _samples(fn, rng)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx().math_eval(fn, xd.data_ptr(), yd.data_ptr(), xd.numel())
    y = yd.cpu().numpy()
    ref = _reference(fn, x)
    keep = np.abs(ref) >= np.longdouble(2.0 ** -1021)      # normal results only
    rel = np.abs((y[keep].astype(np.longdouble) - ref[keep]) / ref[keep])
    worst = float(rel.max()) / ULP
    print(f"max error {worst:.2f} ulp over {keep.sum()} values", flush=True)
    assert worst <= bound_ulp
    # the kernels rely on exact special values
    if fn == qmc.QMC_MATH_LN:
        one = torch.tensor([1.0, 2.0, 0.5], dtype=torch.float64, device="cuda")
        out = torch.empty_like(one)
        ctx().math_eval(fn, one.data_ptr(), out.data_ptr(), 3)
        assert out[0].item() == 0.0
        assert out[1].item() == np.log(2.0) and out[2].item() == -np.log(2.0)


F32 = {qmc.QMC_MATH_LN_F32: qmc.QMC_MATH_LN, qmc.QMC_MATH_LN1P_F32: qmc.QMC_MATH_LN1P,
       qmc.QMC_MATH_EXP_F32: qmc.QMC_MATH_EXP, qmc.QMC_MATH_EXPM1_F32: qmc.QMC_MATH_EXPM1}


def _samples_f32(fn, rng, n=1 << 20):
    u = rng.uniform
    sign = lambda: rng.choice([-1, 1], n)
    if fn == qmc.QMC_MATH_LN_F32:
        parts = [10.0 ** u(-44, 38, n), 1.0 + u(-1e-3, 1e-3, n), u(0.0, 1.0, n),
                 1.0 + 10.0 ** u(-7, -1, n) * sign(), 2.0 ** rng.integers(-149, 127, n)]
    elif fn == qmc.QMC_MATH_LN1P_F32:
        parts = [-1.0 + 10.0 ** u(-7, 0, n), 10.0 ** u(-37, 0, n) * sign(),
                 10.0 ** u(0, 30, n), u(-0.5, 1.0, n)]
    elif fn == qmc.QMC_MATH_EXP_F32:
        parts = [u(-87, 88, n), u(-1, 1, n), 10.0 ** u(-37, 0, n) * sign(),
                 u(-103, -87, n)]
    else:
        parts = [u(-40, 40, n), 10.0 ** u(-37, 0, n) * sign(), u(-0.5, 0.5, n),
                 u(-12, 12, n)]
    x = np.concatenate(parts).astype(np.float32).astype(np.float64)
    ok = np.isfinite(x) & (x > -1.0 if fn == qmc.QMC_MATH_LN1P_F32 else True)
    return x[ok & (x > 0.0) if fn == qmc.QMC_MATH_LN_F32 else ok]


@pytest.mark.parametrize("fn,bound_ulp", [(qmc.QMC_MATH_LN_F32, 4.0),
                                          (qmc.QMC_MATH_LN1P_F32, 8.0),
                                          (qmc.QMC_MATH_EXP_F32, 4.0),
                                          (qmc.QMC_MATH_EXPM1_F32, 10.0)])
def test_relative_error_float(fn, bound_ulp):
    """The float versions of FP32 evaluation (hardware base-2 log and exp
    with Goldberg's log1p and Kahan's expm1), on inputs that are floats,
    against the extended-precision host library; normal float results.
    Errors in units of 2^-24 relative (one ulp is 1 to 2 of them)."""
    print(f"math: float fn {fn}", flush=True)
    rng = np.random.default_rng(fn)
    x = _samples_f32(fn, rng)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx().math_eval(fn, xd.data_ptr(), yd.data_ptr(), xd.numel())
    y = yd.cpu().numpy()
    assert np.all(y == y.astype(np.float32))      # float results
    ref = _reference(F32[fn], x)
    keep = (np.abs(ref) >= np.longdouble(2.0 ** -126)) & (np.abs(ref) < np.longdouble(2.0 ** 127))
    rel = np.abs((y[keep].astype(np.longdouble) - ref[keep]) / ref[keep])
    worst = float(rel.max()) / 2.0 ** -24
    print(f"max error {worst:.2f} ulp over {keep.sum()} values", flush=True)
    assert worst <= bound_ulp
    if fn == qmc.QMC_MATH_LN_F32:
        one = torch.tensor([1.0, 2.0 ** -140], dtype=torch.float64, device="cuda")
        out = torch.empty_like(one)
        ctx().math_eval(fn, one.data_ptr(), out.data_ptr(), 2)
        assert out[0].item() == 0.0
        assert abs(out[1].item() - (-140 * np.log(2.0))) <= 2 * 2.0 ** -24 * 140 * np.log(2.0)


def test_bad_arguments_raise():
    with pytest.raises(qmc.QMCError):
        ctx().math_eval(9, 0, 0, 1)
    with pytest.raises(qmc.QMCError):
        ctx().math_eval(0, 0, 0, -1)
