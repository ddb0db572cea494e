"""Thin ctypes binding of libqmc (include/qmc.h): argument marshalling only.

Every function of the C ABI is exposed under its own name (``qmc_create``,
``qmc_plan_sectors``, ``qmc_integrate`` ...).  The classes ``Context`` and
``Plan`` wrap them for numpy inputs.  The library must have been built
(``python -m paper_1508_02512_amd.build``); there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmc.so")

QMC_OK, QMC_PENDING = 0, 1
ERRORS = {-1: "QMC_EINVAL", -2: "QMC_EUNREGULATED", -3: "QMC_EUNSUPPORTED",
          -4: "QMC_ENOMEM", -5: "QMC_EBUDGET", -6: "QMC_EDEFORM",
          -7: "QMC_ENOTCONVERGED", -8: "QMC_EDEVICE", -9: "QMC_ECANCELLED"}
(QMC_EINVAL, QMC_EUNREGULATED, QMC_EUNSUPPORTED, QMC_ENOMEM, QMC_EBUDGET, QMC_EDEFORM,
 QMC_ENOTCONVERGED, QMC_EDEVICE, QMC_ECANCELLED) = range(-1, -10, -1)
QMC_FP64, QMC_FP32_EVAL = 0, 1
QMC_POLES_SUBTRACT, QMC_POLES_IBP = 0, 1
QMC_MAX_POLES = 4
QMC_MATH_LN, QMC_MATH_LN1P, QMC_MATH_EXP, QMC_MATH_EXPM1, QMC_MATH_RCP = 0, 1, 2, 3, 4
QMC_MATH_LN_F32, QMC_MATH_LN1P_F32, QMC_MATH_EXP_F32, QMC_MATH_EXPM1_F32 = 5, 6, 7, 8
QMC_MAX_DIM = 8
QMC_MAX_ORDERS = 8
QMC_MAX_FACTORS = 4
QMC_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

P = C.POINTER


class qmc_poly(C.Structure):
    _fields_ = [("n_terms", C.c_int32), ("exps", P(C.c_uint8)), ("coef", P(C.c_double))]


class qmc_sector(C.Structure):
    _fields_ = [("dim", C.c_int32), ("mono_a", P(C.c_double)), ("mono_b", P(C.c_double)),
                ("U", qmc_poly), ("F", qmc_poly), ("u_exp", C.c_double * 2),
                ("f_exp", C.c_double * 2), ("coef_re", C.c_double), ("coef_im", C.c_double)]


class qmc_problem(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("sectors", P(qmc_sector)), ("n_inv", C.c_int32),
                ("eps_lo", C.c_int32), ("eps_hi", C.c_int32), ("prefactor", P(C.c_double)),
                ("eps_pref_lo", C.c_int32), ("n_pref", C.c_int32)]


class qmc_plan_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("korobov_r", C.c_int32), ("lambda_", C.c_double),
                ("points_per_lane", C.c_int32), ("pole_method", C.c_int32)]


class qmc_lattice(C.Structure):
    _fields_ = [("n", C.c_uint64), ("z", P(C.c_uint32))]


class qmc_coeff(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double), ("err_re", C.c_double),
                ("err_im", C.c_double)]


class qmc_plan_info(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("n_inv", C.c_int32), ("sec_lo", C.c_int32),
                ("sec_orders", C.c_int32), ("eps_lo", C.c_int32), ("eps_hi", C.c_int32),
                ("max_poles", C.c_int32), ("deform", C.c_int32),
                ("flops_per_point", C.c_double), ("n_input_sectors", C.c_int32),
                ("max_factors", C.c_int32)]


class qmc_sector_info(C.Structure):
    _fields_ = [("origin", C.c_int32), ("dim", C.c_int32), ("poles", C.c_int32),
                ("factors", C.c_int32), ("u_exp", C.c_double * 2), ("f_exp", C.c_double * 2),
                ("coef", (C.c_double * 2) * QMC_MAX_ORDERS), ("coef_lo", C.c_int32)]


class qmc_result(C.Structure):
    _fields_ = [("coeff", P(qmc_coeff)), ("per_shift", P(C.c_double)),
                ("sector_sums", P(C.c_double)), ("evals", C.c_uint64), ("n_final", C.c_uint64),
                ("status", C.c_int32), ("deform_violations", C.c_int32),
                ("kernel_ms", C.c_double), ("algo_flops", C.c_double),
                ("latency_ms", C.c_double), ("steps", C.c_int32), ("lambda_halvings", C.c_int32)]


class qmc_tune_choice(C.Structure):
    _fields_ = [("poles", C.c_int32), ("width", C.c_int32), ("points_per_lane", C.c_int32),
                ("grid_per_cu", C.c_int32), ("occupancy_variant", C.c_int32),
                ("pad", C.c_int32), ("ms", C.c_double)]


class qmc_class_stat(C.Structure):
    _fields_ = [("poles", C.c_int32), ("width", C.c_int32), ("points_per_lane", C.c_int32),
                ("grid", C.c_int32), ("items", C.c_int32), ("precision", C.c_int32),
                ("evals", C.c_uint64), ("algo_flops", C.c_double), ("ms", C.c_double),
                ("variant", C.c_int32), ("pad", C.c_int32)]


class qmc_request(C.Structure):
    _fields_ = [("kin", P(C.c_double)), ("rel_err_target", C.c_double), ("n0", C.c_uint64),
                ("n_max", C.c_uint64), ("m", C.c_int32), ("seed", C.c_uint64),
                ("z", P(C.c_uint32)), ("lambda_halvings", C.c_int32), ("pad", C.c_int32)]


_SIGS = {
    "qmc_create": (C.c_int, [C.c_int, C.c_size_t, C.c_int, P(C.c_void_p)]),
    "qmc_destroy": (None, [C.c_void_p]),
    "qmc_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "qmc_last_error": (C.c_char_p, [C.c_void_p]),
    "qmc_plan_sectors": (C.c_int, [C.c_void_p, P(qmc_problem), P(qmc_plan_opts),
                                   P(C.c_void_p)]),
    "qmc_plan_free": (None, [C.c_void_p]),
    "qmc_plan_get_info": (C.c_int, [C.c_void_p, P(qmc_plan_info)]),
    "qmc_plan_sector_info": (C.c_int, [C.c_void_p, C.c_int32, P(qmc_sector_info)]),
    "qmc_integrate": (C.c_int, [C.c_void_p, C.c_void_p, P(C.c_double), C.c_int32,
                                P(qmc_lattice), P(qmc_lattice), P(C.c_double), C.c_int32,
                                P(qmc_result)]),
    "qmc_size_lattices": (C.c_int, [C.c_void_p, C.c_void_p, P(C.c_double), P(qmc_lattice),
                                    P(C.c_double), C.c_int32, C.c_uint64, P(C.c_uint64),
                                    C.c_int32, P(C.c_uint64)]),
    "qmc_integrate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, P(C.c_double), C.c_int32,
                                        P(qmc_lattice), P(qmc_lattice), P(C.c_double),
                                        C.c_int32, P(qmc_result)]),
    "qmc_bind": (C.c_int, [C.c_void_p, C.c_void_p, P(C.c_double), C.c_int32,
                           P(qmc_lattice), P(qmc_lattice), P(C.c_double), C.c_int32,
                           P(C.c_void_p)]),
    "qmc_run": (C.c_int, [C.c_void_p]),
    "qmc_fetch": (C.c_int, [C.c_void_p, P(qmc_result)]),
    "qmc_job_free": (None, [C.c_void_p]),
    "qmc_job_set_graph": (C.c_int, [C.c_void_p, C.c_int]),
    "qmc_job_set_variant": (C.c_int, [C.c_void_p, C.c_int32]),
    "qmc_job_set_profiling": (C.c_int, [C.c_void_p, C.c_int]),
    "qmc_job_class_stats": (C.c_int, [C.c_void_p, P(qmc_class_stat), C.c_int32,
                                      P(C.c_int32)]),
    "qmc_autotune": (C.c_int, [C.c_void_p, C.c_void_p, P(C.c_double), C.c_int32,
                               P(qmc_lattice), P(qmc_lattice), P(C.c_double), C.c_int32,
                               P(qmc_tune_choice), C.c_int32, P(C.c_int32)]),
    "qmc_math_eval": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64]),
    "qmc_submit": (C.c_int, [C.c_void_p, C.c_void_p, P(qmc_request), P(C.c_uint64)]),
    "qmc_poll": (C.c_int, [C.c_void_p, C.c_uint64, P(qmc_result)]),
    "qmc_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double, P(qmc_result)]),
    "qmc_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "qmc_release": (C.c_int, [C.c_void_p, C.c_uint64]),
}

_lib = None


def lib():
    """Load libqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1508_02512_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def __getattr__(name):          # module-level qmc_* names map to the C functions
    if name in _SIGS:
        return getattr(lib(), name)
    raise AttributeError(name)


class QMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(P(C.c_double))


class Context:
    def __init__(self, device=0, hbm_budget=0, max_slots=0, stream=None):
        self.h = C.c_void_p()
        rc = lib().qmc_create(device, hbm_budget, max_slots, C.byref(self.h))
        if rc != QMC_OK:
            raise QMCError(rc, "qmc_create failed")
        if stream is not None:
            self.check(lib().qmc_set_stream(self.h, C.c_void_p(stream)))

    def check(self, rc):
        if rc < 0:
            raise QMCError(rc, lib().qmc_last_error(self.h).decode())
        return rc

    def math_eval(self, fn, x_ptr, y_ptr, n):
        """The kernels' elementary function fn (QMC_MATH_*) on n device doubles."""
        self.check(lib().qmc_math_eval(self.h, fn, C.c_void_p(x_ptr), C.c_void_p(y_ptr), n))

    def close(self):
        if self.h:
            lib().qmc_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan(self, sectors, info, eps_hi, prefactor, lam=0.0, korobov_r=2,
             precision=QMC_FP64, points_per_lane=0, D=None, pole_method=QMC_POLES_SUBTRACT):
        """qmc_plan_sectors: sectors as frontend.sector_arrays gives them,
        results up to eps^eps_hi, prefactor (lowest order, coefficients);
        lam > 0 deforms the contour; pole_method QMC_POLES_IBP integrates
        the poles by parts instead of subtracting them."""
        return Plan(self, sectors, info, eps_hi, prefactor, lam, korobov_r, precision,
                    points_per_lane, D, pole_method)


class Plan:
    """Sector tables planned and resident on the device."""

    def __init__(self, ctx, sectors, info, eps_hi, prefactor, lam, korobov_r, precision,
                 points_per_lane, D, pole_method=QMC_POLES_SUBTRACT):
        self.ctx = ctx
        self.keep = []
        ns = len(sectors)
        arr = (qmc_sector * ns)()
        ni = len(info["invariants"])
        for i, s in enumerate(sectors):
            r = arr[i]
            r.dim = s["dim"]
            for key in ("a", "b", "EU", "CU", "EF", "CF"):
                self.keep.append(s[key])
            r.mono_a, r.mono_b = _dptr(s["a"]), _dptr(s["b"])
            for name, E, Cm in (("U", s["EU"], s["CU"]), ("F", s["EF"], s["CF"])):
                poly = getattr(r, name)
                poly.n_terms = E.shape[0]
                poly.exps = E.ctypes.data_as(P(C.c_uint8))
                poly.coef = _dptr(Cm)
            r.u_exp[0], r.u_exp[1] = s["u"]
            r.f_exp[0], r.f_exp[1] = s["f"]
            d = s.get("D", 1.0) if D is None else complex(D[i])
            r.coef_re, r.coef_im = complex(d).real, complex(d).imag
        pref_lo, pref = prefactor
        pref = np.asarray(pref, dtype=complex)
        self.pref_arr = np.ascontiguousarray(np.stack([pref.real, pref.imag], axis=1))
        self.sectors_arr = arr
        prob = qmc_problem()
        prob.n_sectors = ns
        prob.sectors = arr
        prob.n_inv = ni
        self.n_inv = ni
        prob.eps_hi = eps_hi
        prob.eps_pref_lo = pref_lo
        prob.n_pref = len(pref)
        prob.prefactor = _dptr(self.pref_arr)
        # lowest order of the result: -max poles + prefactor's lowest order;
        # integration by parts (Eq. 13) can turn an integer a_j < -1 into a
        # pole, so every integer a_j <= -1 counts
        max_poles = max(int(np.sum((s["a"] <= -1.0) & (s["a"] == np.floor(s["a"]))))
                        for s in sectors)
        prob.eps_lo = -max_poles + pref_lo
        opts = qmc_plan_opts(precision, korobov_r, float(lam), points_per_lane, pole_method)
        self.h = C.c_void_p()
        ctx.check(lib().qmc_plan_sectors(ctx.h, C.byref(prob), C.byref(opts),
                                         C.byref(self.h)))
        self.info = qmc_plan_info()
        ctx.check(lib().qmc_plan_get_info(self.h, C.byref(self.info)))
        self.n_input_sectors = ns
        self.n_sectors = self.info.n_sectors      # after Eq. 13

    def sector_info(self, s):
        """Planned sector s: origin, dim, poles, factors, u, f, the
        coefficient series C(eps) (complex array, orders C_lo ..) and C_lo."""
        out = qmc_sector_info()
        self.ctx.check(lib().qmc_plan_sector_info(self.h, int(s), C.byref(out)))
        return {"origin": out.origin, "dim": out.dim, "poles": out.poles,
                "factors": out.factors, "u": tuple(out.u_exp), "f": tuple(out.f_exp),
                "C": np.array([complex(out.coef[k][0], out.coef[k][1])
                               for k in range(QMC_MAX_ORDERS)]),
                "C_lo": out.coef_lo}

    def close(self):
        if self.h:
            lib().qmc_plan_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def orders(self):
        return list(range(self.info.eps_lo, self.info.eps_hi + 1))

    def _lattice(self, n, z):
        z = np.ascontiguousarray(z, dtype=np.uint32)
        assert z.shape == (QMC_MAX_DIM,)
        self.keep.append(z)
        return qmc_lattice(int(n), z.ctypes.data_as(P(C.c_uint32)))

    def _inputs(self, kin, lattice, shifts, lat_per_sector):
        kin = np.ascontiguousarray(np.atleast_2d(kin), dtype=np.float64)
        assert kin.shape[1] == self.n_inv
        shifts = np.ascontiguousarray(shifts, dtype=np.float64)
        assert shifts.ndim == 2 and shifts.shape[1] == QMC_MAX_DIM
        lat = self._lattice(*lattice) if lattice is not None else None
        lps = None
        if lat_per_sector is not None:
            lps = (qmc_lattice * self.n_sectors)()
            for i, (n, z) in enumerate(lat_per_sector):
                lps[i] = self._lattice(n, z)
        return kin, shifts, lat, lps

    def _result(self, n_points, m, sector_sums, per_shift):
        no = len(self.orders)
        coeff = (qmc_coeff * (n_points * no))()
        res = qmc_result()
        res.coeff = coeff
        ss = ps = None
        if sector_sums:
            ss = np.zeros((n_points, self.n_sectors, m, self.info.sec_orders, 2))
            res.sector_sums = _dptr(ss)
        if per_shift:
            ps = np.zeros((n_points, m, no, 2))
            res.per_shift = _dptr(ps)
        return res, coeff, ss, ps

    def _pack(self, res, coeff, ss, ps, n_points):
        no = len(self.orders)
        arr = np.array([[c.re, c.im, c.err_re, c.err_im] for c in coeff]).reshape(n_points, no, 4)
        out = {"orders": self.orders, "mean": arr[..., 0] + 1j * arr[..., 1],
               "err_re": arr[..., 2], "err_im": arr[..., 3], "evals": res.evals,
               "status": res.status, "violations": res.deform_violations,
               "kernel_ms": res.kernel_ms, "algo_flops": res.algo_flops}
        if ss is not None:
            out["sector_sums"] = ss[..., 0] + 1j * ss[..., 1]
            out["sec_lo"] = self.info.sec_lo
        if ps is not None:
            out["per_shift"] = ps[..., 0] + 1j * ps[..., 1]
        return out

    def integrate(self, kin, lattice, shifts, lat_per_sector=None, sector_sums=False,
                  per_shift=False, allow_violations=False, noalloc=False):
        """lattice = (n, z[8]); shifts [m][8]; kin [n_points][n_inv].
        noalloc=True calls qmc_integrate_noalloc instead of qmc_integrate."""
        kin, shifts, lat, lps = self._inputs(kin, lattice, shifts, lat_per_sector)
        res, coeff, ss, ps = self._result(kin.shape[0], shifts.shape[0], sector_sums,
                                          per_shift)
        fn = lib().qmc_integrate_noalloc if noalloc else lib().qmc_integrate
        rc = fn(self.ctx.h, self.h, _dptr(kin), kin.shape[0],
                C.byref(lat) if lat is not None else None, lps,
                _dptr(shifts), shifts.shape[0], C.byref(res))
        if rc < 0 and not (allow_violations and rc == -6):
            self.ctx.check(rc)
        return self._pack(res, coeff, ss, ps, kin.shape[0])

    def bind(self, kin, lattice, shifts, lat_per_sector=None):
        return Job(self, kin, lattice, shifts, lat_per_sector)

    def autotune(self, kin, lattice, shifts, lat_per_sector=None):
        """Time launch shapes per kernel class; later binds use the best."""
        kin, shifts, lat, lps = self._inputs(kin, lattice, shifts, lat_per_sector)
        ch = (qmc_tune_choice * 64)()
        n = C.c_int32()
        self.ctx.check(lib().qmc_autotune(self.ctx.h, self.h, _dptr(kin), kin.shape[0],
                                          C.byref(lat) if lat is not None else None, lps,
                                          _dptr(shifts), shifts.shape[0], ch, 64, C.byref(n)))
        return [{"poles": c.poles, "width": c.width, "points_per_lane": c.points_per_lane,
                 "grid_per_cu": c.grid_per_cu, "occupancy_variant": c.occupancy_variant,
                 "ms": c.ms} for c in ch[:min(n.value, 64)]]


class Request:
    """Handle of one served request (continuous batching, see qmc.h)."""

    def __init__(self, plan, ticket):
        self.plan, self.ticket = plan, ticket

    def _result(self):
        res, coeff, _, _ = self.plan._result(1, 2, False, False)
        return res, coeff

    def wait(self, timeout=-1.0):
        res, coeff = self._result()
        rc = lib().qmc_wait(self.plan.ctx.h, self.ticket, float(timeout), C.byref(res))
        if rc == QMC_PENDING:
            return None
        out = self.plan._pack(res, coeff, None, None, 1)
        out["rc"] = rc
        out["latency_ms"] = res.latency_ms
        out["steps"] = res.steps
        out["n_final"] = res.n_final
        out["lambda_halvings"] = res.lambda_halvings
        return out

    def poll(self):
        res, coeff = self._result()
        rc = lib().qmc_poll(self.plan.ctx.h, self.ticket, C.byref(res))
        if rc == QMC_PENDING:
            return None
        out = self.plan._pack(res, coeff, None, None, 1)
        out.update(rc=rc, latency_ms=res.latency_ms, steps=res.steps, n_final=res.n_final,
                   lambda_halvings=res.lambda_halvings)
        return out

    def cancel(self):
        self.plan.ctx.check(lib().qmc_cancel(self.plan.ctx.h, self.ticket))

    def release(self):
        lib().qmc_release(self.plan.ctx.h, self.ticket)


def submit(plan, kin, target, n0, n_max, m, seed, z, lambda_halvings=0):
    """Queue one request of `plan` at kinematic vector `kin`."""
    kin = np.ascontiguousarray(kin, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.uint32)
    req = qmc_request(_dptr(kin), float(target), int(n0), int(n_max), int(m), int(seed),
                      z.ctypes.data_as(P(C.c_uint32)), int(lambda_halvings), 0)
    t = C.c_uint64()
    plan.ctx.check(lib().qmc_submit(plan.ctx.h, plan.h, C.byref(req), C.byref(t)))
    return Request(plan, t.value)


class Job:
    """Inputs resident on the device; run() enqueues, fetch() waits."""

    def __init__(self, plan, kin, lattice, shifts, lat_per_sector):
        self.plan = plan
        self.kin, self.shifts, lat, lps = plan._inputs(kin, lattice, shifts, lat_per_sector)
        self.h = C.c_void_p()
        plan.ctx.check(lib().qmc_bind(plan.ctx.h, plan.h, _dptr(self.kin), self.kin.shape[0],
                                      C.byref(lat) if lat is not None else None, lps,
                                      _dptr(self.shifts), self.shifts.shape[0],
                                      C.byref(self.h)))

    def run(self):
        self.plan.ctx.check(lib().qmc_run(self.h))

    def use_graph(self, enable=True):
        self.plan.ctx.check(lib().qmc_job_set_graph(self.h, int(enable)))

    def set_variant(self, variant):
        """Run every kernel class with occupancy build `variant` (0 or 1)."""
        self.plan.ctx.check(lib().qmc_job_set_variant(self.h, int(variant)))

    def profile(self, enable=True):
        """Time every kernel-class launch of later eager runs."""
        self.plan.ctx.check(lib().qmc_job_set_profiling(self.h, int(enable)))

    def class_stats(self):
        """One dict per kernel launch of a run: class, shape, evaluations,
        algorithmic flops and the launch time of the last fetched run."""
        n = C.c_int32()
        self.plan.ctx.check(lib().qmc_job_class_stats(self.h, None, 0, C.byref(n)))
        arr = (qmc_class_stat * max(n.value, 1))()
        self.plan.ctx.check(lib().qmc_job_class_stats(self.h, arr, n.value, C.byref(n)))
        return [{f: getattr(arr[i], f) for f, _ in qmc_class_stat._fields_}
                for i in range(n.value)]

    def fetch(self, sector_sums=False, per_shift=False):
        n_points, m = self.kin.shape[0], self.shifts.shape[0]
        res, coeff, ss, ps = self.plan._result(n_points, m, sector_sums, per_shift)
        self.plan.ctx.check(lib().qmc_fetch(self.h, C.byref(res)))
        return self.plan._pack(res, coeff, ss, ps, n_points)

    def close(self):
        if self.h:
            lib().qmc_job_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def size_lattices(plan, kin, total_points, sizes, pilot_n, pilot_z, shifts):
    """Per-sector lattice sizes for a total budget of lattice points: the
    library's variance-weighted sizing (qmc_size_lattices) from a pilot run
    at n = pilot_n; every size is one of `sizes`."""
    kin = np.ascontiguousarray(np.atleast_2d(kin)[0], dtype=np.float64)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    avail = np.ascontiguousarray(sorted(sizes), dtype=np.uint64)
    out = np.zeros(plan.n_sectors, dtype=np.uint64)
    pilot = plan._lattice(pilot_n, pilot_z)
    plan.ctx.check(lib().qmc_size_lattices(
        plan.ctx.h, plan.h, _dptr(kin), C.byref(pilot), _dptr(shifts), shifts.shape[0],
        int(total_points), avail.ctypes.data_as(P(C.c_uint64)), len(avail),
        out.ctypes.data_as(P(C.c_uint64))))
    return [int(v) for v in out]
