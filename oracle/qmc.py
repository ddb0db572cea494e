"""Oracle driver: lattice sums per sector, Laurent assembly, mean and error.
TEST INFRASTRUCTURE: only tests, the smoke check and the CPU baseline of the
benchmark use this module.

Section III: for each shift k the estimate is Q_k = (1/n) sum_i f(x_i + Delta_k)
(Eq. 18); the result is the mean over shifts (Eq. 19) with the unbiased
mean-square-error estimate sum_k (Q_k - Qbar)^2 / (m (m-1)) (Eq. 20), applied
separately to real and imaginary parts.  The Laurent coefficients of the
integral are (Eq. 5 with Eq. 9)

    I(eps) = Gamma(N_nu - L D/2) / prod Gamma(nu_j) * sum_sectors D_s I_s(eps),

so the per-shift estimate of every order is the prefactor series times the
sector sum, taken shift by shift before the variance (sectors share shifts).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import mpmath
import numpy as np

from . import ibp
from .decompose import decompose

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIBQ = os.path.join(_HERE, "liboracle_q.so")     # integrand in binary128


class _Sector(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int),
                ("a", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double)),
                ("nU", ctypes.c_int),
                ("eU", ctypes.POINTER(ctypes.c_int32)),
                ("cU", ctypes.POINTER(ctypes.c_double)),
                ("nF", ctypes.c_int),
                ("eF", ctypes.POINTER(ctypes.c_int32)),
                ("cF", ctypes.POINTER(ctypes.c_double)),
                ("u0", ctypes.c_double), ("u1", ctypes.c_double),
                ("f0", ctypes.c_double), ("f1", ctypes.c_double),
                ("nP", ctypes.c_int),
                ("nPt", ctypes.POINTER(ctypes.c_int32)),
                ("eP", ctypes.POINTER(ctypes.c_int32)),
                ("cP", ctypes.POINTER(ctypes.c_double))]


def build() -> str:
    """Compile the C oracle with gcc (OpenMP): FP64 and binary128 builds."""
    base = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-D_DEFAULT_SOURCE"]
    subprocess.run(base + ["-o", _LIB, _SRC, "-lm"], check=True)
    subprocess.run(base + ["-DORACLE_QUAD", "-o", _LIBQ, _SRC, "-lquadmath", "-lm"],
                   check=True)
    return _LIB


_libs = {}


def lib(quad=False):
    """The FP64 oracle library, or the binary128 build when quad=True."""
    path = _LIBQ if quad else _LIB
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        L.oracle_sector_sums.argtypes = [
            P(_Sector), ctypes.c_uint64, P(ctypes.c_uint32), P(ctypes.c_double),
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double),
            P(ctypes.c_int64), ctypes.c_int]
        L.oracle_sector_sums.restype = ctypes.c_int
        L.oracle_point.argtypes = [P(_Sector), P(ctypes.c_double), ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, P(ctypes.c_double)]
        L.oracle_point.restype = ctypes.c_int
        L.oracle_psi.argtypes = [ctypes.c_double, ctypes.c_int]
        L.oracle_psi.restype = ctypes.c_double
        L.oracle_omega.argtypes = [ctypes.c_double, ctypes.c_int]
        L.oracle_omega.restype = ctypes.c_double
        _libs[path] = L
    return _libs[path]


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def form_value(form, kin):
    """Value of a linear form {invariant: Fraction} at kinematics kin."""
    return float(sum(Fraction(v) * (1 if k == "1" else Fraction(kin[k]))
                     for k, v in form.items()))


class NumericSector:
    """A sector with its coefficients evaluated at one kinematic point."""

    def __init__(self, sec, info, kin):
        d = len(sec["a"])
        self.dim = d
        self.a = np.array([float(x) for x in sec["a"]])
        self.b = np.array([float(x) for x in sec["b"]])
        self.eU = np.array(sorted(sec["U"]), dtype=np.int32).reshape(-1, d)
        self.cU = np.array([form_value(sec["U"][tuple(e)], kin) for e in self.eU])
        self.eF = np.array(sorted(sec["F"]), dtype=np.int32).reshape(-1, d)
        self.cF = np.array([form_value(sec["F"][tuple(e)], kin) for e in self.eF])
        u = sec.get("u", (info["u0"], info["u1"]))
        f = sec.get("f", (info["f0"], info["f1"]))
        self.u = (float(u[0]), float(u[1]))
        self.f = (float(f[0]), float(f[1]))
        self.nJ = int(np.sum(self.a == -1.0))
        # numerator factors (Eq. 13), all terms of all factors in one table
        P = sec.get("P", [])
        self.nPt = np.array([len(p) for p in P] or [0], dtype=np.int32)
        eP = [e for p in P for e in sorted(p)]
        self.eP = np.array(eP or [[0] * d], dtype=np.int32).reshape(-1, d)
        self.cP = np.array([form_value(p[e], kin) for p in P for e in sorted(p)] or [0.0])
        self.nP = len(P)

    def cstruct(self):
        s = _Sector()
        s.dim = self.dim
        s.a, s.b = _ptr(self.a, ctypes.c_double), _ptr(self.b, ctypes.c_double)
        s.nU, s.nF = len(self.cU), len(self.cF)
        s.eU, s.cU = _ptr(self.eU, ctypes.c_int32), _ptr(self.cU, ctypes.c_double)
        s.eF, s.cF = _ptr(self.eF, ctypes.c_int32), _ptr(self.cF, ctypes.c_double)
        s.u0, s.u1 = self.u
        s.f0, s.f1 = self.f
        s.nP = self.nP
        s.nPt = _ptr(self.nPt, ctypes.c_int32)
        s.eP = _ptr(self.eP, ctypes.c_int32)
        s.cP = _ptr(self.cP, ctypes.c_double)
        return s


def effective_lambda(ns: NumericSector, lam):
    """Deformation parameter lambda_i of Eq. 14 for a sector at its point.

    Eq. 14 is needed only where F can vanish inside the cube: when every
    coefficient of the sector's F is non-negative (its constant term is
    positive) F > 0 on the whole cube and the undeformed contour is used.
    Otherwise the paper leaves lambda to be chosen; it is taken
    dimensionless, lam / max |coefficient of F|, so that one value serves
    all kinematic points and integrals."""
    if not np.any(ns.cF < 0.0):
        return 0.0
    return float(lam) / float(np.max(np.abs(ns.cF)))


def sector_sums(ns: NumericSector, n, z, shifts, r=2, lam=0.0,
                out_lo=0, out_len=1, nthreads=0, quad=False):
    """(sums, abss, counts): sums[m][out_len] complex = sum_i w g (no 1/n).

    quad=True evaluates the integrand in binary128 (same formula)."""
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    m, dmax = shifts.shape
    z = np.ascontiguousarray(z, dtype=np.uint32)
    sums = np.zeros((m, out_len, 2))
    abss = np.zeros((m, out_len, 2))
    counts = np.zeros((m, 3), dtype=np.int64)
    st = ns.cstruct()
    rc = lib(quad).oracle_sector_sums(
        ctypes.byref(st), int(n), _ptr(z, ctypes.c_uint32),
        _ptr(shifts, ctypes.c_double), m, dmax, int(r), float(lam),
        int(out_lo), int(out_len), _ptr(sums, ctypes.c_double),
        _ptr(abss, ctypes.c_double), _ptr(counts, ctypes.c_int64), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sector_sums rejected its arguments")
    return sums[..., 0] + 1j * sums[..., 1], abss, counts


def point_value(ns: NumericSector, t, lam=0.0, out_lo=0, out_len=1, quad=False):
    t = np.ascontiguousarray(t, dtype=np.float64)
    out = np.zeros((out_len, 2))
    st = ns.cstruct()
    rc = lib(quad).oracle_point(ctypes.byref(st), _ptr(t, ctypes.c_double), float(lam),
                            int(out_lo), int(out_len), _ptr(out, ctypes.c_double))
    if rc < 0:
        raise ValueError("oracle_point rejected its arguments")
    return out[:, 0] + 1j * out[:, 1]


def gamma_prefactor(info, lo, hi):
    """Laurent coefficients eps^lo..eps^hi of Gamma(g0 + g1 eps)/prod Gamma(nu)."""
    g0, g1 = (float(x) for x in info["gamma"])
    pole = 1 if (g0 <= 0 and g0 == int(g0)) else 0
    mpmath.mp.dps = 40
    norm = mpmath.mpf(1)
    for nu in info["nus"]:
        norm *= mpmath.gamma(nu)

    def f(e):
        return (e ** pole) * mpmath.gamma(g0 + g1 * e) / norm

    if pole:
        # eps Gamma(x), x = g0 + g1 eps with g0 = -j: the recurrence
        # Gamma(x) = Gamma(x + j + 1) / (x (x+1) ... (x+j)) and x + j = g1 eps
        j = int(-g0)

        def f(e):  # noqa: F811
            x = g0 + g1 * e
            den = mpmath.mpf(1)
            for q in range(0, j):
                den *= (x + q)
            return mpmath.gamma(x + j + 1) / den / g1 / norm
    coeffs = mpmath.taylor(f, 0, hi - lo + pole + 2)
    out = {}
    for p in range(lo, hi + 1):
        idx = p + pole
        out[p] = complex(coeffs[idx]) if 0 <= idx < len(coeffs) else 0j
    return out, -pole


def assemble(per_sector, D, pref, pref_lo, sec_lo, n, eps_lo, eps_hi, tot_lo=None):
    """Per-shift Laurent estimates, mean and error (Eqs. 18-20).

    per_sector: list of arrays [m][K] complex of raw sums (no 1/n), orders
    sec_lo.. ; D: list of sector constants, each a number or a Laurent
    series {order: coefficient} in eps (the coefficient C(eps) of a sector
    from Eq. 13); pref: dict order->coeff.  The sum over sectors of C(eps)
    times the sector's series is kept from order tot_lo (default sec_lo;
    lower when some C(eps) starts below eps^0) up to eps_hi - pref_lo.
    """
    m = per_sector[0].shape[0]
    K = per_sector[0].shape[1]
    if tot_lo is None:
        tot_lo = sec_lo
    Kt = eps_hi - pref_lo - tot_lo + 1
    tot = np.zeros((m, Kt), dtype=complex)
    for S, Ds in zip(per_sector, D):
        ser = Ds if isinstance(Ds, dict) else {0: Ds}
        for e, c in ser.items():
            for i in range(K):
                j = sec_lo + i + e - tot_lo
                if 0 <= j < Kt:
                    tot[:, j] += complex(c) * S[:, i] / float(n)
    orders = list(range(eps_lo, eps_hi + 1))
    Q = np.zeros((m, len(orders)), dtype=complex)
    for qi, p in enumerate(orders):
        for j in range(Kt):
            ps = tot_lo + j
            pp = p - ps
            if pp in pref:
                Q[:, qi] += pref[pp] * tot[:, j]
    mean = Q.mean(axis=0)
    err_re = np.sqrt(np.sum((Q.real - mean.real) ** 2, axis=0) / (m * (m - 1))) if m > 1 else np.zeros(len(orders))
    err_im = np.sqrt(np.sum((Q.imag - mean.imag) ** 2, axis=0) / (m * (m - 1))) if m > 1 else np.zeros(len(orders))
    return {"orders": orders, "mean": mean, "err_re": err_re, "err_im": err_im,
            "per_shift": Q}


def integrate(problem, kin, n, z, shifts, r=2, lam=0.0, eps_hi=0, nthreads=0,
              sectors=None, quad=False, poles="subtract"):
    """Whole-problem oracle estimate: dict with orders, mean, errors.

    poles="subtract" takes the poles a_j = -1 out by the subtraction of
    Eq. 11 (integration by parts only below -1); poles="ibp" takes them out
    by the integration by parts of Eq. 13 as well."""
    if poles not in ("subtract", "ibp"):
        raise ValueError(f"unknown pole method {poles!r}")
    if sectors is None:
        sectors, info = decompose(problem)
    else:
        sectors, info = sectors
    by_parts = poles == "ibp"
    if ibp.needs_ibp(sectors, by_parts):
        sectors = ibp.expand(sectors, info, by_parts)
    nums = [NumericSector(s, info, kin) for s in sectors]
    kmax = max(ns.nJ for ns in nums)
    # lowest order of the coefficient series C(eps) (below 0 after Eq. 13 at -1)
    c_lo = min([0] + [min(s["C"]) for s in sectors if "C" in s and s["C"]])
    pref_probe, pref_lo = gamma_prefactor(info, -2, eps_hi + kmax - c_lo + 2)
    sec_lo = -kmax
    sec_hi = eps_hi - pref_lo - c_lo
    K = sec_hi - sec_lo + 1
    per = []
    counts = np.zeros(3, dtype=np.int64)
    for ns in nums:
        S, _, c = sector_sums(ns, n, z, shifts, r, effective_lambda(ns, lam), sec_lo, K,
                              nthreads, quad)
        per.append(S)
        counts += c.sum(axis=0)
    eps_lo = sec_lo + c_lo + pref_lo
    res = assemble(per, [s["C"] if "C" in s else float(s.get("D", 1)) for s in sectors],
                   pref_probe, pref_lo, sec_lo, n, eps_lo, eps_hi, sec_lo + c_lo)
    res["sector_sums"] = per
    res["counts"] = counts
    res["sec_lo"] = sec_lo
    return res
