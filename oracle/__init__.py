"""FP64 CPU oracle of the chemistry advance -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library neither imports nor links it, and the
two share no code: the only common inputs are the seeded generators in
``synth``.  See ``chem_oracle.c`` for the equations (paper Sec. II.B, Eqs. 1-2,
with the textbook rate laws written out there) and ``ann.py`` for the learned
part (Sec. II.B: inputs, Box-Cox transform Eq. 7, MLP with GELU, Adam, loss
Eq. 8).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP, -O2, no hand SIMD)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def default_threads() -> int:
    """Host threads for the oracle: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when set (oversubscribed spinning threads slow it down)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


class _Mech(C.Structure):
    _fields_ = [("E", C.c_int32), ("K", C.c_int32), ("R", C.c_int32),
                ("emass", C.c_void_p), ("comp", C.c_void_p), ("nasa", C.c_void_p),
                ("reac", C.c_void_p), ("prod", C.c_void_p), ("lnA", C.c_void_p),
                ("beta", C.c_void_p), ("Ea", C.c_void_p), ("tb", C.c_void_p),
                ("rev", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("h0_frac", C.c_double), ("max_steps", C.c_int32), ("project", C.c_int32),
                ("newton_T", C.c_int32)]


_lib = None


def lib():
    """The oracle library (built on first use)."""
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def load(path):
    """A build of chem_oracle.c at `path` with its call signatures set (the
    reference build, or a variant compiled by a test)."""
    L = C.CDLL(path)
    mp = C.POINTER(_Mech)
    L.or_molar_mass.restype = C.c_double
    L.or_molar_mass.argtypes = [mp, C.c_int]
    L.or_species_thermo.argtypes = [mp, C.c_double, _f64p, _f64p, _f64p]
    L.or_mixture_cp_h.argtypes = [mp, C.c_double, _f64p, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    L.or_fluxes.argtypes = [mp, C.c_double, C.c_double, _f64p, _f64p, _f64p]
    L.or_rhs.argtypes = [mp, C.c_double, _f64p, _f64p]
    L.or_jacobian.argtypes = [mp, C.c_double, _f64p, _f64p]
    L.or_T_from_h.restype = C.c_int
    L.or_T_from_h.argtypes = [mp, C.c_double, _f64p, C.c_double, C.POINTER(C.c_double)]
    L.or_element_mass.argtypes = [mp, _f64p, _f64p]
    L.or_project.argtypes = [mp, _f64p, _f64p]
    L.or_advance.argtypes = [mp, C.c_int64, _f64p, _f64p, _f64p, C.c_double,
                             C.POINTER(_Opts), _i32p, _i32p, C.c_int]
    L.or_thermo_batch.argtypes = [mp, C.c_int64, _f64p, _f64p, _f64p, _f64p]
    L.or_T_from_h_batch.argtypes = [mp, C.c_int64, _f64p, _f64p, _f64p, _i32p]
    L.or_rhs_batch.argtypes = [mp, C.c_int64, _f64p, _f64p, _f64p, _f64p]
    L.or_jacobian_batch.argtypes = [mp, C.c_int64, _f64p, _f64p, _f64p, _f64p]
    L.or_rodas_coefficients.argtypes = [C.POINTER(C.c_double), _f64p, _f64p]
    L.or_lu.restype = C.c_int
    L.or_lu.argtypes = [C.c_int, _f64p, _i32p]
    L.or_lu_solve.argtypes = [C.c_int, _f64p, _i32p, _f64p]
    L.or_rodas_generic.restype = C.c_int
    return L


RHS_CB = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))


class OracleMech:
    """Keeps the flat arrays alive and exposes the C struct."""

    def __init__(self, mech, library=None):
        self._L = library if library is not None else lib()
        self.src = mech
        self.E = len(mech.elements)
        self.K = int(mech.composition.shape[0])
        self.R = int(mech.reactants.shape[0])
        self._arrs = dict(
            emass=np.ascontiguousarray(mech.element_mass, np.float64),
            comp=np.ascontiguousarray(mech.composition, np.int32),
            nasa=np.ascontiguousarray(mech.nasa7, np.float64),
            reac=np.ascontiguousarray(mech.reactants, np.int32),
            prod=np.ascontiguousarray(mech.products, np.int32),
            lnA=np.ascontiguousarray(mech.log_A, np.float64),
            beta=np.ascontiguousarray(mech.beta, np.float64),
            Ea=np.ascontiguousarray(mech.Ea, np.float64),
            tb=np.ascontiguousarray(mech.third_body, np.int32),
            rev=np.ascontiguousarray(mech.reversible, np.int32))
        a = self._arrs
        self.s = _Mech(self.E, self.K, self.R, *(a[k].ctypes.data for k in
                                                  ("emass", "comp", "nasa", "reac", "prod",
                                                   "lnA", "beta", "Ea", "tb", "rev")))
        self.ref = C.byref(self.s)
        self.W = a["comp"].astype(np.float64) @ a["emass"]       # g/mol

    # ---- thermo ----
    def species_thermo(self, T):
        cp, h, s = (np.zeros(self.K) for _ in range(3))
        self._L.or_species_thermo(self.ref, float(T), cp, h, s)
        return cp, h, s

    def cp_h(self, T, Y):
        cp, h = C.c_double(), C.c_double()
        self._L.or_mixture_cp_h(self.ref, float(T), np.ascontiguousarray(Y, np.float64),
                              C.byref(cp), C.byref(h))
        return cp.value, h.value

    def thermo_batch(self, T, Y):
        T = np.ascontiguousarray(T, np.float64)
        n = T.size
        cp, h = np.zeros(n), np.zeros(n)
        self._L.or_thermo_batch(self.ref, n, T, np.ascontiguousarray(Y, np.float64), cp, h)
        return cp, h

    def T_from_h(self, h0, Y, T_guess):
        T = C.c_double()
        rc = self._L.or_T_from_h(self.ref, float(h0), np.ascontiguousarray(Y, np.float64),
                               float(T_guess), C.byref(T))
        return T.value, rc

    def T_from_h_batch(self, h, Y, T_guess):
        T = np.array(T_guess, np.float64, copy=True)
        st = np.zeros(T.size, np.int32)
        self._L.or_T_from_h_batch(self.ref, T.size, np.ascontiguousarray(h, np.float64),
                                np.ascontiguousarray(Y, np.float64), T, st)
        return T, st

    # ---- kinetics ----
    def fluxes(self, T, p, Y):
        qf, qr = np.zeros(self.R), np.zeros(self.R)
        self._L.or_fluxes(self.ref, float(T), float(p), np.ascontiguousarray(Y, np.float64), qf, qr)
        return qf, qr

    def rhs(self, y, p):
        f = np.zeros(self.K + 1)
        self._L.or_rhs(self.ref, float(p), np.ascontiguousarray(y, np.float64), f)
        return f

    def jacobian(self, y, p):
        J = np.zeros((self.K + 1) * (self.K + 1))
        self._L.or_jacobian(self.ref, float(p), np.ascontiguousarray(y, np.float64), J)
        return J.reshape(self.K + 1, self.K + 1)

    def rhs_batch(self, T, p, Y):
        n = len(T)
        f = np.zeros((n, self.K + 1))
        self._L.or_rhs_batch(self.ref, n, np.ascontiguousarray(T, np.float64),
                           np.ascontiguousarray(p, np.float64),
                           np.ascontiguousarray(Y, np.float64), f)
        return f

    def jacobian_batch(self, T, p, Y):
        n = len(T)
        J = np.zeros((n, self.K + 1, self.K + 1))
        self._L.or_jacobian_batch(self.ref, n, np.ascontiguousarray(T, np.float64),
                                np.ascontiguousarray(p, np.float64),
                                np.ascontiguousarray(Y, np.float64), J)
        return J

    # ---- elements ----
    def element_mass(self, Y):
        me = np.zeros(self.E)
        self._L.or_element_mass(self.ref, np.ascontiguousarray(Y, np.float64), me)
        return me

    def project(self, Yref, Y):
        Y = np.array(Y, np.float64, copy=True)
        self._L.or_project(self.ref, np.ascontiguousarray(Yref, np.float64), Y)
        return Y

    # ---- advance ----
    def advance(self, T, p, Y, dt, rtol=1e-10, atol_Y=1e-18, atol_T=1e-8, h0_frac=1e-3,
                max_steps=100000, project=True, newton_T=True, nthreads=None):
        """Advance every cell over dt.  Returns (T, Y, status, nsteps)."""
        T = np.array(T, np.float64, copy=True)
        Y = np.array(Y, np.float64, copy=True, order="C")
        p = np.ascontiguousarray(np.broadcast_to(np.asarray(p, np.float64), T.shape))
        n = T.size
        st = np.zeros(n, np.int32)
        ns = np.zeros(n, np.int32)
        o = _Opts(rtol, atol_Y, atol_T, h0_frac, max_steps, int(project), int(newton_T))
        self._L.or_advance(self.ref, n, T, p, Y, float(dt), C.byref(o), st, ns,
                         int(nthreads or default_threads()))
        return T, Y, st, ns


def rodas_coefficients():
    g = C.c_double()
    A = np.zeros(30)
    Cc = np.zeros(30)
    lib().or_rodas_coefficients(C.byref(g), A, Cc)
    return g.value, A.reshape(6, 5), Cc.reshape(6, 5)


def rodas_generic(f, jac, y0, tend, atol, rtol, h0=1e-3, max_steps=100000, fixed_h=0.0):
    """RODAS on Python callbacks f(y)->dy, jac(y)->J (small test ODEs)."""
    N = len(y0)

    def fcb(_ctx, yp, out):
        y = np.ctypeslib.as_array(yp, (N,))
        np.ctypeslib.as_array(out, (N,))[:] = f(y.copy())

    def jcb(_ctx, yp, out):
        y = np.ctypeslib.as_array(yp, (N,))
        np.ctypeslib.as_array(out, (N * N,))[:] = np.asarray(jac(y.copy())).ravel()

    cf, cj = RHS_CB(fcb), RHS_CB(jcb)
    y = np.array(y0, np.float64, copy=True)
    at = np.ascontiguousarray(np.broadcast_to(np.asarray(atol, np.float64), (N,)))
    counts = np.zeros(3, np.int32)
    L = lib()
    L.or_rodas_generic.argtypes = [C.c_int, RHS_CB, RHS_CB, _f64p, C.c_double, _f64p,
                                   C.c_double, C.c_double, C.c_int, C.c_double, _i32p]
    rc = L.or_rodas_generic(N, cf, cj, y, float(tend), at, float(rtol), float(h0),
                            int(max_steps), float(fixed_h), counts)
    return y, rc, counts
