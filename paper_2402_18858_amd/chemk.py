"""Python binding of libchemk.so (argument marshalling only).

Every call forwards device pointers of torch tensors and the current HIP
stream to the C ABI declared in include/chemk.h; all arithmetic runs in the
library's gfx950 kernels.  There is no fallback: if the shared library is
missing or cannot be loaded, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchemk.so")

OK, E_ARG, E_MECH, E_HIP, E_DT, E_OOM, E_STATE, E_UNSUPPORTED = range(8)
CELL_OK, CELL_MAX_STEPS, CELL_T_RANGE, CELL_NONFINITE, CELL_NEWTON = 0, 1, 2, 3, 4
CELL_SINGULAR, CELL_ROUTED_DI = 6, 8
MODE_DI, MODE_ANN = 0, 1
DI_AUTO, DI_LDS_LU, DI_REG_LU = 0, 1, 2


class ChemkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"chemk error {code}: {msg}")
        self.code = code


class MechDesc(C.Structure):
    _fields_ = [("n_elements", C.c_int32), ("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("element_mass", C.c_void_p), ("composition", C.c_void_p),
                ("nasa7", C.c_void_p), ("reactants", C.c_void_p), ("products", C.c_void_p),
                ("log_A", C.c_void_p), ("beta", C.c_void_p), ("Ea", C.c_void_p),
                ("third_body", C.c_void_p), ("reversible", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_steps", C.c_int32), ("rtol", C.c_double),
                ("atol_Y", C.c_double), ("atol_T", C.c_double), ("h0_frac", C.c_double),
                ("bins", C.c_int32), ("waves_per_cu", C.c_int32), ("use_graph", C.c_int32),
                ("project", C.c_int32), ("di_kernel", C.c_int32)]


MAX_RATIOS, MAX_ELEMENTS = 4, 8


class AnnChecks(C.Structure):
    _fields_ = [("adj_max", C.c_double), ("dT_lo", C.c_double), ("dT_hi", C.c_double),
                ("n_ratios", C.c_int32),
                ("ratio_num", C.c_double * (MAX_RATIOS * MAX_ELEMENTS)),
                ("ratio_den", C.c_double * (MAX_RATIOS * MAX_ELEMENTS)),
                ("ratio_lo", C.c_double * MAX_RATIOS), ("ratio_hi", C.c_double * MAX_RATIOS)]


class TrainOpts(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("lr0", C.c_float), ("lr1", C.c_float),
                ("seed", C.c_uint64), ("use_graph", C.c_int32), ("w_mass", C.c_float),
                ("w_hrr", C.c_float), ("G", C.c_void_p), ("out_w", C.c_void_p), ("epoch0", C.c_int32),
                ("epochs_total", C.c_int32)]


_vp = C.c_void_p
_i64 = C.c_int64
_SIGS = {
    "chemk_mech_create": (C.c_int, [C.POINTER(MechDesc), C.POINTER(_vp)]),
    "chemk_mech_free": (None, [_vp]),
    "chemk_mech_info": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]),
    "chemk_ctx_create": (C.c_int, [C.c_int, _vp, C.POINTER(_vp)]),
    "chemk_ctx_free": (None, [_vp]),
    "chemk_last_error": (C.c_char_p, []),
    "chemk_thermo": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "chemk_T_from_h": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "chemk_rhs": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "chemk_jacobian": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "chemk_opts_default": (None, [C.POINTER(Opts)]),
    "chemk_advance": (C.c_int, [_vp, _i64, _vp, _vp, _vp, C.c_double, C.POINTER(Opts), _vp,
                                _vp, _vp]),
    "chemk_advance_noalloc": (C.c_int, [_vp, _i64, _vp, _vp, _vp, C.c_double, C.POINTER(Opts), _vp,
                                        _vp, _vp]),
    "chemk_transport_set": (C.c_int, [_vp, _vp, _vp]),
    "chemk_transport": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "chemk_pasr": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, C.c_double, _vp, _vp, _vp, C.c_double,
                             C.c_double, _vp, _vp, _vp, _vp]),
    "chemk_tuning": (C.c_int, [_vp, _vp]),
    "chemk_tune_cache_clear": (None, []),
    "chemk_autotune": (C.c_int, [_vp, _i64, _vp, _vp, _vp, C.c_double, C.POINTER(Opts),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double), _vp]),
    "chemk_last_counters": (C.c_int, [_vp, C.POINTER(C.c_int64), _vp]),
    "chemk_timing": (C.c_int, [_vp, C.c_int32]),
    "chemk_timing_read": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), _vp]),
    "chemk_ann_create": (C.c_int, [_vp, C.POINTER(C.c_int32), C.c_int32]),
    "chemk_ann_create_species": (C.c_int, [_vp, C.POINTER(C.c_int32), C.c_int32]),
    "chemk_ann_param_count": (C.c_int, [_vp, C.POINTER(C.c_int64)]),
    "chemk_ann_set_weights": (C.c_int, [_vp, _vp, _i64]),
    "chemk_ann_get_weights": (C.c_int, [_vp, _vp, _i64]),
    "chemk_ann_set_norm": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double]),
    "chemk_ann_get_norm": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_double)]),
    "chemk_ann_set_envelope": (C.c_int, [_vp, _vp, _vp, C.c_double]),
    "chemk_ann_get_envelope": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_double)]),
    "chemk_ann_set_checks": (C.c_int, [_vp, C.POINTER(AnnChecks)]),
    "chemk_ann_get_checks": (C.c_int, [_vp, C.POINTER(AnnChecks)]),
    "chemk_ann_fit_envelope": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, C.c_double, C.c_double,
                                         _vp]),
    "chemk_ann_fit_norm": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, C.c_double, C.c_double,
                                     C.c_double, _vp]),
    "chemk_ann_pack": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "chemk_ann_forward_packed": (C.c_int, [_vp, _i64, _vp, _vp, _vp]),
    "chemk_ann_train_step": (C.c_int, [_vp, _vp, C.c_int32, _vp, _vp, _vp, C.c_float, C.c_float,
                                       _vp, C.c_float, C.c_int32, _vp, _vp, _vp]),
    "chemk_ann_hrr_weights": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, C.c_double, C.c_double, _vp,
                                        C.POINTER(C.c_double), _vp]),
    "chemk_ann_train": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _i64, C.POINTER(TrainOpts), _vp, _vp,
                                  _vp]),
    "chemk_ann_reset_optimizer": (C.c_int, [_vp]),
}

# torch ships its own HIP runtime (libamdhip64.so.7).  Importing torch first
# makes the library's libamdhip64.so.7 dependency resolve to that same copy, so
# the process has one HIP/HSA runtime shared by torch tensors, streams and the
# library's kernels (a second runtime would hide the GPU from one of them).
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(hipcc, gfx950); there is no fallback path")
lib = C.CDLL(LIB_PATH)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return list(_SIGS)


def _check(code):
    if code != OK:
        raise ChemkError(code, lib.chemk_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def default_opts(**kw) -> Opts:
    o = Opts()
    lib.chemk_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class Mechanism:
    """Validated host copy of a mechanism (chemk_mech)."""

    def __init__(self, mech):
        self._keep = dict(
            em=np.ascontiguousarray(mech.element_mass, np.float64),
            comp=np.ascontiguousarray(mech.composition, np.int32),
            nasa=np.ascontiguousarray(mech.nasa7, np.float64),
            reac=np.ascontiguousarray(mech.reactants, np.int32),
            prod=np.ascontiguousarray(mech.products, np.int32),
            lnA=np.ascontiguousarray(mech.log_A, np.float64),
            beta=np.ascontiguousarray(mech.beta, np.float64),
            Ea=np.ascontiguousarray(mech.Ea, np.float64),
            tb=np.ascontiguousarray(mech.third_body, np.int32),
            rev=np.ascontiguousarray(mech.reversible, np.int32))
        k = self._keep
        d = MechDesc(len(mech.elements), k["comp"].shape[0], k["reac"].shape[0],
                     *(k[n].ctypes.data for n in ("em", "comp", "nasa", "reac", "prod", "lnA",
                                                  "beta", "Ea", "tb", "rev")))
        h = C.c_void_p()
        # bound here: at interpreter exit the module's globals may be gone
        # before this object is
        self._free = lib.chemk_mech_free
        _check(lib.chemk_mech_create(C.byref(d), C.byref(h)))
        self.handle = h
        K, R, E = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.chemk_mech_info(h, C.byref(K), C.byref(R), C.byref(E)))
        self.K, self.R, self.E = K.value, R.value, E.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._free(h)
            self.handle = None


class Context:
    """A chemk_ctx on one GPU: device tables of the mechanism, scratch, graphs."""

    def __init__(self, mech, device: int = 0):
        self.mech = mech if isinstance(mech, Mechanism) else Mechanism(mech)
        self._free = lib.chemk_ctx_free   # bound here, as for the mechanism
        h = C.c_void_p()
        _check(lib.chemk_ctx_create(int(device), self.mech.handle, C.byref(h)))
        self.handle = h
        self.K = self.mech.K
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self._free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    # ---- properties ----
    def thermo(self, T, Y, cp, h, stream=None):
        _check(lib.chemk_thermo(self.handle, T.numel(), _ptr(T), _ptr(Y), _ptr(cp), _ptr(h),
                                _stream(stream)))

    def T_from_h(self, h, Y, T, status, stream=None):
        _check(lib.chemk_T_from_h(self.handle, T.numel(), _ptr(h), _ptr(Y), _ptr(T),
                                  _ptr(status), _stream(stream)))

    def rhs(self, T, p, Y, out, stream=None):
        _check(lib.chemk_rhs(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y), _ptr(out),
                             _stream(stream)))

    def jacobian(self, T, p, Y, out, stream=None):
        _check(lib.chemk_jacobian(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y), _ptr(out),
                                  _stream(stream)))

    # ---- advance ----
    def advance(self, T, p, Y, dt, status, nsteps=None, opts=None, stream=None, n=None):
        o = opts if opts is not None else default_opts()
        n = T.numel() if n is None else n
        _check(lib.chemk_advance(self.handle, n, _ptr(T), _ptr(p), _ptr(Y), float(dt),
                                 C.byref(o), _ptr(status), _ptr(nsteps), _stream(stream)))

    def advance_noalloc(self, T, p, Y, dt, status, nsteps=None, opts=None, stream=None, n=None):
        """chemk_advance_noalloc: DI mode with the library's fixed scratch."""
        o = opts if opts is not None else default_opts()
        n = T.numel() if n is None else n
        _check(lib.chemk_advance_noalloc(self.handle, n, _ptr(T), _ptr(p), _ptr(Y), float(dt),
                                         C.byref(o), _ptr(status), _ptr(nsteps), _stream(stream)))

    def autotune(self, T, p, Y, dt, opts=None, stream=None):
        o = opts if opts is not None else default_opts()
        best = (C.c_int32 * 2)()
        ms = C.c_double()
        _check(lib.chemk_autotune(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y), float(dt),
                                  C.byref(o), best, C.byref(ms), _stream(stream)))
        return int(best[0]), int(best[1]), ms.value

    def transport_set(self, mu_poly, lam_poly):
        mu_poly = np.ascontiguousarray(mu_poly, np.float64)
        lam_poly = np.ascontiguousarray(lam_poly, np.float64)
        _check(lib.chemk_transport_set(self.handle, mu_poly.ctypes.data, lam_poly.ctypes.data))

    def transport(self, T, Y, mu, lam=None, stream=None):
        _check(lib.chemk_transport(self.handle, T.numel(), _ptr(T), _ptr(Y), _ptr(mu), _ptr(lam),
                                   _stream(stream)))

    def pasr(self, T, p, Y0, Y1, dt, k_sgs, delta, mu, kappa=None, omega=None, Y_out=None,
             c_eps=1.048, y_min=1e-6, stream=None):
        _check(lib.chemk_pasr(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y0), _ptr(Y1), float(dt),
                              _ptr(k_sgs), _ptr(delta), _ptr(mu), float(c_eps), float(y_min), _ptr(kappa),
                              _ptr(omega), _ptr(Y_out), _stream(stream)))

    def tuning(self):
        """(bins, waves per CU, DI factorisation) the context uses when opts leave them 0."""
        out = (C.c_int32 * 3)()
        _check(lib.chemk_tuning(self.handle, out))
        return int(out[0]), int(out[1]), int(out[2])

    def last_counters(self, stream=None):
        out = (C.c_int64 * 3)()
        _check(lib.chemk_last_counters(self.handle, out, _stream(stream)))
        return {"routed": out[0], "di_steps": out[1], "failed": out[2]}

    PHASES = ("di", "binning", "ingest", "mlp", "post", "fallback", "layer1", "layer2", "layer3",
              "layer4")

    def timing(self, enable=True):
        _check(lib.chemk_timing(self.handle, int(bool(enable))))

    def timing_read(self, stream=None):
        ms = (C.c_double * len(self.PHASES))()
        nl = (C.c_int64 * len(self.PHASES))()
        _check(lib.chemk_timing_read(self.handle, ms, nl, _stream(stream)))
        return {ph: (ms[i], nl[i]) for i, ph in enumerate(self.PHASES)}

    # ---- learned part ----
    def ann_create(self, dims):
        d = (C.c_int32 * len(dims))(*dims)
        _check(lib.chemk_ann_create(self.handle, d, len(dims) - 1))
        self.dims = list(dims)
        self.species_nets = False

    def ann_create_species(self, dims):
        """K networks of shape dims (dims[-1] = 1), one per species."""
        d = (C.c_int32 * len(dims))(*dims)
        _check(lib.chemk_ann_create_species(self.handle, d, len(dims) - 1))
        self.dims = list(dims)
        self.species_nets = True

    def ann_param_count(self):
        c = C.c_int64()
        _check(lib.chemk_ann_param_count(self.handle, C.byref(c)))
        return c.value

    def ann_set_weights(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        _check(lib.chemk_ann_set_weights(self.handle, p.ctypes.data, p.size))

    def ann_get_weights(self):
        n = self.ann_param_count()
        p = np.zeros(n, np.float32)
        _check(lib.chemk_ann_get_weights(self.handle, p.ctypes.data, n))
        return p

    def ann_set_norm(self, mu_x, sd_x, mu_y, sd_y, dt):
        arrs = [np.ascontiguousarray(a, np.float64) for a in (mu_x, sd_x, mu_y, sd_y)]
        _check(lib.chemk_ann_set_norm(self.handle, *(a.ctypes.data for a in arrs), float(dt)))

    def ann_get_norm(self):
        F, K = self.K + 2, self.K
        mx, sx, my, sy = np.zeros(F), np.zeros(F), np.zeros(K), np.zeros(K)
        dt = C.c_double()
        _check(lib.chemk_ann_get_norm(self.handle, mx.ctypes.data, sx.ctypes.data,
                                      my.ctypes.data, sy.ctypes.data, C.byref(dt)))
        return mx, sx, my, sy, dt.value

    def ann_set_envelope(self, lo, hi, neg_tol):
        lo = np.ascontiguousarray(lo, np.float64)
        hi = np.ascontiguousarray(hi, np.float64)
        _check(lib.chemk_ann_set_envelope(self.handle, lo.ctypes.data, hi.ctypes.data,
                                          float(neg_tol)))

    def ann_get_envelope(self):
        F = self.K + 2
        lo, hi = np.zeros(F), np.zeros(F)
        nt = C.c_double()
        _check(lib.chemk_ann_get_envelope(self.handle, lo.ctypes.data, hi.ctypes.data,
                                          C.byref(nt)))
        return lo, hi, nt.value

    def ann_set_checks(self, adj_max=0.0, dT=(-1e300, 1e300), ratios=()):
        """ratios: up to 4 tuples (num[E], den[E], lo, hi) over the mechanism's
        elements (coefficients of the element mass fractions)."""
        ck = AnnChecks()
        ck.adj_max = float(adj_max)
        ck.dT_lo, ck.dT_hi = float(dT[0]), float(dT[1])
        ck.n_ratios = len(ratios)
        for j, (num, den, lo, hi) in enumerate(ratios):
            for e, (u, d) in enumerate(zip(num, den)):
                ck.ratio_num[j * MAX_ELEMENTS + e] = float(u)
                ck.ratio_den[j * MAX_ELEMENTS + e] = float(d)
            ck.ratio_lo[j], ck.ratio_hi[j] = float(lo), float(hi)
        _check(lib.chemk_ann_set_checks(self.handle, C.byref(ck)))

    def ann_get_checks(self):
        ck = AnnChecks()
        _check(lib.chemk_ann_get_checks(self.handle, C.byref(ck)))
        E = self.mech.E
        ratios = [(np.array(ck.ratio_num[j * MAX_ELEMENTS:j * MAX_ELEMENTS + E]),
                   np.array(ck.ratio_den[j * MAX_ELEMENTS:j * MAX_ELEMENTS + E]),
                   ck.ratio_lo[j], ck.ratio_hi[j]) for j in range(ck.n_ratios)]
        return {"adj_max": ck.adj_max, "dT": (ck.dT_lo, ck.dT_hi), "ratios": ratios}

    def ann_fit_envelope(self, T, p, Y, T_next=None, q=1e-3, widen=0.02, stream=None):
        _check(lib.chemk_ann_fit_envelope(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y),
                                          _ptr(T_next), float(q), float(widen), _stream(stream)))

    def ann_fit_norm(self, T, p, Y, Y_next, dt, widen=0.02, neg_tol=1e-6, stream=None):
        _check(lib.chemk_ann_fit_norm(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y),
                                      _ptr(Y_next), float(dt), float(widen), float(neg_tol),
                                      _stream(stream)))

    def ann_pack(self, T, p, Y, Y_next, X, Z, stream=None):
        _check(lib.chemk_ann_pack(self.handle, T.numel(), _ptr(T), _ptr(p), _ptr(Y),
                                  _ptr(Y_next), _ptr(X), _ptr(Z), _stream(stream)))

    def ann_forward_packed(self, X, out, n=None, stream=None):
        n = X.shape[0] if n is None else n
        _check(lib.chemk_ann_forward_packed(self.handle, n, _ptr(X), _ptr(out), _stream(stream)))

    def ann_train_step(self, idx, X, Z, lr, update=True, loss=None, grads=None, stream=None,
                       G=None, w_mass=0.0, w_hrr=0.0, out_w=None):
        _check(lib.chemk_ann_train_step(self.handle, _ptr(idx), idx.numel(), _ptr(X), _ptr(Z), _ptr(G),
                                        float(w_mass), float(w_hrr), _ptr(out_w), float(lr), int(bool(update)),
                                        _ptr(loss), _ptr(grads), _stream(stream)))

    def ann_hrr_weights(self, T, P, Y, Y_next, dt, G, scale=0.0, stream=None):
        """Heat-release loss weights into G [n, K] (device float32); returns the scale."""
        out = C.c_double(0.0)
        _check(lib.chemk_ann_hrr_weights(self.handle, T.shape[0], _ptr(T), _ptr(P), _ptr(Y), _ptr(Y_next),
                                         float(dt), float(scale), _ptr(G), C.byref(out), _stream(stream)))
        return out.value

    def ann_train(self, X, Z, epochs, batch=4096, lr0=1e-3, lr1=1e-5, seed=3001, X_hold=None,
                  Z_hold=None, use_graph=True, stream=None, G=None, w_mass=0.0, w_hrr=0.0, out_w=None,
                  epoch0=0, epochs_total=0):
        """Returns (epoch_loss, hold_loss) as host arrays [epochs] (this call's
        epochs: [epoch0, epoch0 + epochs) of a schedule over epochs_total)."""
        o = TrainOpts(int(batch), int(epochs), float(lr0), float(lr1), int(seed), int(bool(use_graph)),
                      float(w_mass), float(w_hrr), _ptr(G), _ptr(out_w), int(epoch0), int(epochs_total))
        el = np.zeros(epochs, np.float32)
        hl = np.zeros(epochs, np.float32)
        nh = 0 if X_hold is None else X_hold.shape[0]
        _check(lib.chemk_ann_train(self.handle, X.shape[0], _ptr(X), _ptr(Z), _ptr(X_hold), _ptr(Z_hold),
                                   nh, C.byref(o), el.ctypes.data, hl.ctypes.data, _stream(stream)))
        return el, hl

    def ann_reset_optimizer(self):
        _check(lib.chemk_ann_reset_optimizer(self.handle))


def tune_cache_clear():
    """Empties the process's autotuner cache."""
    lib.chemk_tune_cache_clear()
