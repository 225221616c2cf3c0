"""ctypes binding of libqpat (include/qpat.h).

Argument marshalling only: tensors are checked (device, dtype, contiguity,
size) and their device pointers passed to the C ABI; every computation runs
in the library's HIP kernels. Importing this module loads the shared library
and raises if it is missing -- there is no fallback path.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpat.so")

QPAT_OK, QPAT_ERR_ARG, QPAT_ERR_MESH, QPAT_ERR_NOCONV, QPAT_ERR_BREAKDOWN, \
    QPAT_ERR_DEVICE, QPAT_ERR_OOM, QPAT_ERR_STATE = range(8)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_MESH", 3: "ERR_NOCONV", 4: "ERR_BREAKDOWN",
                5: "ERR_DEVICE", 6: "ERR_OOM", 7: "ERR_STATE"}


class QpatError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_rhs_block", ctypes.c_int32),
                ("pcg_rtol", ctypes.c_double), ("pcg_maxit", ctypes.c_int32),
                ("prior_rtol", ctypes.c_double), ("prior_deflate", ctypes.c_int32),
                ("lsqr_reorth", ctypes.c_int32), ("lsqr_max_steps", ctypes.c_int32),
                ("ru_delta", ctypes.c_double), ("use_graphs", ctypes.c_int32),
                ("operator_format", ctypes.c_int32), ("prior_precond", ctypes.c_int32),
                ("pcg_precond", ctypes.c_int32), ("autotune", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_solves", ctypes.c_int32), ("iters_max", ctypes.c_int32),
                ("iters_sum", ctypes.c_int64), ("updates", ctypes.c_int32),
                ("relres_max", ctypes.c_double), ("rhs_cap", ctypes.c_int32),
                ("rhs_iters", ctypes.POINTER(ctypes.c_int32)), ("rhs_relres", ctypes.POINTER(ctypes.c_double))]
    RHS_CAP = 4096

    def __init__(self):
        super().__init__()
        # host buffers for the per-system report, owned by this object
        self._it = (ctypes.c_int32 * self.RHS_CAP)()
        self._rr = (ctypes.c_double * self.RHS_CAP)()
        self.rhs_cap = self.RHS_CAP
        self.rhs_iters = ctypes.cast(self._it, ctypes.POINTER(ctypes.c_int32))
        self.rhs_relres = ctypes.cast(self._rr, ctypes.POINTER(ctypes.c_double))

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_[:5]}
        n = max(0, min(self.n_solves, self.rhs_cap))
        d["rhs_iters"] = list(self.rhs_iters[:n]) if self.rhs_iters else []
        d["rhs_relres"] = list(self.rhs_relres[:n]) if self.rhs_relres else []
        return d


class KStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("lanes", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["avg_ms"] = self.total_ms / self.launches if self.launches else 0.0
        return d


KSTAT_NAMES = ("K_dir_spmv", "K_update", "prior_dir_spmv", "prior_update",
               "K_mg_dir_spmv", "K_mg_update", "K_mg_resid0", "K_mg_smooth0",
               "prior_mg_dir_spmv", "prior_mg_update", "prior_mg_resid0", "prior_mg_smooth0")

_P = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_S = ctypes.c_int

# name -> (restype, argtypes); the names are those of include/qpat.h
SIGNATURES = {
    "qpat_default_opts": (None, [ctypes.POINTER(Opts)]),
    "qpat_setup_mesh": (_S, [ctypes.POINTER(_P), _I64, _P, _I64, _P, _I64, _P, ctypes.POINTER(Opts), _P]),
    "qpat_set_opts": (_S, [_P, ctypes.POINTER(Opts)]),
    "qpat_get_opts": (_S, [_P, ctypes.POINTER(Opts)]),
    "qpat_set_sources": (_S, [_P, _I32, _P]),
    "qpat_forward": (_S, [_P, _P, _P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_forward_log": (_S, [_P, _D, _D, _P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_jvp": (_S, [_P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_vjp": (_S, [_P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_prior_setup": (_S, [_P, _P, _P, _D, _D, _D]),
    "qpat_prior_setup_r": (_S, [_P, _P, _P, _I32, _D, _D, _D, _D]),
    "qpat_fit_background": (_S, [_P, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D), _I32, _D,
                                 ctypes.POINTER(_I32), ctypes.POINTER(Info)]),
    "qpat_lsqr_init_kappa": (_S, [_P, _P, _P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_prior_apply": (_S, [_P, _P, _P]),
    "qpat_prior_solve": (_S, [_P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_misfit": (_S, [_P, _P, _P, ctypes.POINTER(_D)]),
    "qpat_misfit_noalloc": (_S, [_P, _P, _P, _P]),
    "qpat_init_guess": (_S, [_P, _P, _D, _P]),
    "qpat_lsqr_init": (_S, [_P, _P, _P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_lsqr_step": (_S, [_P, ctypes.POINTER(_D), ctypes.POINTER(Info)]),
    "qpat_lsqr_steps": (_I32, [_P]),
    "qpat_lsqr_basis": (_I32, [_P]),
    "qpat_geometry_classes": (_I32, [_P]),
    "qpat_lsqr_residual": (_D, [_P]),
    "qpat_profile": (_S, [_P, _I32]),
    "qpat_profile_read": (_S, [_P, ctypes.POINTER(KStat)]),
    "qpat_operator_layout": (_S, [_P, ctypes.POINTER(_I64)]),
    "qpat_tile_schedule": (_S, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "qpat_batch": (_S, [ctypes.POINTER(_P), _I32, _I32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                        ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(Info)]),
    "qpat_forward_x0": (_S, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(Info)]),
    "qpat_guess_setup": (_S, [_P, _I32, _I32, _I32]),
    "qpat_guess_set_params": (_S, [_P, _P]),
    "qpat_guess_get_params": (_S, [_P, _P]),
    "qpat_guess_eval": (_S, [_P, _P, _P]),
    "qpat_guess_grad": (_S, [_P, _P, _P, _P, ctypes.POINTER(_D)]),
    "qpat_guess_train_step": (_S, [_P, _P, _P, ctypes.c_float, ctypes.POINTER(_D)]),
    "qpat_guess_train": (_S, [_P, _P, _P, _D, _D, _P, _P, ctypes.c_float, ctypes.POINTER(_D)]),
    "qpat_guess_fluence": (_S, [_P, _P, _P, _D, _D, _P, _P]),
    "qpat_last_error": (ctypes.c_char_p, [_P]),
    "qpat_version": (ctypes.c_char_p, []),
    "qpat_destroy": (None, [_P]),
}


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libqpat.so not found at {path}; build it with "
                          "`python -m paper_1512_02796_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def default_opts(**overrides):
    o = Opts()
    _lib.qpat_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t, dtype, numel=None, name="array", allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One mesh on one GPU; wraps a qpat_ctx."""

    def __init__(self, coords, tets, bfaces, opts=None, stream=None):
        self._h = ctypes.c_void_p()
        N, E, F = coords.shape[0], tets.shape[0], bfaces.shape[0]
        self.N, self.E, self.F_b = N, E, F
        self.device = coords.device
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        o = opts if opts is not None else default_opts()
        st = _lib.qpat_setup_mesh(ctypes.byref(self._h), N, _ptr(coords, torch.float64, 3 * N, "coords"),
                                  E, _ptr(tets, torch.int32, 4 * E, "tets"), F,
                                  _ptr(bfaces, torch.int32, 3 * F, "bfaces"), ctypes.byref(o),
                                  ctypes.c_void_p(s.cuda_stream))
        if st != QPAT_OK:
            msg = self.last_error()
            _lib.qpat_destroy(self._h)
            self._h = ctypes.c_void_p()
            raise QpatError(st, msg)
        self.n_ill = 0

    # ---- helpers
    def last_error(self):
        m = _lib.qpat_last_error(self._h)
        return m.decode() if m else ""

    def _check(self, st):
        if st != QPAT_OK:
            raise QpatError(st, self.last_error())

    def close(self):
        if self._h:
            _lib.qpat_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- options
    def get_opts(self):
        o = Opts()
        self._check(_lib.qpat_get_opts(self._h, ctypes.byref(o)))
        return o

    def set_opts(self, **kw):
        o = self.get_opts()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(_lib.qpat_set_opts(self._h, ctypes.byref(o)))
        return o

    # ---- the path
    def set_sources(self, phi_src):
        n_ill = phi_src.shape[0]
        self._check(_lib.qpat_set_sources(self._h, n_ill, _ptr(phi_src, torch.float64, n_ill * self.F_b * 3,
                                                              "phi_src")))
        self.n_ill = n_ill

    def forward(self, kappa, mu, phi_out=None, h_out=None):
        info = Info()
        nd = self.n_ill * self.N
        self._check(_lib.qpat_forward(self._h, _ptr(kappa, torch.float64, self.N, "kappa"),
                                      _ptr(mu, torch.float64, self.N, "mu"),
                                      _ptr(phi_out, torch.float64, nd, "phi_out", True),
                                      _ptr(h_out, torch.float64, nd, "h_out", True), ctypes.byref(info)))
        return info.as_dict()

    def forward_log(self, kappa0, mu0, beta, phi_out=None, h_out=None):
        info = Info()
        nd = self.n_ill * self.N
        self._check(_lib.qpat_forward_log(self._h, float(kappa0), float(mu0),
                                          _ptr(beta, torch.float64, 2 * self.N, "beta"),
                                          _ptr(phi_out, torch.float64, nd, "phi_out", True),
                                          _ptr(h_out, torch.float64, nd, "h_out", True), ctypes.byref(info)))
        return info.as_dict()

    def forward_x0(self, kappa, mu, x0, phi_out=None, h_out=None):
        info = Info()
        nd = self.n_ill * self.N
        self._check(_lib.qpat_forward_x0(self._h, _ptr(kappa, torch.float64, self.N, "kappa"),
                                         _ptr(mu, torch.float64, self.N, "mu"),
                                         _ptr(x0, torch.float64, nd, "x0"),
                                         _ptr(phi_out, torch.float64, nd, "phi_out", True),
                                         _ptr(h_out, torch.float64, nd, "h_out", True), ctypes.byref(info)))
        return info.as_dict()

    # ---- learned initial guess
    N_PARAMS = 15601

    def guess_setup(self, nx, ny, nz):
        self._check(_lib.qpat_guess_setup(self._h, nx, ny, nz))

    def guess_set_params(self, params):
        self._check(_lib.qpat_guess_set_params(self._h, _ptr(params, torch.float32, self.N_PARAMS, "params")))

    def guess_get_params(self, out):
        self._check(_lib.qpat_guess_get_params(self._h, _ptr(out, torch.float32, self.N_PARAMS, "params")))

    def guess_eval(self, inp, out):
        self._check(_lib.qpat_guess_eval(self._h, _ptr(inp, torch.float32, 3 * self.N, "input"),
                                         _ptr(out, torch.float32, self.N, "out")))

    def guess_grad(self, inp, target, grad=None):
        loss = ctypes.c_double()
        self._check(_lib.qpat_guess_grad(self._h, _ptr(inp, torch.float32, 3 * self.N, "input"),
                                         _ptr(target, torch.float32, self.N, "target"),
                                         _ptr(grad, torch.float32, self.N_PARAMS, "grad", True),
                                         ctypes.byref(loss)))
        return loss.value

    def guess_train_step(self, inp, target, lr):
        loss = ctypes.c_double()
        self._check(_lib.qpat_guess_train_step(self._h, _ptr(inp, torch.float32, 3 * self.N, "input"),
                                               _ptr(target, torch.float32, self.N, "target"), float(lr),
                                               ctypes.byref(loss)))
        return loss.value

    def guess_train(self, kappa, mu, kappa0, mu0, phi_hom, phi, lr):
        loss = ctypes.c_double()
        self._check(_lib.qpat_guess_train(self._h, _ptr(kappa, torch.float64, self.N, "kappa"),
                                          _ptr(mu, torch.float64, self.N, "mu"), float(kappa0), float(mu0),
                                          _ptr(phi_hom, torch.float64, self.N, "phi_hom"),
                                          _ptr(phi, torch.float64, self.N, "phi"), float(lr), ctypes.byref(loss)))
        return loss.value

    def guess_fluence(self, kappa, mu, kappa0, mu0, phi_hom, phi0_out):
        nd = self.n_ill * self.N
        self._check(_lib.qpat_guess_fluence(self._h, _ptr(kappa, torch.float64, self.N, "kappa"),
                                            _ptr(mu, torch.float64, self.N, "mu"), float(kappa0), float(mu0),
                                            _ptr(phi_hom, torch.float64, nd, "phi_hom"),
                                            _ptr(phi0_out, torch.float64, nd, "phi0_out")))

    def jvp(self, s, out):
        info = Info()
        self._check(_lib.qpat_jvp(self._h, _ptr(s, torch.float64, 2 * self.N, "s"),
                                  _ptr(out, torch.float64, self.n_ill * self.N, "out"), ctypes.byref(info)))
        return info.as_dict()

    def vjp(self, t, out):
        info = Info()
        self._check(_lib.qpat_vjp(self._h, _ptr(t, torch.float64, self.n_ill * self.N, "t"),
                                  _ptr(out, torch.float64, 2 * self.N, "out"), ctypes.byref(info)))
        return info.as_dict()

    def prior_setup(self, kt, mt, T=5e-3, b_over_a=1.0, delta=1e-6):
        self._check(_lib.qpat_prior_setup(self._h, _ptr(kt, torch.float64, self.N, "kt"),
                                          _ptr(mt, torch.float64, self.N, "mt"), float(T), float(b_over_a),
                                          float(delta)))

    def prior_setup_r(self, kt, mt, kind, T=5e-3, q=1.0, b_over_a=1.0, delta=1e-6):
        """kind: PRIOR_PM or PRIOR_TVQ (r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q)."""
        self._check(_lib.qpat_prior_setup_r(self._h, _ptr(kt, torch.float64, self.N, "kt"),
                                            _ptr(mt, torch.float64, self.N, "mt"), int(kind), float(T), float(q),
                                            float(b_over_a), float(delta)))

    def prior_apply(self, x, y):
        self._check(_lib.qpat_prior_apply(self._h, _ptr(x, torch.float64, 2 * self.N, "x"),
                                          _ptr(y, torch.float64, 2 * self.N, "y")))

    def prior_solve(self, p, r):
        info = Info()
        self._check(_lib.qpat_prior_solve(self._h, _ptr(p, torch.float64, 2 * self.N, "p"),
                                          _ptr(r, torch.float64, 2 * self.N, "r"), ctypes.byref(info)))
        return info.as_dict()

    def misfit(self, chi, w):
        out = ctypes.c_double()
        nd = self.n_ill * self.N
        self._check(_lib.qpat_misfit(self._h, _ptr(chi, torch.float64, nd, "chi"), _ptr(w, torch.float64, nd, "w"),
                                     ctypes.byref(out)))
        return out.value

    def misfit_noalloc(self, chi, w, out):
        """||W (chi - h)|| into out[0] (a device FP64 tensor), stream-ordered, no
        allocation and no synchronisation (qpat_misfit_noalloc)."""
        nd = self.n_ill * self.N
        self._check(_lib.qpat_misfit_noalloc(self._h, _ptr(chi, torch.float64, nd, "chi"),
                                             _ptr(w, torch.float64, nd, "w"), _ptr(out, torch.float64, 1, "out")))

    def init_guess(self, chi, mu0, beta_out):
        self._check(_lib.qpat_init_guess(self._h, _ptr(chi, torch.float64, self.n_ill * self.N, "chi"),
                                         float(mu0), _ptr(beta_out, torch.float64, 2 * self.N, "beta_out")))

    def fit_background(self, chi, w, kappa0, mu0, maxit=30, tol=1e-10):
        """Homogeneous (kappa0, mu0) minimising |W (chi - h)|; returns (kappa0, mu0, iters, info)."""
        nd = self.n_ill * self.N
        k = ctypes.c_double(kappa0)
        m = ctypes.c_double(mu0)
        it = ctypes.c_int32(0)
        info = Info()
        self._check(_lib.qpat_fit_background(self._h, _ptr(chi, torch.float64, nd, "chi"),
                                             _ptr(w, torch.float64, nd, "w"), ctypes.byref(k), ctypes.byref(m),
                                             int(maxit), float(tol), ctypes.byref(it), ctypes.byref(info)))
        return k.value, m.value, it.value, info.as_dict()

    def lsqr_init_kappa(self, chi, w, beta_lin, beta_out):
        info = Info()
        nd = self.n_ill * self.N
        self._beta_out = beta_out
        self._check(_lib.qpat_lsqr_init_kappa(self._h, _ptr(chi, torch.float64, nd, "chi"),
                                              _ptr(w, torch.float64, nd, "w"),
                                              _ptr(beta_lin, torch.float64, 2 * self.N, "beta_lin", True),
                                              _ptr(beta_out, torch.float64, 2 * self.N, "beta_out"),
                                              ctypes.byref(info)))
        return info.as_dict()

    def lsqr_init(self, chi, w, beta_lin, beta_out):
        info = Info()
        nd = self.n_ill * self.N
        self._beta_out = beta_out      # registered with the library until the next init
        self._check(_lib.qpat_lsqr_init(self._h, _ptr(chi, torch.float64, nd, "chi"),
                                        _ptr(w, torch.float64, nd, "w"),
                                        _ptr(beta_lin, torch.float64, 2 * self.N, "beta_lin", True),
                                        _ptr(beta_out, torch.float64, 2 * self.N, "beta_out"),
                                        ctypes.byref(info)))
        return info.as_dict()

    def lsqr_step(self):
        info = Info()
        res = ctypes.c_double()
        self._check(_lib.qpat_lsqr_step(self._h, ctypes.byref(res), ctypes.byref(info)))
        return res.value, info.as_dict()

    def lsqr_steps(self):
        return _lib.qpat_lsqr_steps(self._h)

    def lsqr_basis(self):
        return _lib.qpat_lsqr_basis(self._h)

    def geometry_classes(self):
        return int(_lib.qpat_geometry_classes(self._h))

    def lsqr_residual(self):
        return _lib.qpat_lsqr_residual(self._h)

    def profile(self, enable):
        self._check(_lib.qpat_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        arr = (KStat * len(KSTAT_NAMES))()
        self._check(_lib.qpat_profile_read(self._h, arr))
        return {KSTAT_NAMES[i]: arr[i].as_dict() for i in range(len(KSTAT_NAMES))}

    def operator_layout(self):
        arr = (_I64 * 6)()
        self._check(_lib.qpat_operator_layout(self._h, arr))
        return {"lattice": bool(arr[0]), "nx": arr[1], "ny": arr[2], "nz": arr[3], "stencil_arrays": arr[4],
                "sell_len": arr[5]}


    def tile_schedule(self, B=16):
        arr = (ctypes.c_int32 * 8)()
        self._check(_lib.qpat_tile_schedule(self._h, B, arr))
        return {"tiled": bool(arr[0]), "zc": arr[1], "zc_model": arr[2], "ps_zc": arr[3], "ps_zc_model": arr[4],
                "ps_zc32": arr[5], "ps_zc32_model": arr[6], "tuned": bool(arr[7])}


PRIOR_PM, PRIOR_TVQ = 0, 1   # QPAT_PRIOR_PM, QPAT_PRIOR_TVQ
BATCH_OPS = {"forward": 0, "jvp": 1, "vjp": 2, "pair": 3, "lsqr_step": 4}


def batch(ctxs, op, in0=None, out0=None, in1=None, out1=None):
    """One call on several contexts at once (each on its own stream); returns
    the per-instance info dicts. Arrays are lists with one tensor per context
    (None where the call takes none)."""
    n = len(ctxs)
    hs = (_P * n)(*[c._h.value for c in ctxs])

    def ptrs(lst, what, dtype=torch.float64):
        if lst is None:
            return None
        arr = (_P * n)()
        for i, t in enumerate(lst):
            arr[i] = None if t is None else _ptr(t, dtype, name=f"{what}[{i}]").value
        return arr
    owners = [Info() for _ in range(n)]     # own the per-system buffers the array entries point at
    infos = (Info * n)(*owners)
    st = _lib.qpat_batch(hs, n, BATCH_OPS[op], ptrs(in0, "in0"), ptrs(out0, "out0"), ptrs(in1, "in1"),
                         ptrs(out1, "out1"), infos)
    if st != 0:
        bad = next((c for c in ctxs if c.last_error()), ctxs[0])
        raise QpatError(st, bad.last_error())
    return [infos[i].as_dict() for i in range(n)]


def version():
    return _lib.qpat_version().decode()
