"""ctypes binding of libile (include/ile.h): argument marshalling only.

Every step of the likelihood runs in the HIP library; this module converts
numpy arrays and device tensors (anything with ``data_ptr()``, e.g. a torch
tensor on the GPU) into the C ABI's plain pointers and raises ``IleError`` on
a non-OK status.  The functions keep the C names; ``Context`` bundles them.
Loading fails loudly when libile.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ILE_LIB names another build of the library (the host-sanitizer build)
LIB_PATH = os.environ.get("ILE_LIB") or os.path.join(HERE, "libile.so")

ILE_OK, ILE_E_ARG, ILE_E_STATE, ILE_E_RANGE, ILE_E_NUMERIC, ILE_E_DEVICE, \
    ILE_E_NOMEM, ILE_E_UNSUPPORTED = range(8)
STATUS_NAMES = ["ILE_OK", "ILE_E_ARG", "ILE_E_STATE", "ILE_E_RANGE",
                "ILE_E_NUMERIC", "ILE_E_DEVICE", "ILE_E_NOMEM",
                "ILE_E_UNSUPPORTED"]
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
ILE_OPT_SORT = 0
ILE_OPT_ENGINE = 1
ILE_OPT_THREADS = 2
ILE_OPT_HARVEST_ROWS = 3
ILE_OPT_LDS_KB = 4
NOALLOC_MAX_N = 65536   # ile_integrate_dev_noalloc: samples per call


class IleError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


class Mode(C.Structure):
    _fields_ = [("l", C.c_int32), ("m", C.c_int32)]


class Detector(C.Structure):
    _fields_ = [("lat_deg", C.c_double), ("lon_deg", C.c_double),
                ("xarm_az_deg", C.c_double)]


class Config(C.Structure):
    _fields_ = [("n_det", C.c_int32), ("n_lm", C.c_int32),
                ("modes", C.POINTER(Mode)), ("srate_hz", C.c_double),
                ("n_t", C.c_int32), ("d_ref_mpc", C.c_double),
                ("gmst_rad", C.c_double), ("earth_radius_m", C.c_double),
                ("t_ref_max_s", C.c_double), ("precision", C.c_int),
                ("device", C.c_int32), ("stream", C.c_void_p)]


SAMPLER = {"prior": 0, "adaptive": 1, "learned": 2}


class RunOpts(C.Structure):
    _fields_ = [("sampler", C.c_int), ("seed", C.c_uint64), ("chunk", C.c_int64),
                ("max_samples", C.c_int64), ("n_eff_target", C.c_double),
                ("d_min_mpc", C.c_double), ("d_max_mpc", C.c_double),
                ("n_bins", C.c_int32), ("floor", C.c_double), ("temper", C.c_double),
                ("adapt_chunks", C.c_int32), ("reset", C.c_int32),
                ("prop", C.c_void_p), ("eps", C.c_double), ("fallback_neff", C.c_double),
                ("train_steps", C.c_int32), ("train_batch", C.c_int32), ("lr", C.c_double),
                ("refine_rounds", C.c_int32), ("refine_steps", C.c_int32),
                ("refine_eff", C.c_double), ("train_ess", C.c_double),
                ("refine_kish", C.c_double), ("sigma_scale", C.c_double),
                ("warm", C.c_int32)]


class LearnedInfo(C.Structure):
    _fields_ = [("n_train_samples", C.c_int64), ("n_refine_samples", C.c_int64),
                ("n_learned_samples", C.c_int64), ("fell_back", C.c_int32),
                ("train_ms", C.c_double), ("final_loss", C.c_double),
                ("last_refine_eff", C.c_double), ("refine_eff", C.c_double * 32),
                ("refine_kish", C.c_double * 32)]


class PropConfig(C.Structure):
    _fields_ = [("d_min_mpc", C.c_double), ("d_max_mpc", C.c_double),
                ("t_ref_max_s", C.c_double), ("sigma_floor", C.c_double),
                ("seed", C.c_uint64), ("device", C.c_int32), ("stream", C.c_void_p),
                ("sigma_scale", C.c_double)]


class PropTrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("ess_frac", C.c_double), ("seed", C.c_uint64), ("fit_transform", C.c_int32)]


PROP_NPARAM = 60880


class BatchConfig(C.Structure):
    _fields_ = [("precision", C.c_int), ("device", C.c_int32), ("stream", C.c_void_p)]


class BatchTuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("wgs_per_cu", C.c_int32), ("order", C.c_int32),
                ("engine", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("ln_L_marg", C.c_double), ("n_eff", C.c_double),
                ("n_eff_kish", C.c_double), ("sigma_ln_L", C.c_double),
                ("max_ln_L", C.c_double), ("n_samples", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_dp = C.POINTER(C.c_double)
_vp = C.c_void_p


def lib():
    """Load libile.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        # PyTorch (device memory and streams for the _dev calls) bundles its
        # own HIP runtime under the same soname as the one libile links to:
        # load PyTorch first so that both bind to that one runtime (a
        # process holding two cannot hand device pointers between them).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.ile_create.argtypes = [C.POINTER(Config), C.POINTER(_vp)]
        L.ile_set_data.argtypes = [_vp, _dp, C.c_int64, C.c_double, _dp, _dp,
                                   C.POINTER(Detector)]
        L.ile_eval.argtypes = [_vp, _dp, C.c_int64, _dp]
        L.ile_eval_series.argtypes = [_vp, _dp, C.c_int64, _dp]
        L.ile_integrate.argtypes = [_vp, _dp, _dp, _dp, C.c_int64, C.POINTER(Result)]
        L.ile_eval_dev.argtypes = [_vp, _vp, C.c_int64, _vp]
        L.ile_integrate_dev.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, _vp]
        L.ile_integrate_dev_noalloc.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, _vp]
        L.ile_set_data_fd.argtypes = [_vp, _dp, _dp, _dp, C.c_int64, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.POINTER(Detector), _dp, _dp, _dp]
        L.ile_qvu_fd_dev.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, C.c_double, C.c_double,
                                     C.c_double, C.c_double, _vp, _vp, _vp]
        L.ile_rom_set.argtypes = [_vp, C.POINTER(Mode), C.c_int32, C.c_int32, _dp]
        L.ile_rom_eval_dev.argtypes = [_vp, _vp, C.c_int64, _vp]
        L.ile_rom_integrate_dev.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, _vp]
        L.ile_harvest_dev.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, _vp, C.c_int64, _vp,
                                      _vp, _vp, _vp]
        L.ile_draw_prior_dev.argtypes = [_vp, C.c_uint64, C.c_int64, C.c_int64,
                                         C.c_double, C.c_double, _vp, C.c_int64, _vp]
        L.ile_run_prior.argtypes = [_vp, C.c_uint64, C.c_int64, C.c_int64,
                                    C.c_double, C.c_double, C.POINTER(Result)]
        L.ile_run.argtypes = [_vp, C.POINTER(RunOpts), C.POINTER(Result),
                              C.POINTER(C.c_int64)]
        L.ile_hist_get.argtypes = [_vp, C.c_int32, _dp, _dp]
        L.ile_hist_set.argtypes = [_vp, C.c_int32, _dp, _dp]
        L.ile_hist_draw_dev.argtypes = [_vp, C.c_uint64, C.c_int64, C.c_int64, C.c_double,
                                        C.c_double, _vp, C.c_int64, _vp, _vp, _vp]
        L.ile_hist_refit_dev.argtypes = [_vp, _vp, C.c_int64, _vp, _vp, _vp, C.c_int64,
                                         C.c_double, C.c_double]
        L.ile_batch_create.argtypes = [C.POINTER(BatchConfig), C.POINTER(_vp)]
        L.ile_batch_add_point.argtypes = [_vp, C.POINTER(Config), _dp, C.c_int64, C.c_double,
                                          _dp, _dp, C.POINTER(Detector), C.POINTER(C.c_int32)]
        L.ile_batch_run.argtypes = [_vp, C.c_uint64, C.c_int64, C.c_double, C.c_double,
                                    C.POINTER(Result)]
        L.ile_batch_run_dev.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, C.POINTER(Result)]
        L.ile_batch_lnL.argtypes = [_vp, _dp, C.c_int64]
        L.ile_batch_n_points.argtypes = [_vp]
        L.ile_batch_set_tuning.argtypes = [_vp, C.POINTER(BatchTuning)]
        L.ile_batch_get_tuning.argtypes = [_vp, C.POINTER(BatchTuning)]
        L.ile_batch_autotune.argtypes = [_vp, C.c_int64, C.c_char_p]
        L.ile_batch_last_ms.argtypes = [_vp]
        L.ile_batch_last_ms.restype = C.c_double
        L.ile_batch_destroy.argtypes = [_vp]
        L.ile_batch_destroy.restype = None
        L.ile_batch_last_error.argtypes = [_vp]
        L.ile_batch_last_error.restype = C.c_char_p
        L.ile_inject.argtypes = [_vp, _dp, C.c_int64, C.c_double, C.POINTER(Detector), _dp,
                                 C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.ile_last_learned_info.argtypes = [_vp, C.POINTER(LearnedInfo)]
        L.ile_get_stream.argtypes = [_vp, C.POINTER(_vp)]
        _fp = C.POINTER(C.c_float)
        L.ile_prop_create.argtypes = [C.POINTER(PropConfig), C.POINTER(_vp)]
        L.ile_prop_set_params.argtypes = [_vp, _fp]
        L.ile_prop_get_params.argtypes = [_vp, _fp]
        L.ile_prop_set_transform.argtypes = [_vp, _dp, _dp, _dp]
        L.ile_prop_get_transform.argtypes = [_vp, _dp, _dp, _dp]
        L.ile_prop_set_sigma_scale.argtypes = [_vp, C.c_double]
        L.ile_prop_fit_transform_dev.argtypes = [_vp, _vp, C.c_int64, _vp, C.c_int64,
                                                 C.c_double]
        L.ile_prop_grad_dev.argtypes = [_vp, _vp, C.c_int64, _vp, C.c_int64, _vp, _dp]
        L.ile_prop_train_dev.argtypes = [_vp, _vp, C.c_int64, _vp, C.c_int64,
                                         C.POINTER(PropTrainOpts), _dp]
        L.ile_prop_logpdf_dev.argtypes = [_vp, _vp, C.c_double, _vp, C.c_int64, C.c_int64,
                                          _vp]
        L.ile_prop_sample_dev.argtypes = [_vp, _vp, C.c_double, C.c_uint64, C.c_int64,
                                          C.c_int64, _vp, C.c_int64, _vp, _vp]
        L.ile_prop_sync.argtypes = [_vp]
        L.ile_prop_last_ms.argtypes = [_vp]
        L.ile_prop_last_ms.restype = C.c_double
        L.ile_prop_destroy.argtypes = [_vp]
        L.ile_prop_destroy.restype = None
        L.ile_prop_last_error.argtypes = [_vp]
        L.ile_prop_last_error.restype = C.c_char_p
        L.ile_sync.argtypes = [_vp]
        L.ile_set_option.argtypes = [_vp, C.c_int, C.c_int64]
        L.ile_last_kernel_ms.argtypes = [_vp]
        L.ile_last_kernel_ms.restype = C.c_double
        L.ile_destroy.argtypes = [_vp]
        L.ile_destroy.restype = None
        L.ile_last_error.argtypes = [_vp]
        L.ile_last_error.restype = C.c_char_p
        L.ile_status_string.argtypes = [C.c_int]
        L.ile_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != ILE_OK:
        msg = ""
        if ctx:
            m = lib().ile_last_error(ctx)
            msg = m.decode() if m else ""
        if not msg:
            msg = lib().ile_status_string(status).decode()
        raise IleError(status, msg)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _dev(t):
    return None if t is None else C.c_void_p(int(t.data_ptr()))


# ----------------------------------------------------------- C-named calls
def ile_create(dets, modes, srate_hz, n_t, *, d_ref_mpc=100.0, gmst_rad=0.0,
               earth_radius_m=6378.0e3, t_ref_max_s=0.01, precision="fp64",
               device=0, stream=None):
    modes_arr = (Mode * len(modes))(*[Mode(int(l), int(m)) for (l, m) in modes])
    cfg = Config(len(dets), len(modes), modes_arr, float(srate_hz), int(n_t),
                 d_ref_mpc, gmst_rad, earth_radius_m, t_ref_max_s,
                 PRECISION[precision], int(device),
                 C.c_void_p(stream) if stream else None)
    h = _vp()
    _check(lib().ile_create(C.byref(cfg), C.byref(h)))
    return h


def ile_set_data(h, Q, t0_s, U, V, dets):
    Qa = np.ascontiguousarray(Q, np.complex128)
    n_q = Qa.shape[-1]
    Qf, Qp = _f64(Qa.view(np.float64))
    Uf, Up = _f64(np.ascontiguousarray(U, np.complex128).view(np.float64))
    Vf, Vp = _f64(np.ascontiguousarray(V, np.complex128).view(np.float64))
    darr = (Detector * len(dets))(*[Detector(*d) for d in dets])
    _check(lib().ile_set_data(h, Qp, n_q, float(t0_s), Up, Vp, darr), h)


def ile_eval(h, samples):
    s, sp = _f64(samples)
    n = s.shape[1]
    out = np.empty(n)
    _check(lib().ile_eval(h, sp, n, out.ctypes.data_as(_dp)), h)
    return out


def ile_eval_series(h, samples, n_t):
    s, sp = _f64(samples)
    n = s.shape[1]
    out = np.empty((n, n_t))
    _check(lib().ile_eval_series(h, sp, n, out.ctypes.data_as(_dp)), h)
    return out


def ile_integrate(h, samples, ln_p, ln_q):
    s, sp = _f64(samples)
    lp, lpp = _f64(ln_p)
    lq, lqp = _f64(ln_q)
    r = Result()
    _check(lib().ile_integrate(h, sp, lpp, lqp, s.shape[1], C.byref(r)), h)
    return r.as_dict()


def ile_eval_dev(h, samples_dev, n, out_dev):
    _check(lib().ile_eval_dev(h, _dev(samples_dev), int(n), _dev(out_dev)), h)


def ile_integrate_dev(h, samples_dev, ln_p_dev, ln_q_dev, n, result_dev):
    _check(lib().ile_integrate_dev(h, _dev(samples_dev), _dev(ln_p_dev),
                                   _dev(ln_q_dev), int(n), _dev(result_dev)), h)


def ile_integrate_dev_noalloc(h, samples_dev, ln_p_dev, ln_q_dev, n, result_dev):
    _check(lib().ile_integrate_dev_noalloc(h, _dev(samples_dev), _dev(ln_p_dev),
                                           _dev(ln_q_dev), int(n), _dev(result_dev)), h)


def ile_set_data_fd(h, h_f, d_f, psd, df, f_min, f_max, t0_s, dets, want_data=False):
    """Q, U, V from frequency-domain series (see ile.h); with want_data,
    returns the host Q, U, V it installed."""
    hf = np.ascontiguousarray(h_f, np.complex128)
    dfa = np.ascontiguousarray(d_f, np.complex128)
    ps = np.ascontiguousarray(psd, np.float64)
    n_lm, n_q = hf.shape
    n_det = dfa.shape[0]
    det_arr = (Detector * n_det)(*[Detector(*d) for d in dets])
    Q = np.zeros((n_det, n_lm, n_q), np.complex128) if want_data else None
    U = np.zeros((n_det, n_lm, n_lm), np.complex128) if want_data else None
    V = np.zeros((n_det, n_lm, n_lm), np.complex128) if want_data else None
    vp = (lambda a: a.view(np.float64).ctypes.data_as(_dp)) if want_data else (lambda a: None)
    _check(lib().ile_set_data_fd(h, hf.view(np.float64).ctypes.data_as(_dp),
                                 dfa.view(np.float64).ctypes.data_as(_dp), ps.ctypes.data_as(_dp),
                                 int(n_q), float(df), float(f_min), float(f_max), float(t0_s),
                                 det_arr, vp(Q), vp(U), vp(V)), h)
    return (Q, U, V) if want_data else None


def ile_qvu_fd_dev(h, h_f_dev, d_f_dev, psd_dev, n_q, df, f_min, f_max, t0_s, Q_dev, U_dev,
                   V_dev):
    _check(lib().ile_qvu_fd_dev(h, _dev(h_f_dev), _dev(d_f_dev), _dev(psd_dev), int(n_q),
                                float(df), float(f_min), float(f_max), float(t0_s),
                                _dev(Q_dev), _dev(U_dev), _dev(V_dev)), h)


def ile_rom_set(h, modes, A):
    """Surrogate form (see ile.h): physical modes [(l, m)] and the complex
    coefficient table A [n_lm][n_b][n_pow]."""
    a = np.ascontiguousarray(A, np.complex128)
    marr = (Mode * len(modes))(*[Mode(int(l), int(m)) for (l, m) in modes])
    _check(lib().ile_rom_set(h, marr, len(modes), int(a.shape[2]),
                             a.view(np.float64).ctypes.data_as(_dp)), h)


def ile_rom_eval_dev(h, samples_dev, n, out_dev):
    _check(lib().ile_rom_eval_dev(h, _dev(samples_dev), int(n), _dev(out_dev)), h)


def ile_rom_integrate_dev(h, samples_dev, ln_p_dev, ln_q_dev, n, result_dev):
    _check(lib().ile_rom_integrate_dev(h, _dev(samples_dev), _dev(ln_p_dev), _dev(ln_q_dev),
                                       int(n), _dev(result_dev)), h)


def ile_harvest_dev(h, samples_dev, ln_p_dev, ln_q_dev, n, u_dev, n_out, idx_dev,
                    bin_dev, theta_dev=None, result_dev=None):
    _check(lib().ile_harvest_dev(h, _dev(samples_dev), _dev(ln_p_dev), _dev(ln_q_dev),
                                 int(n), _dev(u_dev), int(n_out), _dev(idx_dev),
                                 _dev(bin_dev), _dev(theta_dev), _dev(result_dev)), h)


def ile_draw_prior_dev(h, seed, first, n, d_min, d_max, samples_dev, ld,
                       ln_p_dev=None):
    _check(lib().ile_draw_prior_dev(h, int(seed), int(first), int(n), float(d_min),
                                    float(d_max), _dev(samples_dev), int(ld),
                                    _dev(ln_p_dev)), h)


def ile_run_prior(h, seed, n, chunk, d_min=10.0, d_max=1000.0):
    r = Result()
    _check(lib().ile_run_prior(h, int(seed), int(n), int(chunk), float(d_min),
                               float(d_max), C.byref(r)), h)
    return r.as_dict()


def ile_run(h, sampler="adaptive", seed=1, chunk=100_000, max_samples=1_000_000,
            n_eff_target=0.0, d_min=10.0, d_max=1000.0, n_bins=50, floor=0.1,
            temper=10.0, adapt_chunks=-1, reset=True, prop=None, eps=-1.0,
            fallback_neff=-1.0, train_steps=0, train_batch=0, lr=0.0, refine_rounds=-1,
            refine_steps=0, refine_eff=0.0, train_ess=0.0, refine_kish=0.0, sigma_scale=0.0,
            warm=False):
    o = RunOpts(SAMPLER[sampler], int(seed), int(chunk), int(max_samples),
                float(n_eff_target), float(d_min), float(d_max), int(n_bins),
                float(floor), float(temper), int(adapt_chunks), 1 if reset else 0,
                prop, float(eps), float(fallback_neff), int(train_steps),
                int(train_batch), float(lr), int(refine_rounds), int(refine_steps),
                float(refine_eff), float(train_ess), float(refine_kish), float(sigma_scale),
                1 if warm else 0)
    r = Result()
    nc = C.c_int64()
    _check(lib().ile_run(h, C.byref(o), C.byref(r), C.byref(nc)), h)
    d = r.as_dict()
    d["n_chunks"] = nc.value
    if sampler == "learned":
        li = LearnedInfo()
        _check(lib().ile_last_learned_info(h, C.byref(li)), h)
        d.update({f: getattr(li, f) for f, _ in li._fields_
                  if f not in ("refine_eff", "refine_kish")})
        nr = d["n_refine_samples"] // max(int(chunk), 1)
        d["refine_eff"] = [li.refine_eff[i] for i in range(min(nr, 32))]
        d["refine_kish"] = [li.refine_kish[i] for i in range(min(nr, 32))]
    return d


def ile_inject(h, h_lm, t0_s, dets, theta, snr=0.0, want_data=False):
    """Device zero-noise injection (see ile.h); returns (rho2, d_inj) and,
    with want_data, the host Q, U, V it installed."""
    hl = np.ascontiguousarray(h_lm, np.complex128)
    n_lm, n_q = hl.shape
    hv = hl.view(np.float64)
    th, thp = _f64(theta)
    d = (Detector * len(dets))(*[Detector(*x) for x in dets])
    rho2, dinj = C.c_double(), C.c_double()
    outs = [None, None, None]
    if want_data:
        n_det = len(dets)
        outs = [np.zeros((n_det, n_lm, n_q), np.complex128),
                np.zeros((n_det, n_lm, n_lm), np.complex128),
                np.zeros((n_det, n_lm, n_lm), np.complex128)]
    ptr = [None if o is None else o.view(np.float64).ctypes.data_as(_dp) for o in outs]
    _check(lib().ile_inject(h, hv.ctypes.data_as(_dp), int(n_q), float(t0_s), d, thp,
                            float(snr), C.byref(rho2), C.byref(dinj), *ptr), h)
    if want_data:
        return rho2.value, dinj.value, outs[0], outs[1], outs[2]
    return rho2.value, dinj.value


def ile_get_stream(h):
    s = _vp()
    _check(lib().ile_get_stream(h, C.byref(s)), h)
    return s.value


def ile_hist_get(h, n_bins):
    a = np.zeros(n_bins)
    b = np.zeros(n_bins)
    _check(lib().ile_hist_get(h, int(n_bins), a.ctypes.data_as(_dp),
                              b.ctypes.data_as(_dp)), h)
    return a, b


def ile_hist_set(h, P_ra, P_sd):
    a, ap = _f64(P_ra)
    b, bp = _f64(P_sd)
    _check(lib().ile_hist_set(h, int(a.size), ap, bp), h)


def ile_hist_draw_dev(h, seed, first, n, d_min, d_max, samples_dev, ld,
                      ln_p_dev=None, ln_q_dev=None, bins_dev=None):
    _check(lib().ile_hist_draw_dev(h, int(seed), int(first), int(n), float(d_min),
                                   float(d_max), _dev(samples_dev), int(ld),
                                   _dev(ln_p_dev), _dev(ln_q_dev), _dev(bins_dev)), h)


def ile_hist_refit_dev(h, bins_dev, ld, lnL_dev, ln_p_dev, ln_q_dev, n, floor=0.1,
                       temper=10.0):
    _check(lib().ile_hist_refit_dev(h, _dev(bins_dev), int(ld), _dev(lnL_dev),
                                    _dev(ln_p_dev), _dev(ln_q_dev), int(n), float(floor),
                                    float(temper)), h)


def ile_sync(h):
    _check(lib().ile_sync(h), h)


def ile_set_option(h, opt, value):
    _check(lib().ile_set_option(h, int(opt), int(value)), h)


def ile_last_kernel_ms(h):
    return lib().ile_last_kernel_ms(h)


def ile_destroy(h):
    lib().ile_destroy(h)


# -------------------------------------------------------------- Context
class Context:
    """One intrinsic point on one GPU: create + set_data, then evaluate."""

    def __init__(self, inst, precision="fp64", device=0, stream=None, sort=True,
                 engine=None, threads=None, lds_kb=None):
        self.inst = inst
        self.n_t = inst.n_t
        self.h = ile_create(inst.dets, inst.modes, inst.srate_hz, inst.n_t,
                            d_ref_mpc=inst.d_ref_mpc, gmst_rad=inst.gmst_rad,
                            earth_radius_m=inst.earth_radius_m,
                            t_ref_max_s=inst.t_ref_max_s, precision=precision,
                            device=device, stream=stream)
        try:
            ile_set_data(self.h, inst.Q, inst.t0_s, inst.U, inst.V, inst.dets)
            if not sort:
                ile_set_option(self.h, ILE_OPT_SORT, 0)
            if engine is not None:
                ile_set_option(self.h, ILE_OPT_ENGINE,
                               {"valu": 0, "mfma": 1, "pipelined": 2}[engine])
            if threads is not None:
                ile_set_option(self.h, ILE_OPT_THREADS, threads)
            if lds_kb is not None:
                ile_set_option(self.h, ILE_OPT_LDS_KB, lds_kb)
        except Exception:
            self.close()
            raise

    def eval(self, samples):
        return ile_eval(self.h, samples)

    def eval_series(self, samples):
        return ile_eval_series(self.h, samples, self.n_t)

    def integrate(self, samples, ln_p, ln_q):
        return ile_integrate(self.h, samples, ln_p, ln_q)

    def eval_dev(self, samples_dev, n, out_dev):
        ile_eval_dev(self.h, samples_dev, n, out_dev)

    def integrate_dev(self, samples_dev, ln_p_dev, ln_q_dev, n, result_dev):
        ile_integrate_dev(self.h, samples_dev, ln_p_dev, ln_q_dev, n, result_dev)

    def integrate_dev_noalloc(self, samples_dev, ln_p_dev, ln_q_dev, n, result_dev):
        ile_integrate_dev_noalloc(self.h, samples_dev, ln_p_dev, ln_q_dev, n, result_dev)

    def harvest_dev(self, samples_dev, ln_p_dev, ln_q_dev, n, u_dev, n_out, idx_dev,
                    bin_dev, theta_dev=None, result_dev=None):
        ile_harvest_dev(self.h, samples_dev, ln_p_dev, ln_q_dev, n, u_dev, n_out, idx_dev,
                        bin_dev, theta_dev, result_dev)

    def draw_prior_dev(self, seed, first, n, samples_dev, ld, ln_p_dev=None,
                       d_min=10.0, d_max=1000.0):
        ile_draw_prior_dev(self.h, seed, first, n, d_min, d_max, samples_dev, ld,
                           ln_p_dev)

    def run_prior(self, seed, n, chunk=0, d_min=10.0, d_max=1000.0):
        return ile_run_prior(self.h, seed, n, chunk, d_min, d_max)

    def run(self, **kw):
        if isinstance(kw.get("prop"), Proposal):
            kw["prop"] = kw["prop"].h
        return ile_run(self.h, **kw)

    def stream(self):
        """The context's hipStream_t (as an integer)."""
        return ile_get_stream(self.h)

    def sync(self):
        ile_sync(self.h)

    def set_sort(self, on):
        ile_set_option(self.h, ILE_OPT_SORT, 1 if on else 0)

    def last_kernel_ms(self):
        return ile_last_kernel_ms(self.h)

    def close(self):
        if getattr(self, "h", None):
            ile_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ batched form
def _bcheck(status, b):
    if status != ILE_OK:
        m = lib().ile_batch_last_error(b) if b else b""
        raise IleError(status, (m or b"").decode() or lib().ile_status_string(status).decode())


class Batch:
    """Many intrinsic points evaluated in one graph-captured run
    (ile_batch_* of include/ile.h)."""

    def __init__(self, precision="fp32", device=0, stream=None):
        cfg = BatchConfig(PRECISION[precision], int(device),
                          C.c_void_p(stream) if stream else None)
        self.h = _vp()
        _bcheck(lib().ile_batch_create(C.byref(cfg), C.byref(self.h)), None)

    def add_point(self, inst):
        modes_arr = (Mode * inst.n_lm)(*[Mode(int(l), int(m)) for (l, m) in inst.modes])
        cfg = Config(inst.n_det, inst.n_lm, modes_arr, float(inst.srate_hz), int(inst.n_t),
                     inst.d_ref_mpc, inst.gmst_rad, inst.earth_radius_m, inst.t_ref_max_s,
                     0, 0, None)
        Qa = np.ascontiguousarray(inst.Q, np.complex128)
        Qf, Qp = _f64(Qa.view(np.float64))
        Uf, Up = _f64(np.ascontiguousarray(inst.U, np.complex128).view(np.float64))
        Vf, Vp = _f64(np.ascontiguousarray(inst.V, np.complex128).view(np.float64))
        darr = (Detector * inst.n_det)(*[Detector(*d) for d in inst.dets])
        pid = C.c_int32()
        _bcheck(lib().ile_batch_add_point(self.h, C.byref(cfg), Qp, Qa.shape[-1],
                                          float(inst.t0_s), Up, Vp, darr, C.byref(pid)),
                self.h)
        return pid.value

    @property
    def n_points(self):
        return lib().ile_batch_n_points(self.h)

    def run(self, seed, n_per_point, d_min=10.0, d_max=1000.0):
        res = (Result * self.n_points)()
        _bcheck(lib().ile_batch_run(self.h, int(seed), int(n_per_point), float(d_min),
                                    float(d_max), res), self.h)
        return [r.as_dict() for r in res]

    def run_dev(self, n_per_point, samples_dev, ln_p_dev=None, ln_q_dev=None):
        """Evaluate caller-supplied device draws: samples_dev [P][7][n],
        ln_p_dev / ln_q_dev [P][n] (None = 0)."""
        res = (Result * self.n_points)()
        _bcheck(lib().ile_batch_run_dev(self.h, int(n_per_point), _dev(samples_dev),
                                        _dev(ln_p_dev), _dev(ln_q_dev), res), self.h)
        return [r.as_dict() for r in res]

    def lnL(self, n_per_point):
        out = np.empty(self.n_points * int(n_per_point))
        _bcheck(lib().ile_batch_lnL(self.h, out.ctypes.data_as(_dp), out.size), self.h)
        return out.reshape(self.n_points, -1)

    def set_tuning(self, threads=256, wgs_per_cu=2, order=0, engine=1):
        t = BatchTuning(threads, wgs_per_cu, order, engine)
        _bcheck(lib().ile_batch_set_tuning(self.h, C.byref(t)), self.h)

    def get_tuning(self):
        t = BatchTuning()
        _bcheck(lib().ile_batch_get_tuning(self.h, C.byref(t)), self.h)
        return dict(threads=t.threads, wgs_per_cu=t.wgs_per_cu, order=t.order, engine=t.engine)

    def autotune(self, n_per_point, cache_path=None):
        _bcheck(lib().ile_batch_autotune(self.h, int(n_per_point),
                                         cache_path.encode() if cache_path else None), self.h)
        return self.get_tuning()

    def last_ms(self):
        return lib().ile_batch_last_ms(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().ile_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -------------------------------------------------------- learned proposal
def _pcheck(status, p):
    if status != ILE_OK:
        m = lib().ile_prop_last_error(p) if p else b""
        raise IleError(status, (m or b"").decode() or lib().ile_status_string(status).decode())


class Proposal:
    """The learned proposal (ile_prop_*).  Pass ctx to share its stream and
    its histograms (for the defensive mixture)."""

    def __init__(self, ctx=None, *, d_min=10.0, d_max=1000.0, t_ref_max=0.01,
                 sigma_floor=1e-3, seed=1, device=0, stream=None, sigma_scale=1.0):
        if ctx is not None and stream is None:
            stream = ctx.stream()
        self.ctx = ctx
        cfg = PropConfig(float(d_min), float(d_max), float(t_ref_max), float(sigma_floor),
                         int(seed), int(device), stream, float(sigma_scale))
        h = _vp()
        st = lib().ile_prop_create(C.byref(cfg), C.byref(h))
        if st != ILE_OK:
            raise IleError(st, lib().ile_status_string(st).decode())
        self.h = h.value

    def set_params(self, params):
        a = np.ascontiguousarray(params, np.float32)
        assert a.size == PROP_NPARAM
        _pcheck(lib().ile_prop_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))),
                self.h)

    def get_params(self):
        a = np.zeros(PROP_NPARAM, np.float32)
        _pcheck(lib().ile_prop_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))),
                self.h)
        return a

    def set_transform(self, origin, mean, scale):
        o, op = _f64(origin)
        m, mp = _f64(mean)
        s, sp = _f64(scale)
        _pcheck(lib().ile_prop_set_transform(self.h, op, mp, sp), self.h)

    def set_sigma_scale(self, kappa):
        _pcheck(lib().ile_prop_set_sigma_scale(self.h, float(kappa)), self.h)

    def get_transform(self):
        o, m, s = np.zeros(3), np.zeros(7), np.zeros(7)
        _pcheck(lib().ile_prop_get_transform(self.h, o.ctypes.data_as(_dp),
                                             m.ctypes.data_as(_dp), s.ctypes.data_as(_dp)),
                self.h)
        return o, m, s

    def fit_transform_dev(self, x_dev, ld, lnw_dev, n, ess_frac=0.01):
        _pcheck(lib().ile_prop_fit_transform_dev(self.h, _dev(x_dev), int(ld), _dev(lnw_dev),
                                                 int(n), float(ess_frac)), self.h)

    def grad_dev(self, x_dev, ld, n, w_dev=None, grad_dev=None):
        loss = C.c_double()
        _pcheck(lib().ile_prop_grad_dev(self.h, _dev(x_dev), int(ld), _dev(w_dev), int(n),
                                        _dev(grad_dev), C.byref(loss)), self.h)
        return loss.value

    def train_dev(self, x_dev, ld, lnw_dev, n, *, steps=1000, batch=4096, lr=1e-3,
                  ess_frac=0.01, seed=1, fit_transform=True):
        o = PropTrainOpts(int(steps), int(batch), float(lr), float(ess_frac), int(seed),
                          1 if fit_transform else 0)
        loss = C.c_double()
        _pcheck(lib().ile_prop_train_dev(self.h, _dev(x_dev), int(ld), _dev(lnw_dev), int(n),
                                         C.byref(o), C.byref(loss)), self.h)
        return loss.value

    def logpdf_dev(self, x_dev, ld, n, lnq_dev, eps=0.0):
        mix = self.ctx.h if (self.ctx is not None and eps > 0) else None
        _pcheck(lib().ile_prop_logpdf_dev(self.h, mix, float(eps), _dev(x_dev), int(ld),
                                          int(n), _dev(lnq_dev)), self.h)

    def sample_dev(self, seed, first, n, x_dev, ld, lnp_dev, lnq_dev, eps=0.0):
        mix = self.ctx.h if (self.ctx is not None and eps > 0) else None
        _pcheck(lib().ile_prop_sample_dev(self.h, mix, float(eps), int(seed), int(first),
                                          int(n), _dev(x_dev), int(ld), _dev(lnp_dev),
                                          _dev(lnq_dev)), self.h)

    def sync(self):
        _pcheck(lib().ile_prop_sync(self.h), self.h)

    def last_ms(self):
        return lib().ile_prop_last_ms(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().ile_prop_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
