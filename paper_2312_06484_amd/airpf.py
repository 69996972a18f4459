"""Thin ctypes binding of the AIRPF C ABI (include/airpf.h).

Argument marshalling only: every step of the filter runs in the HIP kernels
of libairpf.so.  The library must have been built (``__graft_entry__.build()``
or ``python paper_2312_06484_amd/build.py``); there is no fallback path.

Naming follows the paper: m islands (filters), N particles per island (the
paper's M), T observations, tau the ENF threshold of Algorithm 1.
"""
import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libairpf.so")

LG1, SV, LGD, BIN, BCP = 0, 1, 2, 3, 4
SYSTEMATIC, MULTINOMIAL = 0, 1
FP32, FP64 = 0, 1
PATHSPACE, PATHWISE = 0, 1
FLAG_Y_ON_DEVICE = 1
FLAG_AUTOTUNE = 2

OK, E_INVALID_ARG, E_DOMAIN, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_TOO_LARGE = range(7)

# every symbol include/airpf.h declares
EXPORTS = ["airpf_ctx_create", "airpf_ctx_destroy", "airpf_run", "airpf_run_noalloc", "airpf_score",
           "airpf_run_batch", "airpf_status_str", "airpf_ctx_last_kernel_ms", "airpf_debug_eval"]

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)
_u64p = C.POINTER(C.c_uint64)


class AirpfError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, status_str(status), status))


class _Model(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dx", C.c_int32), ("dy", C.c_int32),
                ("consts", _dp), ("n_consts", C.c_int32)]


class _Options(C.Structure):
    _fields_ = [("tau", C.c_double), ("resampling", C.c_int32), ("precision", C.c_int32),
                ("score_mode", C.c_int32), ("ckpt_every", C.c_int32), ("flags", C.c_uint32),
                ("resample_ess", C.c_double), ("arity", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("theta", _dp), ("d_theta", C.c_int32), ("y", C.c_void_p), ("T", C.c_int64),
                ("m", C.c_int32), ("N", C.c_int32), ("seed", C.c_uint64)]


class _Trace(C.Structure):
    _fields_ = [("sstar", _i32p), ("enf", _dp), ("lpost", _dp), ("anc", _i32p),
                ("pi", _i32p), ("digest", _u64p), ("fmean", _dp)]


_lib = None
_live = weakref.WeakSet()          # open contexts, closed at interpreter exit


def _close_all():
    """At interpreter exit: destroy every open context (each synchronises its
    stream first), so no work of this library is in flight when the process
    tears down the HIP runtime."""
    for ctx in list(_live):
        try:
            ctx.close()
        except Exception:
            pass


def lib():
    """Load libairpf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libairpf.so is missing: build it with paper_2312_06484_amd/build.py "
                               "(or __graft_entry__.build()); the filter has no CPU fallback")
        # torch first: its HIP runtime (soname libamdhip64.so.7) is then the
        # one the library binds to.  Loaded the other way round, torch would
        # bring up a second HIP/HSA runtime by file name that finds no device.
        import torch  # noqa: F401
        L = C.CDLL(LIBPATH)
        L.airpf_status_str.restype = C.c_char_p
        L.airpf_status_str.argtypes = [C.c_int]
        L.airpf_ctx_create.restype = C.c_int
        L.airpf_ctx_create.argtypes = [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
        L.airpf_ctx_destroy.restype = C.c_int
        L.airpf_ctx_destroy.argtypes = [C.c_void_p]
        L.airpf_run.restype = C.c_int
        L.airpf_run.argtypes = [C.c_void_p, C.POINTER(_Model), _dp, C.c_int32, C.c_void_p, C.c_int64,
                                C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_Options), _dp,
                                C.POINTER(_Trace)]
        L.airpf_run_noalloc.restype = C.c_int
        L.airpf_run_noalloc.argtypes = [C.c_void_p, C.POINTER(_Model), _dp, C.c_int32, C.c_void_p, C.c_int64,
                                        C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_Options), _dp]
        L.airpf_score.restype = C.c_int
        L.airpf_score.argtypes = [C.c_void_p, C.POINTER(_Model), _dp, C.c_int32, C.c_void_p, C.c_int64,
                                  C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_Options), _dp, _dp,
                                  C.POINTER(_Trace)]
        L.airpf_run_batch.restype = C.c_int
        L.airpf_run_batch.argtypes = [C.c_void_p, C.POINTER(_Model), C.c_int32, C.POINTER(_Problem),
                                      C.POINTER(_Options), C.c_int32, _dp, _dp, C.POINTER(C.c_int)]
        L.airpf_ctx_last_kernel_ms.restype = C.c_int
        L.airpf_ctx_last_kernel_ms.argtypes = [C.c_void_p, _dp]
        L.airpf_debug_eval.restype = C.c_int
        L.airpf_debug_eval.argtypes = [C.c_void_p, C.c_int32, C.c_int64, _dp, _u32p, _dp, _dp, _u32p]
        _lib = L
        atexit.register(_close_all)
    return _lib


def status_str(s):
    return lib().airpf_status_str(int(s)).decode()


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


class Trace:
    """Host arrays a run fills (see airpf_trace in include/airpf.h)."""

    def __init__(self, T, m, N, sstar=True, enf=True, lpost=True, anc=True, pi=True, digest=True, fmean=False):
        S = int(m).bit_length() - 1
        self.sstar = np.zeros(T, np.int32) if sstar else None
        self.enf = np.zeros(T * (S + 1)) if enf else None
        self.lpost = np.zeros(T * m) if lpost else None
        self.anc = np.zeros(max(T - 1, 0) * m * N, np.int32) if anc else None
        self.pi = np.zeros(max(T - 1, 0) * m, np.int32) if pi else None
        self.digest = np.zeros(2 * T, np.uint64) if digest else None
        self.fmean = np.zeros(T * m) if fmean else None

    def _c(self):
        t = _Trace()
        t.sstar, t.enf, t.lpost = _p(self.sstar, _i32p), _p(self.enf, _dp), _p(self.lpost, _dp)
        t.anc, t.pi, t.digest = _p(self.anc, _i32p), _p(self.pi, _i32p), _p(self.digest, _u64p)
        t.fmean = _p(self.fmean, _dp)
        return t


class Context:
    """An airpf_ctx: device workspaces reused across calls."""

    def __init__(self, device=0, stream=None):
        self._h = C.c_void_p()
        st = lib().airpf_ctx_create(int(device), C.c_void_p(stream) if stream else None, C.byref(self._h))
        if st != OK:
            raise AirpfError(st, "airpf_ctx_create")
        _live.add(self)

    def close(self):
        if self._h:
            lib().airpf_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------ calls

    @staticmethod
    def _args(kind, theta, y, tau, fp64, dx, dy, consts, y_device_ptr, T, score_mode=PATHSPACE, ckpt_every=0,
              resampling=SYSTEMATIC, resample_ess=0.0, arity=2):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        model = _Model()
        model.kind, model.dx, model.dy = int(kind), int(dx), int(dy)
        cst = None if consts is None else np.ascontiguousarray(consts, dtype=np.float64)
        model.consts = _p(cst, _dp)
        model.n_consts = 0 if cst is None else cst.size
        opt = _Options()
        opt.tau, opt.resampling, opt.precision = float(tau), int(resampling), FP64 if fp64 else FP32
        opt.score_mode, opt.ckpt_every, opt.flags = int(score_mode), int(ckpt_every), 0
        opt.resample_ess, opt.arity = float(resample_ess), int(arity)
        if y_device_ptr is not None:
            ptr = C.c_void_p(int(y_device_ptr))
            opt.flags |= FLAG_Y_ON_DEVICE
            Tn = int(T)
            yy = None
        else:
            yy = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
            ptr = yy.ctypes.data_as(C.c_void_p)
            Tn = yy.size // int(dy)
        return theta, model, cst, opt, ptr, Tn, yy

    def run(self, kind, theta, y, m, N, seed, tau=0.3, fp64=False, dx=1, dy=1, consts=None,
            trace=None, y_device_ptr=None, T=None, raise_on_error=True, resampling=SYSTEMATIC, resample_ess=0.0,
            arity=2):
        """airpf_run: returns (status, log Zhat).  ``y`` is a host array, or
        pass ``y_device_ptr`` (int) and ``T`` for observations already in HBM.
        ``resampling``: SYSTEMATIC or MULTINOMIAL internal resampling;
        ``resample_ess`` > 0: adaptive internal resampling (an island
        resamples iff its ESS < resample_ess * N); ``arity`` r: islands
        interact in groups of r (m a power of r)."""
        theta, model, cst, opt, ptr, Tn, keep = self._args(kind, theta, y, tau, fp64, dx, dy, consts,
                                                           y_device_ptr, T, resampling=resampling,
                                                           resample_ess=resample_ess, arity=arity)
        out = C.c_double(np.nan)
        tr = trace._c() if trace is not None else None
        st = lib().airpf_run(self._h, C.byref(model), _p(theta, _dp), theta.size, ptr, Tn, int(m), int(N),
                             C.c_uint64(int(seed)), C.byref(opt), C.byref(out),
                             C.byref(tr) if tr is not None else None)
        if st != OK and raise_on_error:
            raise AirpfError(st, "airpf_run")
        return st, out.value

    def run_noalloc(self, kind, theta, y, m, N, seed, tau=0.3, fp64=False, dx=1, dy=1, consts=None,
                    y_device_ptr=None, T=None, raise_on_error=True, resampling=SYSTEMATIC, resample_ess=0.0,
                    arity=2):
        """airpf_run_noalloc (workspaces in the library's fixed device
        scratch, nothing allocated): returns (status, log Zhat)."""
        theta, model, cst, opt, ptr, Tn, keep = self._args(kind, theta, y, tau, fp64, dx, dy, consts,
                                                           y_device_ptr, T, resampling=resampling,
                                                           resample_ess=resample_ess, arity=arity)
        out = C.c_double(np.nan)
        st = lib().airpf_run_noalloc(self._h, C.byref(model), _p(theta, _dp), theta.size, ptr, Tn, int(m), int(N),
                                     C.c_uint64(int(seed)), C.byref(opt), C.byref(out))
        if st != OK and raise_on_error:
            raise AirpfError(st, "airpf_run_noalloc")
        return st, out.value

    def score(self, kind, theta, y, m, N, seed, tau=0.3, fp64=False, dx=1, dy=1, consts=None,
              ckpt_every=0, score_mode=PATHSPACE, trace=None, y_device_ptr=None, T=None, raise_on_error=True,
              resampling=SYSTEMATIC, resample_ess=0.0, arity=2):
        """airpf_score: returns (status, log Zhat, gradient)."""
        theta, model, cst, opt, ptr, Tn, keep = self._args(kind, theta, y, tau, fp64, dx, dy, consts,
                                                           y_device_ptr, T, score_mode, ckpt_every, resampling,
                                                           resample_ess, arity)
        out = C.c_double(np.nan)
        grad = np.full(theta.size, np.nan)
        tr = trace._c() if trace is not None else None
        st = lib().airpf_score(self._h, C.byref(model), _p(theta, _dp), theta.size, ptr, Tn, int(m), int(N),
                               C.c_uint64(int(seed)), C.byref(opt), C.byref(out), _p(grad, _dp),
                               C.byref(tr) if tr is not None else None)
        if st != OK and raise_on_error:
            raise AirpfError(st, "airpf_score")
        return st, out.value, grad

    def run_batch(self, kind, problems, tau=0.3, fp64=False, dx=1, dy=1, consts=None, want_score=False,
                  ckpt_every=0, y_on_device=False, autotune=False, raise_on_error=True, resampling=SYSTEMATIC,
                  score_mode=PATHSPACE, resample_ess=0.0, arity=2):
        """airpf_run_batch.  ``problems``: dicts with theta, y (host array, or a
        device pointer int with ``y_on_device`` and then T), m, N, seed;
        ``autotune`` sets AIRPF_FLAG_AUTOTUNE (measured tiling, cached per
        batch shape in the context); ``resampling`` MULTINOMIAL is forward
        only.
        Returns (status, log_z[B], grad[B, d_theta] or None, item_status[B])."""
        B = len(problems)
        model = _Model()
        model.kind, model.dx, model.dy = int(kind), int(dx), int(dy)
        cst = None if consts is None else np.ascontiguousarray(consts, dtype=np.float64)
        model.consts = _p(cst, _dp)
        model.n_consts = 0 if cst is None else cst.size
        opt = _Options()
        opt.tau, opt.resampling, opt.precision = float(tau), int(resampling), FP64 if fp64 else FP32
        opt.score_mode, opt.ckpt_every = int(score_mode), int(ckpt_every)
        opt.resample_ess, opt.arity = float(resample_ess), int(arity)
        opt.flags = (FLAG_Y_ON_DEVICE if y_on_device else 0) | (FLAG_AUTOTUNE if autotune else 0)
        arr = (_Problem * max(B, 1))()
        keep = []
        for i, pr in enumerate(problems):
            th = np.ascontiguousarray(pr["theta"], dtype=np.float64)
            keep.append(th)
            arr[i].theta, arr[i].d_theta = _p(th, _dp), th.size
            if y_on_device:
                arr[i].y, arr[i].T = C.c_void_p(int(pr["y"])), int(pr["T"])
            else:
                yy = np.ascontiguousarray(pr["y"], dtype=np.float64).reshape(-1)
                keep.append(yy)
                arr[i].y, arr[i].T = yy.ctypes.data_as(C.c_void_p), yy.size // int(dy)
            arr[i].m, arr[i].N, arr[i].seed = int(pr["m"]), int(pr["N"]), int(pr["seed"])
        P = int(dx) * int(dx) if kind == LGD else {BIN: 0, BCP: 1}.get(kind, 3)
        lz = np.full(max(B, 1), np.nan)
        gr = np.full((max(B, 1), P), np.nan) if want_score else None
        ist = (C.c_int * max(B, 1))()
        st = lib().airpf_run_batch(self._h, C.byref(model), B, arr, C.byref(opt), int(bool(want_score)),
                                   _p(lz, _dp), _p(gr, _dp) if gr is not None else None, ist)
        if st != OK and raise_on_error:
            raise AirpfError(st, "airpf_run_batch")
        return st, lz[:B], (gr[:B] if gr is not None else None), np.array(ist[:B])

    def last_kernel_ms(self):
        """Event-timed device duration of the last call's filter kernel (ms)."""
        v = C.c_double()
        st = lib().airpf_ctx_last_kernel_ms(self._h, C.byref(v))
        if st != OK:
            raise AirpfError(st, "airpf_ctx_last_kernel_ms")
        return v.value

    def debug_eval(self, which, values=None, words=None):
        """Evaluate the device's own exp (0), log (1), cossin 2 pi (2),
        Box-Muller (3) or Philox (4) on host arrays; 5-8 are the binary32
        exp, log, cossin and Box-Muller."""
        L = lib()
        if which in (0, 1, 2, 5, 6, 7):
            v = np.ascontiguousarray(values, dtype=np.float64)
            n = v.size
            out, out2 = np.zeros(n), np.zeros(n)
            st = L.airpf_debug_eval(self._h, which, n, _p(v, _dp), None, _p(out, _dp), _p(out2, _dp), None)
            if st != OK:
                raise AirpfError(st, "airpf_debug_eval")
            return (out, out2) if which in (2, 7) else out
        w = np.ascontiguousarray(words, dtype=np.uint32)
        if which in (3, 8):
            n = w.size // 2
            out, out2 = np.zeros(n), np.zeros(n)
            st = L.airpf_debug_eval(self._h, which, n, None, _p(w, _u32p), _p(out, _dp), _p(out2, _dp), None)
            if st != OK:
                raise AirpfError(st, "airpf_debug_eval")
            return out, out2
        n = w.size // 6
        o = np.zeros(4 * n, np.uint32)
        st = L.airpf_debug_eval(self._h, 4, n, None, _p(w, _u32p), None, None, _p(o, _u32p))
        if st != OK:
            raise AirpfError(st, "airpf_debug_eval")
        return o.reshape(n, 4)
