"""ctypes front end of the AIRPF CPU oracle (oracle/liborc.so).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Shares no code with
the HIP library.

Model kinds and parameters (Section 1.2's HMM; concrete models as stated in
orc_models.c):
    LG1 theta = (a, sx, sy);  SV theta = (mu, phi, sigma);
    LGD theta = vec(A), consts = (q, r, p0, H.ravel());  BIN (toy HMM);
    BCP theta = (p,), consts = (alpha, beta) integers, alpha + beta <= 7,
    dx = dy = 2, y rows (k_n, n_n).
Argument ``N`` is the number of particles PER ISLAND (the paper's M).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liborc.so")

LG1, SV, LGD, BIN, BCP = 0, 1, 2, 3, 4
TAG_NORMAL, TAG_SYS, TAG_MULT, TAG_ISL, TAG_BIN, TAG_BCP = 1, 2, 3, 4, 5, 6

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_u64p = C.POINTER(C.c_uint64)


class _Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dx", C.c_int32), ("dy", C.c_int32),
                ("d_theta", C.c_int32), ("theta", _dp), ("consts", _dp),
                ("y", _dp), ("T", C.c_int64), ("m", C.c_int32), ("N", C.c_int32),
                ("seed", C.c_uint64)]


class _Opts(C.Structure):
    _fields_ = [("tau", C.c_double), ("scheme", C.c_int32),
                ("f32", C.c_int32), ("replay", C.c_int32),
                ("exact_weights", C.c_int32), ("ess_frac", C.c_double), ("arity", C.c_int32)]


class _Trace(C.Structure):
    _fields_ = [("sstar", _i32p), ("enf", _dp), ("lpost", _dp), ("anc", _i32p),
                ("pi", _i32p), ("digest", _u64p), ("x", _dp), ("logz_inc", _dp), ("fmean", _dp),
                ("lpre", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIBPATH)
        L.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_exp.restype = C.c_double; L.orc_exp.argtypes = [C.c_double]
        L.orc_log.restype = C.c_double; L.orc_log.argtypes = [C.c_double]
        L.orc_cossin2pi.argtypes = [C.c_double, _dp, _dp]
        L.orc_boxmuller.argtypes = [C.c_uint32, C.c_uint32, _dp, _dp]
        L.orc_expf.restype = C.c_float; L.orc_expf.argtypes = [C.c_float]
        L.orc_logf.restype = C.c_float; L.orc_logf.argtypes = [C.c_float]
        L.orc_cossin2pif.argtypes = [C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_boxmullerf.argtypes = [C.c_uint32, C.c_uint32, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_island_normalsf.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int64, _dp]
        L.orc_u53.restype = C.c_double; L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_bounded.restype = C.c_uint64
        L.orc_bounded.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
        L.orc_island_normals.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int64, _dp]
        L.orc_quantise.argtypes = [_dp, C.c_int32, _u64p, _dp]
        L.orc_systematic.argtypes = [_u64p, C.c_int32, C.c_uint64, _i32p]
        L.orc_digest_term.restype = C.c_uint64
        L.orc_digest_term.argtypes = [C.c_int64] * 4
        L.orc_airpf_run.restype = C.c_double
        L.orc_airpf_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.POINTER(_Trace)]
        L.orc_airpf_score.restype = C.c_double
        L.orc_airpf_score.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.POINTER(_Trace), _dp, _dp]
        L.orc_airpf_frozen.restype = C.c_double
        L.orc_airpf_frozen.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.POINTER(_Trace), _dp, _dp]
        L.orc_bpf_run.restype = C.c_double
        L.orc_bpf_run.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_int32, _i32p]
        _lib = L
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


# ---------------------------------------------------------------- primitives

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return tuple(o)


def exp(x):
    return lib().orc_exp(float(x))


def log(x):
    return lib().orc_log(float(x))


def cossin2pi(v):
    c, s = C.c_double(), C.c_double()
    lib().orc_cossin2pi(float(v), C.byref(c), C.byref(s))
    return c.value, s.value


def boxmuller(wa, wb):
    a, b = C.c_double(), C.c_double()
    lib().orc_boxmuller(int(wa), int(wb), C.byref(a), C.byref(b))
    return a.value, b.value


def expf(x):
    """binary32 counterpart of exp (runs with binary32 particles)"""
    return lib().orc_expf(float(x))


def logf(x):
    return lib().orc_logf(float(x))


def cossin2pif(v):
    c, s = C.c_float(), C.c_float()
    lib().orc_cossin2pif(float(v), C.byref(c), C.byref(s))
    return c.value, s.value


def boxmullerf(wa, wb):
    a, b = C.c_float(), C.c_float()
    lib().orc_boxmullerf(int(wa), int(wb), C.byref(a), C.byref(b))
    return a.value, b.value


def island_normalsf(seed, n, k, count):
    z = np.zeros(count, dtype=np.float64)
    lib().orc_island_normalsf(int(seed), int(n), int(k), int(count), _ptr(z, _dp))
    return z


def u53(hi, lo):
    return lib().orc_u53(int(hi), int(lo))


def bounded(seed, c0, c1, c2, tag, Q):
    return int(lib().orc_bounded(int(seed), int(c0), int(c1), int(c2), int(tag), int(Q)))


def island_normals(seed, n, k, count):
    z = np.zeros(count, dtype=np.float64)
    lib().orc_island_normals(int(seed), int(n), int(k), int(count), _ptr(z, _dp))
    return z


def quantise(lw):
    lw = np.ascontiguousarray(lw, dtype=np.float64)
    q = np.zeros(lw.size, dtype=np.uint64)
    mx = C.c_double()
    lib().orc_quantise(_ptr(lw, _dp), lw.size, _ptr(q, _u64p), C.byref(mx))
    return q, mx.value


def systematic(q, U):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    a = np.zeros(q.size, dtype=np.int32)
    lib().orc_systematic(_ptr(q, _u64p), q.size, int(U), _ptr(a, _i32p))
    return a


def digest_term(n, k, j, v):
    return int(lib().orc_digest_term(int(n), int(k), int(j), int(v)))


# ------------------------------------------------------------------ problems

class Problem:
    """One filtering problem: model, theta, data, sizes, seed."""

    def __init__(self, kind, theta, y, m, N, seed, dx=1, dy=1, consts=None):
        self.kind = int(kind)
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        self.dx, self.dy = int(dx), int(dy)
        self.T = self.y.size // self.dy
        self.m, self.N, self.seed = int(m), int(N), int(seed)
        self.consts = None if consts is None else np.ascontiguousarray(consts, dtype=np.float64)

    def _c(self):
        p = _Problem()
        p.kind, p.dx, p.dy, p.d_theta = self.kind, self.dx, self.dy, self.theta.size
        p.theta = _ptr(self.theta, _dp)
        p.consts = _ptr(self.consts, _dp)
        p.y = _ptr(self.y, _dp)
        p.T, p.m, p.N, p.seed = self.T, self.m, self.N, self.seed
        return p

    def with_theta(self, theta):
        q = Problem(self.kind, theta, self.y, self.m, self.N, self.seed, self.dx, self.dy, self.consts)
        return q


class Trace:
    """Host arrays the oracle fills (or, in replay mode, reads)."""

    def __init__(self, prob, anc=True, pi=True, lpost=True, enf=True, digest=True,
                 x=False, logz_inc=True, fmean=False, lpre=False):
        T, m, N = prob.T, prob.m, prob.N
        S = m.bit_length() - 1
        self.sstar = np.zeros(T, dtype=np.int32)
        self.enf = np.full(T * (S + 1), np.nan) if enf else None
        self.lpost = np.zeros(T * m) if lpost else None
        self.anc = np.zeros(T * m * N, dtype=np.int32) if anc else None
        self.pi = np.zeros(T * m, dtype=np.int32) if pi else None
        self.digest = np.zeros(2 * T, dtype=np.uint64) if digest else None
        self.x = np.zeros(T * m * N * prob.dx) if x else None
        self.logz_inc = np.zeros(T) if logz_inc else None
        self.fmean = np.zeros(T * m) if fmean else None
        self.lpre = np.zeros(T * m) if lpre else None
        self.S = S

    def _c(self):
        t = _Trace()
        t.sstar = _ptr(self.sstar, _i32p)
        t.enf = _ptr(self.enf, _dp)
        t.lpost = _ptr(self.lpost, _dp)
        t.anc = _ptr(self.anc, _i32p)
        t.pi = _ptr(self.pi, _i32p)
        t.digest = _ptr(self.digest, _u64p)
        t.x = _ptr(self.x, _dp)
        t.logz_inc = _ptr(self.logz_inc, _dp)
        t.fmean = _ptr(self.fmean, _dp)
        t.lpre = _ptr(self.lpre, _dp)
        return t


def _opts(tau, scheme, f32, replay=0, ess_frac=0.0, arity=2):
    o = _Opts()
    o.tau, o.scheme, o.f32, o.replay, o.exact_weights = float(tau), int(scheme), int(f32), int(replay), 0
    o.ess_frac, o.arity = float(ess_frac), int(arity)
    return o


def run(prob, tau=0.3, scheme=0, f32=False, trace=None, ess_frac=0.0, arity=2):
    """Forward AIRPF; returns log Zhat (fixed-point weights).  ``f32``:
    binary32 particles (state, normals, model, weights; island log-weights
    and log Zhat in double).  ``ess_frac`` > 0: adaptive internal
    resampling (an island resamples iff its ESS < ess_frac * N).
    ``arity`` r: islands interact in groups of r (m a power of r)."""
    p, o = prob._c(), _opts(tau, scheme, f32, ess_frac=ess_frac, arity=arity)
    t = trace._c() if trace is not None else None
    return lib().orc_airpf_run(C.byref(p), C.byref(o), C.byref(t) if t is not None else None)


def score(prob, tau=0.3, scheme=0, f32=False, trace=None, arity=2):
    """Forward-mode score; returns (log Zhat, grad_pathwise, grad_pathspace)."""
    p, o = prob._c(), _opts(tau, scheme, f32, arity=arity)
    t = trace._c() if trace is not None else None
    gpw = np.zeros(prob.theta.size)
    gps = np.zeros(prob.theta.size)
    lz = lib().orc_airpf_score(C.byref(p), C.byref(o), C.byref(t) if t is not None else None,
                               _ptr(gpw, _dp), _ptr(gps, _dp))
    return lz, gpw, gps


def frozen(prob, trace, f32=False):
    """Replay the genealogy in ``trace`` at prob.theta with exact weights.

    Returns (F, S, logw): F the exact-weight log Zhat along that genealogy,
    S[k*N+i] the summed log g along final particle (k,i)'s ancestral path and
    logw[k*N+i] its unnormalised final log-weight."""
    p, o = prob._c(), _opts(0.0, 0, f32, replay=1)
    t = trace._c()
    S = np.zeros(prob.m * prob.N)
    lw = np.zeros(prob.m * prob.N)
    F = lib().orc_airpf_frozen(C.byref(p), C.byref(o), C.byref(t), _ptr(S, _dp), _ptr(lw, _dp))
    return F, S, lw


def bpf(prob, k=0, f32=False, want_anc=False):
    """Textbook bootstrap filter on island k's draws; returns (loglik, anc)."""
    p = prob._c()
    a = np.zeros(prob.T * prob.N, dtype=np.int32) if want_anc else None
    ll = lib().orc_bpf_run(C.byref(p), int(k), int(f32), _ptr(a, _i32p))
    return ll, a
