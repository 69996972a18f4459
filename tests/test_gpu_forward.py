"""GPU parity of the AIRPF forward pass against the CPU oracle (Algorithm 1).

Every case runs the HIP library through its C ABI and the oracle on the same
seeded inputs and compares:
  * island log-weights after every weighting: bit-identical (the same
    double-precision operation sequence on both sides);
  * within-island ancestors, island source maps, interacting-stage counts and
    the order-free digests: bit-identical (integer decisions);
  * log Zhat: to 1e-12 relative (only the final log-sum-exp's summation
    order differs);
  * ENF values: to 1e-12 relative (tree vs sequential sums).
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from paper_2312_06484_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def make_case(orc, model, m, N, T, seed, dx=None):
    if model == "lg1":
        y = W.lg1_data(T)
        return dict(kind=0, theta=np.array(W.LG1_THETA), y=y, dx=1, dy=1, consts=None), \
            orc.Problem(orc.LG1, W.LG1_THETA, y, m, N, seed)
    if model == "sv":
        y = W.sv_data(T)
        return dict(kind=1, theta=np.array(W.SV_THETA), y=y, dx=1, dy=1, consts=None), \
            orc.Problem(orc.SV, W.SV_THETA, y, m, N, seed)
    dy = 4 if dx == 8 else 2
    A, H = W.lgd_model(dx=dx, dy=dy, rho=0.95)
    y = W.lgd_data(A, H, T)
    cst = W.lgd_consts(H)
    return dict(kind=2, theta=A.reshape(-1), y=y, dx=dx, dy=dy, consts=cst), \
        orc.Problem(orc.LGD, A.reshape(-1), y, m, N, seed, dx=dx, dy=dy, consts=cst)


def run_both(ctx, orc, model, m, N, T, tau, f64, seed=1, dx=None):
    from paper_2312_06484_amd import airpf
    g, P = make_case(orc, model, m, N, T, seed, dx)
    print("case", model, dx, m, N, T, tau, "f64" if f64 else "f32", flush=True)
    gt = airpf.Trace(T, m, N, fmean=True)
    st, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, seed, tau=tau, fp64=f64, dx=g["dx"], dy=g["dy"],
                     consts=g["consts"], trace=gt)
    ot = orc.Trace(P, fmean=True)
    lo = orc.run(P, tau=tau, f32=not f64, trace=ot)
    return lz, gt, lo, ot, P


def assert_parity(lz, gt, lo, ot, P):
    T, m, N, S = P.T, P.m, P.N, ot.S
    assert np.isfinite(lo)
    assert abs(lz - lo) <= 1e-12 * max(1.0, abs(lo)), (lz, lo)
    np.testing.assert_array_equal(gt.lpost, ot.lpost)
    if T > 1:
        np.testing.assert_array_equal(gt.anc, ot.anc[: (T - 1) * m * N])
        np.testing.assert_array_equal(gt.pi, ot.pi[: (T - 1) * m])
    np.testing.assert_array_equal(gt.sstar, ot.sstar)
    np.testing.assert_array_equal(gt.digest[: 2 * (T - 1)], ot.digest[: 2 * (T - 1)])
    ge = gt.enf.reshape(T, S + 1)[: T - 1, 1:]
    oe = ot.enf.reshape(T, S + 1)[: T - 1, 1:]
    np.testing.assert_allclose(ge, oe, rtol=1e-12, atol=0)
    if gt.fmean is not None and ot.fmean is not None:
        # island weighted means: the same terms summed in another order
        np.testing.assert_allclose(gt.fmean, ot.fmean, rtol=1e-12, atol=1e-12)


CASES = [
    # model, m, N, T, tau, f64, dx
    ("lg1", 8, 32, 100, 0.3, True, None),      # 1-D linear-Gaussian, T=100, 8 x 32, FP64
    ("lg1", 16, 37, 50, 0.7, False, None),     # ragged island size
    ("lg1", 64, 256, 30, 2.0, False, None),    # always interact
    ("lg1", 1, 100, 20, 0.3, False, None),     # one island = bootstrap filter
    ("lg1", 4, 1, 10, 0.9, False, None),       # one particle per island
    ("lg1", 256, 5, 20, 0.9, True, None),      # many tiny islands
    ("lg1", 2, 3, 1, 0.3, False, None),        # a single observation
    ("lg1", 1024, 256, 12, 0.0, False, None),  # independent filters at full width
    ("lg1", 16384, 16, 6, 0.95, False, None),  # deep butterfly, multi-level upper tree
    ("sv", 32, 128, 40, 0.3, False, None),
    ("sv", 128, 512, 10, 0.5, False, None),    # two-wave island teams
    ("sv", 8, 2048, 5, 2.0, True, None),       # largest island
    ("sv", 4096, 128, 8, 0.6, False, None),    # stochastic volatility width
    ("lgd", 16, 64, 20, 0.5, False, 8),        # 8-D linear-Gaussian
    ("lgd", 4, 300, 8, 2.0, True, 8),
    ("lgd", 8, 33, 10, 0.7, False, 3),
    ("lgd", 8, 20, 10, 0.8, False, 2),
    ("lgd", 4, 16, 10, 0.9, True, 4),
]


@pytest.mark.parametrize("model,m,N,T,tau,f64,dx", CASES)
def test_forward_parity(ctx, orc, model, m, N, T, tau, f64, dx):
    lz, gt, lo, ot, P = run_both(ctx, orc, model, m, N, T, tau, f64, dx=dx)
    assert_parity(lz, gt, lo, ot, P)


def test_lg1_width_of_the_benchmark_long_run(ctx, orc):
    # the 1024 x 256 FP32 linear-Gaussian width over 300 observations: the
    # launch configuration the benchmark times, checked on digests and log Zhat
    lz, gt, lo, ot, P = run_both(ctx, orc, "lg1", 1024, 256, 300, 0.3, False)
    assert_parity(lz, gt, lo, ot, P)


def test_deterministic(ctx):
    y = W.sv_data(30)
    a = ctx.run(1, W.SV_THETA, y, 64, 64, 7)[1]
    b = ctx.run(1, W.SV_THETA, y, 64, 64, 7)[1]
    c = ctx.run(1, W.SV_THETA, y, 64, 64, 8)[1]
    assert a == b and a != c


@pytest.mark.parametrize("kind,m,N,T,tau", [(0, 1024, 256, 400, 0.3), (1, 4096, 128, 200, 0.6), (0, 512, 64, 300, 0.97)])
def test_pipelined_runs_are_deterministic(ctx, kind, m, N, T, tau):
    """Untraced runs (the pipelined kernel: records exchanged through a
    ring of NaN-initialised slots, blocks far apart in time) repeated with one
    seed give one value bit for bit, and another seed another."""
    y = W.lg1_data(T) if kind == 0 else W.sv_data(T)
    th = W.LG1_THETA if kind == 0 else W.SV_THETA
    vals = [ctx.run(kind, th, y, m, N, 11)[1] for _ in range(6)]
    assert all(v == vals[0] for v in vals), vals
    assert ctx.run(kind, th, y, m, N, 12)[1] != vals[0]


def test_close_to_kalman(ctx):
    from oracle import kalman
    T = 1000
    y = W.lg1_data(T)
    lzk, _ = kalman.lg1(W.LG1_THETA, y, grad=False)
    vals = [ctx.run(0, W.LG1_THETA, y, 1024, 256, s)[1] for s in range(1, 6)]
    # 262144 particles over 1000 steps: standard deviation about 0.1
    assert abs(np.mean(vals) - lzk) < 0.5, (vals, lzk)


def test_math_bit_identical(ctx, orc):
    g = np.random.default_rng(0)
    xs = np.concatenate([g.uniform(-745, 709, 20000), g.uniform(-40, 0, 20000),
                         [0.0, -0.0, -1e-300, 709.78, -745.0, -740.0, 1e-10, np.inf, -np.inf]])
    ge = ctx.debug_eval(0, xs)
    oe = np.array([orc.exp(v) for v in xs])
    np.testing.assert_array_equal(ge.view(np.uint64), oe.view(np.uint64))
    ls = np.concatenate([np.exp(g.uniform(-700, 700, 20000)), g.uniform(0.5, 2, 20000),
                         g.integers(1, 2**51, 5000).astype(float), [5e-324, 1.0, 0.0, np.inf]])
    gl = ctx.debug_eval(1, ls)
    ol = np.array([orc.log(v) for v in ls])
    np.testing.assert_array_equal(gl.view(np.uint64), ol.view(np.uint64))
    vs = g.integers(0, 2**32, 20000) * 2.0**-32
    gc, gs = ctx.debug_eval(2, vs)
    oc = np.array([orc.cossin2pi(v) for v in vs])
    np.testing.assert_array_equal(gc.view(np.uint64), oc[:, 0].copy().view(np.uint64))
    np.testing.assert_array_equal(gs.view(np.uint64), oc[:, 1].copy().view(np.uint64))
    words = g.integers(0, 2**32, 40000, dtype=np.uint64).astype(np.uint32)
    z0, z1 = ctx.debug_eval(3, words=words)
    ob = np.array([orc.boxmuller(int(words[2 * i]), int(words[2 * i + 1])) for i in range(words.size // 2)])
    np.testing.assert_array_equal(z0.view(np.uint64), ob[:, 0].copy().view(np.uint64))
    np.testing.assert_array_equal(z1.view(np.uint64), ob[:, 1].copy().view(np.uint64))
    pw = g.integers(0, 2**32, 6 * 3000, dtype=np.uint64).astype(np.uint32)
    gp = ctx.debug_eval(4, words=pw)
    for i in range(3000):
        k0, k1, c0, c1, c2, c3 = (int(v) for v in pw[6 * i:6 * i + 6])
        assert tuple(int(v) for v in gp[i]) == orc.philox((c0, c1, c2, c3), (k0, k1))


def test_math_f32_bit_identical(ctx, orc):
    """The binary32 functions of runs with binary32 particles: device and
    oracle bit for bit, including special and extreme inputs."""
    g = np.random.default_rng(1)
    f = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)    # binary32 inputs
    xs = f(np.concatenate([g.uniform(-104, 89, 40000), g.uniform(-30, 0, 40000), g.uniform(-1e-3, 1e-3, 2000),
                           [0.0, -0.0, -87.3, -87.4, 88.72, 88.73, -125.0, -200.0, 1e-30, np.inf, -np.inf]]))
    ge = ctx.debug_eval(5, xs)
    oe = np.array([orc.expf(v) for v in xs])
    np.testing.assert_array_equal(ge, oe)
    ls = f(np.concatenate([np.exp(g.uniform(-87, 88, 40000)), g.uniform(0.5, 2, 40000),
                           g.integers(1, 2**24, 5000) * 2.0**-24, [1e-40, 1e-45, 1.0, 0.0, np.inf, 2.0**-33]]))
    gl = ctx.debug_eval(6, ls)
    ol = np.array([orc.logf(v) for v in ls])
    np.testing.assert_array_equal(gl, ol)
    vs = f(g.integers(0, 2**32, 40000).astype(np.float32) * np.float32(2.0**-32))
    gc, gs = ctx.debug_eval(7, vs)
    oc = np.array([orc.cossin2pif(v) for v in vs])
    np.testing.assert_array_equal(gc, oc[:, 0])
    np.testing.assert_array_equal(gs, oc[:, 1])
    words = np.concatenate([g.integers(0, 2**32, 80000, dtype=np.uint64).astype(np.uint32),
                            np.array([0, 0, 2**32 - 1, 2**32 - 1, 255, 2**31, 2**32 - 128, 1], dtype=np.uint32)])
    z0, z1 = ctx.debug_eval(8, words=words)
    ob = np.array([orc.boxmullerf(int(words[2 * i]), int(words[2 * i + 1])) for i in range(words.size // 2)])
    np.testing.assert_array_equal(z0, ob[:, 0])
    np.testing.assert_array_equal(z1, ob[:, 1])


def test_invalid_arguments(ctx):
    from paper_2312_06484_amd import airpf
    y = W.lg1_data(10)
    th = W.LG1_THETA
    bad = [dict(m=3, N=4), dict(m=0, N=4), dict(m=4, N=0), dict(m=4, N=4096)]
    for b in bad:
        st, v = ctx.run(0, th, y, b["m"], b["N"], 1, raise_on_error=False)
        assert st == airpf.E_INVALID_ARG and math.isnan(v)
    st, v = ctx.run(0, th, np.array([0.0, np.nan]), 4, 4, 1, raise_on_error=False)
    assert st == airpf.E_INVALID_ARG
    st, v = ctx.run(0, [0.9, 1.0], y, 4, 4, 1, raise_on_error=False)      # wrong d_theta
    assert st == airpf.E_INVALID_ARG
    st, v = ctx.run(1, [-1.0, 1.0, 0.3], y, 4, 4, 1, raise_on_error=False)  # phi = 1
    assert st == airpf.E_DOMAIN and v == -np.inf
    st, v = ctx.run(0, [0.9, 1.0, -1.0], y, 4, 4, 1, raise_on_error=False)  # sy < 0
    assert st == airpf.E_DOMAIN and v == -np.inf
    st, v = ctx.run(2, np.eye(5).ravel(), y, 4, 4, 1, dx=5, dy=1, consts=np.ones(8), raise_on_error=False)
    assert st == airpf.E_INVALID_ARG
    # a valid call still works after the failures
    st, v = ctx.run(0, th, y, 4, 4, 1)
    assert st == airpf.OK and np.isfinite(v)


@pytest.mark.parametrize("where", [0, 7, 29])
def test_device_observations_are_checked(ctx, where):
    """A NaN or infinite observation in device memory, which the host cannot
    look at, is caught by the kernels: INVALID_ARG with NaN outputs from
    airpf_run (pipelined, serial and no-allocation paths), airpf_score and per
    item in a batch; the other items and the next calls are unaffected."""
    import torch
    from paper_2312_06484_amd import airpf
    T = 30
    y = W.lg1_data(T)
    for badv in (np.nan, np.inf):
        yb = y.copy()
        yb[where] = badv
        yd = torch.tensor(yb, dtype=torch.float64, device="cuda")
        good = torch.tensor(y, dtype=torch.float64, device="cuda")
        for tau in (0.3, 2.0, 0.0):
            st, v = ctx.run(0, W.LG1_THETA, None, 256, 64, 1, tau=tau, y_device_ptr=yd.data_ptr(), T=T,
                            raise_on_error=False)
            assert st == airpf.E_INVALID_ARG and math.isnan(v), (tau, st, v)
        st, v = ctx.run_noalloc(0, W.LG1_THETA, None, 64, 32, 1, y_device_ptr=yd.data_ptr(), T=T,
                                raise_on_error=False)
        assert st == airpf.E_INVALID_ARG and math.isnan(v)
        st, v, g = ctx.score(0, W.LG1_THETA, None, 16, 32, 1, y_device_ptr=yd.data_ptr(), T=T,
                             raise_on_error=False)
        assert st == airpf.E_INVALID_ARG and math.isnan(v) and np.isnan(g).all()
        probs = [dict(theta=W.LG1_THETA, y=good.data_ptr(), T=T, m=16, N=32, seed=1),
                 dict(theta=W.LG1_THETA, y=yd.data_ptr(), T=T, m=16, N=32, seed=2)]
        for want in (False, True):
            st, lz, gr, ist = ctx.run_batch(0, probs, want_score=want, y_on_device=True)
            assert st == airpf.OK and ist[0] == airpf.OK and ist[1] == airpf.E_INVALID_ARG
            assert np.isfinite(lz[0]) and np.isnan(lz[1])
            _, ref = ctx.run(0, W.LG1_THETA, y, 16, 32, 1)
            assert lz[0] == ref
        torch.cuda.synchronize()
    st, v = ctx.run(0, W.LG1_THETA, y, 4, 4, 1)
    assert st == airpf.OK and np.isfinite(v)


def test_workspace_cap_reports_nomem(ctx, monkeypatch):
    """AIRPF_WORKSPACE_CAP makes a buffer that would have to grow past it fail
    as an allocation failure does: AIRPF_E_NOMEM, NaN outputs, and the
    context usable again once the cap is lifted."""
    from paper_2312_06484_amd import airpf
    y = W.lg1_data(20)
    fresh = airpf.Context(0)
    try:
        monkeypatch.setenv("AIRPF_WORKSPACE_CAP", str(1 << 20))
        st, v = fresh.run(0, W.LG1_THETA, y, 4096, 256, 1, raise_on_error=False)     # 4 MiB of states
        assert st == airpf.E_NOMEM and math.isnan(v)
        st, v, g = fresh.score(0, W.LG1_THETA, y, 1024, 256, 1, raise_on_error=False)
        assert st == airpf.E_NOMEM and math.isnan(v) and np.isnan(g).all()
        st, v = fresh.run(0, W.LG1_THETA, y, 16, 32, 1, raise_on_error=False)         # fits
        assert st == airpf.OK
        monkeypatch.delenv("AIRPF_WORKSPACE_CAP")
        st, v = fresh.run(0, W.LG1_THETA, y, 4096, 256, 1)
        assert st == airpf.OK and np.isfinite(v)
    finally:
        fresh.close()


@pytest.mark.parametrize("tau", [0.5, 0.25, 0.125])
def test_enf_threshold_at_a_stage_bound(ctx, orc, tau):
    # after s-1 interacting stages the ENF of stage s cannot fall below
    # 2^(s-1)/m, and it sits exactly on that bound whenever one block's weight
    # swamps the others' (common with sharp 8-D likelihoods); tau equal to
    # such a bound must be decided as the definition decides it (not < tau)
    lz, gt, lo, ot, P = run_both(ctx, orc, "lgd", 16, 64, 25, tau, False, dx=8)
    assert_parity(lz, gt, lo, ot, P)


@pytest.mark.parametrize("model,m,N,T,tau,f64,dx", [
    ("lg1", 1024, 256, 120, 0.0, False, None),     # the benchmark width, interactions off
    ("sv", 64, 37, 50, 0.005, False, None),        # tau <= 1/(2m), ragged N
    ("lgd", 32, 20, 30, 0.0, True, 4),
])
def test_untraced_run_without_interactions(ctx, orc, model, m, N, T, tau, f64, dx):
    """With tau <= 1/(2m) no stage can interact (ENF >= 1/m), and an untraced
    run skips the per-step synchronisation entirely; its log Zhat must be the
    traced run's bit for bit, and the oracle's."""
    g, P = make_case(orc, model, m, N, T, 3, dx)
    print("case", model, dx, m, N, T, tau, flush=True)
    from paper_2312_06484_amd import airpf
    gt = airpf.Trace(T, m, N, enf=False, anc=False, digest=False)
    _, lz_traced = ctx.run(g["kind"], g["theta"], g["y"], m, N, 3, tau=tau, fp64=f64, dx=g["dx"], dy=g["dy"],
                           consts=g["consts"], trace=gt)
    _, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, 3, tau=tau, fp64=f64, dx=g["dx"], dy=g["dy"],
                    consts=g["consts"])
    assert lz == lz_traced
    assert (gt.sstar == 0).all()
    lo = orc.run(P, tau=tau, f32=not f64)
    assert abs(lz - lo) <= 1e-12 * max(1.0, abs(lo)), (lz, lo)


@pytest.mark.parametrize("model,m,N,T,tau,f64,dx", [
    ("lg1", 1024, 256, 300, 0.3, False, None),     # the benchmark width: s* = 0 on most steps
    ("sv", 4096, 128, 150, 0.3, False, None),      # 16 islands per block
    ("lg1", 64, 64, 200, 0.9, True, None),         # frequent interactions
    ("lgd", 256, 32, 60, 0.5, False, 4),
    ("sv", 512, 37, 80, 0.6, False, None),         # ragged N
    ("lg1", 1, 64, 40, 0.7, True, None),           # one island: no stages
    ("sv", 2048, 64, 1, 0.3, False, None),         # a single observation
    ("lg1", 256, 256, 2, 0.9, False, None),        # two observations
    ("lg1", 1024, 64, 200, 0.97, False, None),     # stages reaching across blocks on many steps
    ("sv", 16384, 16, 60, 0.8, False, None),       # 64 islands per block
    ("lg1", 65536, 4, 30, 0.6, False, None),       # 256 islands per block
    ("lgd", 2048, 64, 20, 1.5, False, 8),          # untraced serial kernel (every stage interacts) on 512 blocks
    ("lg1", 1024, 256, 70, 0.0, False, None),      # independent filters: the pipelined kernel exchanges nothing
])
def test_untraced_run_matches_traced(ctx, orc, model, m, N, T, tau, f64, dx):
    """An untraced run may take each step's passes before the step's
    interaction count is known (assuming no stage interacts) and redo them
    when some stage does; its log Zhat must equal the traced run's bit for
    bit, and the oracle's."""
    g, P = make_case(orc, model, m, N, T, 5, dx)
    print("case", model, dx, m, N, T, tau, flush=True)
    from paper_2312_06484_amd import airpf
    gt = airpf.Trace(T, m, N, enf=False, anc=False, digest=False, lpost=False)
    _, lz_traced = ctx.run(g["kind"], g["theta"], g["y"], m, N, 5, tau=tau, fp64=f64, dx=g["dx"], dy=g["dy"],
                           consts=g["consts"], trace=gt)
    _, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, 5, tau=tau, fp64=f64, dx=g["dx"], dy=g["dy"],
                    consts=g["consts"])
    print("steps with interactions:", int((gt.sstar[:-1] > 0).sum()), "of", T - 1, flush=True)
    assert lz == lz_traced
    lo = orc.run(P, tau=tau, f32=not f64)
    assert abs(lz - lo) <= 1e-12 * max(1.0, abs(lo)), (lz, lo)


@pytest.mark.parametrize("model,m,N,T,tau", [
    ("lg1", 1024, 256, 200, 0.3),                  # the benchmark width
    ("sv", 4096, 128, 100, 0.6),                   # two passes per block, more than 256 blocks
])
def test_untraced_serial_kernel_matches_traced(ctx, orc, model, m, N, T, tau):
    """With the pipelined kernel switched off (AIRPF_PIPELINE=0) an untraced
    run takes the serial kernel (speculative passes between publishing a step
    and the barrier); its log Zhat must equal the traced run's bit for bit."""
    import os
    g, P = make_case(orc, model, m, N, T, 7, None)
    print("case", model, m, N, T, tau, flush=True)
    from paper_2312_06484_amd import airpf
    gt = airpf.Trace(T, m, N, enf=False, anc=False, digest=False, lpost=False)
    _, lz_traced = ctx.run(g["kind"], g["theta"], g["y"], m, N, 7, tau=tau, trace=gt)
    old = os.environ.get("AIRPF_PIPELINE")
    os.environ["AIRPF_PIPELINE"] = "0"
    try:
        _, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, 7, tau=tau)
    finally:
        if old is None:
            os.environ.pop("AIRPF_PIPELINE", None)
        else:
            os.environ["AIRPF_PIPELINE"] = old
    assert lz == lz_traced


@pytest.mark.parametrize("model,m,N,T,tau,f64,dx", [
    ("lg1", 8, 32, 60, 0.5, True, None),
    ("sv", 64, 37, 30, 0.7, False, None),          # ragged island size
    ("lgd", 16, 64, 12, 0.8, True, 4),
    ("lg1", 256, 256, 20, 0.3, False, None),       # the benchmark's island size, several blocks
    ("sv", 4, 1000, 8, 2.0, False, None),          # islands of several waves, every stage interacts
    ("lg1", 1, 64, 20, 0.5, True, None),           # one island: no stages
    ("sv", 16, 1, 12, 0.9, False, None),           # one particle per island
    ("lg1", 32, 48, 1, 0.3, False, None),          # a single observation: no resampling
])
def test_multinomial_parity(ctx, orc, model, m, N, T, tau, f64, dx):
    """Multinomial internal resampling (N independent draws, slot j from its
    own uniform on [0, Q)): ancestors, island maps, s* and digests bit-exact
    against the oracle, log Zhat to 1e-12; the untraced run equals the traced."""
    from paper_2312_06484_amd import airpf
    g, P = make_case(orc, model, m, N, T, 4, dx)
    print("case", model, dx, m, N, T, tau, flush=True)
    gt = airpf.Trace(T, m, N)
    kw = dict(tau=tau, fp64=f64, dx=g["dx"], dy=g["dy"], consts=g["consts"], resampling=airpf.MULTINOMIAL)
    _, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, 4, trace=gt, **kw)
    ot = orc.Trace(P)
    lo = orc.run(P, tau=tau, scheme=1, f32=not f64, trace=ot)
    assert_parity(lz, gt, lo, ot, P)
    _, lz2 = ctx.run(g["kind"], g["theta"], g["y"], m, N, 4, **kw)
    assert lz2 == lz

