"""r-ary interactions on the GPU (Section 2: m = r^S islands interacting in
groups of r per stage, here r a power of two) against the oracle: island
log-weights, ancestors, island maps, stage counts and digests bit-identical,
every evaluated stage's ENF to 1e-12 and log Zhat to 1e-12 relative, over
the serial kernel's cases (groups inside one block and across blocks, the
tree above the block roots, tau > 1); untraced runs equal traced ones; with
adaptive or multinomial internal resampling too.  The score and the batch
refuse it."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_forward import make_case  # noqa: E402

from paper_2312_06484_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def _parity(lz, gt, lo, ot, P, r):
    T, m, N, S = P.T, P.m, P.N, ot.S
    Sr = round(math.log(m, r)) if m > 1 else 0
    assert np.isfinite(lo)
    assert abs(lz - lo) <= 1e-12 * max(1.0, abs(lo)), (lz, lo)
    np.testing.assert_array_equal(gt.lpost, ot.lpost)
    np.testing.assert_array_equal(gt.sstar, ot.sstar)
    if T > 1:
        np.testing.assert_array_equal(gt.anc, ot.anc[: (T - 1) * m * N])
        np.testing.assert_array_equal(gt.pi, ot.pi[: (T - 1) * m])
    np.testing.assert_array_equal(gt.digest[: 2 * (T - 1)], ot.digest[: 2 * (T - 1)])
    ge = gt.enf.reshape(T, S + 1)[: T - 1, 1: Sr + 1]
    oe = ot.enf.reshape(T, S + 1)[: T - 1, 1: Sr + 1]
    np.testing.assert_allclose(ge, oe, rtol=1e-12, atol=0)


CASES = [
    # model, m, N, T, tau, r, fp64, dx
    ("lg1", 16, 32, 40, 0.7, 4, True, None),
    ("lg1", 64, 64, 30, 0.9, 8, False, None),
    ("sv", 256, 37, 20, 0.95, 4, True, None),        # ragged N, groups across blocks
    ("lgd", 4096, 16, 10, 0.9, 16, False, 2),        # the tree above the block roots
    ("lg1", 16384, 8, 8, 0.97, 4, True, None),
    ("lg1", 1024, 64, 16, 2.0, 32, False, None),     # every stage interacts
    ("sv", 64, 300, 12, 1.5, 64, True, None),        # one stage of 64, islands of two waves
]


@pytest.mark.parametrize("model,m,N,T,tau,r,fp64,dx", CASES)
def test_rary_parity(ctx, orc, model, m, N, T, tau, r, fp64, dx):
    from paper_2312_06484_amd import airpf
    g, P = make_case(orc, model, m, N, T, 5, dx)
    print("case rary", model, dx, m, N, T, tau, r, fp64, flush=True)
    gt = airpf.Trace(T, m, N)
    kw = dict(tau=tau, fp64=fp64, dx=g["dx"], dy=g["dy"], consts=g["consts"], arity=r)
    _, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, 5, trace=gt, **kw)
    ot = orc.Trace(P)
    lo = orc.run(P, tau=tau, f32=not fp64, trace=ot, arity=r)
    _parity(lz, gt, lo, ot, P, r)
    assert (gt.sstar[: T - 1] > 0).any()
    _, lz2 = ctx.run(g["kind"], g["theta"], g["y"], m, N, 5, **kw)
    assert lz2 == lz


def test_rary_with_adaptive_and_multinomial_resampling(ctx, orc):
    from paper_2312_06484_amd import airpf
    g, P = make_case(orc, "lg1", 64, 48, 30, 2)
    for extra, okw in ((dict(resample_ess=0.6), dict(ess_frac=0.6)),
                       (dict(resampling=airpf.MULTINOMIAL), dict(scheme=1))):
        print("case rary", extra, flush=True)
        gt = airpf.Trace(30, 64, 48)
        _, lz = ctx.run(0, g["theta"], g["y"], 64, 48, 2, tau=0.8, fp64=True, arity=4, trace=gt, **extra)
        ot = orc.Trace(P)
        lo = orc.run(P, tau=0.8, trace=ot, arity=4, **okw)
        _parity(lz, gt, lo, ot, P, 4)


def test_rary_independent_filters_are_the_pair_filter(ctx):
    y = W.lg1_data(50)
    a = ctx.run(0, W.LG1_THETA, y, 1024, 256, 3, tau=0.0)[1]
    b = ctx.run(0, W.LG1_THETA, y, 1024, 256, 3, tau=0.0, arity=32)[1]
    assert a == b


def test_rary_one_island(ctx, orc):
    """m = 1 is a power of every r: no stages, the bootstrap filter."""
    y = W.lg1_data(15)
    a = ctx.run(0, W.LG1_THETA, y, 1, 64, 3, tau=2.0, fp64=True, arity=8)[1]
    b = ctx.run(0, W.LG1_THETA, y, 1, 64, 3, tau=2.0, fp64=True)[1]
    P = orc.Problem(orc.LG1, W.LG1_THETA, y, 1, 64, 3)
    assert a == b and abs(a - orc.run(P, tau=2.0, arity=8)) <= 1e-12 * abs(a)


def test_rary_without_allocation(ctx):
    """airpf_run_noalloc runs the same kernels: equal to airpf_run."""
    y = W.lg1_data(30)
    a = ctx.run(0, W.LG1_THETA, y, 256, 64, 7, tau=0.9, arity=4)[1]
    b = ctx.run_noalloc(0, W.LG1_THETA, y, 256, 64, 7, tau=0.9, arity=4)[1]
    assert a == b and np.isfinite(a)


def test_rary_invalid_and_unsupported(ctx):
    from paper_2312_06484_amd import airpf
    y = W.lg1_data(10)
    kw = dict(raise_on_error=False)
    for r in (3, 6, 1, -4):
        assert ctx.run(0, W.LG1_THETA, y, 16, 16, 1, arity=r, **kw)[0] == airpf.E_INVALID_ARG, r
    assert ctx.run(0, W.LG1_THETA, y, 32, 16, 1, arity=4, **kw)[0] == airpf.E_INVALID_ARG      # 32 is no power of 4
    assert ctx.score(0, W.LG1_THETA, y, 16, 16, 1, arity=4, **kw)[0] == airpf.E_UNSUPPORTED
    pr = [dict(theta=W.LG1_THETA, y=y, m=16, N=16, seed=1)]
    assert ctx.run_batch(0, pr, arity=4, **kw)[0] == airpf.E_UNSUPPORTED
    assert ctx.run(0, W.LG1_THETA, y, 16, 16, 1, arity=4, **kw)[0] == airpf.OK
