"""GPU parity against the oracle at the widths the benchmark times.

* The 8-D linear-Gaussian forward at 16384 islands of 64 (resampled states
  too large for a block's LDS copy, so the serial kernel reads every source
  block from HBM), untraced as the benchmark runs it and traced: log Zhat of
  both equal bit for bit, the traced stage counts, island maps and digests
  equal to the oracle's, log Zhat to 1e-12.
* The score at the stochastic-volatility width (4096 x 128, checkpoints
  every 10 steps) and at the 8-D width (16384 x 64, all 64 entries of A,
  two segments): both seeds, every component against the oracle's
  forward-mode tangents.
* One item of each (N, m) class of the 64-proposal batch at T = 500, run as
  one forward-only batch (the eight-particles-per-lane batch kernel), each
  log Zhat against the oracle's to 1e-12.
* The variants the benchmark times at the 1-D width (1024 x 256): the
  multinomial and r-ary instantiations of the pipelined kernel and the
  adaptive kernel, untraced as timed, log Zhat against the oracle's to
  1e-12 and equal to the traced run's, whose stage counts and island maps
  equal the oracle's.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_forward import make_case  # noqa: E402
from test_gpu_score import assert_grad_close  # noqa: E402

from paper_2312_06484_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def test_lgd8_forward_at_benchmark_width(ctx, orc):
    from paper_2312_06484_amd import airpf
    m, N, T, tau, seed = 16384, 64, 16, 0.3, 3
    g, P = make_case(orc, "lgd", m, N, T, seed, 8)
    print("case lgd8", m, N, T, tau, flush=True)
    _, lz = ctx.run(g["kind"], g["theta"], g["y"], m, N, seed, tau=tau, dx=8, dy=4, consts=g["consts"])
    gt = airpf.Trace(T, m, N, enf=False, lpost=False, anc=False)
    _, lz_traced = ctx.run(g["kind"], g["theta"], g["y"], m, N, seed, tau=tau, dx=8, dy=4, consts=g["consts"],
                           trace=gt)
    print("steps with interactions:", int((gt.sstar[:-1] > 0).sum()), "of", T - 1, flush=True)
    assert lz == lz_traced
    ot = orc.Trace(P, anc=False, lpost=False, enf=False)
    lo = orc.run(P, tau=tau, f32=True, trace=ot)
    assert abs(lz - lo) <= 1e-12 * abs(lo), (lz, lo)
    np.testing.assert_array_equal(gt.sstar, ot.sstar)
    np.testing.assert_array_equal(gt.pi, ot.pi[: (T - 1) * m])
    np.testing.assert_array_equal(gt.digest[: 2 * (T - 1)], ot.digest[: 2 * (T - 1)])


@pytest.mark.parametrize("model,m,N,T,tau,dx,K", [
    ("sv", 4096, 128, 30, 0.3, None, 10),          # stochastic-volatility width, three segments
    ("lgd", 16384, 64, 3, 0.3, 8, 2),              # 8-D width, all 64 entries of A, two segments
])
def test_score_at_benchmark_width(ctx, orc, model, m, N, T, tau, dx, K):
    from paper_2312_06484_amd import airpf
    g, P = make_case(orc, model, m, N, T, 1, dx)
    print("case", model, dx, m, N, T, tau, "K", K, flush=True)
    _, lz, gps_gpu = ctx.score(g["kind"], g["theta"], g["y"], m, N, 1, tau=tau, dx=g["dx"], dy=g["dy"],
                               consts=g["consts"], ckpt_every=K)
    _, lz2, gpw_gpu = ctx.score(g["kind"], g["theta"], g["y"], m, N, 1, tau=tau, dx=g["dx"], dy=g["dy"],
                                consts=g["consts"], ckpt_every=K, score_mode=airpf.PATHWISE)
    assert lz == lz2
    lo, gpw, gps = orc.score(P, tau=tau, f32=True)
    assert abs(lz - lo) <= 1e-12 * abs(lo), (lz, lo)
    assert_grad_close(gps_gpu, gps, 1e-5)
    assert_grad_close(gpw_gpu, gpw, 1e-5)


def _oracle_logz(args):
    theta, T, m, N, seed = args
    from oracle import oracle as orc
    P = orc.Problem(orc.SV, theta, W.sv_data(T), m, N, seed)
    return orc.run(P, tau=0.3, f32=True)


def test_proposal_batch_classes_against_oracle(ctx):
    import multiprocessing as mp
    thetas = W.sv_chain_thetas(8)
    T = 500
    y = W.sv_data(T)
    items = []
    for i, (N, m) in enumerate([(n, mm) for n in (64, 128, 256, 512) for mm in (256, 1024)]):
        items.append(dict(theta=thetas[i], y=y, T=T, m=m, N=N, seed=100 + i))
    print("case batch of the eight (N, m) classes, T", T, flush=True)
    st, lz, _, ist = ctx.run_batch(1, items, tau=0.3)
    assert (ist == 0).all()
    with mp.get_context("spawn").Pool(8) as pool:
        ref = pool.map(_oracle_logz, [(it["theta"], T, it["m"], it["N"], it["seed"]) for it in items])
    for it, v, r in zip(items, lz, ref):
        assert abs(v - r) <= 1e-12 * abs(r), (it["m"], it["N"], v, r)


@pytest.mark.parametrize("variant", ["multinomial", "arity4", "adaptive"])
def test_variants_at_benchmark_width(ctx, orc, variant):
    from paper_2312_06484_amd import airpf
    m, N, T, tau, seed = 1024, 256, 40, 0.3, 2
    y = W.lg1_data(T)
    P = orc.Problem(orc.LG1, W.LG1_THETA, y, m, N, seed)
    kw, okw, f64 = {
        "multinomial": (dict(resampling=airpf.MULTINOMIAL), dict(scheme=1), False),
        "arity4": (dict(arity=4), dict(arity=4), False),
        "adaptive": (dict(resample_ess=0.5), dict(ess_frac=0.5), True),
    }[variant]
    print("case variant", variant, m, N, T, tau, flush=True)
    _, lz = ctx.run(0, W.LG1_THETA, y, m, N, seed, tau=tau, fp64=f64, **kw)
    gt = airpf.Trace(T, m, N, enf=False, lpost=False, anc=False)
    _, lz_traced = ctx.run(0, W.LG1_THETA, y, m, N, seed, tau=tau, fp64=f64, trace=gt, **kw)
    assert lz == lz_traced
    ot = orc.Trace(P, anc=False, lpost=False, enf=False)
    lo = orc.run(P, tau=tau, f32=not f64, trace=ot, **okw)
    assert abs(lz - lo) <= 1e-12 * abs(lo), (lz, lo)
    np.testing.assert_array_equal(gt.sstar, ot.sstar)
    np.testing.assert_array_equal(gt.pi, ot.pi[: (T - 1) * m])
