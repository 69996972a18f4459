"""Runs in which every island's weight vanishes (Algorithm 1 with an
observation no particle can explain: log g = -inf for all of them).  The
estimate is then exactly zero, log Zhat = -inf with status OK, and the
oracle says the same; the score of such a run is zero (the oracle's
final-weight average has no live term).  The kernels stop at the step where
the last island dies, so these cases also check that every block and wave
leaves together (no barrier left waiting), in the serial and the pipelined
forward kernels, the multinomial kernel, the score and the batch, and that
the next call on the same context is unaffected."""
import numpy as np
import pytest

from paper_2312_06484_amd import workloads as W

pytestmark = pytest.mark.gpu

HUGE = 1e160          # (y - x)^2 and y^2 overflow to +inf in double precision


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def _lg1(T, dead_at):
    y = W.lg1_data(T).copy()
    if dead_at is not None:
        y[dead_at] = HUGE
    return y


@pytest.mark.parametrize("pipeline", ["1", "0"])
@pytest.mark.parametrize("dead_at", [0, 17, 49])
@pytest.mark.parametrize("m,N,fp64", [(1024, 64, False), (64, 128, True), (1, 64, False)])
def test_run_with_every_island_dead(ctx, orc, monkeypatch, pipeline, dead_at, m, N, fp64):
    from paper_2312_06484_amd import airpf
    monkeypatch.setenv("AIRPF_PIPELINE", pipeline)
    y = _lg1(50, dead_at)
    print(f"dead run m={m} N={N} fp64={fp64} dead_at={dead_at} pipeline={pipeline}", flush=True)
    ref = orc.run(orc.Problem(orc.LG1, list(W.LG1_THETA), y, m, N, 5), tau=0.5, f32=not fp64)
    assert ref == -np.inf
    st, v = ctx.run(0, W.LG1_THETA, y, m, N, 5, tau=0.5, fp64=fp64)
    assert st == airpf.OK and v == -np.inf
    # the next call on the context is unaffected
    y2 = _lg1(50, None)
    ref2 = orc.run(orc.Problem(orc.LG1, list(W.LG1_THETA), y2, m, N, 6), tau=0.5, f32=not fp64)
    st, v2 = ctx.run(0, W.LG1_THETA, y2, m, N, 6, tau=0.5, fp64=fp64)
    assert st == airpf.OK and np.isclose(v2, ref2, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("dead_at", [0, 30])
def test_sv_and_multinomial_dead(ctx, orc, dead_at):
    from paper_2312_06484_amd import airpf
    y = W.sv_data(40).copy()
    y[dead_at] = HUGE
    print(f"dead sv run dead_at={dead_at}", flush=True)
    assert orc.run(orc.Problem(orc.SV, list(W.SV_THETA), y, 256, 64, 3), tau=0.5, f32=True) == -np.inf
    st, v = ctx.run(1, W.SV_THETA, y, 256, 64, 3, tau=0.5)
    assert st == airpf.OK and v == -np.inf
    yl = _lg1(40, dead_at)
    st, v = ctx.run(0, W.LG1_THETA, yl, 256, 64, 3, tau=0.5, resampling=airpf.MULTINOMIAL)
    assert st == airpf.OK and v == -np.inf


@pytest.mark.parametrize("ckpt", [0, 8])
@pytest.mark.parametrize("dead_at", [0, 21, 39])
def test_score_with_every_island_dead(ctx, orc, ckpt, dead_at):
    from paper_2312_06484_amd import airpf
    y = _lg1(40, dead_at)
    print(f"dead score ckpt={ckpt} dead_at={dead_at}", flush=True)
    ref_lz, _, ref_g = orc.score(orc.Problem(orc.LG1, list(W.LG1_THETA), y, 64, 128, 7), tau=0.5, f32=True)
    assert ref_lz == -np.inf and np.array_equal(ref_g, np.zeros(3))
    st, lz, g = ctx.score(0, W.LG1_THETA, y, 64, 128, 7, tau=0.5, ckpt_every=ckpt)
    assert st == airpf.OK and lz == -np.inf and np.array_equal(g, np.zeros(3))
    # a live score right after is unaffected
    y2 = _lg1(40, None)
    r_lz, _, r_g = orc.score(orc.Problem(orc.LG1, list(W.LG1_THETA), y2, 64, 128, 8), tau=0.5, f32=True)
    st, lz, g = ctx.score(0, W.LG1_THETA, y2, 64, 128, 8, tau=0.5, ckpt_every=ckpt)
    assert st == airpf.OK and np.isclose(lz, r_lz, rtol=1e-12, atol=0.0)
    assert np.all(np.abs(g - r_g) <= 1e-5 * np.abs(r_g).max() + 1e-12), (g, r_g)


@pytest.mark.parametrize("want_score", [False, True])
def test_batch_with_dead_problems(ctx, want_score):
    from paper_2312_06484_amd import airpf
    probs = [dict(theta=W.LG1_THETA, y=_lg1(60, None), m=64, N=128, seed=1),
             dict(theta=W.LG1_THETA, y=_lg1(60, 12), m=128, N=64, seed=2),
             dict(theta=W.LG1_THETA, y=_lg1(45, None), m=32, N=256, seed=3),
             dict(theta=W.LG1_THETA, y=_lg1(50, 49), m=64, N=64, seed=4)]
    print(f"dead batch want_score={want_score}", flush=True)
    st, lz, gr, ist = ctx.run_batch(0, probs, tau=0.5, want_score=want_score, ckpt_every=16)
    assert st == airpf.OK and (ist == airpf.OK).all()
    for i, p in enumerate(probs):
        if want_score:
            s1, l1, g1 = ctx.score(0, p["theta"], p["y"], p["m"], p["N"], p["seed"], tau=0.5, ckpt_every=16)
            assert np.array_equal(gr[i], g1), i
        else:
            s1, l1 = ctx.run(0, p["theta"], p["y"], p["m"], p["N"], p["seed"], tau=0.5)
        assert s1 == airpf.OK and (lz[i] == l1), i
    assert lz[1] == -np.inf and lz[3] == -np.inf and np.isfinite(lz[0]) and np.isfinite(lz[2])
    if want_score:
        assert np.array_equal(gr[1], np.zeros(3)) and np.array_equal(gr[3], np.zeros(3))
