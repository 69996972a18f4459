"""Results do not depend on how islands are tiled onto blocks.

The same problem is run with the launch capped at different block counts
(AIRPF_MAX_BLOCKS): log Zhat, island log-weights, ancestors, island maps and
the score must be bit-identical.  Island sums are taken over fixed
adjacent-pair trees of island indices, and the score accumulates per island,
so the block count cannot change the order of any floating-point sum.
"""
import os

import numpy as np
import pytest

from paper_2312_06484_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


def _with_cap(cap, fn):
    old = os.environ.get("AIRPF_MAX_BLOCKS")
    if cap is None:
        os.environ.pop("AIRPF_MAX_BLOCKS", None)
    else:
        os.environ["AIRPF_MAX_BLOCKS"] = str(cap)
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop("AIRPF_MAX_BLOCKS", None)
        else:
            os.environ["AIRPF_MAX_BLOCKS"] = old


@pytest.mark.parametrize("kind,m,N,T,tau", [(0, 256, 64, 30, 0.6), (1, 1024, 32, 20, 0.95), (1, 64, 256, 25, 2.0),
                                            (0, 4096, 256, 12, 0.6)])   # more than 256 blocks uncapped
def test_forward_tiling_invariant(ctx, kind, m, N, T, tau):
    from paper_2312_06484_amd import airpf
    y = W.lg1_data(T) if kind == 0 else W.sv_data(T)
    th = W.LG1_THETA if kind == 0 else W.SV_THETA
    outs = []
    lo = max(1, m // 256)                  # a block holds at most 256 islands
    for cap in (None, lo, 2 * lo, 8 * lo):
        tr = airpf.Trace(T, m, N, enf=False, digest=False)
        _, lz = _with_cap(cap, lambda: ctx.run(kind, th, y, m, N, 3, tau=tau, trace=tr))
        outs.append((lz, tr))
    lz0, t0 = outs[0]
    for lz, tr in outs[1:]:
        assert lz == lz0
        for f in ("lpost", "anc", "pi", "sstar"):
            assert np.array_equal(getattr(tr, f), getattr(t0, f)), f


def test_too_few_blocks_is_unsupported(ctx):
    from paper_2312_06484_amd import airpf
    st, v = _with_cap(1, lambda: ctx.run(0, W.LG1_THETA, W.lg1_data(5), 1024, 8, 1, raise_on_error=False))
    assert st == airpf.E_UNSUPPORTED


def test_score_tiling_invariant(ctx):
    y = W.sv_data(20)
    ref = None
    for cap in (None, 1, 4):
        _, lz, g = _with_cap(cap, lambda: ctx.score(1, W.SV_THETA, y, 128, 64, 2, tau=0.7, ckpt_every=6))
        if ref is None:
            ref = (lz, g)
        else:
            assert lz == ref[0] and np.array_equal(g, ref[1])


@pytest.mark.parametrize("tau", [0.3, 0.9])
def test_score_tiling_invariant_many_blocks(ctx, tau):
    """SV 4096 x 128 over 500 observations, checkpoints every 50 steps: 16 to
    256 blocks, so stages stay inside a block on some steps and reach across
    blocks on others (more often at tau = 0.9); the score and log Zhat must
    not depend on the block count."""
    T = 500
    y = W.sv_data(T)
    ref = None
    for cap in (None, 16, 64):
        _, lz, g = _with_cap(cap, lambda: ctx.score(1, W.SV_THETA, y, 4096, 128, 11, tau=tau, ckpt_every=50))
        if ref is None:
            ref = (lz, g)
        else:
            assert lz == ref[0] and np.array_equal(g, ref[1]), cap
