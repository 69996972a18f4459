"""The Beta change-point model (the change-point experiment of Section 4.2)
on the GPU against the oracle: island log-weights after every weighting,
ancestors, island maps, interacting-stage counts and digests bit-exact, log
Zhat to 1e-12, at small sizes and at the experiment's own filter shape (64
islands of 200 and of 500 particles, 523 daily observations, interaction
below a normalised ENF of 0.3), with synthetic counts standing in for its
news data."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_forward import assert_parity  # noqa: E402

from paper_2312_06484_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
AB = [float(v) for v in W.BCP_AB]


@pytest.fixture(scope="module")
def ctx():
    from paper_2312_06484_amd import airpf
    c = airpf.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("m,N,T,p,tau,mult", [
    (4, 8, 12, 0.2, 0.5, False),
    (16, 37, 40, 0.05, 0.7, False),        # ragged island size
    (8, 16, 30, 0.1, 2.0, True),           # multinomial, every stage interacting
    (64, 200, 523, 0.01, 0.3, False),      # the experiment's filter, M = 200
    (64, 500, 523, 0.01, 0.3, False),      # and M = 500
])
def test_bcp_parity(ctx, orc, m, N, T, p, tau, mult):
    from paper_2312_06484_amd import airpf
    y = W.bcp_data(T)
    seed = 5
    print("case bcp", m, N, T, p, tau, "mult" if mult else "sys", flush=True)
    res = airpf.MULTINOMIAL if mult else airpf.SYSTEMATIC
    gt = airpf.Trace(T, m, N)
    _, lz = ctx.run(airpf.BCP, [p], y, m, N, seed, tau=tau, fp64=True, dx=2, dy=2, consts=AB, trace=gt,
                    resampling=res)
    P = orc.Problem(orc.BCP, [p], y, m, N, seed, dx=2, dy=2, consts=AB)
    ot = orc.Trace(P)
    lo = orc.run(P, tau=tau, scheme=1 if mult else 0, trace=ot)
    assert_parity(lz, gt, lo, ot, P)
    _, lz2 = ctx.run(airpf.BCP, [p], y, m, N, seed, tau=tau, fp64=True, dx=2, dy=2, consts=AB, resampling=res)
    assert lz2 == lz


def test_bcp_rejects_bad_shapes_and_score(ctx):
    from paper_2312_06484_amd import airpf
    y = W.bcp_data(5)
    kw = dict(fp64=True, dx=2, dy=2, raise_on_error=False)
    assert ctx.run(airpf.BCP, [0.1], y, 4, 8, 1, consts=[2.5, 5.0], **kw)[0] == airpf.E_INVALID_ARG   # not integer
    assert ctx.run(airpf.BCP, [0.1], y, 4, 8, 1, consts=[3.0, 5.0], **kw)[0] == airpf.E_INVALID_ARG   # sum > 7
    assert ctx.run(airpf.BCP, [1.5], y, 4, 8, 1, consts=AB, **kw)[0] == airpf.E_DOMAIN                 # p > 1
    assert ctx.score(airpf.BCP, [0.1], y, 4, 8, 1, consts=AB, **kw)[0] == airpf.E_UNSUPPORTED
