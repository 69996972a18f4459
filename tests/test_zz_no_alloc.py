"""GPU test of airpf_run_noalloc, the forward entry point that takes every
workspace from the library's fixed device scratch array instead of
allocating: through the C ABI, its log Zhat must equal airpf_run's bit for bit
on the same inputs, over calls in a row whose sizes shrink (the array keeps
the previous call's contents, so whatever must start cleared has to be
cleared by the call), and a request larger than the array is refused.
"""
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


# (model, m, N, T, tau, fp64): the pipelined kernel (tau = 0.3, 1-D), the
# serial kernel (tau > 1, always interacting), one without interactions
# (tau = 0), and the 8-D model at its benchmark island size
CASES = [
    ("lg1", 1024, 256, 300, 0.3, False),
    ("lg1", 64, 37, 50, 0.3, True),
    ("sv", 4096, 128, 120, 2.0, False),
    ("sv", 256, 64, 80, 0.0, False),
    ("lgd8", 1024, 64, 40, 0.3, False),
    ("lgd8", 16, 64, 20, 0.7, False),
]


def _args(model, T):
    if model == "lg1":
        return dict(kind=0, theta=W.LG1_THETA, y=W.lg1_data(T), dx=1, dy=1, consts=None)
    if model == "sv":
        return dict(kind=1, theta=W.SV_THETA, y=W.sv_data(T), dx=1, dy=1, consts=None)
    A, H = W.lgd_model()
    return dict(kind=2, theta=A.reshape(-1), y=W.lgd_data(A, H, T).reshape(-1), dx=8, dy=4,
                consts=W.lgd_consts(H))


def test_noalloc_equals_run_over_shrinking_calls(ctx):
    from paper_2312_06484_amd import airpf
    for seed in (5, 6):
        for model, m, N, T, tau, fp64 in CASES:       # each case is smaller than the one before it in its group
            a = _args(model, T)
            print("noalloc case", model, m, N, T, tau, fp64, "seed", seed, flush=True)
            st0, lz0 = ctx.run(a["kind"], a["theta"], a["y"], m, N, seed, tau=tau, fp64=fp64, dx=a["dx"],
                               dy=a["dy"], consts=a["consts"])
            st1, lz1 = ctx.run_noalloc(a["kind"], a["theta"], a["y"], m, N, seed, tau=tau, fp64=fp64, dx=a["dx"],
                                       dy=a["dy"], consts=a["consts"])
            assert st0 == airpf.OK and st1 == airpf.OK
            assert np.isfinite(lz0)
            assert lz1 == lz0, (model, m, N, T, tau, fp64, lz0, lz1)


def test_noalloc_with_device_observations(ctx):
    import torch
    T, m, N = 200, 512, 128
    y = W.lg1_data(T)
    yd = torch.tensor(y, dtype=torch.float64, device="cuda")
    _, lz0 = ctx.run(0, W.LG1_THETA, y, m, N, 9, tau=0.3)
    _, lz1 = ctx.run_noalloc(0, W.LG1_THETA, None, m, N, 9, tau=0.3, y_device_ptr=yd.data_ptr(), T=T)
    torch.cuda.synchronize()
    assert lz1 == lz0


def test_noalloc_refuses_requests_beyond_the_scratch(ctx):
    from paper_2312_06484_amd import airpf
    # 8-D states of 16384 x 64 islands: 2 x 32 MiB of resampled states alone
    a = _args("lgd8", 4)
    st, lz = ctx.run_noalloc(a["kind"], a["theta"], a["y"], 16384, 64, 1, tau=0.3, dx=8, dy=4,
                             consts=a["consts"], raise_on_error=False)
    assert st == airpf.E_TOO_LARGE and np.isnan(lz)
    # the next call on the same context still works and agrees with airpf_run
    a = _args("lg1", 30)
    _, lz0 = ctx.run(0, a["theta"], a["y"], 8, 32, 2, tau=0.3)
    st, lz1 = ctx.run_noalloc(0, a["theta"], a["y"], 8, 32, 2, tau=0.3)
    assert st == airpf.OK and lz1 == lz0
