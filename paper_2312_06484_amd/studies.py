"""Effective number of filters along a run: independent island filters
(IBPF) against AIRPF, the comparison of the paper's Section 4.2.

The ENF of the m island weights, (sum W)^2 / (m sum W^2) in the normalised
form the library uses, is traced by the GPU run at every stage of every step
(``airpf_trace.enf``).  With tau = 0 no stage ever interacts and the run is
IBPF: m independent bootstrap filters, whose ENF before interaction decays
towards 1/m as the data record grows (only one filter ends up carrying the
estimate).  With tau > 0 AIRPF interacts over as many stages as it takes to
lift the ENF to at least tau, so the ENF after adaptation stays above tau
at every step whose stages did not run out.
"""
import numpy as np

from . import airpf


def enf_trajectory(ctx, kind, theta, y, m, N, seed, tau, **kw):
    """One traced GPU run.  Returns dict(log_z, sstar[T-1], enf[T-1, S+1],
    enf_before[T-1], enf_after[T-1]): per step n < T-1 (the last step has no
    interaction stages), the number of interacting stages s*, the traced ENF
    of every stage (column s = the ENF stage s saw; column 0 unused),
    the ENF before any interaction (stage 1's), and the ENF after adaptation
    (stage s*+1's; NaN when every stage interacted, s* = log2 m)."""
    y = np.asarray(y, dtype=np.float64)
    dy = int(kw.get("dy", 1))
    T = y.size // dy
    S = int(m).bit_length() - 1
    tr = airpf.Trace(T, m, N, sstar=True, enf=True, lpost=False, anc=False, pi=False, digest=False)
    _, lz = ctx.run(kind, theta, y, m, N, seed, tau=tau, trace=tr, **kw)
    enf = tr.enf.reshape(T, S + 1)[: T - 1]
    ss = tr.sstar[: T - 1].astype(np.int64)
    rows = np.arange(T - 1)
    before = enf[:, 1] if S > 0 else np.full(T - 1, np.nan)
    after = np.where(ss < S, enf[rows, np.minimum(ss + 1, S)], np.nan) if S > 0 else np.full(T - 1, np.nan)
    return dict(log_z=lz, sstar=ss, enf=enf, enf_before=before, enf_after=after)


def ibpf_vs_airpf(ctx, kind, theta, y, m, N, seed, tau=0.3, **kw):
    """The same data, seed and sizes run as IBPF (tau = 0) and as AIRPF with
    threshold tau.  Returns dict(ibpf=..., airpf=...) of enf_trajectory
    results, each with a summary: mean ENF before interaction over the first
    and the last quarter of the steps, the smallest ENF after adaptation, and
    the mean number of interacting stages."""
    out = {}
    for name, t in (("ibpf", 0.0), ("airpf", tau)):
        r = enf_trajectory(ctx, kind, theta, y, m, N, seed, t, **kw)
        q = max(1, r["enf_before"].size // 4)
        r["summary"] = dict(tau=t, enf_first_quarter=float(np.mean(r["enf_before"][:q])),
                            enf_last_quarter=float(np.mean(r["enf_before"][-q:])),
                            min_enf_after=float(np.nanmin(r["enf_after"])) if np.isfinite(r["enf_after"]).any()
                            else float("nan"),
                            mean_stages=float(np.mean(r["sstar"])))
        out[name] = r
    return out
