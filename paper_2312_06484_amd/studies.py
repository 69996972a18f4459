"""Studies of the filter on the GPU.

Effective number of filters along a run: independent island filters
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


def filter_means(lpost, fmean, T, m):
    """The filter's estimate of E[x_n | y_0..y_n] per step from the traced
    island log-weights after each weighting and the islands' weighted means
    (the filtering measure of Algorithm 1 is the island-weighted mixture of
    the islands' weighted particle sets)."""
    L = np.asarray(lpost, dtype=np.float64).reshape(T, m)
    F = np.asarray(fmean, dtype=np.float64).reshape(T, m)
    w = np.exp(L - L.max(axis=1, keepdims=True))
    w = np.where(np.isfinite(F), w, 0.0)
    return (w * np.where(np.isfinite(F), F, 0.0)).sum(axis=1) / w.sum(axis=1)


def error_vs_islands(ctx, theta, y, total, ms, seeds, tau=0.3, exact_means=None):
    """Filtering error against the number of islands at a fixed total number
    of particles (Theorem 2 of Section 3.2: for AIRPF whose ENF stays above
    tau, the L_r error of the filtering estimates is at most
    C sqrt(log2(m) / (m M tau))).  The 1-D linear-Gaussian model, whose
    exact filtering means (``exact_means``, e.g. the Kalman filter's) are
    the reference.  For each m in ``ms`` (N = total / m particles per
    island) and each seed: one traced GPU run; the error is the root mean
    square over steps and seeds of the filter's estimate of E[x_n | y_0..n]
    minus the exact mean.  Returns dict(m=[...], N=[...], rmse=[...],
    rate=[...]) with rate = sqrt(log2(m) / (m N tau)) (log2 m taken as at
    least 1; NaN for tau = 0, independent filters, which the theorem does
    not cover)."""
    y = np.asarray(y, dtype=np.float64)
    T = y.size
    out = dict(m=[], N=[], rmse=[], rate=[])
    for m in ms:
        N = total // m
        sq = []
        for seed in seeds:
            tr = airpf.Trace(T, m, N, sstar=False, enf=False, lpost=True, anc=False, pi=False, digest=False,
                             fmean=True)
            ctx.run(airpf.LG1, theta, y, m, N, seed, tau=tau, trace=tr)
            est = filter_means(tr.lpost, tr.fmean, T, m)
            sq.append(np.mean((est - exact_means) ** 2))
        out["m"].append(m)
        out["N"].append(N)
        out["rmse"].append(float(np.sqrt(np.mean(sq))))
        out["rate"].append(float(np.sqrt(max(1.0, np.log2(m)) / (m * N * tau))) if tau > 0 else float("nan"))
    return out
