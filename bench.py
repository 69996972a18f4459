#!/usr/bin/env python3
"""Throughput benchmark of the AIRPF hot path on one MI355X.

One benchmark step = one full filter run (all T observations: mutation,
weighting, internal resampling, the ENF test and island interactions, log
Zhat) over the synthetic workload, a fresh seed per step as a PMMH sampler
would use.  Observations are resident in HBM before the timed region.

Prints ONE JSON line (metric, value, roofline of the filter kernel, the CPU
oracle timed on a bounded sample of the same workload).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s, fwd and fwd+score, batched vs plain AIRPF, at stated logZ err"
HBM_PEAK_GBS = 8000.0


# Peak issue rate of wave64 VALU instructions: 256 CUs x 4 SIMDs x 2.4 GHz,
# one wave64 instruction occupying a 16-lane SIMD for 4 cycles.
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def measured_counters(workload):
    """The committed counter record of the benchmark kernel on this workload
    (profiles/counters.json: HBM bytes per launch from FETCH_SIZE/WRITE_SIZE,
    wave64 VALU instructions per launch from SQ_INSTS_VALU), or None when the
    kernel sources changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ["forward_impl.h", "dev_math.h", "dev_models.h", "dev_sync.h", "internal.h"]:
        h.update(open(os.path.join(ROOT, "paper_2312_06484_amd", "csrc", f), "rb").read())
    for key, rec in json.load(open(path)).items():
        if key.endswith(" " + workload) and rec.get("kernel_sources_sha256") == h.hexdigest():
            return rec
    return None


def workload_inputs(name):
    from paper_2312_06484_amd import workloads as W
    wl = dict(W.WORKLOADS[name])
    T = wl["T"]
    if wl["model"] == W.LG1:
        y = W.lg1_data(T)
        extra = dict(kind=0, theta=list(W.LG1_THETA), dx=1, dy=1, consts=None)
    elif wl["model"] == W.SV:
        y = W.sv_data(T)
        extra = dict(kind=1, theta=list(W.SV_THETA), dx=1, dy=1, consts=None)
    else:
        A, H = W.lgd_model()
        y = W.lgd_data(A, H, T)
        extra = dict(kind=2, theta=A.reshape(-1).tolist(), dx=8, dy=4, consts=W.lgd_consts(H))
    wl.update(extra)
    return wl, y


def _oracle_sample(args):
    """One oracle run on the sample (a pool worker: imports only the oracle)."""
    kind, theta, ys, m, N, seed, dx, dy, consts, f32 = args
    from oracle import oracle as orc
    P = orc.Problem(kind, theta, ys, m, N, seed, dx=dx, dy=dy, consts=consts)
    t0 = time.perf_counter()
    orc.run(P, tau=0.3, f32=f32)
    return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, y, gpu_ctx, budget_steps):
    """The CPU oracle on the first `budget_steps` observations of the same
    workload: single-threaded, then one process per usable host core running
    the same sample with different seeds (the oracle as it stands, no
    threading of its own); also the GPU's log Zhat on that sample for the
    stated error."""
    import multiprocessing as mp
    from oracle import oracle as orc
    kinds = {0: orc.LG1, 1: orc.SV, 2: orc.LGD}
    Ts = min(budget_steps, wl["T"])
    ys = y[:Ts]
    P = orc.Problem(kinds[wl["kind"]], wl["theta"], ys, wl["m"], wl["N"], 1, dx=wl["dx"], dy=wl["dy"],
                    consts=wl["consts"])
    t0 = time.perf_counter()
    lo = orc.run(P, tau=0.3, f32=wl["f32"])
    dt = time.perf_counter() - t0
    _, lg = gpu_ctx.run(wl["kind"], wl["theta"], ys, wl["m"], wl["N"], 1, tau=0.3, fp64=not wl["f32"],
                        dx=wl["dx"], dy=wl["dy"], consts=wl["consts"])
    ps = wl["m"] * wl["N"] * Ts
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 16))
    args = [(kinds[wl["kind"]], wl["theta"], ys, wl["m"], wl["N"], 1 + i, wl["dx"], wl["dy"], wl["consts"],
             wl["f32"]) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_sample, args)
    dt_all = time.perf_counter() - t0
    return dict(value=cores * ps / dt_all, unit="particle-steps/s", cores=cores, kind="oracle",
                sample="%s, first %d of %d observations; %d processes (one per usable core), seeds 1..%d, "
                       "pool start-up included" % (wl["name"], Ts, wl["T"], cores, cores),
                single_core_value=ps / dt, cpu_model=_cpu_model(), nproc=os.cpu_count()), abs(lg - lo)


def fwd_bytes(dx, store_bytes):
    """Algorithmic HBM bytes per particle-step of the forward filter: the
    selected island block read once, the resampled block written once."""
    return 2 * store_bytes * dx


def fwd_score_bytes(dx, store_bytes):
    """Algorithmic HBM bytes per particle-step of forward + score: the
    forward with checkpoints (read + write the state), the segment recompute
    (read + write the state, record the state entering the weighting and the
    16-bit ancestors) and the reverse pass (read the recorded state and
    ancestors, read the children's (lam, D) and write the parents')."""
    fwd = 2 * store_bytes * dx
    rec = 2 * store_bytes * dx + store_bytes * dx + 2
    rev = store_bytes * dx + 2 + 2 * store_bytes * (dx + 1)
    return fwd + rec + rev


def mode_record(particle_steps, seconds, bpp, **extra):
    gbs = bpp * particle_steps / seconds / 1e9
    rec = {"value": particle_steps / seconds, "unit": "particle-steps/s", "ms": seconds * 1e3,
           "bytes_per_particle_step": bpp, "algorithmic_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    rec.update(extra)
    return rec


REPEATS = 3          # timed calls per mode; the record gives the median and the spread


def timed(torch, fn, spread=None):
    """Median wall time of REPEATS calls after one warm-up call (which also
    sizes the workspaces); `spread`, if given, receives min and max (ms)."""
    fn(True)
    torch.cuda.synchronize()
    ts, r = [], None
    for _ in range(REPEATS):
        t0 = time.perf_counter()
        r = fn(False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    if spread is not None:
        spread.update(ms_min=ts[0] * 1e3, ms_max=ts[-1] * 1e3, repeats=REPEATS)
    return ts[len(ts) // 2], r


def measure_modes(ctx, torch):
    """Every configuration of the benchmark table besides the headline one,
    each timed once (wall clock, inputs resident in HBM) after one warm-up
    call: the 1-D LG workload with interactions off, with multinomial or
    adaptive internal resampling and with groups of four islands, the SV
    workload forward
    and forward + score, the 64-chain SV proposal batch forward alone and
    forward + score in one batched call, the latter also one theta at a
    time, 64 PMMH chains (random walk, and Langevin proposals from the
    batched scores) with their effective sample sizes, the ENF study (IBPF
    against AIRPF, traced runs), and the 8-D LG workload forward and
    forward + score."""
    from paper_2312_06484_amd import workloads as W
    from oracle import kalman
    out = {}
    dev = "cuda"

    # the latency configuration: 1-D LG, T = 100, 8 islands of 32, FP64 state;
    # log Zhat against the oracle's on the same seed and against Kalman
    T, m, N = 100, 8, 32
    y1 = W.lg1_data(T)
    yd = torch.tensor(y1, dtype=torch.float64, device=dev)
    sp = {}
    dt, lz = timed(torch, lambda w: ctx.run(0, W.LG1_THETA, None, m, N, 77 if w else 1, tau=0.3, fp64=True,
                                            y_device_ptr=yd.data_ptr(), T=T)[1], sp)
    from oracle import oracle as orc
    lo = orc.run(orc.Problem(orc.LG1, W.LG1_THETA, y1, m, N, 1), tau=0.3)
    out["fwd_lg1_t100_m8_n32_f64"] = mode_record(m * N * T, dt, fwd_bytes(1, 8), log_z=lz,
                                                 device_ms=ctx.last_kernel_ms(), logz_abs_vs_oracle=abs(lz - lo),
                                                 logz_minus_kalman=lz - kalman.lg1(W.LG1_THETA, y1, grad=False)[0],
                                                 **sp)

    # interactions off (tau = 0: independent bootstrap filters), 1-D LG, T=1000, 1024 x 256
    T, m, N = 1000, 1024, 256
    y1 = W.lg1_data(T)
    yd = torch.tensor(y1, dtype=torch.float64, device=dev)
    sp = {}
    dt, lz = timed(torch, lambda w: ctx.run(0, W.LG1_THETA, None, m, N, 77 if w else 1, tau=0.0,
                                            y_device_ptr=yd.data_ptr(), T=T)[1], sp)
    out["fwd_lg1_t1000_m1024_n256_f32_tau0"] = mode_record(m * N * T, dt, fwd_bytes(1, 4), log_z=lz,
                                                          device_ms=ctx.last_kernel_ms(),
                                                          logz_minus_kalman=lz - kalman.lg1(W.LG1_THETA, y1,
                                                                                            grad=False)[0], **sp)

    # the variants of the internal step and of the interactions on the same
    # workload: multinomial internal resampling, adaptive internal
    # resampling (rho = 0.5, double states), groups of four islands
    for name, kw, nb in (("multinomial", dict(resampling=1), fwd_bytes(1, 4)),
                         ("adaptive_rho0.5", dict(resample_ess=0.5), fwd_bytes(1, 8) + 16),   # + carried log-weights
                         ("arity4", dict(arity=4), fwd_bytes(1, 4))):
        sp = {}
        dt, lz = timed(torch, lambda w, kw=kw: ctx.run(0, W.LG1_THETA, None, m, N, 77 if w else 1, tau=0.3,
                                                       y_device_ptr=yd.data_ptr(), T=T, **kw)[1], sp)
        out["fwd_lg1_t1000_m1024_n256_" + name] = mode_record(
            m * N * T, dt, nb, log_z=lz, device_ms=ctx.last_kernel_ms(),
            logz_minus_kalman=lz - kalman.lg1(W.LG1_THETA, y1, grad=False)[0], **sp)

    # SV, T = 2000, 4096 x 128: forward, and forward + path-space score with checkpoints every 100 steps
    T, m, N = 2000, 4096, 128
    yd = torch.tensor(W.sv_data(T), dtype=torch.float64, device=dev)
    sp = {}
    dt, lz = timed(torch, lambda w: ctx.run(1, W.SV_THETA, None, m, N, 99 if w else 1, tau=0.3,
                                            y_device_ptr=yd.data_ptr(), T=T)[1], sp)
    out["fwd_sv_t2000_m4096_n128_f32"] = mode_record(m * N * T, dt, fwd_bytes(1, 4), log_z=lz,
                                                     device_ms=ctx.last_kernel_ms(), **sp)
    sp = {}
    dt, (_, lz, g) = timed(torch, lambda w: ctx.score(1, W.SV_THETA, None, m, N, 99 if w else 1, tau=0.3,
                                                      ckpt_every=100, y_device_ptr=yd.data_ptr(), T=T), sp)
    out["fwd_score_sv_t2000_m4096_n128_f32_k100"] = mode_record(m * N * T, dt, fwd_score_bytes(1, 4), log_z=lz,
                                                                grad=list(g), **sp)

    # 64 chains' proposals, uneven T, m, N: forward + score, batched and one at a time
    items = W.batch_c4(64)
    ydev = {}
    probs = []
    for it in items:
        if it["T"] not in ydev:
            ydev[it["T"]] = torch.tensor(W.sv_data(it["T"]), dtype=torch.float64, device=dev)
        probs.append(dict(theta=it["theta"], y=ydev[it["T"]].data_ptr(), T=it["T"], m=it["m"], N=it["N"],
                          seed=it["seed"]))
    total = sum(it["m"] * it["N"] * it["T"] for it in items)
    bpp = fwd_score_bytes(1, 4)
    # the warm-up call has the timed call's shape, so it also measures and
    # caches the tiling (AIRPF_FLAG_AUTOTUNE) outside the timed region
    spb = {}
    tb, (st, lzb, grb, ist) = timed(torch, lambda w: ctx.run_batch(1, probs, tau=0.3, want_score=True,
                                                                   ckpt_every=100, y_on_device=True,
                                                                   autotune=True), spb)
    # the forward alone (what a PMMH step calls), batched: the warm-up call
    # measures and caches its tiling too
    sp = {}
    tf, (stf, lzf, _, istf) = timed(torch, lambda w: ctx.run_batch(1, probs, tau=0.3, want_score=False,
                                                                    y_on_device=True, autotune=True), sp)
    out["batched_fwd_sv_64_chains"] = mode_record(total, tf, fwd_bytes(1, 4), total_particle_steps=total,
                                                  items_ok=int((istf == 0).sum()), tiling="autotuned", **sp)
    # PMMH on the SV posterior: 64 chains, each iteration's 64 proposals
    # scored by one batched forward (T = 500, 256 islands of 128 particles);
    # then particle MALA, each iteration one batched forward + score.  The
    # effective sample size per coordinate (mu, phi, sigma) is taken over the
    # iterations after the first 10, across the 64 chains
    import numpy as np
    from paper_2312_06484_amd import pmmh
    Tp, mp_, Np, iters, burn = 500, 256, 128, 60, 10
    ysv = W.sv_data(Tp)
    th0 = np.tile(np.array(W.SV_THETA), (64, 1))

    def chain_record(res, bpp):
        ess = [pmmh.effective_sample_size(res["theta"][burn + 1:, :, i]) for i in range(3)]
        return mode_record(res["runs"] * mp_ * Np * Tp, res["seconds"], bpp, iterations=iters,
                           chain_iterations_per_s=64 * iters / res["seconds"],
                           acceptance=float(res["accepted"].mean()), ms_per_iteration=res["seconds"] / iters * 1e3,
                           ess_mu_phi_sigma=ess, ess_per_s_mu_phi_sigma=[e / res["seconds"] for e in ess],
                           lag1_acf_mu_phi_sigma=[float(pmmh.autocorrelation(res["theta"][burn + 1:, :, i], 1)[1])
                                                  for i in range(3)])
    ll = pmmh.BatchedLogLik(ctx, 1, ysv, mp_, Np, tau=0.3)
    step = [0.05, 0.01, 0.02]
    pmmh.run(ll, pmmh.sv_log_prior, th0, 2, step, seed=1)          # warm-up (workspaces, tiling)
    res = pmmh.run(ll, pmmh.sv_log_prior, th0, iters, step, seed=2)
    out["pmmh_sv_t500_m256_n128_64_chains"] = chain_record(res, fwd_bytes(1, 4))
    sc = pmmh.BatchedScore(ctx, 1, ysv, mp_, Np, tau=0.3)
    step = [0.08, 0.015, 0.03]
    pmmh.run_mala(sc, pmmh.sv_log_prior, pmmh.sv_grad_log_prior, th0, 2, step, seed=1)
    res = pmmh.run_mala(sc, pmmh.sv_log_prior, pmmh.sv_grad_log_prior, th0, iters, step, seed=2)
    out["pmala_sv_t500_m256_n128_64_chains"] = chain_record(res, fwd_score_bytes(1, 4))
    # effective number of filters along a run: IBPF (tau = 0) against AIRPF
    # (tau = 0.3) on the same 400 observations of the 1-D LG model, 256 x 8
    from paper_2312_06484_amd import studies
    Te = 400
    t0 = time.perf_counter()
    enf = studies.ibpf_vs_airpf(ctx, 0, W.LG1_THETA, W.lg1_data(Te), 256, 8, 3, tau=0.3)
    out["enf_study_lg1_t400_m256_n8"] = {"seconds": time.perf_counter() - t0,
                                         "ibpf": enf["ibpf"]["summary"], "airpf": enf["airpf"]["summary"],
                                         "log_z": {"ibpf": enf["ibpf"]["log_z"], "airpf": enf["airpf"]["log_z"]}}
    out["batched_fwd_score_sv_64_chains"] = mode_record(total, tb, bpp, total_particle_steps=total,
                                                        items_ok=int((ist == 0).sum()), tiling="autotuned", **spb)
    t0 = time.perf_counter()
    same = True
    for p, lzv, gv in zip(probs, lzb, grb):
        _, l1, g1 = ctx.score(1, p["theta"], None, p["m"], p["N"], p["seed"], tau=0.3, ckpt_every=100,
                              y_device_ptr=p["y"], T=p["T"])
        same = same and bool(l1 == lzv) and bool((g1 == gv).all())
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    out["plain_fwd_score_sv_64_chains"] = mode_record(total, tp, bpp, batched_speedup=tp / tb,
                                                      batched_items_bit_identical=same)

    # 8-D LG, T = 500, 16384 x 64: forward, and forward + score wrt the 64 entries of A (K = 50)
    A, H = W.lgd_model()
    T, m, N = 500, 16384, 64
    yd = torch.tensor(W.lgd_data(A, H, T).reshape(-1), dtype=torch.float64, device=dev)
    cst = W.lgd_consts(H)
    th = A.reshape(-1).tolist()
    lzk8 = kalman.lgd(A, H, cst[0], cst[1], cst[2], W.lgd_data(A, H, T), grad=False)[0]
    sp = {}
    dt, lz = timed(torch, lambda w: ctx.run(2, th, None, m, N, 99 if w else 1, tau=0.3, dx=8, dy=4, consts=cst,
                                            y_device_ptr=yd.data_ptr(), T=T)[1], sp)
    out["fwd_lgd8_t500_m16384_n64_f32"] = mode_record(m * N * T, dt, fwd_bytes(8, 4), log_z=lz,
                                                      device_ms=ctx.last_kernel_ms(), logz_minus_kalman=lz - lzk8,
                                                      **sp)
    sp = {}
    dt, (_, lz, g) = timed(torch, lambda w: ctx.score(2, th, None, m, N, 99 if w else 1, tau=0.3, dx=8, dy=4,
                                                      consts=cst, ckpt_every=50, y_device_ptr=yd.data_ptr(),
                                                      T=T), sp)
    out["fwd_score_lgd8_t500_m16384_n64_f32_k50"] = mode_record(m * N * T, dt, fwd_score_bytes(8, 4), log_z=lz,
                                                                logz_minus_kalman=lz - lzk8, **sp)
    return out


PROFILE_MODES = ("headline", "c1", "batch_fwd", "batch_fwd_score", "lgd8_fwd", "sv_fwd_score", "all")


def profile_mode(name, ctx, torch, runs):
    """One configuration alone, `runs` calls after one warm-up call, for the
    counter passes of a profiler (each pass a run of its own): c1 (1-D LG,
    T = 100, 8 x 32, FP64), batch_fwd / batch_fwd_score (the 64-chain SV
    proposal batch, forward alone or with scores, K = 100), lgd8_fwd (8-D LG,
    T = 500, 16384 x 64), sv_fwd_score (SV, T = 2000, 4096 x 128, K = 100),
    headline (the benchmark workload), all (each of these in turn, so that
    one profiler pass covers every kernel: their names differ)."""
    from paper_2312_06484_amd import workloads as W
    dev = "cuda"
    if name == "all":
        for n in PROFILE_MODES[:-1]:
            profile_mode(n, ctx, torch, runs)
        return
    if name == "headline":
        wl, y = workload_inputs("lg1_t1000_m1024_n256_f32")
        yd = torch.tensor(y.reshape(-1), dtype=torch.float64, device=dev)
        fn = lambda s: ctx.run(0, wl["theta"], None, wl["m"], wl["N"], s, tau=0.3, y_device_ptr=yd.data_ptr(),
                               T=wl["T"])
    elif name == "c1":
        yd = torch.tensor(W.lg1_data(100), dtype=torch.float64, device=dev)
        fn = lambda s: ctx.run(0, W.LG1_THETA, None, 8, 32, s, tau=0.3, fp64=True, y_device_ptr=yd.data_ptr(),
                               T=100)
    elif name in ("batch_fwd", "batch_fwd_score"):
        probs, keep = [], {}
        for it in W.batch_c4(64):
            if it["T"] not in keep:
                keep[it["T"]] = torch.tensor(W.sv_data(it["T"]), dtype=torch.float64, device=dev)
            probs.append(dict(theta=it["theta"], y=keep[it["T"]].data_ptr(), T=it["T"], m=it["m"], N=it["N"],
                              seed=it["seed"]))
        score = name == "batch_fwd_score"
        fn = lambda s: ctx.run_batch(1, probs, tau=0.3, want_score=score, ckpt_every=100 if score else 0,
                                     y_on_device=True, autotune=True)
    elif name == "lgd8_fwd":
        A, H = W.lgd_model()
        yd = torch.tensor(W.lgd_data(A, H, 500).reshape(-1), dtype=torch.float64, device=dev)
        cst = W.lgd_consts(H)
        fn = lambda s: ctx.run(2, A.reshape(-1).tolist(), None, 16384, 64, s, tau=0.3, dx=8, dy=4, consts=cst,
                               y_device_ptr=yd.data_ptr(), T=500)
    elif name == "sv_fwd_score":
        yd = torch.tensor(W.sv_data(2000), dtype=torch.float64, device=dev)
        fn = lambda s: ctx.score(1, W.SV_THETA, None, 4096, 128, s, tau=0.3, ckpt_every=100,
                                 y_device_ptr=yd.data_ptr(), T=2000)
    else:
        raise SystemExit("unknown profile mode %r (one of %s)" % (name, ", ".join(PROFILE_MODES)))
    fn(99)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(runs):
        fn(k + 1)
    torch.cuda.synchronize()
    print(json.dumps({"profile_mode": name, "runs": runs, "ms_per_run": (time.perf_counter() - t0) / runs * 1e3}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lg1_t1000_m1024_n256_f32")
    ap.add_argument("--tau", type=float, default=0.3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=300)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the forward+score and batched-vs-plain measurements")
    ap.add_argument("--profile-mode", choices=PROFILE_MODES, default=None,
                    help="run only this configuration (a warm-up call and --steps calls) and exit: "
                         "for profiler counter passes")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (the "
                         "reference reading for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the filter of one parameter value is one "
              "device's work here (no multi-GPU path is built); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch                                     # device memory and the stream
    from paper_2312_06484_amd import airpf

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": 4 * n, "copies": 5}))
        return

    if args.profile_mode:
        ctx = airpf.Context(0, stream=torch.cuda.current_stream().cuda_stream)
        profile_mode(args.profile_mode, ctx, torch, args.steps)
        ctx.close()
        return

    wl, y = workload_inputs(args.workload)
    wl["name"] = args.workload
    T, m, N = wl["T"], wl["m"], wl["N"]
    dev = torch.device("cuda", 0)
    y_dev = torch.tensor(y.reshape(-1), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    ctx = airpf.Context(0, stream=stream.cuda_stream)

    def one(seed):
        st, lz = ctx.run(wl["kind"], wl["theta"], None, m, N, seed, tau=args.tau, fp64=not wl["f32"],
                         dx=wl["dx"], dy=wl["dy"], consts=wl["consts"], y_device_ptr=y_dev.data_ptr(), T=T)
        return lz

    for w in range(args.warmup):
        one(1000 + w)
    torch.cuda.synchronize()
    kernel_ms, logz = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        logz.append(one(k + 1))
        kernel_ms.append(ctx.last_kernel_ms())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ps_per_step = m * N * T
    value = ps_per_step * args.steps / elapsed
    avg_k = sum(kernel_ms) / len(kernel_ms)
    bpp = fwd_bytes(wl["dx"], 4 if wl["f32"] else 8)
    achieved = bpp * ps_per_step / (avg_k * 1e-3) / 1e9

    err = {}
    if wl["kind"] == 0:
        from oracle import kalman
        lzk, _ = kalman.lg1(wl["theta"], y, grad=False)
        mean = sum(logz) / len(logz)
        sd = math.sqrt(sum((v - mean) ** 2 for v in logz) / max(1, len(logz) - 1))
        err["mean_minus_kalman"] = mean - lzk
        err["sd_over_seeds"] = sd
    cpu = None
    if not args.no_cpu_baseline:
        cpu, d = cpu_baseline(wl, y, ctx, args.cpu_sample_steps)
        err["max_abs_vs_oracle_on_sample"] = d

    extras = None if args.no_extras else measure_modes(ctx, torch)

    counters = measured_counters(args.workload)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["f32"] else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "T": T, "m": m, "N_per_island": N, "tau": args.tau,
                   "state_storage": "f32" if wl["f32"] else "f64", "mode": "forward",
                   "arithmetic": ("particles binary32, weights 40-bit fixed point (uint64), island "
                                  "log-weights and log Zhat f64") if wl["f32"] else "particles, island "
                                 "log-weights and log Zhat f64, weights 40-bit fixed point (uint64)",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counters["traffic_bytes_per_launch"] if counters else None,
                     "valu_frac": (counters["valu_insts_per_launch"] / (avg_k * 1e-3) / VALU_PEAK_WAVE_INSTS
                                   if counters else None),
                     "valu_peak_wave_insts_per_s": VALU_PEAK_WAVE_INSTS,
                     "kernel": ("forward_kernel" if os.environ.get("AIRPF_PIPELINE", "1").startswith("0")
                                else "forward_pipe_kernel"), "kernel_ms": avg_k,
                     "bytes_per_particle_step": bpp},
        "logz_err": err,
        "cpu_baseline": cpu,
        "modes": extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
