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
# algorithmic HBM bytes per particle-step of the forward filter: the state of
# the selected island block is read once (mutation input) and the resampled
# block written once, each d_x values of the storage type
FWD_BYTES_PER_PARTICLE_STEP = {(1, "f32"): 8, (1, "f64"): 16, (8, "f32"): 64, (8, "f64"): 128}


def measured_traffic(workload):
    """HBM bytes per launch from the committed counter record, or None when the
    kernel sources changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ["forward.hip", "dev_math.h", "dev_models.h", "dev_sync.h", "internal.h"]:
        h.update(open(os.path.join(ROOT, "paper_2312_06484_amd", "csrc", f), "rb").read())
    for key, rec in json.load(open(path)).items():
        if key.endswith(" " + workload) and rec.get("kernel_sources_sha256") == h.hexdigest():
            return rec["traffic_bytes_per_launch"]
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


def cpu_baseline(wl, y, gpu_ctx, budget_steps):
    """The CPU oracle, single-threaded, on the first `budget_steps`
    observations of the same workload; also the GPU's log Zhat on that same
    sample for the stated error."""
    from oracle import oracle as orc
    kinds = {0: orc.LG1, 1: orc.SV, 2: orc.LGD}
    Ts = min(budget_steps, wl["T"])
    ys = y[:Ts]
    P = orc.Problem(kinds[wl["kind"]], wl["theta"], ys, wl["m"], wl["N"], 1, dx=wl["dx"], dy=wl["dy"],
                    consts=wl["consts"])
    t0 = time.perf_counter()
    lo = orc.run(P, tau=0.3, store_f32=wl["f32"])
    dt = time.perf_counter() - t0
    _, lg = gpu_ctx.run(wl["kind"], wl["theta"], ys, wl["m"], wl["N"], 1, tau=0.3, fp64=not wl["f32"],
                        dx=wl["dx"], dy=wl["dy"], consts=wl["consts"])
    ps = wl["m"] * wl["N"] * Ts
    return dict(value=ps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample="%s, first %d of %d observations, seed 1, single thread" % (wl["name"], Ts, wl["T"])), \
        abs(lg - lo)


def measure_extras(ctx, torch):
    """Forward+score on the stochastic-volatility workload, and the 64-chain
    proposal batch (forward+score) run in one batched call versus one theta
    at a time.  Each is timed once after one warm-up call."""
    from paper_2312_06484_amd import workloads as W
    out = {}
    # forward + path-space score, SV, T = 2000, 4096 x 128, checkpoints every 100 steps
    T, m, N = 2000, 4096, 128
    y = W.sv_data(T)
    yd = torch.tensor(y, dtype=torch.float64, device="cuda")
    run = lambda seed: ctx.score(1, W.SV_THETA, None, m, N, seed, tau=0.3, ckpt_every=100,
                                 y_device_ptr=yd.data_ptr(), T=T)
    run(99)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, lz, g = run(1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["fwd_score_sv_t2000_m4096_n128_k100"] = {
        "value": m * N * T / dt, "unit": "particle-steps/s", "ms": dt * 1e3, "device_ms": ctx.last_kernel_ms(),
        "log_z": lz, "grad": list(g)}
    # 64 chains' proposals, uneven T, m, N: forward + score
    items = W.batch_c4(64)
    ydev = {}
    probs = []
    for it in items:
        if it["T"] not in ydev:
            ydev[it["T"]] = torch.tensor(W.sv_data(it["T"]), dtype=torch.float64, device="cuda")
        probs.append(dict(theta=it["theta"], y=ydev[it["T"]].data_ptr(), T=it["T"], m=it["m"], N=it["N"],
                          seed=it["seed"]))
    total = sum(it["m"] * it["N"] * it["T"] for it in items)
    ctx.run_batch(1, probs[:4], tau=0.3, want_score=True, ckpt_every=100, y_on_device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, lzb, grb, ist = ctx.run_batch(1, probs, tau=0.3, want_score=True, ckpt_every=100, y_on_device=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    out["batched_sv_64_chains_fwd_score"] = {"value": total / tb, "unit": "particle-steps/s", "ms": tb * 1e3,
                                             "particle_steps": total, "items_ok": int((ist == 0).sum())}
    t0 = time.perf_counter()
    same = True
    for p, lzv, gv in zip(probs, lzb, grb):
        _, l1, g1 = ctx.score(1, p["theta"], None, p["m"], p["N"], p["seed"], tau=0.3, ckpt_every=100,
                              y_device_ptr=p["y"], T=p["T"])
        same = same and (l1 == lzv) and bool((g1 == gv).all())
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    out["plain_sv_64_chains_fwd_score"] = {"value": total / tp, "unit": "particle-steps/s", "ms": tp * 1e3,
                                           "batched_speedup": tp / tb, "batched_items_bit_identical": same}
    return out


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
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (the "
                         "reference reading for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the filter of one parameter value is one "
              "device's work here (see DESIGN.md for how it would shard); got --gpus %d" % args.gpus,
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
    bpp = FWD_BYTES_PER_PARTICLE_STEP[(wl["dx"], "f32" if wl["f32"] else "f64")]
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

    extras = None if args.no_extras else measure_extras(ctx, torch)

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "T": T, "m": m, "N_per_island": N, "tau": args.tau,
                   "state_storage": "f32" if wl["f32"] else "f64", "mode": "forward",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload),
                     "kernel": "forward_kernel", "kernel_ms": avg_k,
                     "bytes_per_particle_step": bpp},
        "logz_err": err,
        "cpu_baseline": cpu,
        "modes": extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
