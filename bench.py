#!/usr/bin/env python3
"""EnSF analysis benchmark on one MI355X.

A "step" is one full analysis (ensf_analysis: prior prep, particle init and the K
pseudo-steps of Gram -> softmax -> W.X/update) over one synthetic ensemble that is already
resident in HBM.  The metric is member-dim updates per second, N * d * K / (time of one
analysis), with M_p = N particles.

Default workload: d = 2 x 128 x 128 = 32768, N = 256, arctan observations of a random 25 %
of the components with sigma_o = 0.05, K = 100, FP32 form; the split-BF16 form of the same
workload is reported alongside.  The dominant kernel's roofline point comes from HIP events
recorded around every launch on the launch stream (ensf_profile_phases).  The CPU baseline
is the FP64 oracle on a bounded particle subset, scaled to the full analysis.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2|1|3] [--precision fp32]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "bf16": 2500.0}
WORKLOAD = {
    1: "EnSF analysis d=2x64x64=8192, N=M_p=20, arctan obs of all components, sigma_o=0.05, K=100",
    2: "EnSF analysis d=2x128x128=32768, N=M_p=256, arctan obs of a random 25% subset, "
       "sigma_o=0.05, K=100",
    3: "EnSF analysis d=2x256x256=131072, N=M_p=1024, arctan obs of all components, "
       "sigma_o=0.02, K=200",
}


def run_form(p, precision, steps, warmup, dev):
    import torch
    from paper_2407_12168_amd import ensf

    X = torch.from_numpy(p.X).to(dev)
    post = torch.empty_like(X)
    idx = torch.from_numpy(p.obs_idx).to(dev)
    val = torch.from_numpy(p.obs_val).to(dev)
    stream = torch.cuda.current_stream()
    ctx = ensf.Context(precision=precision, use_graph=True)
    h = ctx.handle

    def one():
        ensf.ensf_analysis(h, X, post, idx, val, p.sigma_o, p.n_steps, p.seed, p.filter_id,
                           stream)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, bad = ensf.ensf_sync_status(h)
    if st != ensf.ENSF_OK:
        raise RuntimeError(f"analysis status {st} ({bad} non-finite values)")
    ms = (t1 - t0) / steps * 1e3

    # per-kernel durations: HIP events around every launch, on the launch stream
    ensf.ensf_profile_phases(h, True)
    for _ in range(max(1, min(steps, 3))):
        one()
    phase_ms, n_launch = ensf.ensf_phase_times(h)
    ensf.ensf_profile_phases(h, False)
    ctx.destroy()
    return ms, [m / n_launch for m in phase_ms], post


def roofline(p, precision, phase_avg_ms):
    # algorithmic flops per launch: Gram = 2*M_p*N*d, W.X = 2*M_p*N*d (split forms issue 3x)
    flops = 2.0 * p.n_members * p.n_members * p.dim
    names = ("k_gram", "k_softmax", "k_wx")
    dom = 0 if phase_avg_ms[0] >= phase_avg_ms[2] else 2
    achieved = flops / (phase_avg_ms[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    return {"kernel": names[dom], "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "avg_launch_ms": round(phase_avg_ms[dom], 5),
            "phase_avg_ms": {n: round(v, 5) for n, v in zip(names, phase_avg_ms)}}


def cpu_baseline(p, n_sample):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import ensf as oracle_ensf

    rows = np.linspace(0, p.n_members - 1, n_sample).astype(int)
    t0 = time.perf_counter()
    oracle_ensf.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, p.n_steps, p.seed,
                         particle_ids=rows)
    t = time.perf_counter() - t0
    full_t = t * p.n_members / n_sample   # cost is linear in the particle count
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": p.n_members * p.dim * p.n_steps / full_t, "unit": "member-dim updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{n_sample} of {p.n_members} particles, full K={p.n_steps}, "
                      f"{t:.1f}s measured, scaled by {p.n_members / n_sample:.0f}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, choices=(1, 2, 3))
    ap.add_argument("--precision", default="fp32", choices=("fp32", "bf16x3", "bf16"))
    ap.add_argument("--other-form", default=None,
                    help="second precision reported alongside (default: the other of fp32/bf16x3)")
    ap.add_argument("--cpu-particles", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (the analysis shards over particles or "
              "filters; no multi-GPU path is built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    dev = torch.device("cuda:0")
    p = workloads.config_problem(a.config)
    print(f"# workload: {WORKLOAD[a.config]}", file=sys.stderr, flush=True)
    ms, phase, _ = run_form(p, a.precision, a.steps, a.warmup, dev)
    print(f"# {a.precision}: {ms:.3f} ms per analysis", file=sys.stderr, flush=True)
    other = a.other_form or ("bf16x3" if a.precision == "fp32" else "fp32")
    ms2, phase2, _ = run_form(p, other, max(2, a.steps // 2), 1, dev)
    print(f"# {other}: {ms2:.3f} ms per analysis", file=sys.stderr, flush=True)
    ndk = p.n_members * p.dim * p.n_steps
    line = {
        "metric": "EnSF member-dim updates/s (N*d*K/s)",
        "value": ndk / (ms * 1e-3),
        "unit": "member-dim updates/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else a.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOAD[a.config], "precision": a.precision,
                   "members": p.n_members, "particles": p.n_members, "dim": p.dim,
                   "pseudo_steps": p.n_steps, "obs": int(p.obs_idx.size)},
        "roofline": roofline(p, a.precision, phase),
        "forms": {other: {"value": ndk / (ms2 * 1e-3), "ms_per_step": ms2,
                          "roofline": roofline(p, other, phase2)},
                  "speedup_bf16x3_over_fp32": (ms / ms2) if a.precision == "fp32" else (ms2 / ms)},
    }
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, a.cpu_particles)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
