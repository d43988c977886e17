#!/usr/bin/env python3
"""EnSF analysis benchmark on one MI355X.

A "step" is one full analysis (ensf_analysis: prior prep, particle init and the K
pseudo-steps of Gram -> softmax -> W.X/update) over one synthetic ensemble that is already
resident in HBM.  The metric is member-dim updates per second, N * d * K / (time of one
analysis), with M_p = N particles.

Default workload: the largest single-filter configuration, d = 2 x 256 x 256 = 131072,
N = M_p = 1024, arctan observations of every component with sigma_o = 0.02, K = 200, FP32
form, with the likelihood drift advanced linearly implicitly (the step whose trajectories
match the FP64 oracle at this K; the explicit step needs K >= 1/sigma_o^2 = 2500 to be
stable and costs the same per pseudo-step).  The split-BF16 form of the same workload is
reported alongside.  The dominant kernel's roofline point comes from HIP events recorded
around every launch on the launch stream (ensf_profile_phases).  The CPU baseline is the
FP64 oracle on a bounded sample (a particle subset, and at this size also a subset of the
pseudo-steps: every step costs the same), scaled to the full analysis.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3|1|2|4|5] [--precision fp32]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "bf16": 2500.0}
# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# calibrated with a plain copy of known size (profiles/hbm_traffic_*.md);
# keyed by (workload config, precision, kernel).  Absent entries are reported as null.
MEASURED_TRAFFIC = {(2, "fp32", "k_wx"): 103.32e6, (2, "bf16x3", "k_wx"): 103.32e6,
                    (3, "fp32", "k_wx"): 2620.9e6, (3, "bf16x3", "k_wx"): 2645.9e6}
WORKLOAD = {
    1: "EnSF analysis d=2x64x64=8192, N=M_p=20, arctan obs of all components, sigma_o=0.05, K=100",
    2: "EnSF analysis d=2x128x128=32768, N=M_p=256, arctan obs of a random 25% subset, "
       "sigma_o=0.05, K=100",
    3: "EnSF analysis d=2x256x256=131072, N=M_p=1024, arctan obs of all components, "
       "sigma_o=0.02, K=200",
    4: "64 independent EnSF filters in one batched call: d uniform in {2x64x64, 2x128x128, "
       "2x256x256}, N=M_p uniform in 32..512, arctan obs of 10-100% of components, "
       "sigma_o=0.05, K=100",
    5: "learned-forecast assimilation cycle: 50 cycles on 2x128x128 SQG states, N=M_p=512, "
       "forecast (0.125 time units) by a 6-layer 3x3 conv net (64 channels) trained on 2000 "
       "SQG pairs, split-BF16 EnSF analysis of identity obs every 4th grid point "
       "(sigma_o=0.05, K=400)",
}


def run_cycle_bench(a):
    """Config 5: train the surrogate, cycle with it, with the SQG model and with no forecast
    model; the metric is the analyses' member-dim updates per second."""
    import numpy as np
    import torch

    from paper_2407_12168_amd import cycle
    dev = torch.device("cuda:0")
    cfg = cycle.CycleConfig(cycles=a.cycles)
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    x, y = cycle.training_pairs(2000, cfg, dev)
    xv, yv = cycle.training_pairs(64, cfg, dev, seed=cfg.seed + 77, perturbed=0.0)
    log(f"2000 SQG training pairs in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    sur, hist = cycle.train_surrogate(x, y, epochs=a.epochs, batch=32, lr=1e-3, val=(xv, yv),
                                      log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    n_steps_train = a.epochs * (2000 // 32)
    train_flops = 3 * 4.91e9 * 32 * n_steps_train
    del x, y
    runs = {}
    for name in ("conv", "sqg", "persistence"):
        runs[name] = cycle.run_cycle(cfg, name, surrogate=sur if name == "conv" else None,
                                     dev=dev, log=log)
    sur.destroy()
    conv = runs["conv"]
    ndk = cfg.members * 2 * cfg.grid * cfg.grid * cfg.pseudo_steps
    ms = 1e3 * float(np.mean(conv.analysis_s))
    summary = {n: {"rmse_analysis_mean": float(np.mean(r.rmse[5:])),
                   "rmse_forecast_mean": float(np.mean(r.rmse_forecast[5:])),
                   "forecast_ms_per_cycle": 1e3 * float(np.mean(r.forecast_s)),
                   "analysis_ms_per_cycle": 1e3 * float(np.mean(r.analysis_s)),
                   "rmse_analysis": [round(v, 5) for v in r.rmse]}
               for n, r in runs.items()}
    line = {
        "metric": "EnSF member-dim updates/s (N*d*K/s)",
        "value": ndk / (ms * 1e-3), "unit": "member-dim updates/s",
        "n_gpus": 1, "steps": cfg.cycles, "warmup": 0, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": WORKLOAD[5], "precision": "bf16x3", "members": cfg.members,
                   "dim": 2 * cfg.grid * cfg.grid, "pseudo_steps": cfg.pseudo_steps,
                   "obs": int(2 * (cfg.grid // cfg.obs_stride) ** 2)},
        "cycle": summary,
        "surrogate_training": {"seconds": train_s, "steps": n_steps_train,
                               "tflops_per_s": train_flops / train_s / 1e12,
                               "final_val_mse": hist[-1].get("val_mse"),
                               "persistence_val_mse": float(torch.mean((xv - yv) ** 2))},
    }
    print(json.dumps(line), flush=True)


def run_vit_cycle_bench(a):
    """The Table II 64^2 ViT surrogate as the cycle's forecast model: trained on SQG pairs by
    the library's kernels, then cycled against the truth with the SQG forecast, with no
    forecast model, with the ViT, and with the ViT trained online on the observations; the
    metric is the analyses' member-dim updates per second of the ViT cycle."""
    import numpy as np
    import torch

    from paper_2407_12168_amd import cycle
    dev = torch.device("cuda:0")
    cfg = cycle.CycleConfig(grid=64, members=256, cycles=a.cycles, pseudo_steps=400,
                            sqg_dt=0.025, steps_per_cycle=10, spinup_steps=800)
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)
    x, y = cycle.training_pairs(2000, cfg, dev)
    xv, yv = cycle.training_pairs(64, cfg, dev, seed=cfg.seed + 77, perturbed=0.0)
    t0 = time.perf_counter()
    net, hist = cycle.train_vit(x, y, epochs=a.epochs, batch=32, lr=5e-5, val=(xv, yv),
                                log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del x, y
    online = cycle.OnlineTuning(steps=2, lr=3e-6, window=8)
    runs = {}
    for name, fc, kw in (("sqg", "sqg", {}), ("persistence", "persistence", {}),
                         ("vit", "vit", {"surrogate": net}),
                         ("vit_online", "vit", {"surrogate": net, "online": online})):
        runs[name] = cycle.run_cycle(cfg, fc, dev=dev, log=log, **kw)
    net.destroy()
    r = runs["vit"]
    ndk = cfg.members * 2 * cfg.grid * cfg.grid * cfg.pseudo_steps
    ms = 1e3 * float(np.mean(r.analysis_s))
    first = min(5, cfg.cycles - 1)
    line = {
        "metric": "EnSF member-dim updates/s (N*d*K/s)",
        "value": ndk / (ms * 1e-3), "unit": "member-dim updates/s",
        "n_gpus": 1, "steps": cfg.cycles, "warmup": 0, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"ViT-forecast assimilation cycle: {cfg.cycles} cycles on "
                               f"2x64x64 SQG states, N=M_p={cfg.members}, forecast by the "
                               f"Table II 64x64 ViT (151M parameters) trained on 2000 SQG "
                               f"pairs for {a.epochs} epochs, obs every 4th point, "
                               f"sigma_o=0.05, K=400", "members": cfg.members,
                   "dim": 2 * cfg.grid * cfg.grid, "pseudo_steps": cfg.pseudo_steps},
        "cycle": {n: {"rmse_analysis_mean": float(np.mean(v.rmse[first:])),
                      "rmse_forecast_mean": float(np.mean(v.rmse_forecast[first:])),
                      "forecast_ms_per_cycle": 1e3 * float(np.mean(v.forecast_s)),
                      "analysis_ms_per_cycle": 1e3 * float(np.mean(v.analysis_s))}
                  for n, v in runs.items()},
        "vit_training": {"seconds": train_s, "final_val_mse": hist[-1]["val_mse"],
                         "persistence_val_mse": float(torch.mean((xv - yv) ** 2))},
    }
    print(json.dumps(line), flush=True)


def vit_training_flops(layers, tokens, embed, mlp_hidden, patch_dim, batch):
    """Matrix-product flops of one ViT training step (2 per multiply-add): forward, and the
    weight gradients of every linear layer plus the input gradients of all but the patch
    embedding (3x the forward for the blocks and the head, 2x for the embedding); attention's
    q k^T and P v per head, forward (2) and backward (4)."""
    D, F, P, T = embed, mlp_hidden, patch_dim, tokens
    body = layers * (3 * D * D + D * D + 2 * D * F) + D * P
    per_token = 3 * 2 * body + 2 * 2 * P * D
    attn = 3 * layers * 2 * 2 * T * T * D
    return batch * (T * per_token + attn)


# Table II rows this library can run (the 256^2 row has 4096 tokens, beyond its attention's
# 1024): input size -> (layers, embed); patch 4, 8 heads, MLP ratio 4 throughout
VIT_TABLE2 = {64: (12, 1024), 128: (24, 2048)}


def run_vit_bench(a):
    """Training throughput of a Table II ViT surrogate (default the 64^2 row: patch 4, 12
    layers, 8 heads, embed 1024, MLP ratio 4) on synthetic 2-level states, as matrix-product
    TFLOP/s."""
    import torch

    from paper_2407_12168_amd import ensf, vit
    dev = torch.device("cuda:0")
    B = a.vit_batch
    S = a.vit_size
    L, D = VIT_TABLE2[S]
    T = (S // 4) ** 2
    g = torch.Generator(device="cpu").manual_seed(2407)
    x = torch.randn((B, 2, S, S), generator=g).to(dev)
    t = (x + 0.1 * torch.randn(x.shape, generator=g).to(dev)).contiguous()
    m = vit.ViT(channels=2, height=S, width=S, patch=4, layers=L, heads=8, embed=D,
                mlp_hidden=4 * D, max_batch=B, seed=1)
    h = m.handle
    for _ in range(a.warmup):
        vit.ensf_vit_train_step(h, x, t, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        vit.ensf_vit_train_step(h, x, t, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / a.steps * 1e3
    loss = vit.ensf_vit_train_step(h, x, t, 1e-4)
    n_params = vit.ensf_vit_num_params(h)
    m.destroy()
    flops = vit_training_flops(L, T, D, 4 * D, 32, B)
    tf = flops / (ms * 1e-3) / 1e12
    rate = ensf.ensf_measure_mfma_rate("bf16")
    line = {
        "metric": "ViT surrogate training TFLOP/s (matrix products)", "value": tf,
        "unit": "TFLOP/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"ViT {S}x{S} input, patch 4, {L} layers, 8 heads, embed {D}, "
                               f"MLP {4 * D} ({n_params} parameters), batch {B}, forward + "
                               f"backward + Adam", "batch": B, "params": n_params},
        "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4), "traffic": None,
                     "mfma_rate_measured": round(rate, 1),
                     "frac_of_measured_rate": round(tf / rate, 4)},
        "flops_per_step": flops, "final_loss": loss,
    }
    print(json.dumps(line), flush=True)


def run_form(probs, precision, steps, warmup, dev, lik_step="explicit", wx_sparse=False):
    """Times ensf_analysis (one problem) or ensf_analysis_batched (several) on `probs`."""
    import torch
    from paper_2407_12168_amd import ensf

    stream = torch.cuda.current_stream()
    tens, descs = [], []
    for p in probs:
        X = torch.from_numpy(p.X).to(dev)
        post = torch.empty_like(X)
        idx = torch.from_numpy(p.obs_idx).to(dev)
        val = torch.from_numpy(p.obs_val).to(dev)
        tens.append((X, post, idx, val))
        descs.append(ensf.make_problem(X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                                       p.filter_id))
    ctx = ensf.Context(precision=precision, use_graph=True, lik_step=lik_step,
                       wx_sparse=wx_sparse)
    h = ctx.handle

    def one():
        if len(probs) == 1:
            p, (X, post, idx, val) = probs[0], tens[0]
            ensf.ensf_analysis(h, X, post, idx, val, p.sigma_o, p.n_steps, p.seed, p.filter_id,
                               stream)
        else:
            ensf.ensf_analysis_batched(h, descs, stream)

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
    return ms, [m / n_launch for m in phase_ms]


def roofline(probs, precision, phase_avg_ms, config=None, wx_sparse=False, mfma_rate=None):
    # algorithmic flops per launch: Gram = sum 2*M_p*N*d, W.X the same (split forms issue 3x).
    # With the degenerate-weight W.X most of its tiles are gathers, not contractions, so the
    # Gram is the kernel priced against the MFMA peak.
    flops = sum(2.0 * p.n_members * p.n_members * p.dim for p in probs)
    names = ("k_gram", "k_softmax", "k_wx")
    dom = 0 if wx_sparse or phase_avg_ms[0] >= phase_avg_ms[2] else 2
    achieved = flops / (phase_avg_ms[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    traffic = MEASURED_TRAFFIC.get((config, precision, names[dom]))
    out = {"kernel": names[dom], "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
           "avg_launch_ms": round(phase_avg_ms[dom], 5),
           "phase_avg_ms": {n: round(v, 5) for n, v in zip(names, phase_avg_ms)}}
    if precision == "bf16x3":
        # the split form issues three BF16 products per algorithmic one (hi*hi + hi*lo + lo*hi)
        out["issued_tflops"] = round(3 * achieved, 3)
        out["frac_issued"] = round(3 * achieved / peak, 4)
        # both GEMM kernels at their issued rate
        out["frac_issued_per_kernel"] = {
            n: round(3 * flops / (phase_avg_ms[i] * 1e-3) / 1e12 / peak, 4)
            for i, n in ((0, "k_gram"), (2, "k_wx"))}
    if mfma_rate:
        # the same work against the matrix-core rate this card sustains (ensf_measure_mfma_rate:
        # register-only MFMA chains under its own clock and power limits)
        issued = 3 * achieved if precision == "bf16x3" else achieved
        out["mfma_rate_measured"] = round(mfma_rate, 1)
        out["frac_of_measured_rate"] = round(issued / mfma_rate, 4)
    return out


def cpu_baseline(probs, n_sample, lik_step="explicit", n_steps=None):
    """FP64 oracle on `n_sample` particles of the first problem and its first `n_steps`
    pseudo-steps (all of them by default), scaled to the whole job: the cost is linear in
    the particle count (particles are independent given the prior), the same for every
    pseudo-step, and proportional to each filter's N*d*K."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import ensf as oracle_ensf

    p = probs[0]
    n_sample = min(n_sample, p.n_members)
    k_sample = min(n_steps or p.n_steps, p.n_steps)
    rows = np.linspace(0, p.n_members - 1, n_sample).astype(int)
    t0 = time.perf_counter()
    oracle_ensf.analysis(p.X, p.obs_idx, p.obs_val, p.sigma_o, k_sample, p.seed,
                         filter_id=p.filter_id, particle_ids=rows, lik_step=lik_step)
    t = time.perf_counter() - t0
    work = lambda q: float(q.n_members) * q.n_members * q.dim * q.n_steps
    scale = sum(work(q) for q in probs) / (
        work(p) * (n_sample / p.n_members) * (k_sample / p.n_steps))
    full_t = t * scale
    ndk = sum(q.n_members * q.dim * q.n_steps for q in probs)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    steps_txt = f", {k_sample} of K={p.n_steps} pseudo-steps" if k_sample < p.n_steps else \
        f", K={p.n_steps}"
    return {"value": ndk / full_t, "unit": "member-dim updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_sample} of {p.n_members} particles of filter 0 (N={p.n_members}, "
                      f"d={p.dim}{steps_txt}), {t:.1f}s measured, scaled by {scale:.0f}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3, 4, 5))
    ap.add_argument("--cycles", type=int, default=50, help="config 5: assimilation cycles")
    ap.add_argument("--epochs", type=int, default=30, help="config 5: surrogate epochs")
    ap.add_argument("--precision", default="fp32", choices=("fp32", "bf16x3", "bf16"))
    ap.add_argument("--other-form", default=None,
                    help="second precision reported alongside (default: the other of "
                         "fp32/bf16x3; 'none' to skip)")
    ap.add_argument("--lik-step", default="implicit", choices=("explicit", "implicit"),
                    help="time stepping of the likelihood drift (implicit: stable and "
                         "oracle-matched at the workloads' K; explicit: plain Euler-Maruyama, "
                         "chaotic at K < 1/sigma_o^2)")
    ap.add_argument("--wx-sparse", action="store_true",
                    help="degenerate-weight W.X variant (reported apart from the dense path)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the degenerate-weight W.X variant reported beside the dense path")
    ap.add_argument("--cpu-particles", type=int, default=None,
                    help="particles of the oracle's timed sample (default per workload, "
                         "10-30 s of CPU work)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="pseudo-steps of the oracle's timed sample (default: all, except "
                         "10 at d = 131072)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--vit", action="store_true",
                    help="time the Table II 64x64 ViT surrogate's training step instead")
    ap.add_argument("--vit-batch", type=int, default=32)
    ap.add_argument("--vit-size", type=int, default=64, choices=sorted(VIT_TABLE2),
                    help="Table II row by input size")
    ap.add_argument("--vit-cycle", action="store_true",
                    help="cycle with the Table II ViT as the forecast model (2x64x64 SQG; "
                         "--cycles, --epochs apply)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: runs on one GPU only (the analysis would shard over particles or "
              "filters; there is no multi-GPU path).", file=sys.stderr)
        sys.exit(2)

    if a.vit:
        run_vit_bench(a)
        return
    if a.vit_cycle:
        run_vit_cycle_bench(a)
        return
    if a.config == 5:
        run_cycle_bench(a)
        return

    import torch

    import workloads
    from paper_2407_12168_amd import ensf
    dev = torch.device("cuda:0")
    if a.config == 4:
        probs = workloads.batched_problems(n_filters=64, n_steps=100, sigma_o=0.05)
    else:
        probs = [workloads.config_problem(a.config)]
    print(f"# workload: {WORKLOAD[a.config]}", file=sys.stderr, flush=True)
    ms, phase = run_form(probs, a.precision, a.steps, a.warmup, dev, a.lik_step, a.wx_sparse)
    print(f"# {a.precision}: {ms:.3f} ms per analysis", file=sys.stderr, flush=True)
    other = a.other_form or ("bf16x3" if a.precision == "fp32" else "fp32")
    if other != "none":
        ms2, phase2 = run_form(probs, other, max(2, a.steps // 2), 1, dev, a.lik_step,
                               a.wx_sparse)
        print(f"# {other}: {ms2:.3f} ms per analysis", file=sys.stderr, flush=True)
    variant = None
    if not a.wx_sparse and not a.no_variants:
        ms3, phase3 = run_form(probs, a.precision, max(2, a.steps // 2), 1, dev, a.lik_step,
                               True)
        print(f"# {a.precision} degenerate-weight W.X: {ms3:.3f} ms per analysis",
              file=sys.stderr, flush=True)
        # the gather tiles are bound by HBM, not by the matrix cores: priced on the bytes every
        # W.X launch must move (Z read and written, the weights: 2*M_p*d*4 + M_p*N*4); the X
        # rows the gathers read depend on the weights and are left out
        wx_bytes = sum(4.0 * (2 * p.n_members * p.dim + p.n_members ** 2) for p in probs)
        gbs = wx_bytes / (phase3[2] * 1e-3) / 1e9
        variant = {"value": None, "ms_per_step": ms3,
                   "k_wx_hbm": {"achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                                "frac": round(gbs / 8000.0, 4)},
                   "phase_avg_ms": {k: round(v, 5) for k, v in
                                    zip(("k_gram", "k_softmax", "k_wx"), phase3)},
                   "note": "same analysis; W.X tiles whose weight rows have at most 8 weights "
                           ">= 2^-30 gather xhat from those members (dense tiles otherwise)"}
    # after the timed runs: the attainable MFMA rate of each form's instruction on this card
    rates = {pr: ensf.ensf_measure_mfma_rate(pr) for pr in {a.precision, other} - {"none"}}
    ndk = sum(p.n_members * p.dim * p.n_steps for p in probs)
    p0 = probs[0]
    cfg = {"workload": WORKLOAD[a.config], "precision": a.precision}
    if a.lik_step != "explicit":
        cfg["lik_step"] = a.lik_step
    if a.wx_sparse:
        cfg["wx"] = "degenerate-weight variant (sparse W.X where rows allow)"
    if len(probs) == 1:
        cfg.update(members=p0.n_members, particles=p0.n_members, dim=p0.dim,
                   pseudo_steps=p0.n_steps, obs=int(p0.obs_idx.size))
    else:
        cfg.update(filters=len(probs), total_member_dims=int(sum(p.n_members * p.dim
                                                                  for p in probs)))
    line = {
        "metric": "EnSF member-dim updates/s (N*d*K/s)",
        "value": ndk / (ms * 1e-3),
        "unit": "member-dim updates/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else a.precision,
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline(probs, a.precision, phase, a.config, a.wx_sparse,
                             rates.get(a.precision)),
    }
    if other != "none":
        line["forms"] = {other: {"value": ndk / (ms2 * 1e-3), "ms_per_step": ms2,
                                 "roofline": roofline(probs, other, phase2, a.config,
                                                      a.wx_sparse, rates.get(other))},
                         "speedup_bf16x3_over_fp32":
                             (ms / ms2) if a.precision == "fp32" else (ms2 / ms)}
    if variant is not None:
        variant["value"] = ndk / (variant["ms_per_step"] * 1e-3)
        line["variants"] = {"wx_sparse": variant}
    if not a.no_cpu:
        n_cpu = a.cpu_particles or {1: 20, 2: 80, 3: 128, 4: 16}[a.config]
        k_cpu = a.cpu_steps or {3: 10}.get(a.config)
        line["cpu_baseline"] = cpu_baseline(probs, n_cpu, a.lik_step, k_cpu)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
