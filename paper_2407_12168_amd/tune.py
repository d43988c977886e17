"""Measures kernel variants with ensf_autotune / ensf_autotune_batched on this GPU and records
the fastest per problem shape in a tune table (the JSON file a context reads through
ensf_options.tune_cache).

    python -m paper_2407_12168_amd.tune --configs 3 --precisions fp32 bf16x3 \\
        --out tune.json [--base paper_2407_12168_amd/tune_gfx950.json]

Entries of --base are kept unless re-measured.  Workloads are the seeded benchmark
problems (workloads.config_problem; config 4 is the 64-filter batch, tuned as a batch).
"""
import argparse
import os
import shutil
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main():
    import torch

    import workloads
    from paper_2407_12168_amd import ensf
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--precisions", nargs="+", default=["fp32", "bf16x3"])
    ap.add_argument("--lik-step", default="implicit")
    ap.add_argument("--base", default=ensf.DEFAULT_TUNE_CACHE)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.base and os.path.abspath(a.base) != os.path.abspath(a.out):
        shutil.copyfile(a.base, a.out)
    os.environ["ENSF_TUNE_LOG"] = "1"
    dev = torch.device("cuda:0")
    for c in a.configs:
        probs = (workloads.batched_problems(n_filters=64, n_steps=100, sigma_o=0.05) if c == 4
                 else [workloads.config_problem(c)])
        keep, descs = [], []
        for p in probs:
            X = torch.from_numpy(p.X).to(dev)
            post = torch.empty_like(X)
            idx = torch.from_numpy(p.obs_idx).to(dev)
            val = torch.from_numpy(p.obs_val).to(dev)
            keep.append((X, post, idx, val))
            descs.append(ensf.make_problem(X, post, idx, val, p.sigma_o, p.n_steps, p.seed,
                                           p.filter_id))
        for prec in a.precisions:
            print(f"# tuning config {c} {prec}", file=sys.stderr, flush=True)
            with ensf.Context(precision=prec, tune_cache=a.out, lik_step=a.lik_step) as ctx:
                if len(descs) == 1:
                    ensf.ensf_autotune(ctx.handle, descs[0])
                else:
                    ensf.ensf_autotune_batched(ctx.handle, descs)
                torch.cuda.synchronize()
        del keep
    print(open(a.out).read())


if __name__ == "__main__":
    main()
