"""Data-assimilation cycle of the paper's framework (Fig. 1, Sec. III; twin experiment of
Sec. IV-A): forecast every member, observe the truth, run the EnSF analysis, repeat.

Everything runs on the GPU through libensf: the truth and the physics forecast are the
FP64 SQG model (ensf_sqg), the learned forecast is the conv surrogate (ensf_surrogate) or
the ViT surrogate (ensf_vit, Sec. III-B), the analysis is ensf_analysis.  A learned forecast
can keep training online on the cycle's own analyses (Sec. I, Sec. V).  Host code only draws
the synthetic observation noise and the initial ensemble and orchestrates the calls.
"""
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CycleConfig:
    grid: int = 128
    members: int = 512
    cycles: int = 50
    obs_stride: int = 4          # observe every 4th grid point in x and y on both levels
    sigma_o: float = 0.05
    obs_op: str = "linear"       # the paper's twin experiment observes the state itself
    pseudo_steps: int = 400      # EM-stable for sigma_o = 0.05
    precision: str = "bf16x3"
    spread_relax: float = 1.0    # relax the analysis spread to the prior spread
    sqg_dt: float = 0.0125       # CFL-safe at 128^2 through the spin-up transient
    relax_time: float = 5.0      # SQG thermal relaxation (lets the turbulence equilibrate)
    # forecast length between analyses: 0.125 time units, over which features move a few
    # grid lengths, within the conv surrogate's 13 x 13 receptive field
    steps_per_cycle: int = 10
    spinup_steps: int = 1600     # 20 time units
    trajectories: int = 16       # independent SQG runs the climatological states come from
    # surrogate training set: this fraction of the pairs starts from a climatological state
    # plus a random perturbation (a red-spectrum field and white noise, amplitudes drawn
    # uniformly up to these multiples of the climatological standard deviation), with the
    # SQG evolution of the perturbed state as the target, so that the surrogate also sees
    # states off the attractor such as analysis ensembles
    train_perturbed: float = 0.5
    perturb_smooth: float = 0.5
    perturb_white: float = 0.1
    seed: int = 2412
    filter_seed: int = 12173


@dataclass
class OnlineTuning:
    """Online training of the learned forecast on observations during the cycle (the paper
    adapts the surrogate with observational data, Sec. I and V).  The loss is the forecast's
    misfit at the observed components only: for each of the latest `window` cycles the input
    is the previous analysis mean x and the target is the network's own forecast f(x) with
    the observed components replaced by that cycle's observations, so the squared error (and
    its gradient) lives on the observed components.  After each analysis the surrogate takes
    `steps` Adam steps at rate `lr`.  Needs the identity observation operator."""
    steps: int = 2
    lr: float = 3e-6
    window: int = 8


@dataclass
class CycleResult:
    rmse: list = field(default_factory=list)          # analysis mean vs truth, per cycle
    rmse_forecast: list = field(default_factory=list)  # forecast mean vs truth, per cycle
    rmse_obs: list = field(default_factory=list)       # analysis mean, observed components
    rmse_forecast_obs: list = field(default_factory=list)  # forecast mean, observed components
    spread: list = field(default_factory=list)
    forecast_s: list = field(default_factory=list)
    analysis_s: list = field(default_factory=list)


def obs_indices(grid, stride):
    lv, iy, ix = np.meshgrid(np.arange(2), np.arange(0, grid, stride), np.arange(0, grid, stride),
                             indexing="ij")
    return np.sort((lv * grid * grid + iy * grid + ix).reshape(-1)).astype(np.int32)


def sqg_model(cfg, max_batch):
    from .sqg import SQGModel
    return SQGModel(n=cfg.grid, dt=cfg.sqg_dt, relax_time=cfg.relax_time, max_batch=max_batch)


def climate_trajectories(sqg, cfg, samples, rng, dev, n_traj=None):
    """States of n_traj independent SQG runs from red-spectrum random fields, after a
    spin-up, sampled every forecast interval: tensor (n_traj, samples, 2, n, n) float64."""
    import torch

    import workloads
    n_traj = n_traj or cfg.trajectories
    x = workloads.smooth_fields(rng, 2 * n_traj, cfg.grid, cfg.grid).reshape(
        n_traj, 2, cfg.grid, cfg.grid)
    cur = torch.from_numpy(x).to(dev)
    sqg.run(cur, cur, cfg.spinup_steps)
    out = torch.empty((n_traj, samples, 2, cfg.grid, cfg.grid), dtype=torch.float64, device=dev)
    for k in range(samples):
        out[:, k] = cur
        sqg.run(cur, cur, cfg.steps_per_cycle)
    return out


def _surrogate_ops(forecast, surrogate):
    """(forward(x, y), train_step(x, target, lr)) of a learned forecast model."""
    if forecast == "conv":
        from .surrogate import ensf_surrogate_forward, ensf_surrogate_train_step
        return (lambda x, y: ensf_surrogate_forward(surrogate.handle, x, y),
                lambda x, t, lr: ensf_surrogate_train_step(surrogate.handle, x, t, lr,
                                                           want_loss=False))
    if forecast == "vit":
        from .vit import ensf_vit_forward, ensf_vit_train_step
        return (lambda x, y: ensf_vit_forward(surrogate.handle, x, y),
                lambda x, t, lr: ensf_vit_train_step(surrogate.handle, x, t, lr, want_loss=False))
    return None, None


def run_cycle(cfg, forecast="sqg", surrogate=None, dev=None, log=None, online=None):
    """forecast: "sqg" (the physics model, which is also the truth's model), "conv" or "vit"
    (a trained surrogate) or "persistence" (no forecast model: the analysis is carried over).
    online: an OnlineTuning to keep training a learned forecast on the analyses."""
    import torch

    from . import ensf

    if forecast not in ("sqg", "conv", "vit", "persistence"):
        raise ValueError(forecast)
    if forecast in ("conv", "vit") and surrogate is None:
        raise ValueError(f"forecast '{forecast}' needs a trained surrogate")
    net_forward, net_train = _surrogate_ops(forecast, surrogate)
    if online is not None and net_train is None:
        raise ValueError("online training needs a learned forecast")
    if online is not None and cfg.obs_op != "linear":
        raise ValueError("online training on observations needs obs_op='linear'")
    dev = dev or torch.device("cuda:0")
    rng = np.random.default_rng(cfg.seed)
    n = cfg.grid
    res = CycleResult()
    with sqg_model(cfg, min(cfg.members, 256)) as sqg:
        truth = climate_trajectories(sqg, cfg, 1, rng, dev, n_traj=1)[0]       # (1, 2, n, n)
        # initial ensemble: climatological states of independent long runs (Sec. IV-A)
        per = -(-cfg.members // cfg.trajectories)
        clim = climate_trajectories(sqg, cfg, per, rng, dev).reshape(-1, 2 * n * n)
        ens = clim[:cfg.members].float().contiguous()               # (N, d) float32
        del clim
        post = torch.empty_like(ens)
        idx = torch.from_numpy(obs_indices(n, cfg.obs_stride)).to(dev)
        ctx = ensf.Context(precision=cfg.precision, obs_op=cfg.obs_op,
                           spread_relax=cfg.spread_relax)
        fc_out = torch.empty_like(ens) if forecast == "vit" else None
        pairs = []
        try:
            for c in range(cfg.cycles):
                sqg.run(truth, truth, cfg.steps_per_cycle)
                torch.cuda.synchronize()
                prev_mean = ens.mean(0).view(1, 2, n, n).clone() if online is not None else None
                t0 = time.perf_counter()
                states = ens.view(cfg.members, 2, n, n)
                if forecast == "sqg":
                    sqg.run(states, states, cfg.steps_per_cycle)
                elif forecast == "conv":
                    net_forward(states, states)
                elif forecast == "vit":   # output may not alias the input
                    net_forward(states, fc_out.view(states.shape))
                    ens.copy_(fc_out)
                elif forecast != "persistence":
                    raise ValueError(forecast)
                torch.cuda.synchronize()
                res.forecast_s.append(time.perf_counter() - t0)
                tv = truth.reshape(-1).float()
                clean = torch.atan(tv[idx.long()]) if cfg.obs_op == "arctan" else tv[idx.long()]
                noise = torch.from_numpy(rng.standard_normal(idx.numel()).astype(np.float32)).to(dev)
                y = (clean + cfg.sigma_o * noise).contiguous()
                res.rmse_forecast.append(float(torch.sqrt(torch.mean((ens.mean(0) - tv) ** 2))))
                t0 = time.perf_counter()
                ensf.ensf_analysis(ctx.handle, ens, post, idx, y, cfg.sigma_o, cfg.pseudo_steps,
                                   cfg.filter_seed, c)
                st, nbad = ensf.ensf_sync_status(ctx.handle)
                res.analysis_s.append(time.perf_counter() - t0)
                if st != ensf.ENSF_OK:
                    raise RuntimeError(f"analysis status {st} at cycle {c} ({nbad} non-finite)")
                ens, post = post, ens
                res.rmse.append(float(torch.sqrt(torch.mean((ens.mean(0) - tv) ** 2))))
                res.rmse_obs.append(float(torch.sqrt(torch.mean(
                    (ens.mean(0)[idx.long()] - tv[idx.long()]) ** 2))))
                res.rmse_forecast_obs.append(float(torch.sqrt(torch.mean(
                    (post.mean(0)[idx.long()] - tv[idx.long()]) ** 2))))
                res.spread.append(float(torch.sqrt(torch.mean(ens.var(0)))))
                if online is not None:
                    pairs = (pairs + [(prev_mean, y)])[-online.window:]
                    xs = torch.cat([p[0] for p in pairs]).contiguous()
                    ys = torch.stack([p[1] for p in pairs])
                    li = idx.long()
                    for _ in range(online.steps):
                        ts = torch.empty_like(xs)
                        net_forward(xs, ts)
                        tv_ = ts.view(len(pairs), -1)
                        tv_[:, li] = ys
                        net_train(xs, ts, online.lr)
                if log:
                    log(f"cycle {c}: forecast rmse {res.rmse_forecast[-1]:.4f}, analysis rmse "
                        f"{res.rmse[-1]:.4f}, spread {res.spread[-1]:.4f}, forecast "
                        f"{res.forecast_s[-1] * 1e3:.1f} ms, analysis {res.analysis_s[-1] * 1e3:.1f} ms")
        finally:
            ctx.destroy()
    return res


def training_pairs(count, cfg, dev, seed=None, perturbed=None):
    """(x, SQG(x)) pairs over one forecast interval: consecutive samples of independent
    spun-up SQG trajectories from seeded random initial fields; a fraction `perturbed`
    (default cfg.train_perturbed) of the inputs is perturbed first and evolved again."""
    import torch

    import workloads
    rng = np.random.default_rng(cfg.seed + 1 if seed is None else seed)
    n_traj = min(cfg.trajectories, count)
    per = -(-count // n_traj) + 1
    frac = cfg.train_perturbed if perturbed is None else perturbed
    with sqg_model(cfg, 256) as sqg:
        traj = climate_trajectories(sqg, cfg, per, rng, dev, n_traj=n_traj)
        x = traj[:, :-1].reshape(-1, 2, cfg.grid, cfg.grid)[:count].clone()
        y = traj[:, 1:].reshape(-1, 2, cfg.grid, cfg.grid)[:count].clone()
        del traj
        n_pert = int(round(frac * count))
        if n_pert > 0:
            sel = torch.from_numpy(rng.choice(count, n_pert, replace=False)).to(dev)
            clim_std = float(x.std())
            a_s = rng.uniform(0.0, cfg.perturb_smooth, n_pert) * clim_std
            a_w = rng.uniform(0.0, cfg.perturb_white, n_pert) * clim_std
            red = workloads.smooth_fields(rng, 2 * n_pert, cfg.grid, cfg.grid).reshape(
                n_pert, 2, cfg.grid, cfg.grid)
            white = rng.standard_normal((n_pert, 2, cfg.grid, cfg.grid))
            pert = a_s[:, None, None, None] * red + a_w[:, None, None, None] * white
            xp = x[sel] + torch.from_numpy(pert).to(dev)
            yp = torch.empty_like(xp)
            sqg.run(xp, yp, cfg.steps_per_cycle)
            x[sel] = xp
            y[sel] = yp
    if not (bool(torch.isfinite(x).all()) and bool(torch.isfinite(y).all())):
        raise RuntimeError("SQG trajectory became non-finite (reduce sqg_dt)")
    return x.float().contiguous(), y.float().contiguous()


def train_vit(x, y, epochs=20, batch=32, lr=1e-4, seed=0, log=None, val=None, **arch):
    """Trains a ViT surrogate (Sec. III-B; architecture keywords as vit.ViT, default the
    Table II 64^2 model) on pairs (x, y) with the library's Adam; returns it and the
    per-epoch history (as train_surrogate)."""
    import torch

    from .vit import ViT, ensf_vit_forward, ensf_vit_train_step
    n = x.shape[0]
    a = dict(patch=4, layers=12, heads=8, embed=1024, mlp_hidden=4096)
    a.update(arch)
    net = ViT(channels=x.shape[1], height=x.shape[2], width=x.shape[3], max_batch=batch,
              seed=seed, **a)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(x.device)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            loss = ensf_vit_train_step(net.handle, x[sel].contiguous(), y[sel].contiguous(), lr,
                                       want_loss=(b0 == 0))
            if loss is not None:
                tot += loss
                cnt += 1
        entry = {"epoch": ep, "train_loss_first_batch": tot / max(cnt, 1)}
        if val is not None:
            xv, yv = val
            pred = torch.empty_like(xv)
            ensf_vit_forward(net.handle, xv, pred)
            entry["val_mse"] = float(torch.mean((pred - yv) ** 2))
        hist.append(entry)
        if log:
            log(str(entry))
    return net, hist


def train_surrogate(x, y, epochs=30, batch=32, lr=1e-3, seed=0, log=None, val=None):
    """Trains the conv surrogate on pairs (x, y) with the library's Adam; returns it and
    the per-epoch mean training loss (and validation loss if val = (xv, yv))."""
    import torch

    from .surrogate import Surrogate, ensf_surrogate_forward, ensf_surrogate_train_step
    n = x.shape[0]
    sur = Surrogate(c0=x.shape[1], width=64, layers=6, h=x.shape[2], w=x.shape[3],
                    max_batch=batch, seed=seed)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(x.device)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            loss = ensf_surrogate_train_step(sur.handle, x[sel].contiguous(), y[sel].contiguous(),
                                             lr, want_loss=(b0 == 0))
            if loss is not None:
                tot += loss
                cnt += 1
        entry = {"epoch": ep, "train_loss_first_batch": tot / max(cnt, 1)}
        if val is not None:
            xv, yv = val
            vl = []
            for b0 in range(0, xv.shape[0], batch):
                pred = torch.empty_like(xv[b0:b0 + batch])
                ensf_surrogate_forward(sur.handle, xv[b0:b0 + batch].contiguous(), pred)
                vl.append(float(torch.mean((pred - yv[b0:b0 + batch]) ** 2)))
            entry["val_mse"] = float(np.mean(vl))
        hist.append(entry)
        if log:
            log(str(entry))
    return sur, hist
