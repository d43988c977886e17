"""Every kernel variant the tuner can choose (Gram tile, W.X tile, k-step depth, LDS stage
count, split-K scale), forced through a tune-cache file, against the FP64 oracle on a
problem that is ragged in members, particles and components and spans several tiles."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ensf as O
from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu

N, M, D, K, SIG = 70, 130, 3001, 20, 0.5
N_GRAM, N_WX = 7, 9
PREC_ID = {"fp32": 0, "bf16x3": 1}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(4242)
    X = rng.standard_normal((N, D)).astype(np.float32)
    idx = np.sort(rng.choice(D, D // 2, replace=False)).astype(np.int32)
    y = np.arctan(rng.standard_normal(idx.size)).astype(np.float32)
    want = O.analysis(X, idx, y, SIG, K, 77, filter_id=1, n_particles=M)
    return X, idx, y, want


def _key(prec):
    b = lambda v: int(v).bit_length() - 1
    return f"gfx950/p{PREC_ID[prec]}/n{b(N)}/m{b(M)}/d{b(D)}"


def _variants():
    out = []
    for g in range(N_GRAM):
        for w in range(N_WX):
            i = g * N_WX + w
            gbk = 32 if g == 4 else (32, 64)[i % 2]     # the 256x256 Gram has k-step 32 only
            out.append((g, w, (0.5, 1.0, 2.0)[i % 3], gbk, (32, 64)[(i // 2) % 2],
                        1 + i % 2, 1 + (i // 3) % 2))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_every_tile_variant_matches_oracle(dev, tmp_path, case, prec):
    X, idx, y, want = case
    Xg = torch.from_numpy(X).to(dev)
    ig = torch.from_numpy(idx).to(dev)
    yg = torch.from_numpy(y).to(dev)
    worst = 0.0
    for v in _variants():
        g, w, sc, gbk, wbk, gst, wst = v
        cache = tmp_path / f"{prec}_{g}_{w}.json"
        cache.write_text(json.dumps({_key(prec): [g, w, sc, gbk, wbk, gst, wst]}))
        post = torch.empty((M, D), device=dev)
        with ensf.Context(precision=prec, tune_cache=str(cache)) as ctx:
            ensf.ensf_analysis(ctx.handle, Xg, post, ig, yg, SIG, K, 77, 1)
            st, nbad = ensf.ensf_sync_status(ctx.handle)
        assert st == ensf.ENSF_OK, (v, st, nbad)
        got = post.cpu().numpy().astype(np.float64)
        err = np.abs(got - want).max() / np.abs(want).max()
        worst = max(worst, err)
        assert err <= 5e-4, (v, err)
    print(f"{prec}: {len(_variants())} variants, worst max rel diff {worst:.2e}")
