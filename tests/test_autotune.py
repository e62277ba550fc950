"""The schedule autotuner: seeded samples, its cache, and (GPU) a tuned
launch that gives the same bits as the default one."""
import json

import numpy as np
import pytest

from paper_1611_02274_amd import autotune
from paper_1611_02274_amd import inputs as I


def test_sample_indices_seeded_sorted_and_bounded():
    a = autotune.sample_indices(1000, 0.05, 64, seed=3)
    b = autotune.sample_indices(1000, 0.05, 64, seed=3)
    assert np.array_equal(a, b) and a.size == 64 and np.all(np.diff(a) > 0)
    assert autotune.sample_indices(1000, 0.5, 64, seed=3).size == 500
    assert autotune.sample_indices(10, 0.5, 64, seed=3).size == 10


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv(autotune.CACHE_ENV, str(path))
    autotune._store("k", {"best": {"schedule": 1}})
    autotune._store("k2", {"best": {"schedule": 2}})
    assert autotune._load()["k"]["best"] == {"schedule": 1}
    assert json.loads(path.read_text())["k2"]["best"] == {"schedule": 2}


@pytest.mark.gpu
def test_tuned_network_launch_equals_default(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_02274_amd as rk
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 4096, 31, (1000.0, 2500.0))
    prob = rk.Problem.network(net)
    best = autotune.tune_network(prob, "rkc", y0, g, 0.0, 1e-7, 1e-8, 1e-12, fraction=0.5,
                                 minimum=2048, seed=1)
    assert best in [c for c in autotune.NETWORK_CANDIDATES if c["schedule"] != 3]
    assert autotune.tune_network(prob, "rkc", y0, g, 0.0, 1e-7, 1e-8, 1e-12) == best
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    ya, sa, sta = rk.integrate_rkc(prob, yd, gd, 0.0, 1e-7, 1e-8, 1e-12)
    yb, sb, stb = rk.integrate_rkc(prob, yd, gd, 0.0, 1e-7, 1e-8, 1e-12, **best)
    torch.cuda.synchronize()
    assert torch.equal(ya.view(torch.int64), yb.view(torch.int64))
    assert torch.equal(sa, sb) and torch.equal(sta, stb)
