"""Host-side logic that needs no GPU: the tile autotuner's choice and cache,
the seeded input recipes, the network shape agreement with the oracle, and
the benchmark's refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import unet as U
from paper_1204_5125_amd import autotune, glnk, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class FakeMesh:
    dim, shape, n = 2, (65, 65), 65 * 65


def test_autotune_picks_fastest_and_caches(tmp_path, monkeypatch):
    times = {t: 1.0 + 0.1 * k for k, t in enumerate(autotune.CANDIDATES)}
    best = (1, 2048)
    times[best] = 0.5
    calls = []

    def fake_time(mesh, psi, pre, tiles, iters=24, reps=3):
        calls.append(tiles)
        return times[tiles]

    monkeypatch.setattr(autotune, "time_tiles", fake_time)
    monkeypatch.setattr(autotune, "_key", lambda mesh, p, mc: f"dev|{mesh.shape}|{p}|{mc}")
    monkeypatch.setattr(glnk, "Precond", lambda *a, **k: object())
    cache = str(tmp_path / "tiles.json")
    assert autotune.tune(FakeMesh(), None, cache=cache) == best
    assert sorted(calls) == sorted(autotune.CANDIDATES)
    table = json.load(open(cache))
    (entry,) = table.values()
    assert tuple(entry["tiles"]) == best
    calls.clear()
    assert autotune.tune(FakeMesh(), None, cache=cache) == best  # from the cache
    assert calls == []


def test_sweep_mus_recipe():
    mus = inputs.sweep_mus(2.0, 0.01, 0.002, seed=0)
    d = np.diff(mus)
    assert mus[0] == 0.0 and mus[-1] == pytest.approx(2.0)
    assert np.all(d[:-1] >= 0.008 - 1e-12) and np.all(d[:-1] <= 0.012 + 1e-12)
    assert 170 <= len(mus) <= 230
    assert inputs.sweep_mus(2.0, 0.01, 0.002, seed=0) == mus


def test_unet_shapes_and_init_match_the_oracle_layout():
    for levels, base in [(4, 32), (3, 32), (2, 64)]:
        shapes = glnk.unet_layer_shapes(levels, base)
        assert shapes == U.layer_specs(levels, base)
        theta = inputs.unet_init(shapes, seed=1)
        assert theta.size == U.num_params(shapes) and theta.dtype == np.float32
        # head weights start at zero (a fresh network is the secant start)
        ci, co, k = shapes[-1]
        assert np.all(theta[-(co * ci + co):] == 0.0)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
