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


class FakePrecond:
    INFO = {"nlev": 3, "sizes": [4225, 700, 90], "nnz": [0, 0, 0], "ncolors": [2, 4, 5]}

    def __init__(self, *a, **k):
        pass

    def info(self):
        return self.INFO


def test_tile_split_rule():
    """The (lane_shift, bottom level, dense level) the library derives from a
    tile set, for the level sizes of the 1025 x 1025 hierarchy."""
    info = {"sizes": [1050625, 175446, 19580, 2181, 252], "ncolors": [2, 4, 4, 6, 5]}
    assert autotune.split(info, (1, 2048, 0)) == (1, 4, 4)
    assert autotune.split(info, (1, 2048, 4096)) == (1, 3, 3)
    assert autotune.split(info, (0, 8192, 0)) == (0, 3, 4)
    # a 2181-row sub-cycle is too large for the one-work-group bottom kernel
    assert autotune.split(info, (0, 65536, 4096)) == (0, 3, 3)
    small = {"sizes": [16641, 2827, 318, 40], "ncolors": [2, 4, 6, 7]}  # 129^2, max_coarse 64
    assert autotune.split(small, (0, 65536, 512)) == (0, 1, 2)
    assert autotune.split(small, (0, 65536, 4096)) == (0, 1, 1)
    assert autotune.split(info, (0, 0, 100)) == (0, 4, 4)      # no level above the coarsest small enough
    assert autotune.split(info, (0, 0, 200000)) == (0, 1, 1)
    many = dict(info, ncolors=[2, 4, 4, 70, 5])                  # too many colours for the bottom kernel
    assert autotune.split(many, (0, 8192, 4096)) == (0, 4, 4)
    cube = {"sizes": [2146689, 255871, 5592, 66], "ncolors": [2, 16, 31, 23]}  # 129^3
    assert autotune.split(cube, (1, 64, 4096)) == (1, 3, 3)
    assert autotune.split(cube, (1, 64, 8192)) == (1, 2, 2)      # the rule itself has no upper bound


def test_autotune_picks_fastest_and_caches(tmp_path, monkeypatch):
    times = {t: 1.0 + 0.1 * k for k, t in enumerate(autotune.CANDIDATES)}
    best = (1, 2048, 0)
    times[best] = 0.5
    calls = []
    l0 = {0: 0.5, 1: 0.45, 2: 0.4, 3: 0.42}  # seconds per iteration of the chosen set by level-0 form

    def fake_time(mesh, psi, pre, tiles, iters=24, reps=3):
        calls.append(tiles)
        return l0[tiles[3]] if len(tiles) == 4 else times[tiles]

    monkeypatch.setattr(autotune, "time_tiles", fake_time)
    monkeypatch.setattr(autotune, "_key", lambda mesh, p, mc: f"dev|{mesh.shape}|{p}|{mc}")
    monkeypatch.setattr(glnk, "Precond", FakePrecond)
    cache = str(tmp_path / "tiles.json")
    assert autotune.tune(FakeMesh(), None, cache=cache) == best + (2,)
    # each distinct split timed once, by its first candidate; then every
    # level-0 form of the fastest
    coarse = [t for t in calls if len(t) == 3]
    assert sorted(t for t in calls if len(t) == 4) == [best + (k,) for k in range(4)]
    splits = [autotune.split(FakePrecond.INFO, t) for t in coarse]
    assert len(set(splits)) == len(splits)
    assert set(splits) == {autotune.split(FakePrecond.INFO, t) for t in autotune.CANDIDATES}
    assert len(coarse) < len(autotune.CANDIDATES)
    table = json.load(open(cache))
    (entry,) = table.values()
    assert tuple(entry["tiles"]) == best + (2,)
    calls.clear()
    assert autotune.tune(FakeMesh(), None, cache=cache) == best + (2,)  # from the cache
    assert calls == []
    # the one-dispatch form when it is the faster; none tried in a batch
    l0.update({1: 0.6, 2: 0.6, 3: 0.6})
    assert autotune.tune(FakeMesh(), None) == best + (0,)
    calls.clear()
    assert autotune.tune(FakeMesh(), None, batch=True)[3] == 0
    assert all(len(t) == 3 for t in calls)


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
