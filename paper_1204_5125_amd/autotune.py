"""Autotuner for the V-cycle launch shapes (gl_tiles) per grid shape.

For one representative instance of each grid shape it times a fixed number
of preconditioned MINRES iterations (graph-replayed, as in the solvers) for
every candidate tile set, keeps the fastest, and caches the choice in a JSON
file keyed by device name, grid shape, precision and coarse-size limit.  The
candidates change only the order of rounding in row sums (lanes per row) and
which levels run inside the one-work-group bottom kernel.
"""
import json
import os
import time

from . import glnk

CANDIDATES = [(ls, br) for ls in (-1, 0, 1) for br in (64, 512, 2048, 8192)]


def _key(mesh, precision, max_coarse):
    import torch
    dev = torch.cuda.get_device_name(0).replace(" ", "_")
    return f"{dev}|dim{mesh.dim}|{'x'.join(str(n) for n in mesh.shape)}|p{precision}|mc{max_coarse}"


def time_tiles(mesh, psi, pre, tiles, iters=24, reps=3):
    """Seconds per MINRES iteration of J(psi) with preconditioner `pre` under
    `tiles`, over a fixed iteration count (rtol = 0)."""
    import torch
    glnk.gl_precond_set_tiles(pre, *tiles)
    b = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)
    best = float("inf")
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        glnk.gl_jacobian_solve(mesh, psi, pre, b, x, rtol=0.0, max_iter=iters, poll_every=iters,
                               inner_rtol=1e-30, raise_on_fail=False)
        torch.cuda.synchronize()
        if r:  # the first run builds the graph
            best = min(best, (time.perf_counter() - t0) / iters)
    return best


def tune(mesh, psi, precision=glnk.GL_FP32, max_coarse=64, cache=None, candidates=CANDIDATES,
         log=None):
    """Best (lane_shift, bottom_rows) for this grid shape; read from / written
    to the JSON file `cache` when given."""
    key = _key(mesh, precision, max_coarse)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return tuple(table[key]["tiles"])
    pre = glnk.Precond(mesh, psi, precision=precision, max_coarse=max_coarse)
    times = {}
    for t in candidates:
        times[t] = time_tiles(mesh, psi, pre, t)
        if log:
            log(f"[autotune] {key} tiles {t}: {times[t] * 1e6:.1f} us/iteration")
    best = min(times, key=times.get)
    if cache:
        table[key] = {"tiles": list(best), "us_per_iteration": times[best] * 1e6,
                      "default_us_per_iteration": times.get((0, 512), float("nan")) * 1e6}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best
