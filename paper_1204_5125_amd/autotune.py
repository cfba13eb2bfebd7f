"""Autotuner for the V-cycle launch shapes (gl_tiles) per grid shape.

For one representative instance of each grid shape it times a fixed number
of preconditioned MINRES iterations (graph-replayed, as in the solvers) for
every candidate tile set, keeps the fastest, and caches the choice in a JSON
file keyed by device name, grid shape, precision and coarse-size limit.  The
candidates change only the order of rounding (lanes per row; a sub-cycle
applied as an explicit matrix; level 0 of a 2D grid in two LDS-tiled kernels,
on one of L0_SHAPES) and which levels run inside the one-work-group bottom
kernel; candidates that give the same split of the hierarchy are timed once.
The level-0 forms are timed on the best coarse-level choice only.
"""
import json
import os
import time

from . import glnk

CANDIDATES = [(ls, br, dr) for ls in (-1, 0, 1) for br in (64, 512, 2048, 8192) for dr in (0, 4096, 8192)]
# A batch runs many instances per dispatch: the launches an explicit
# sub-cycle saves are shared there, its matrix reads are not, so batches
# choose among the tile sets without one.
BATCH_CANDIDATES = [c for c in CANDIDATES if c[2] == 0]
MAX_COLOURS = 64   # colours per level the bottom kernel handles
DEFAULT_BOTTOM = 512
L0_SHAPES = (1, 2, 3)  # gl_tiles.l0_tiled: 32 x 32, 32 x 16, 16 x 16 node tiles
BOTTOM_DENSE_ROWS = 512  # largest explicit sub-cycle the bottom kernel applies


def split(info, tiles):
    """(lane_shift, first level of the bottom kernel, level applied as a dense
    operator) that a preconditioner with these level sizes and colour counts
    (`Precond.info()`) derives from `tiles`, by the rule of
    gl_precond_set_tiles."""
    ls, br, dr = tiles
    sizes, colours = info["sizes"], info["ncolors"]
    last = len(sizes) - 1
    tail = last
    if dr > 0:
        for lev in range(1, last):
            if sizes[lev] <= dr:
                if all(c <= MAX_COLOURS for c in colours[lev:last]):
                    tail = lev
                break
    first = tail
    if tail == last or sizes[tail] <= BOTTOM_DENSE_ROWS:
        for lev in range(tail - 1, 0, -1):
            if sizes[lev] > (br or DEFAULT_BOTTOM) or colours[lev] > MAX_COLOURS:
                break
            first = lev
    return ls, first, tail


def _key(mesh, precision, max_coarse):
    import torch
    dev = torch.cuda.get_device_name(0).replace(" ", "_")
    shape = 'x'.join(str(n) for n in mesh.shape) if mesh.shape else f"simplicial{mesh.n}"
    return f"{dev}|dim{mesh.dim}|{shape}|p{precision}|mc{max_coarse}"


# Tile sets also change the numeric setup (an explicit sub-cycle is formed at
# every setup), so a candidate is charged its setup time spread over this many
# iterations, a typical Jacobian solve (170-400 MINRES iterations on the
# 1025^2 grid from a random-phase start, about 100 on the 129^3 grid).
SETUP_AMORTIZED_OVER = 100


def time_tiles(mesh, psi, pre, tiles, iters=24, reps=3):
    """Seconds per MINRES iteration of J(psi) with preconditioner `pre` under
    `tiles`, over a fixed iteration count (rtol = 0), plus the numeric setup
    time over SETUP_AMORTIZED_OVER iterations."""
    import torch
    glnk.gl_precond_set_tiles(pre, *tiles)
    setup = float("inf")
    for r in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre.update(psi)
        torch.cuda.synchronize()
        setup = min(setup, time.perf_counter() - t0)
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
    return best + setup / SETUP_AMORTIZED_OVER


def tune(mesh, psi, precision=glnk.GL_FP32, max_coarse=64, cache=None, candidates=None,
         log=None, batch=False):
    """Best (lane_shift, bottom_rows, dense_rows, l0_tiled) for this grid
    shape, among `candidates` (default: CANDIDATES, or BATCH_CANDIDATES for a
    batch) and, on a 2D grid outside a batch, both level-0 forms; read from /
    written to the JSON file `cache` when given."""
    if candidates is None:
        candidates = BATCH_CANDIDATES if batch else CANDIDATES
    key = _key(mesh, precision, max_coarse) + ("|batch" if batch else "")
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table and len(table[key]["tiles"]) == 4:
            return tuple(table[key]["tiles"])
    pre = glnk.Precond(mesh, psi, precision=precision, max_coarse=max_coarse)
    info = pre.info()
    times, seen = {}, {}
    for t in candidates:
        sp = split(info, t)
        if sp in seen:  # same launches as an earlier candidate
            times[t] = times[seen[sp]]
            continue
        seen[sp] = t
        times[t] = time_tiles(mesh, psi, pre, t)
        if log:
            log(f"[autotune] {key} tiles {t}: {times[t] * 1e6:.1f} us/iteration")
    best = min(times, key=times.get)
    times = {t + (0,): v for t, v in times.items()}
    best = best + (0,)
    if mesh.dim == 2 and mesh.shape and not batch:  # the LDS-tiled level 0 is for grids
        forms = [best]
        for shape in L0_SHAPES:
            tiled = best[:3] + (shape,)
            times[tiled] = time_tiles(mesh, psi, pre, tiled)
            forms.append(tiled)
            if log:
                log(f"[autotune] {key} tiles {tiled}: {times[tiled] * 1e6:.1f} us/iteration")
        # re-time the one-dispatch form beside them, so all see the same state
        times[best] = min(times[best], time_tiles(mesh, psi, pre, best))
        best = min(forms, key=times.get)
    if cache:
        table[key] = {"tiles": list(best), "us_per_iteration": times[best] * 1e6,
                      "default_us_per_iteration": times.get((0, 512, 0, 0), float("nan")) * 1e6}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best
