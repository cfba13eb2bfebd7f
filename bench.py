#!/usr/bin/env python3
"""Jacobian-solve benchmark on one MI355X.

Workload (one "step"): the 2D 1025 x 1025 grid (1,050,625 nodes), side 10,
uniform field mu = 1 along z, psi0 = 0.9 exp(i theta) with theta ~ U[0, 2 pi)
from seed 0; four Newton steps from psi0, each one preconditioned MINRES solve
of the Jacobian system to relative residual 1e-10 (preconditioner numeric
setup, MINRES, update, GL residual).  The hierarchy's grid-only part is built
once during warm-up.  The headline value uses the FP32 V-cycle under the FP64
outer iteration, in MINRES with the Krylov basis stored and reorthogonalised
(the remedy for the loss of orthogonality the paper names in Sec. 4; with it
the FP32 V-cycle needs the iterations of the FP64 one); plain MINRES with the
FP32 and the FP64 V-cycle, the relaxed switch and the reorthogonalised FP64
solve are timed beside it.

Prints one JSON line.  Roofline: the dominant kernel's algorithmic bytes per
launch over its HIP-event-measured average duration in an identical timed
pass.  cpu_baseline: the plain C oracle on this host, one full solve of the
workload's second Newton system.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Jacobian solves/s + HBM GB/s at 1M nodes, FP32-precond vs FP64 at 1e-10"
HBM_PEAK_GBS = 8000.0
N_AXIS = (1025, 1025)
SIDE = (10.0, 10.0)
MU = 1.0
NEWTON_STEPS = 4
RTOL = 1e-10
L0_TILED_NAME = "L0 Gauss-Seidel in LDS tiles (L0PreTile, L0PostTile)"
KERNEL_NAMES = {1: "MinresJapply", 2: "L0 Gauss-Seidel sweeps (L0PreBlack, L0Sweep, L0Last)",
                3: "L0Residual", 4: "level-0 transfers (CsrSpmv restriction, L0ProlongBlack)", 5: "MinresVupdate", 6: "k_minres_wx",
                7: "GlResidual", 8: "EllSgs (Gauss-Seidel colour sweep, levels >= 1)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


MAX_COARSE = 512
BATCH_HALVINGS = 3   # batched continuation: halvings of a step whose Newton fails
# tiles of the single counter pass (--one-pass): the autotuner's choice for
# this grid on MI355X, FP32 and FP64 alike (lane_shift, bottom_rows, dense_rows)
ONE_PASS_TILES = (0, 64, 4096)
# the autotuner's full choice without the profiler (--fixed-tiles): level 0 in
# 16 x 16-node LDS tiles with the FP32 V-cycle, one dispatch per pass in FP64
FIXED_TILES = {"fp32": ONE_PASS_TILES + (3,), "fp64": ONE_PASS_TILES + (0,)}
COPY_BYTES = 256 << 20   # counter calibration copy: reads and writes this many bytes
# HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter passes
# (calibrated on the copy), valid for the kernel sources with this fingerprint;
# "2t2", "2t3": the level-0 class in 32 x 16 and 16 x 16 LDS tiles
TRAFFIC = {"csrc_sha256": "001a72ced063a46ec0329231d3fb9f116a665765e5dd16b1156c50e0eaf5befd",
           8: 4971861.0, 2: 21189661.2, "2t2": 48767097.9, "2t3": 48785225.5}


def csrc_fingerprint():
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1204_5125_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()
RELAX = 1e-4   # relaxed variant: FP64 V-cycle until the MINRES estimate falls below this
REORTH = 400   # Krylov basis of the reorthogonalised solves (above every solve's count here)
BATCH_REORTH = 300  # per instance in the batch (64 bases: 32 B per node and vector in FP64, 28 in FP32)


def run_steps(glnk, torch, mesh, psi0, psi, handle, precision, steps, relax=0.0, reorth=0):
    # every variant stops on the true residual (plain FP64: a restart when the
    # recurrence estimate and the true residual part; plain FP32: refinement,
    # or with relax > 0 one recurrence with the FP64 V-cycle above relax;
    # reorthogonalised: each start measures the true residual)
    inner = RTOL if precision == glnk.GL_FP64 and reorth == 0 else 0.0
    infos = []
    for _ in range(steps):
        psi.copy_(psi0)
        rc, info = glnk.gl_newton_solve(mesh, psi, fixed_steps=NEWTON_STEPS, krylov_rtol=RTOL,
                                        krylov_max_iter=8000, poll_every=16, precision=precision,
                                        inner_rtol=inner, relax_rtol=relax, max_coarse=MAX_COARSE,
                                        precond=handle, reorth=reorth)
        infos.append(info)
    return infos


def timed(glnk, torch, mesh, psi0, psi, handle, precision, steps, relax=0.0, reorth=0):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = run_steps(glnk, torch, mesh, psi0, psi, handle, precision, steps, relax, reorth)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos


def host_stream_add():
    """Host memory bandwidth on one thread: a = b + c over 2^25 doubles per
    array (24 bytes moved per element), best of 5 (numpy)."""
    import numpy as np
    n = 1 << 25
    b, c = np.ones(n), np.ones(n)
    a = np.empty(n)
    best = float("inf")
    for _ in range(5):
        t0 = time.perf_counter()
        np.add(b, c, out=a)
        best = min(best, time.perf_counter() - t0)
    return 24.0 * n / best / 1e9


def cpu_baseline():
    """The serial C oracle on one full Jacobian solve of the same workload:
    the second Newton step's system (the first step, untimed, reaches its
    state from the same psi0), timed from the preconditioner setup to the
    MINRES solution at rtol 1e-10."""
    import platform

    import oracle
    from paper_1204_5125_amd import inputs
    m = oracle.Mesh(2, N_AXIS, SIDE, mu=MU)
    psi0 = inputs.random_phase_state(m.n, seed=0)
    psi, info = oracle.newton(m, psi0, fixed_steps=1, krylov_rtol=RTOL, krylov_max_iter=4000,
                              max_coarse=MAX_COARSE)
    t0 = time.perf_counter()
    amg = oracle.Amg.for_state(m, psi, max_coarse=MAX_COARSE)
    t_setup = time.perf_counter() - t0
    _, ki, _ = oracle.minres(m, psi, -m.gl(psi), amg=amg, rtol=RTOL, max_iter=4000)
    t_solve = time.perf_counter() - t0
    t_iter = (t_solve - t_setup) / max(1, ki["iterations"])
    bw = host_stream_add()
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    # the survey's per-iteration byte model of the FP64 path (594 B per node)
    model = 594.0 * m.n
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of the workload's second Newton system (1025x1025, from the same psi0 "
                      f"after one untimed oracle Newton step): preconditioner setup {t_setup:.2f} s + "
                      f"{ki['iterations']} MINRES iterations to 1e-10 ({t_iter * 1e3:.0f} ms each), "
                      f"{t_solve:.1f} s, serial C on one host core",
            "seconds_per_solve": t_solve, "minres_iterations": ki["iterations"],
            "converged": bool(ki["converged"]), "res_true": ki["res_true"],
            "host_cpu": cpu, "host_threads": os.cpu_count(),
            "host_stream_add_gbs_1thread": bw,
            "roofline": {"bound": "host memory", "achieved": model / t_iter / 1e9, "peak": bw, "unit": "GB/s",
                         "frac": model / t_iter / 1e9 / bw,
                         "note": "594 B per node per MINRES iteration (FP64 byte model) over the oracle's "
                                 "time per iteration, against one thread's measured a = b + c bandwidth"}}


def iteration_bytes(glnk, pre, precision):
    """Algorithmic bytes of the V-cycle kernels the profiler does not count,
    per MINRES iteration, from the handle's hierarchy: per multi-kernel
    level >= 1 the residual (operator, b, x, r) and the transfers
    (P / R entries, both vectors), and the dense product of the explicit
    sub-cycle or coarsest inverse."""
    info = pre.info()
    tiles = glnk.gl_precond_get_tiles(pre)
    sz = 16.0 if precision == glnk.GL_FP64 else 8.0
    sizes, nnz = info["sizes"], info["nnz"]
    nlev = info["nlev"]
    dense = next((l for l in range(1, nlev) if sizes[l] <= tiles["dense_rows"]), nlev - 1)
    total = 0.0
    for l in range(1, dense):
        total += nnz[l] * (4 + sz) + (sizes[l] + 1) * 4 + 3 * sizes[l] * sz          # residual
    for l in range(1, dense):
        pn = int(pre.export(l, "P_rp")[-1])
        total += 2 * (pn * (4 + sz) + (sizes[l] + sizes[l + 1] + 2) * 4) + 3 * (sizes[l] + sizes[l + 1]) * sz
    total += sizes[dense] ** 2 * sz + 2 * sizes[dense] * sz                          # dense product
    return total


def one_pass(l0_tiled=0, reorth=0):
    """One Newton step of the headline workload (FP32 V-cycle, plain MINRES;
    level 0 in LDS tiles of the given shape when l0_tiled > 0) and a plain
    copy of known size, for rocprofv3 counter passes.  reorth > 0: two Newton
    steps with the basis reorthogonalised instead (the second solve is the
    long one)."""
    import torch

    from paper_1204_5125_amd import glnk, inputs
    torch.cuda.set_device(0)
    mesh = glnk.Mesh(2, N_AXIS, SIDE, mu=MU)
    psi = torch.from_numpy(inputs.random_phase_state(mesh.n, seed=0)).cuda()
    h = glnk.PrecondHandle(mesh)
    # builds the hierarchy (two MINRES iterations), then the tiles the autotuner picks here
    glnk.gl_newton_solve(mesh, psi.clone(), fixed_steps=1, krylov_rtol=RTOL, krylov_max_iter=2,
                         poll_every=2, precision=glnk.GL_FP32, max_coarse=MAX_COARSE, precond=h,
                         raise_on_fail=False)
    glnk.gl_precond_set_tiles(h, *ONE_PASS_TILES, l0_tiled)
    glnk.gl_newton_solve(mesh, psi, fixed_steps=2 if reorth else 1, krylov_rtol=RTOL, krylov_max_iter=8000,
                         poll_every=16, precision=glnk.GL_FP32, max_coarse=MAX_COARSE, precond=h, reorth=reorth)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.add(a, 0.0, out=b)
    torch.cuda.synchronize()


def newton_rounds(batch, psis, max_rounds, tag, totals=None, **kw):
    """Batched Newton one lock-step round per call (the same work as one call
    with max_steps = max_rounds, with a progress line per round); the
    library's per-call statistics are added up in `totals`."""
    solves = iters = 0
    infos = None
    hist = [[] for _ in psis]  # per instance: (GL residual, MINRES iterations) of each Newton step
    for r in range(max_rounds):
        rc, infos = batch.newton_solve(psis, max_steps=1, raise_on_fail=False, **kw)
        st = batch.stats()
        if totals is not None:
            totals["graph_launches"] += st["graph_launches"]
            totals["dispatches_per_graph"] = max(totals["dispatches_per_graph"], st["dispatches_per_graph"])
            totals["groups"] = max(totals["groups"], st["groups"])
            for k, v in st["seconds"].items():
                totals["seconds"][k] += v
        n = sum(i["steps"] for i in infos)
        if n == 0:
            break
        solves += n
        iters += sum(sum(i["krylov_iters"]) for i in infos)
        for k, i in enumerate(infos):
            if i["steps"]:
                hist[k].append((i["res"][-1], i["krylov_iters"][-1]))
        sec = st["seconds"]
        log(f"[bench] {tag} round {r + 1}: {n} solves, {iters} iterations so far; "
            f"setup {sec['setup']:.2f} s, solve {sec['solve']:.2f} s")
    bad = [k for k, i in enumerate(infos) if not i["res"][-1] < kw["tol"]]
    return solves, iters, len(infos) - len(bad), {k: hist[k] for k in bad}


def bench_batch(args):
    """Batched continuation: 64 instances on 2D grids of 129^2, 257^2 or 513^2
    nodes (drawn with seed 0), side 10, mu_k = 2k/63, FP32 V-cycle under FP64
    outer iterations.  Untimed: autotuning of the tiles per grid size and the
    warm start (Newton from psi = 1 at mu_k).  Timed: `steps` continuation
    steps of dmu = 0.02 (secant predictor after the first), each one batched
    Newton solve of all instances; an instance whose Newton does not converge
    within 15 steps retries from its last solution with the step halved (at
    most 3 times: the tracked branch can end at a fold), in a batched solve
    of the retrying instances."""
    import numpy as np
    import torch

    from paper_1204_5125_amd import autotune, glnk
    torch.cuda.set_device(0)
    count, side, dmu = 64, 10.0, 0.02
    sizes = np.random.default_rng(0).choice([129, 257, 513], count)
    mus = [2.0 * k / (count - 1) for k in range(count)]
    meshes = [glnk.Mesh(2, (int(N), int(N)), (side, side), mu=mu) for N, mu in zip(sizes, mus)]
    psis = [torch.ones(m.n, dtype=torch.complex128, device="cuda") for m in meshes]
    prec = glnk.GL_FP64 if args.batch_fp64 else glnk.GL_FP32
    kw = dict(tol=1e-10, krylov_rtol=1e-10, poll_every=16, precision=prec,
              max_coarse=args.batch_max_coarse, deflate=not args.batch_plain,
              reorth=BATCH_REORTH if args.batch_reorth else 0)
    batch = glnk.Batch(meshes)
    tiles = {}
    for N in sorted(set(int(v) for v in sizes)):
        i = int(np.nonzero(sizes == N)[0][0])
        tiles[N] = autotune.tune(meshes[i], psis[i], precision=prec, max_coarse=args.batch_max_coarse,
                                 cache=args.tile_cache, log=log, batch=True)
        log(f"[bench] tiles for {N}^2: lane_shift {tiles[N][0]}, bottom_rows {tiles[N][1]}")
    for i, N in enumerate(sizes):
        batch.set_tiles(*tiles[int(N)], index=i)
    log(f"[bench] warm start of {count} instances, sizes "
        f"{ {int(k): int(v) for k, v in zip(*np.unique(sizes, return_counts=True))} }")
    t0 = time.perf_counter()
    ws, wi, wc, _ = newton_rounds(batch, psis, 40, "warm start", krylov_max_iter=4000, **kw)
    log(f"[bench] warm start: {time.perf_counter() - t0:.2f} s, {ws} solves, converged {wc}/{count}")
    prev = [p.clone() for p in psis]
    pred = [torch.empty_like(p) for p in psis]
    mu_now = list(mus)
    hlast = [None] * count   # each instance's last continuation step (none before the first)
    solves = iters = conv = first = 0
    unconverged, halved, folds = [], [], []
    totals = {"graph_launches": 0, "dispatches_per_graph": 0, "groups": 0,
              "seconds": {"residual": 0.0, "setup": 0.0, "solve": 0.0}}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        # every instance tries the full step; one that does not converge
        # within 15 Newton steps retries from its last solution with the step
        # halved (at most BATCH_HALVINGS times), as natural continuation does
        h = [dmu] * count
        todo = list(range(count))
        for attempt in range(BATCH_HALVINGS + 1):
            for i in todo:
                meshes[i].set_field(mu_now[i] + h[i])
                if hlast[i] is None:
                    pred[i].copy_(psis[i])
                else:
                    glnk.gl_secant_predict(meshes[i], psis[i], prev[i], h[i] / hlast[i], pred[i])
            tag = f"step {step + 1}" + (f" retry {attempt}" if attempt else "")
            s_, i_, c_, bad = newton_rounds(batch, pred, 15, tag, totals, krylov_max_iter=1000, **kw)
            solves += s_
            iters += i_
            if attempt == 0:
                first += c_
                unconverged += [{"step": step + 1, "instance": i, "N": int(sizes[i]), "mu": mu_now[i] + dmu,
                                 "gl_residual_and_minres_iterations": hh} for i, hh in bad.items()]
            else:
                halved += [{"step": step + 1, "instance": i, "N": int(sizes[i]), "mu": mu_now[i] + h[i],
                            "dmu": h[i]} for i in todo if i not in bad]
            todo = [i for i in todo if i in bad]
            if not todo:
                break
            for i in todo:
                h[i] *= 0.5
        for i in todo:  # no step size worked: the instance stays where it is
            folds.append({"step": step + 1, "instance": i, "N": int(sizes[i]), "mu": mu_now[i]})
            meshes[i].set_field(mu_now[i])
        conv += count - len(todo)
        for i in range(count):
            if i in todo:
                continue
            prev[i].copy_(psis[i])
            psis[i].copy_(pred[i])
            mu_now[i] += h[i]
            hlast[i] = h[i]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = totals
    out = {
        "metric": "batched Jacobian solves/s (continuation, 64 instances)",
        "value": solves / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (outer) / " + ("f64" if args.batch_fp64 else "f32") + " (V-cycle)",
        "data": "synthetic: 64 continuation instances, grid sizes drawn with seed 0",
        "config": {"workload": "64 instances, 2D grids of 129^2 / 257^2 / 513^2 nodes (seed 0), side 10, "
                               "mu_k = 2k/63, continuation steps of 0.02 with the secant predictor (an "
                               "instance that fails retries with the step halved, up to 3 times), "
                               "Newton to 1e-10 within 15 steps, MINRES to 1e-10 (deflated unless --batch-plain), "
                               "FP32 V-cycle (FP64 with --batch-fp64)",
                   "sizes": {str(k): int(v) for k, v in zip(*np.unique(sizes, return_counts=True))},
                   "tiles": {str(k): list(v) for k, v in tiles.items()},
                   "amg_max_coarse": args.batch_max_coarse},
        "jacobian_solves": solves, "minres_iterations": iters,
        "dispatches_per_graph": st["dispatches_per_graph"], "groups": st["groups"],
        "graph_launches": st["graph_launches"], "host_seconds": st["seconds"],
        "deflate": not args.batch_plain,
        "reorth": BATCH_REORTH if args.batch_reorth else 0,
        "converged_fraction": conv / (count * args.steps),
        "converged_first_try_fraction": first / (count * args.steps), "unconverged_first_try": unconverged,
        "halved_steps": halved, "folds": folds,
        "graph_launches_per_step": st["graph_launches"] / args.steps,
        "warm_start": {"solves": ws, "iterations": wi, "converged": wc},
    }
    print(json.dumps(out), flush=True)


def bench_continuation(args):
    """Learned predictor (config: 2D 513^2, side 8, mu 0 -> 2): a seeded
    training sweep (steps 0.01 +- U(0.002)), U-Net training (4 levels, 32 base
    channels) on pairs (psi_i, psi_{i+s}), s = 1..3, then the canonical sweep
    mu = 0, 0.02, ..., 2 twice: secant start, and learned start with the
    secant as fallback (whichever start has the smaller GL residual)."""
    import numpy as np
    import torch

    from paper_1204_5125_amd import continuation, glnk, inputs, predictor
    torch.cuda.set_device(0)
    N, side, levels, base = 513, 8.0, 4, 32
    mesh = glnk.Mesh(2, (N, N), (side, side), mu=0.0)
    ones = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
    common = dict(tol=1e-10, krylov_rtol=1e-10, krylov_max_iter=3000, max_newton=25, max_coarse=64,
                  poll_every=16)

    def progress(tag):
        def cb(rec, _):
            if int(round(rec["mu"] / 0.02)) % 10 == 0 or rec["status"] != 0:
                log(f"[bench] {tag}: mu {rec['mu']:.4f} newton {rec['newton_steps']} "
                    f"krylov {sum(rec['krylov_iters'])} status {rec['status']} ({rec['predictor']})")
        return cb

    mus_train = inputs.sweep_mus(2.0, 0.01, 0.002, seed=0)
    t0 = time.perf_counter()
    recs, states = predictor.sweep(mesh, mus_train, ones, precision=glnk.GL_FP64, callback=progress("train sweep"),
                                   **common)
    t_sweep = time.perf_counter() - t0
    log(f"[bench] training sweep: {len(states)} states in {t_sweep:.1f} s")
    pairs = predictor.make_pairs(mesh, states)
    net = glnk.UNet(levels, base)
    net.set_params(predictor.init_params(levels, base, seed=0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = predictor.train(net, mesh, pairs, epochs=args.epochs, batch=4, lr=1e-3, lr_end=5e-5, seed=0,
                           log=lambda m: log(f"{m} ({time.perf_counter() - t0:.1f} s)"))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # U-Net forward throughput on the matrix cores (BF16, FP32 accumulation)
    shapes = glnk.unet_layer_shapes(levels, base)
    Nl = [(N - 1) // (1 << l) + 1 for l in range(levels)]
    lvl = [l for l in range(levels) for _ in range(2)] + [l for l in range(levels - 2, -1, -1) for _ in range(2)]
    flops = sum(2.0 * Nl[l] ** 2 * 9 * ci * co for l, (ci, co, k) in zip(lvl, shapes[:-1]))
    flops += 2.0 * Nl[0] ** 2 * shapes[-1][0] * shapes[-1][1]
    out_t = torch.empty_like(ones)
    net.predict(mesh, states[1][1], states[1][1], states[1][0], 0.02, out_t)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        net.predict(mesh, states[1][1], states[1][1], states[1][0], 0.02, out_t)
    ev1.record()
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1) / 10
    unet_roof = {"bound": "mfma", "kernel": "U-Net forward (k_conv3x3 and transfers)",
                 "achieved": flops / (fwd_ms * 1e-3) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                 "frac": flops / (fwd_ms * 1e-3) / 1e12 / 2500.0, "traffic": None,
                 "forward_ms": fwd_ms, "flop_per_forward": flops}
    log(f"[bench] U-Net forward: {fwd_ms:.2f} ms, {unet_roof['achieved']:.1f} TFLOP/s")
    mus = [0.02 * k for k in range(101)]
    runs = {}
    variants = [("fp64_secant", glnk.GL_FP64, None, False, 0),
                ("fp64_learned", glnk.GL_FP64, "residual", False, 0),
                ("fp64_learned_always", glnk.GL_FP64, "always", False, 0),
                ("fp64_secant_deflated", glnk.GL_FP64, None, True, 0),
                ("fp32_secant_deflated", glnk.GL_FP32, None, True, 0),
                ("fp64_learned_always_deflated", glnk.GL_FP64, "always", True, 0),
                ("fp32_learned_always_deflated", glnk.GL_FP32, "always", True, 0),
                # MINRES with the Krylov basis reorthogonalised (Sec. 4's
                # remedy), where the FP32 V-cycle keeps the FP64 count
                ("fp32_secant_deflated_reorth", glnk.GL_FP32, None, True, REORTH),
                ("fp32_learned_always_deflated_reorth", glnk.GL_FP32, "always", True, REORTH)]
    for name, prec, learned, defl, reorth in variants:
        pred = predictor.LearnedPredictor(net, mesh, select=learned) if learned else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, _, _ = continuation.continuation_path(mesh, ones, mus, precision=prec, predictor=pred,
                                                    callback=progress(name), deflate=defl, reorth=reorth, **common)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        runs[name] = {"seconds": dt, "steps": len(recs) - 1,
                      "newton_steps": sum(r["newton_steps"] + r.get("failed_newton_steps", 0) for r in recs[1:]),
                      "krylov_iterations": sum(sum(r["krylov_iters"]) + r.get("failed_krylov_iters", 0)
                                               for r in recs[1:]),
                      "secant_fallbacks": sum(r["predictor"].startswith("custom->") for r in recs),
                      "failed": sum(r["status"] != 0 for r in recs), "reached_mu": recs[-1]["mu"]}
        if pred is not None:
            runs[name]["starts"] = pred.used
            ratio = [rn / rs for rs, rn in pred.residuals if rs > 0 and np.isfinite(rn)]
            runs[name]["start_residual_ratio_median"] = float(np.median(ratio)) if ratio else None
        log(f"[bench] {name}: {runs[name]}")
    base_run = runs["fp64_secant"]
    mixed = runs["fp32_learned_always_deflated"]
    best_learned = min((runs["fp64_learned"], runs["fp64_learned_always"]), key=lambda r: (r["failed"], r["seconds"]))
    best_name = min((k for k in runs if k != "fp64_secant" and runs[k]["failed"] == 0),
                    key=lambda k: runs[k]["seconds"])
    best = runs[best_name]
    out = {
        "metric": "continuation speedup over the plain FP64 secant path (learned start, deflation, precision)",
        "value": base_run["seconds"] / best["seconds"], "unit": "x", "n_gpus": 1, "steps": 100, "warmup": 0,
        "best_variant": best_name,
        "ms_per_step": 1e3 * best["seconds"] / max(1, best["steps"]), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (outer) / f32 (V-cycle) / bf16 (U-Net, f32 accumulation)",
        "speedups": {"learned_vs_secant_fp64": base_run["seconds"] / best_learned["seconds"],
                     "deflated_vs_plain_fp64_secant": base_run["seconds"] / runs["fp64_secant_deflated"]["seconds"],
                     "fp32_vs_fp64_deflated_secant": runs["fp64_secant_deflated"]["seconds"]
                     / runs["fp32_secant_deflated"]["seconds"],
                     "mixed_learned_deflated_vs_plain_fp64": base_run["seconds"] / mixed["seconds"],
                     "mixed_learned_deflated_reorth_vs_plain_fp64":
                         base_run["seconds"] / runs["fp32_learned_always_deflated_reorth"]["seconds"]},
        "data": "synthetic: continuation of psi = 1 from mu = 0 on a uniform grid; training states from a seeded sweep",
        "config": {"workload": "2D 513x513 grid, side 8, mu 0 -> 2 in steps of 0.02 (Newton to 1e-10); U-Net 4 levels, "
                               "32 base channels, BF16 / FP32 accumulation",
                   "training_states": len(states), "training_pairs": len(pairs), "epochs": args.epochs},
        "runs": runs, "roofline": unet_roof,
        "training": {"sweep_seconds": t_sweep, "train_seconds": t_train,
                                   "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]},
    }
    print(json.dumps(out), flush=True)


def bench_arclength(args):
    """Pseudo-arclength continuation (Sec. 4) on the continuation grid: 2D
    513^2, side 8, from psi = 1 at mu = 0, arclength steps of 0.05 in
    <(u, a), (v, b)> = <u, v>_R / |Omega| + a b, deflated Jacobian solves,
    FP64 and FP32 V-cycle; beside it natural continuation in steps of 0.02
    over the same mu range, which cannot pass the branch's fold."""
    import torch

    from paper_1204_5125_amd import continuation, glnk
    torch.cuda.set_device(0)
    N, side, ds = 513, 8.0, 0.05
    mesh = glnk.Mesh(2, (N, N), (side, side), mu=0.0)
    ones = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
    runs = {}
    # plain MINRES, and MINRES with the basis reorthogonalised (the paper's
    # remedy for the iteration peaks of its continuation runs, Sec. 4)
    for name, prec, reorth in (("fp64", glnk.GL_FP64, 0), ("fp32", glnk.GL_FP32, 0),
                               ("fp64_reorth", glnk.GL_FP64, REORTH), ("fp32_reorth", glnk.GL_FP32, REORTH)):
        def cb(rec, _):
            log(f"[bench] arclength {name}: mu {rec['mu']:.4f} ds {rec['ds']:.4f} newton {rec['newton_steps']} "
                f"krylov {sum(a + b for a, b in rec['krylov_iters'])}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, states = continuation.arclength_path(mesh, ones, 0.0, ds, args.arc_steps, precision=prec,
                                                   max_coarse=64, poll_every=16, callback=cb, reorth=reorth)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mus = [r["mu"] for r in recs]
        turns = sum(1 for a, b, c in zip(mus, mus[1:], mus[2:]) if (b - a) * (c - b) < 0)
        per_solve = [k for r in recs[1:] for pair in r["krylov_iters"] for k in pair]
        runs[name] = {"seconds": dt, "points": len(recs) - 1, "converged": sum(r["converged"] for r in recs[1:]),
                      "newton_steps": sum(r["newton_steps"] for r in recs[1:]),
                      "krylov_iterations": sum(a + b for r in recs[1:] for a, b in r["krylov_iters"]),
                      "krylov_max_per_solve": max(per_solve) if per_solve else 0,
                      "krylov_per_point": [sum(a + b for a, b in r["krylov_iters"]) for r in recs[1:]],
                      "mu_max": max(mus), "mu_final": mus[-1], "turning_points": turns}
        log(f"[bench] arclength {name}: {runs[name]}")
    mu_max = runs["fp64"]["mu_max"]
    mus = [0.02 * k for k in range(int(mu_max / 0.02) + 4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, _, _ = continuation.continuation_path(mesh, ones, mus, precision=glnk.GL_FP64, max_coarse=64,
                                                poll_every=16, deflate=True, krylov_max_iter=3000, max_newton=25)
    dt = time.perf_counter() - t0
    runs["natural_fp64"] = {"seconds": dt, "points": len(recs) - 1,
                            "newton_steps": sum(r["newton_steps"] for r in recs[1:]),
                            "newton_steps_per_point": [r["newton_steps"] for r in recs[1:]],
                            "mu": [r["mu"] for r in recs[1:]], "failed": sum(r["status"] != 0 for r in recs)}
    log(f"[bench] natural continuation to {mus[-1]:.2f}: {runs['natural_fp64']['newton_steps']} Newton steps")
    r64 = runs["fp64"]
    out = {
        "metric": "pseudo-arclength continuation points/s",
        "value": r64["points"] / r64["seconds"], "unit": "points/s", "n_gpus": 1, "steps": args.arc_steps,
        "warmup": 0, "ms_per_step": 1e3 * r64["seconds"] / max(1, r64["points"]), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (solver)",
        "data": "synthetic: continuation of psi = 1 from mu = 0 on a uniform grid",
        "config": {"workload": "2D 513x513 grid, side 8, pseudo-arclength steps of 0.05 from psi = 1 at mu = 0, "
                               "Newton to 1e-10, deflated MINRES to 1e-10 (two solves per Newton step)"},
        "runs": runs,
    }
    print(json.dumps(out), flush=True)


def bench_fig1(args):
    """Fig. 1 protocol: J(psi = 1) x = 1 from x = 0 on the square of side
    5 sqrt 2 with 1001^2 nodes (about the paper's 1000^2 unknowns), A_z with
    mu = 1; MINRES without preconditioner and with R_k, k = 1, 2, 5, 10, and
    R_inf (conjugate gradients with the V-cycle, fixed steps); iterations to
    1e-8, 1e-10, 1e-11, 1e-12, and the cost per iteration and per solve in
    units of one Jacobian application, measured."""
    import math

    import torch

    from paper_1204_5125_amd import glnk
    torch.cuda.set_device(0)
    N, side = 1001, 5.0 * math.sqrt(2.0)
    mesh = glnk.Mesh(2, (N, N), (side, side), mu=1.0)
    ones = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(ones)
    out = torch.empty_like(ones)
    for _ in range(3):
        glnk.gl_jacobian_apply(mesh, ones, ones, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        glnk.gl_jacobian_apply(mesh, ones, ones, out)
    e1.record()
    torch.cuda.synchronize()
    t_mv = e0.elapsed_time(e1) / 50 * 1e-3
    tols = (1e-8, 1e-10, 1e-11, 1e-12)
    paper = {"0": None, "1": [20, 26, 28, 30], "2": [14, 21, 25, 27], "5": [7, 13, 15, 18], "10": [7, 9, 9, 10]}
    rows = {}
    for k in (0, 1, 2, 5, 10, "inf"):
        pre = None
        if k != 0:
            pre = glnk.Precond(mesh, ones, cycles=0 if k == "inf" else k, max_coarse=64)
        counts, secs = [], []
        for tol in tols:
            glnk.gl_jacobian_solve(mesh, ones, pre, ones, x, rtol=tol, max_iter=500 if k == 0 else 200,
                                   poll_every=16, raise_on_fail=False)  # graph capture and warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, info = glnk.gl_jacobian_solve(mesh, ones, pre, ones, x, rtol=tol, max_iter=500 if k == 0 else 200,
                                              poll_every=16, raise_on_fail=False)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            counts.append(info["iterations"] if info["converged"] else None)
        it10 = counts[1]
        row = {"iterations": dict(zip(["1e-8", "1e-10", "1e-11", "1e-12"], counts)),
               "vcycles_per_iteration": pre.inner_steps() if pre is not None else 0,
               "seconds_to_1e-10": secs[1],
               "matvec_equiv_per_iteration": (secs[1] / it10 / t_mv) if it10 else None,
               "matvec_equiv_to_1e-10": secs[1] / t_mv,
               "paper_iterations": paper.get(str(k))}
        rows[str(k)] = row
        log(f"[bench] fig1 k={k}: {row}")
    best = min((r for r in rows.values() if r["iterations"]["1e-10"]), key=lambda r: r["seconds_to_1e-10"])
    out = {
        "metric": "Jacobian solve time to 1e-10 with the cheapest R_k (Fig. 1 protocol)",
        "value": best["seconds_to_1e-10"] * 1e3, "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best["seconds_to_1e-10"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic: psi = 1, b = 1, x0 = 0",
        "config": {"workload": "2D 1001x1001 grid (1,002,001 nodes), side 5 sqrt 2, A_z with mu = 1; MINRES "
                               "with R_k, k = 0 (none), 1, 2, 5, 10, inf"},
        "matvec_seconds": t_mv, "rows": rows,
        "cheapest_k": [k for k, r in rows.items() if r is best][0],
    }
    print(json.dumps(out), flush=True)


def bench_meshind(args):
    """Mesh independence of R_1 (Fig. 3 protocol): J(psi = 1) x = 1 from x = 0
    to rtol 1e-11 with one V-cycle per MINRES step, uniform field mu = 1 along
    z; 2D squares of side 10 with N = 33 ... 1025 nodes per axis, 3D cubes of
    side 10/sqrt(3) (circumradius 5) with N = 9 ... 129.  Reports the MINRES
    iterations per grid with the FP64 and the FP32 V-cycle; the cube in the
    dipole potential; and the triangle, disc, tetrahedron and ball of
    circumradius 5 as simplicial meshes (137 to 1.05 M nodes) in both
    potentials with R_1, R_inf and, up to 3000 nodes, no preconditioner."""
    import torch

    from paper_1204_5125_amd import glnk
    torch.cuda.set_device(0)
    rows = []
    grids = [(2, n, 10.0) for n in (33, 65, 129, 257, 513, 1025)] + \
            [(3, n, 10.0 / 3 ** 0.5) for n in (9, 17, 33, 65, 129)]
    t0 = time.perf_counter()
    for dim, n, side in grids:
        mesh = glnk.Mesh(dim, (n,) * dim, (side,) * dim, mu=1.0)
        ones = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
        x = torch.empty_like(ones)
        row = {"dim": dim, "N": n, "nodes": mesh.n}
        for name, prec in (("fp64", glnk.GL_FP64), ("fp32", glnk.GL_FP32)):
            pre = glnk.Precond(mesh, ones, precision=prec, max_coarse=MAX_COARSE)
            rc, info = glnk.gl_jacobian_solve(mesh, ones, pre, ones, x, rtol=1e-11, max_iter=4000, poll_every=8,
                                              raise_on_fail=False)
            row[name] = {"iterations": info["iterations"], "res_true": info["res_true"], "status": rc}
        row["levels"] = pre.info()["sizes"]
        log(f"[bench] meshind {row}")
        rows.append(row)
    # Fig. 3, cube in the dipole potential A_d (m = e_z at (0, 0, 6)), the
    # paper's grids N = 5 ... 40 and two finer ones; the paper's R_1 counts
    # for this panel are 6, 22, 29, 31, 31, 32, 32, 31
    dip_rows = []
    for n in (5, 10, 15, 20, 25, 30, 35, 40, 65, 129):
        mesh = glnk.Mesh(3, (n,) * 3, (10.0 / 3 ** 0.5,) * 3, mu=1.0, dipole=((0, 0, 1), (0, 0, 6)))
        ones = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
        x = torch.empty_like(ones)
        pre = glnk.Precond(mesh, ones, max_coarse=64)
        rc, info = glnk.gl_jacobian_solve(mesh, ones, pre, ones, x, rtol=1e-11, max_iter=4000, poll_every=8,
                                          raise_on_fail=False)
        dip_rows.append({"N": n, "nodes": mesh.n, "iterations": info["iterations"], "status": rc})
        log(f"[bench] meshind cube A_d {dip_rows[-1]}")
    # Fig. 3 protocol on the paper's other domains as simplicial meshes: the
    # triangle and the disc of circumradius 5 (A_d: m = e_z at (0, 0, 1)),
    # the tetrahedron and the ball (A_d at (0, 0, 6); tetrahedron k = 7 ... 55
    # and ball m = 4 ... 49 give about the paper's 2n = 406 ... 112580 and
    # 250 ... 273598), A_z and A_d, mu = 1: R_1, R_inf and (small meshes) no
    # preconditioner
    from paper_1204_5125_amd import meshes
    simp_rows = []
    sizes = {"tri": (16, 32, 64, 128, 256, 512, 1024, 1448), "circ": (8, 16, 32, 64, 128, 256, 512),
             "tet": (7, 15, 23, 31, 39, 47, 55, 80, 128), "ball": (4, 7, 15, 22, 29, 36, 43, 49, 64, 80)}
    for dom, ks in sizes.items():
        x0 = (0, 0, 6) if dom in ("tet", "ball") else (0, 0, 1)
        for k in ks:
            xy, tri = meshes.domain(dom, k)
            for pot, kw in (("Az", {}), ("Ad", {"dipole": ((0, 0, 1), x0)})):
                mesh = glnk.Mesh.simplicial(xy, tri, mu=1.0, **kw)
                ones = torch.ones(mesh.n, dtype=torch.complex128, device="cuda")
                x = torch.empty_like(ones)
                row = {"domain": dom, "potential": pot, "k": k, "nodes": mesh.n}
                for name, cyc in (("R1", 1), ("Rinf", 0)):
                    if cyc == 0 and mesh.n > 300000:
                        continue
                    pre = glnk.Precond(mesh, ones, cycles=cyc, max_coarse=64)
                    rc, info = glnk.gl_jacobian_solve(mesh, ones, pre, ones, x, rtol=1e-11, max_iter=4000,
                                                      poll_every=8, raise_on_fail=False)
                    row[name] = info["iterations"] if rc == 0 else None
                    if cyc == 1:
                        row["levels"] = pre.info()["sizes"]
                if mesh.n <= 3000:
                    rc, info = glnk.gl_jacobian_solve(mesh, ones, None, ones, x, rtol=1e-11, max_iter=3000,
                                                      poll_every=8, raise_on_fail=False)
                    row["unpreconditioned"] = info["iterations"] if rc == 0 else None
                log(f"[bench] meshind simplicial {row}")
                simp_rows.append(row)
    it2 = [r["fp64"]["iterations"] for r in rows if r["dim"] == 2]
    it3 = [r["fp64"]["iterations"] for r in rows if r["dim"] == 3]
    out = {
        "metric": "MINRES iterations to 1e-11 with R_1 against grid size (mesh independence)",
        "value": max(it2[1:]) / min(it2[1:]), "unit": "max/min iterations, 2D N >= 65",
        "n_gpus": 1, "steps": len(rows), "warmup": 0, "ms_per_step": 1e3 * (time.perf_counter() - t0) / len(rows),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64 / f32 (V-cycle)",
        "data": "synthetic: psi = 1, b = 1 on square and cube grids",
        "config": {"workload": "2D N = 33..1025 (side 10), 3D N = 9..129 (side 10/sqrt 3), mu 1 along z, "
                               "x0 = 0, rtol 1e-11, one V-cycle per step, max_coarse 512"},
        "iterations_2d_fp64": it2, "iterations_3d_fp64": it3, "grids": rows,
        "cube_dipole_fig3": {"iterations": [r["iterations"] for r in dip_rows], "N": [r["N"] for r in dip_rows],
                             "paper_R1": [6, 22, 29, 31, 31, 32, 32, 31]},
        "simplicial": simp_rows,
        "tet_fig3_paper": {"2n": [406, 3018, 9676, 22270, 42748, 71832, 112580],
                           "Az_R1": [20, 22, 22, 22, 22, 22, 22], "Az_Rinf": [20, 19, 19, 18, 18, 18, 18],
                           "Ad_R1": [26, 29, 27, 29, 27, 28, 28], "Ad_Rinf": [26, 25, 23, 23, 22, 22, 22],
                           "unpreconditioned_406": {"Az": 75, "Ad": 91}},
        "ball_fig3_paper": {"2n": [250, 1222, 8024, 24248, 54920, 104160, 176708, 273598],
                            "Az_R1": [3, 20, 19, 19, 19, 18, 18, 18], "Az_Rinf": [3, 18, 17, 16, 15, 14, 14, 14],
                            "Ad_R1": [6, 37, 34, 34, 32, 34, 32, 32], "Ad_Rinf": [6, 33, 29, 27, 27, 27, 27, 26],
                            "unpreconditioned": {"Az": [14, 70], "Ad": [15, 122]}},
    }
    print(json.dumps(out), flush=True)


def bench_cube(args):
    """Mixed precision in 3D: cube grid 129^3 (2,146,689 nodes), side 5, mu 0.6
    along (1,1,1)/sqrt(3), psi0 random phase (seed 0); 4 Newton steps with the
    FP32 V-cycle (FP64 outer iteration) and with the FP64 V-cycle.  Reports
    solves/s of both, the FP32 V-cycle output error against the FP64 V-cycle
    on the same input, and the first Newton update against the oracle's."""
    import numpy as np
    import torch

    from paper_1204_5125_amd import glnk, inputs
    torch.cuda.set_device(0)
    N, side, mu = (129, 129, 129), (5.0, 5.0, 5.0), 0.6
    bdir = tuple(np.ones(3) / np.sqrt(3.0))
    mesh = glnk.Mesh(3, N, side, mu=mu, b_dir=bdir)
    psi0 = torch.from_numpy(inputs.random_phase_state(mesh.n, seed=0)).cuda()
    # preconditioner outputs: FP32 against FP64 on the same input
    p64 = glnk.Precond(mesh, psi0, precision=glnk.GL_FP64, max_coarse=512)
    p32 = glnk.Precond(mesh, psi0, precision=glnk.GL_FP32, max_coarse=512)
    r = torch.from_numpy(inputs.random_complex(mesh.n, seed=1)).cuda()
    z64, z32 = torch.empty_like(r), torch.empty_like(r)
    p64.apply(r, z64)
    p32.apply(r, z32)
    torch.cuda.synchronize()
    prec_err = float(torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64))
    del p64, p32
    log(f"[bench] cube {N}: n = {mesh.n}; FP32 V-cycle output error {prec_err:.2e}")
    psi = torch.empty_like(psi0)
    out = {}
    first = {}
    from paper_1204_5125_amd import autotune
    tiles = {}
    for name, prec, reorth in [("fp32", glnk.GL_FP32, 0), ("fp64", glnk.GL_FP64, 0),
                               ("fp32_reorth", glnk.GL_FP32, REORTH), ("fp64_reorth", glnk.GL_FP64, REORTH)]:
        tname = name.split("_")[0]
        if tname not in tiles:
            tiles[tname] = autotune.tune(mesh, psi0, precision=prec, max_coarse=MAX_COARSE, cache=args.tile_cache,
                                         log=log)
        h = glnk.PrecondHandle(mesh)
        inner = RTOL if prec == glnk.GL_FP64 and reorth == 0 else 0.0
        kw = dict(krylov_rtol=RTOL, krylov_max_iter=8000, poll_every=16, precision=prec, inner_rtol=inner,
                  max_coarse=MAX_COARSE, precond=h, reorth=reorth)
        psi.copy_(psi0)
        glnk.gl_newton_solve(mesh, psi, fixed_steps=1, **kw)  # warm-up: hierarchy + graphs
        first[name] = psi.clone()
        glnk.gl_precond_set_tiles(h, *tiles[tname])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            psi.copy_(psi0)
            rc, info = glnk.gl_newton_solve(mesh, psi, fixed_steps=NEWTON_STEPS, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"value": NEWTON_STEPS * args.steps / dt, "unit": "solves/s",
                     "ms_per_step": 1e3 * dt / args.steps, "krylov_iters_per_solve": info["krylov_iters"],
                     "final_gl_residual": info["res"][-1]}
        log(f"[bench] cube {name}: {out[name]}")
        h.close()
    d32, d64 = first["fp32"] - psi0, first["fp64"] - psi0
    upd_err = float(torch.linalg.norm(d32 - d64) / torch.linalg.norm(d64))
    res = {
        "metric": "Jacobian solves/s at 2.1M nodes (3D), FP32 V-cycle vs FP64",
        "value": out["fp32_reorth"]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": out["fp32_reorth"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (outer) / f32 (V-cycle)",
        "data": "synthetic: seeded random-phase psi0 on a uniform cube grid",
        "config": {"workload": "3D 129^3 grid (2,146,689 nodes), side 5, mu 0.6 along (1,1,1)/sqrt3; 4 Newton "
                               "steps from psi0 = 0.9 exp(i theta), seed 0, MINRES + R_1 to rtol 1e-10; value: "
                               f"FP32 V-cycle, Krylov basis reorthogonalised (at most {REORTH})",
                   "nodes": mesh.n, "amg_max_coarse": MAX_COARSE,
                   "tiles": {k: list(v) for k, v in tiles.items()}},
        "fp32_precond_plain": out["fp32"], "fp64_precond": out["fp64"],
        "fp32_precond_reorth": out["fp32_reorth"], "fp64_precond_reorth": out["fp64_reorth"],
        "fp32_vcycle_output_rel_error": prec_err,
        "first_newton_update_fp32_vs_fp64_rel_error": upd_err,
    }
    if not args.no_cpu_baseline:
        import oracle
        log("[bench] cube: oracle, first Newton step")
        mo = oracle.Mesh(3, N, side, mu=mu, bdir=np.asarray(bdir))
        t0 = time.perf_counter()
        pso, io = oracle.newton(mo, inputs.random_phase_state(mo.n, seed=0), fixed_steps=1, krylov_rtol=RTOL,
                                krylov_max_iter=4000, max_coarse=MAX_COARSE)
        dto = time.perf_counter() - t0
        do = pso - inputs.random_phase_state(mo.n, seed=0)
        dg = d32.cpu().numpy()
        res["first_newton_update_fp32_vs_oracle_rel_error"] = float(np.linalg.norm(dg - do) / np.linalg.norm(do))
        res["cpu_baseline"] = {"value": 1.0 / dto, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"first Newton step ({io['krylov_iters'][0]} MINRES iterations) of the "
                                         f"same workload: {dto:.1f} s, serial C (one host core)"}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["jacobian", "batch", "continuation", "cube", "meshind", "arclength",
                                           "fig1"],
                    default="jacobian",
                    help="jacobian: the 1M-node Jacobian solves (headline); batch: batched continuation; "
                         "continuation: learned vs secant predictor; cube: 3D 129^3 mixed precision; "
                         "meshind: R_1 iteration counts against grid size")
    ap.add_argument("--epochs", type=int, default=12,
                    help="continuation: training epochs of the U-Net (12 take about 34 s at 513^2)")
    ap.add_argument("--arc-steps", type=int, default=60)
    ap.add_argument("--batch-max-coarse", type=int, default=64)
    ap.add_argument("--batch-plain", action="store_true",
                    help="batch: Newton without deflation of the gauge mode")
    ap.add_argument("--batch-fp64", action="store_true", help="batch: FP64 V-cycle")
    ap.add_argument("--batch-reorth", action="store_true",
                    help="batch: MINRES with the Krylov basis stored and reorthogonalised")
    ap.add_argument("--tile-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "glnk_tiles.json"))
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fixed-tiles", action="store_true",
                    help="jacobian: skip the autotuner and use the tiles it picks on MI355X for this grid "
                         "(lane_shift 0, bottom_rows 64, dense_rows 4096; level 0 in 16 x 16 LDS tiles with "
                         "the FP32 V-cycle, one dispatch per pass with FP64), so that a profiled run times "
                         "the configuration of an unprofiled one")
    ap.add_argument("--profile-kernel", type=int, default=8,
                    help="internal kernel id for the roofline (see gl_profile_start)")
    ap.add_argument("--one-pass", action="store_true",
                    help="for hardware-counter runs: one Newton step of the headline workload with the "
                         "FP32 V-cycle (tiles lane_shift 0, bottom_rows 64, dense_rows 4096), then a 256 MiB elementwise "
                         "copy whose bytes calibrate the counters; prints nothing")
    ap.add_argument("--one-pass-l0-tiled", type=int, default=0, choices=[0, 1, 2, 3],
                    help="with --one-pass: level 0 in LDS tiles of this shape (gl_tiles.l0_tiled)")
    ap.add_argument("--one-pass-reorth", action="store_true",
                    help="with --one-pass: two Newton steps with the Krylov basis reorthogonalised")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)

    if args.one_pass:
        one_pass(args.one_pass_l0_tiled, REORTH if args.one_pass_reorth else 0)
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "continuation":
        bench_continuation(args)
        return
    if args.workload == "cube":
        bench_cube(args)
        return
    if args.workload == "meshind":
        bench_meshind(args)
        return
    if args.workload == "arclength":
        bench_arclength(args)
        return
    if args.workload == "fig1":
        bench_fig1(args)
        return

    import torch

    from paper_1204_5125_amd import glnk, inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mesh = glnk.Mesh(2, N_AXIS, SIDE, mu=MU)
    psi0 = torch.from_numpy(inputs.random_phase_state(mesh.n, seed=0)).cuda()
    psi = torch.empty_like(psi0)
    h32, h64 = glnk.PrecondHandle(mesh), glnk.PrecondHandle(mesh)

    from paper_1204_5125_amd import autotune
    tiles = {}
    for name, prec in (("fp32", glnk.GL_FP32), ("fp64", glnk.GL_FP64)):
        if args.fixed_tiles:
            tiles[name] = FIXED_TILES[name]
        else:
            tiles[name] = autotune.tune(mesh, psi0, precision=prec, max_coarse=MAX_COARSE, cache=args.tile_cache,
                                        log=log)
        log(f"[bench] tiles {name}: lane_shift {tiles[name][0]}, bottom_rows {tiles[name][1]}, "
            f"dense_rows {tiles[name][2]}")
    log(f"[bench] grid {N_AXIS} n={mesh.n}; warm-up {args.warmup} step(s)")
    run_steps(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, 1)
    run_steps(glnk, torch, mesh, psi0, psi, h64, glnk.GL_FP64, 1)
    glnk.gl_precond_set_tiles(h32, *tiles["fp32"])
    glnk.gl_precond_set_tiles(h64, *tiles["fp64"])
    if args.warmup > 1:
        run_steps(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, args.warmup - 1)
        run_steps(glnk, torch, mesh, psi0, psi, h64, glnk.GL_FP64, args.warmup - 1)

    log(f"[bench] timing {args.steps} step(s), FP32 preconditioner")
    t32, info32 = timed(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, args.steps)
    final_res32 = info32[-1]["res"][-1]
    log(f"[bench] FP32: {t32:.3f} s, krylov iterations {info32[-1]['krylov_iters']}")
    log(f"[bench] timing {args.steps} step(s), FP64 preconditioner")
    t64, info64 = timed(glnk, torch, mesh, psi0, psi, h64, glnk.GL_FP64, args.steps)
    log(f"[bench] FP64: {t64:.3f} s, krylov iterations {info64[-1]['krylov_iters']}")
    log(f"[bench] timing {args.steps} step(s), FP32 preconditioner below relative residual {RELAX}")
    run_steps(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, 1, RELAX)
    tr, infor = timed(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, args.steps, RELAX)
    log(f"[bench] FP32 relaxed: {tr:.3f} s, krylov iterations {infor[-1]['krylov_iters']}")
    # MINRES with the basis stored and reorthogonalised (Sec. 4's remedy for
    # the loss of orthogonality), both V-cycle precisions
    reo = {}
    for name, prec, h in (("fp32", glnk.GL_FP32, h32), ("fp64", glnk.GL_FP64, h64)):
        run_steps(glnk, torch, mesh, psi0, psi, h, prec, 1, reorth=REORTH)
        t, inf = timed(glnk, torch, mesh, psi0, psi, h, prec, args.steps, reorth=REORTH)
        reo[name] = (t, inf)
        log(f"[bench] {name.upper()} reorthogonalised: {t:.3f} s, krylov iterations {inf[-1]['krylov_iters']}")

    solves = NEWTON_STEPS * args.steps
    # the headline: the FP32 V-cycle in MINRES with the basis reorthogonalised
    # (the library's FP32 mode for these indefinite solves; plain FP32 beside)
    t_head, info_head = reo["fp32"]
    value = solves / t_head

    # roofline: an identical pass per kernel class with its launches timed by
    # HIP events on the stream they run on.  The coarse-level Gauss-Seidel
    # sweeps take the most GPU time (latency-bound small launches); the
    # level-0 sweeps move the most bytes.
    # level 0 of the FP32 V-cycle: one dispatch per pass, or LDS tiles of
    # shape l0_tiled (the same profile id; the counters are per form)
    l0_form = tiles["fp32"][3] if len(tiles["fp32"]) > 3 else 0
    names = dict(KERNEL_NAMES)
    if l0_form:
        names[2] = L0_TILED_NAME

    def profile(kid):
        log(f"[bench] profiling kernel {kid} ({names.get(kid)})")
        glnk.gl_profile_start(kid)
        run_steps(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, 1)
        ms, nbytes, launches = glnk.gl_profile_stop()
        avg_ms = ms / max(1, launches)
        achieved = (nbytes / max(1, launches)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0
        key = f"{kid}t{l0_form}" if kid == 2 and l0_form else kid
        traffic = TRAFFIC.get(key) if TRAFFIC["csrc_sha256"] == csrc_fingerprint() else None
        return {"bound": "hbm", "kernel": names.get(kid), "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_unit": "bytes per launch", "avg_launch_us": 1e3 * avg_ms,
                "launches": launches, "bytes_per_launch": nbytes / max(1, launches),
                "kernel_ms_per_step": ms}
    roof = profile(args.profile_kernel)
    roof_l0 = profile(2) if args.profile_kernel != 2 else roof
    # whole iteration: the algorithmic bytes of every profiled kernel class in
    # one pass of the workload, plus the coarse residuals, transfers and the
    # dense product from the hierarchy, per MINRES iteration, over the timed
    # run's time per iteration
    by_class = {}
    for kid in sorted(KERNEL_NAMES):
        glnk.gl_profile_start(kid)
        infos = run_steps(glnk, torch, mesh, psi0, psi, h32, glnk.GL_FP32, 1)
        _, nbytes, _ = glnk.gl_profile_stop()
        by_class[names[kid]] = nbytes / max(1, sum(infos[-1]["krylov_iters"]))
    rest = iteration_bytes(glnk, h32, glnk.GL_FP32)
    bytes_iter = sum(by_class.values()) + rest
    t_iter32 = t32 / args.steps / sum(info32[-1]["krylov_iters"])
    roof_iter = {"bound": "hbm", "kernel": "one plain MINRES iteration, FP32 V-cycle (all kernels)",
                 "achieved": bytes_iter / t_iter32 / 1e9,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bytes_iter / t_iter32 / 1e9 / HBM_PEAK_GBS,
                 "bytes_per_iteration": bytes_iter, "us_per_iteration": t_iter32 * 1e6,
                 "bytes_by_kernel_class": by_class, "bytes_coarse_residual_transfer_dense": rest,
                 "traffic": None}
    # the headline leg: the same kernels per iteration plus the basis traffic
    # of the reorthogonalisation, per node 4 (j + 1) bytes read by the dots
    # (BF16 Z) and 8 (j + 1) by the update (FP32 V) in iteration j, 28 bytes
    # written (Z in FP64 and BF16, V in FP32), and 16 read per stored vector
    # by x = Z y at the end of each solve
    its = info_head[-1]["krylov_iters"]
    basis = sum(sum(12.0 * (j + 1) + 28.0 for j in range(k)) + 16.0 * k for k in its) * mesh.n
    bytes_iter_r = bytes_iter + basis / sum(its)
    t_iter_r = t_head / args.steps / sum(its)
    roof_iter_r = {"bound": "hbm", "kernel": "one reorthogonalised MINRES iteration, FP32 V-cycle (all kernels)",
                   "achieved": bytes_iter_r / t_iter_r / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": bytes_iter_r / t_iter_r / 1e9 / HBM_PEAK_GBS, "bytes_per_iteration": bytes_iter_r,
                   "basis_bytes_per_iteration": basis / sum(its), "us_per_iteration": t_iter_r * 1e6,
                   "traffic": None}
    # the peak measured two ways: vendor 8 TB/s, and a plain copy of the size
    # of one level-0 FP64 vector set (256 MiB in, 256 MiB out)
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * COPY_BYTES * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    for r in (roof, roof_l0):
        r["copy_peak_gbs"] = copy_gbs
        r["frac_of_copy"] = r["achieved"] / copy_gbs
    del a, c

    iters32 = info32[-1]["krylov_iters"]
    iters64 = info64[-1]["krylov_iters"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_head / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (outer) / f32 (V-cycle)",
        "data": "synthetic: seeded random-phase psi0 on a uniform grid",
        "config": {"workload": "2D 1025x1025 grid (1,050,625 nodes), side 10, mu 1.0 along z; "
                               "4 Newton steps from psi0 = 0.9 exp(i theta), seed 0, each one "
                               "Jacobian solve by MINRES + R_1 (SA-AMG V-cycle) to rtol 1e-10 on the "
                               "true residual",
                   "nodes": mesh.n, "newton_steps": NEWTON_STEPS, "precond": "fp32",
                   "krylov": f"MINRES, Krylov basis stored and reorthogonalised (at most {REORTH})",
                   "amg_max_coarse": MAX_COARSE, "tiles": {k: list(v) for k, v in tiles.items()}},
        "krylov_iters_per_solve": info_head[-1]["krylov_iters"],
        "final_gl_residual": info_head[-1]["res"][-1],
        "ms_per_iteration": 1e3 * t_head / args.steps / sum(info_head[-1]["krylov_iters"]),
        "fp32_precond_plain": {"value": solves / t32, "unit": "solves/s", "ms_per_step": 1e3 * t32 / args.steps,
                               "krylov_iters_per_solve": iters32, "final_gl_residual": final_res32,
                               "ms_per_iteration": 1e3 * t32 / args.steps / sum(iters32)},
        "fp64_precond": {"value": solves / t64, "unit": "solves/s", "ms_per_step": 1e3 * t64 / args.steps,
                         "krylov_iters_per_solve": iters64,
                         "ms_per_iteration": 1e3 * t64 / args.steps / sum(iters64)},
        "fp32_precond_relaxed": {"value": solves / tr, "unit": "solves/s", "relax_rtol": RELAX,
                                 "ms_per_step": 1e3 * tr / args.steps,
                                 "krylov_iters_per_solve": infor[-1]["krylov_iters"],
                                 "final_gl_residual": infor[-1]["res"][-1]},
        **{f"{name}_precond_reorth": {"value": solves / t, "unit": "solves/s", "reorth_basis": REORTH,
                                      "ms_per_step": 1e3 * t / args.steps,
                                      "krylov_iters_per_solve": inf[-1]["krylov_iters"],
                                      "ms_per_iteration": 1e3 * t / args.steps / sum(inf[-1]["krylov_iters"]),
                                      "final_gl_residual": inf[-1]["res"][-1]}
           for name, (t, inf) in reo.items() if name != "fp32"},
        "roofline": roof,
        "roofline_level0": roof_l0,
        "roofline_iteration": roof_iter,
        "roofline_iteration_reorth": roof_iter_r,
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, one full solve of the workload's second Newton system)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
