"""Benchmark of the tree ray-shooting hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the configuration the headline metric is quoted on): 1e6 smoothed
NFW particles (c = 5, truncated at r200 = 1, equal masses summing to 1,
smoothing length = distance to the 32nd neighbour, q = 3) and the 2048 x 2048
cell-centred ray grid over [-0.5, 0.5]^2; theta = 0.3, multipole order 8, leaf
size 16.  Synthetic, seeded inputs (no dataset exists for this workload).

A step is one pass of the hot path over that batch: build the tree from the
particles (bounding square, Morton sort, boxes, lists, FP64 moments) and shoot
every ray (ray sort + walk), inputs already in HBM.  `value` = rays / step time.

Printed as one JSON line, with:
  roofline     -- the walk kernel alone, timed with HIP events on the stream it
                  runs on; algorithmic FLOPs from its own per-ray interaction
                  counts times fixed per-interaction weights;
  fwd_adjoint  -- the same particles and grid with the fitting loss: build +
                  alpha walk + adjoint walk, and the adjoint call's roofline;
  cpu_baseline -- the FP64 brute-force oracle on a bounded ray sample on the
                  host cores, on all threads and on one (also yields the
                  sample's error vs FP64), and the FP64 reference tree;
  extras       -- build time, walk-only rate, plain GPU direct sum rates, and
                  the fitting (forward + adjoint), refinement and 64-lens
                  workloads (--no-extras leaves these out).

`roofline.traffic` is the walk's HBM bytes per launch from the committed
rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the counters'
reading for a plain 1 GiB device copy, which every run performs last); it is
null when the walk's sources differ from those the counters were taken on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s (α,κ,γ) at 1e6 particles, rel err ≤1e-4 vs FP64; fwd+adjoint rays/s"
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (dense)
THETA, ORDER, LEAF = 0.3, 8, 16

# algorithmic FLOPs per interaction (FMA = 2): opening test, accepted box at
# order p, leaf particle, big-particle correction
def flops_per_ray(counts: np.ndarray, p: int) -> np.ndarray:
    return 5.0 * counts[:, 0] + (20.0 + 16.0 * p) * counts[:, 1] + 22.0 * counts[:, 2] + 60.0 * counts[:, 3]


# algorithmic FLOPs per interaction of the adjoint walk (FMA = 2): opening
# test; accepted box at order p (1/w and t = r_cm / w: 7, g v: 6, g v t^k for
# k <= p + 1: 6 (p + 1), one add per box-adjoint word per ray for the sum over
# the rays: 2 p + 4); leaf particle (point-mass gradient of alpha and its four
# FP64 sums); big-particle correction (profile minus point gradient)
def adjoint_flops_per_ray(counts: np.ndarray, p: int) -> np.ndarray:
    return 5.0 * counts[:, 0] + (23.0 + 8.0 * p) * counts[:, 1] + 38.0 * counts[:, 2] + 90.0 * counts[:, 3]


WALK_SOURCES = ["walk.hip", "walk.hpp", "eval.hpp", "common.hpp"]
HBM_PROFILE = os.path.join(ROOT, "profiles", "k_walk_nfw1e6_grid2048_hbm.txt")


def walk_sources_sha256() -> str:
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, "paper_1312_1128_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per walk launch from the committed counter summary, or None
    when there is none or the walk has changed since it was taken."""
    try:
        with open(HBM_PROFILE) as fh:
            kv = dict(l.split(":", 1) for l in fh.read().splitlines() if ":" in l and not l.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("walk_sources_sha256") != walk_sources_sha256():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SQ_PROFILE = os.path.join(ROOT, "profiles", "k_walk_nfw1e6_grid2048_sq.txt")


def issued_valu(flop: float) -> dict:
    """Issued VALU lane-operations per walk launch (wavefront instructions x 64,
    masked lanes included) from the committed counter summary, and the
    algorithmic FLOPs over them (an FMA counts 2 FLOPs and one lane-operation);
    empty when there is no summary for the current walk sources."""
    try:
        with open(SQ_PROFILE) as fh:
            kv = dict(l.split(":", 1) for l in fh.read().splitlines() if ":" in l and not l.startswith(" "))
    except OSError:
        return {}
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("walk_sources_sha256") != walk_sources_sha256():
        return {}
    try:
        ops = 64.0 * float(kv["valu_insts_per_launch"])
    except (KeyError, ValueError):
        return {}
    return {"issued_valu_lane_ops_per_launch": ops, "algorithmic_flop_over_issued_lane_ops": flop / ops}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads() -> int:
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(aff, int(env))) if env and env.isdigit() else aff


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads (direct sum, fitting, refinement, 64 lenses)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_1312_1128_amd as g
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    lens = synth.nfw_halo(1_000_000, synth.BASE_SEED + 2)
    rx_t, ry_t = synth.ray_grid_tiled(2048)  # grid stored in 8x8-tile order
    R = rx_t.size
    log(f"inputs generated in {time.time() - t0:.1f}s: n={lens.n} rays={R}")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    x, y, m, s = d(lens.x), d(lens.y), d(lens.m), d(lens.s)
    rx, ry = d(rx_t), d(ry_t)
    stream = torch.cuda.current_stream()

    tree = g.Tree()
    out = {k: torch.empty(R, dtype=torch.float32, device=dev) for k in ["a1", "a2", "kappa", "g1", "g2"]}
    ws = torch.empty(g.workspace_bytes(R), dtype=torch.uint8, device=dev)

    # one step: the tree build on the current stream and, on a second stream at
    # the same time, the ray staging (it reads only the rays; it waits for the
    # previous step's walk, which read the same workspace); then the walk
    main, side = torch.cuda.current_stream(), torch.cuda.Stream()

    def step():
        side.wait_stream(main)
        g.stage_rays(rx, ry, ws, stream=side)
        staged = torch.cuda.Event()
        staged.record(side)
        tree.build(x, y, m, s, theta=THETA, q=lens.q, leaf_size=LEAF, order=ORDER)
        main.wait_event(staged)
        g.shoot(tree, rx, ry, out=out, workspace=ws, staged=True)

    def step_one_stream():
        tree.build(x, y, m, s, theta=THETA, q=lens.q, leaf_size=LEAF, order=ORDER)
        g.shoot(tree, rx, ry, out=out, workspace=ws)

    def timed_steps(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    el1 = timed_steps(step_one_stream)
    el = timed_steps(step)
    ms_step = 1e3 * el / args.steps
    ms_step_one_stream = 1e3 * el1 / args.steps
    value = R * args.steps / el
    log(f"step (build + shoot, ray staging beside the build): {ms_step:.3f} ms -> {value:.4e} rays/s "
        f"(all on one stream: {ms_step_one_stream:.3f} ms)")

    # build alone
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tb = []
    for _ in range(5):
        t = time.perf_counter()
        tree.build(x, y, m, s, theta=THETA, q=lens.q, leaf_size=LEAF, order=ORDER)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
    build_ms = 1e3 * float(np.median(tb))
    info = tree.info()

    # walk kernel alone: rays already in tile order, so the launch is k_walk only
    nrep = 10
    ev0.record(stream)
    for _ in range(nrep):
        g.shoot(tree, rx, ry, out=out, ordered=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    walk_ms = ev0.elapsed_time(ev1) / nrep
    # per-ray interaction counts (separate launch, outside every timed region)
    cnt = g.shoot(tree, rx, ry, counts=True, ordered=True)["counts"].cpu().numpy().astype(np.float64)
    flop = float(flops_per_ray(cnt, ORDER).sum())
    achieved = flop / (walk_ms * 1e-3) / 1e12
    # rays in tile order: each wavefront walks 64 consecutive rays, which carry its counts
    lane_use = {"accepted_boxes": float(cnt[:, 1].sum() / cnt[:, 5].sum()),
                "leaf_particles": float(cnt[:, 2].sum() / cnt[:, 6].sum()),
                "list_candidates": float(cnt[:, 3].sum() / cnt[:, 7].sum())}
    scan_flop = 5.0 * float(cnt[:, 4].sum())  # list-entry distance checks: search overhead, not algorithmic
    log(f"lane use: {lane_use}; list entries tested per ray {cnt[:, 4].mean():.0f} "
        f"(search overhead {scan_flop:.3e} FLOP per launch)")
    log(f"walk: {walk_ms:.3f} ms, {flop:.3e} algorithmic FLOP -> {achieved:.2f} TFLOP/s "
        f"({achieved / PEAK_FP32_TFLOPS:.3f} of FP32 peak); counts/ray {cnt.mean(0)}")

    # the tree's error over every ray of the grid, against the library's FP64
    # direct sum (itself held to 1e-10 of the CPU oracle by the tests)
    g.shoot(tree, rx, ry, out=out, workspace=ws)
    full = g.shoot_direct(x, y, m, s, lens.q, rx, ry, fp64=True)
    ref_a = torch.stack([full["a1"], full["a2"]], 1)
    ref_g = torch.stack([full["g1"], full["g2"]], 1)
    e_a = (torch.stack([out["a1"], out["a2"]], 1).double() - ref_a).norm(dim=1) / ref_a.norm(dim=1)
    e_g = (torch.stack([out["g1"], out["g2"]], 1).double() - ref_g).norm(dim=1) / ref_g.norm(dim=1)
    e_k = (out["kappa"].double() - full["kappa"]).abs() / full["kappa"].abs()
    full_err = {"rays": R, "alpha_max": float(e_a.max()), "kappa_max": float(e_k.max()),
                "gamma_max": float(e_g.max()), "alpha_median": float(e_a.median()),
                "gamma_median": float(e_g.median())}
    del ref_a, ref_g, e_a, e_g, e_k
    log(f"tree vs GPU FP64 direct over all {R} rays: max rel err alpha {full_err['alpha_max']:.2e} "
        f"kappa {full_err['kappa_max']:.2e} gamma {full_err['gamma_max']:.2e}")

    # forward + adjoint at the headline size: the fitting loss L = sum |x - alpha - beta*|^2
    # over the 2048^2 grid, beta* = x - alpha_true + N(0, 1e-4) per component (alpha_true:
    # the FP64 direct sum above); step = build + alpha walk + dL/dalpha + adjoint walk
    # (dL/d(m, x, y, s) of the 1e6 particles, FP64)
    noise = synth.rng(synth.BASE_SEED + 14).normal(0.0, 1e-4, size=(2, R))
    bx = rx - full["a1"] + torch.from_numpy(noise[0]).to(dev)
    by = ry - full["a2"] + torch.from_numpy(noise[1]).to(dev)
    del full, noise
    outa = {k: torch.empty(R, dtype=torch.float32, device=dev) for k in ["a1", "a2"]}
    grads = [torch.zeros(lens.n, dtype=torch.float64, device=dev) for _ in range(4)]
    ws_adj = torch.empty(g.adjoint_workspace_bytes(tree, R), dtype=torch.uint8, device=dev)

    def step_fa():
        # the rays are staged once, on the second stream beside the build, into the
        # adjoint's workspace, whose start both walks read
        side.wait_stream(main)
        g.stage_rays(rx, ry, ws_adj, stream=side)
        staged = torch.cuda.Event()
        staged.record(side)
        tree.build(x, y, m, s, theta=THETA, q=lens.q, leaf_size=LEAF, order=ORDER)
        main.wait_event(staged)
        g.shoot(tree, rx, ry, out=outa, workspace=ws_adj, alpha_only=True, staged=True)
        ga1 = (-2.0 * (rx - outa["a1"] - bx)).float()
        ga2 = (-2.0 * (ry - outa["a2"] - by)).float()
        for t_ in grads:
            t_.zero_()
        g.shoot_adjoint(tree, rx, ry, ga1, ga2, *grads, workspace=ws_adj, staged=True)
        return ga1, ga2

    for _ in range(args.warmup):
        step_fa()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        ga1, ga2 = step_fa()
    torch.cuda.synchronize()
    fa_ms = 1e3 * (time.perf_counter() - t) / args.steps
    # the adjoint call alone on ordered rays (box-adjoint clear + adjoint walk + push-down)
    nrep = 5
    ev0.record(stream)
    for _ in range(nrep):
        g.shoot_adjoint(tree, rx, ry, ga1, ga2, *grads, workspace=ws_adj, ordered=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    adj_ms = ev0.elapsed_time(ev1) / nrep
    adj_flop = float(adjoint_flops_per_ray(cnt, ORDER).sum())
    adj_tf = adj_flop / (adj_ms * 1e-3) / 1e12
    log(f"fwd+adjoint (1e6 particles, {R} rays): {fa_ms:.3f} ms -> {R / (fa_ms * 1e-3):.4e} rays/s; adjoint call "
        f"{adj_ms:.3f} ms, {adj_flop:.3e} algorithmic FLOP -> {adj_tf:.2f} TFLOP/s ({adj_tf / PEAK_FP32_TFLOPS:.3f})")
    fwd_adjoint = {"value": R / (fa_ms * 1e-3), "unit": "rays/s", "ms_per_step": fa_ms,
                   "workload": "nfw_1e6_particles_grid2048, L = sum |x - alpha - beta*|^2, "
                               "beta* = x - alpha_true + N(0, 1e-4)",
                   "step": "build_tree + shoot (alpha) + dL/dalpha + shoot_adjoint -> dL/d(m, x, y, s); the rays are "
                           "staged once, on a second stream beside the build",
                   "roofline": {"bound": "alu", "kernel": "glm_shoot_adjoint (k_fill_zero + k_adjoint_walk + "
                                                          "k_pushdown)",
                                "achieved": adj_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                "frac": adj_tf / PEAK_FP32_TFLOPS, "kernel_ms": adj_ms, "flop_per_launch": adj_flop}}
    del grads, ws_adj, outa, bx, by, ga1, ga2

    extras = {}
    if not args.no_extras:
        # plain GPU direct sum on a slice of the rays
        nd = 262144
        res = {}
        for fp64 in (False, True):
            g.shoot_direct(x, y, m, s, lens.q, rx[:256], ry[:256], fp64=fp64)
            torch.cuda.synchronize()
            t = time.perf_counter()
            g.shoot_direct(x, y, m, s, lens.q, rx[:nd], ry[:nd], fp64=fp64)
            torch.cuda.synchronize()
            res[fp64] = nd / (time.perf_counter() - t)
        log(f"direct sum: fp32 {res[False]:.3e} rays/s, fp64 {res[True]:.3e} rays/s")

        # deflection + potential + time delay of the headline grid in one walk
        pot = g.shoot_potential(tree, rx, ry, ordered=True, workspace=ws)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(3):
            pot = g.shoot_potential(tree, rx, ry, ordered=True, workspace=ws)
        ev1.record(stream)
        torch.cuda.synchronize()
        pot_ms = ev0.elapsed_time(ev1) / 3
        log(f"alpha + potential + time delay walk: {pot_ms:.3f} ms -> {R / (pot_ms * 1e-3):.4e} rays/s")
        del pot

        # smoothing lengths of the 1e6 particles on the GPU (tree of the positions + k = 32 walk)
        g.smoothing_lengths(x, y, k=32)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            s_gpu = g.smoothing_lengths(x, y, k=32)
        torch.cuda.synchronize()
        knn_ms = 1e3 * (time.perf_counter() - t) / 3
        knn_diff = float(((s_gpu - s).abs() / s).max())
        log(f"smoothing lengths (k = 32, 1e6 particles): {knn_ms:.3f} ms; max rel diff vs the inputs' host k-d tree "
            f"{knn_diff:.1e}")
        # the same from raw positions on the bounding-box hierarchy: 2D, 3D (the positions
        # before projection), and two species (the halo plus 1e5 stars around (0.25, 0))
        x3d, y3d, z3d = (d(a) for a in synth.nfw_3d(1_000_000, synth.BASE_SEED + 2))
        stars_b = synth.star_patch(100_000, synth.BASE_SEED + 20)
        xs2, ys2 = torch.cat([x, d(stars_b.x)]), torch.cat([y, d(stars_b.y)])
        sp2 = torch.cat([torch.zeros(lens.n, dtype=torch.int32), torch.ones(100_000, dtype=torch.int32)]).to(dev)
        knn_pos = {}
        for name, args_k in (("2d", (x, y, None, None)), ("3d", (x3d, y3d, z3d, None)),
                             ("2d_two_species", (xs2, ys2, None, sp2))):
            wsk = torch.empty(max(1, g.knn_workspace_bytes(args_k[0].numel(), args_k[3] is not None)),
                              dtype=torch.uint8, device=dev)
            g.knn(args_k[0], args_k[1], 32, z=args_k[2], species=args_k[3], workspace=wsk)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                sk = g.knn(args_k[0], args_k[1], 32, z=args_k[2], species=args_k[3], workspace=wsk)
            torch.cuda.synchronize()
            knn_pos[name] = 1e3 * (time.perf_counter() - t) / 3
            if name == "2d":
                knn_pos["2d_equals_quadtree"] = bool(torch.equal(sk, s_gpu))
        del x3d, y3d, z3d, xs2, ys2, sp2, wsk, sk
        log(f"smoothing lengths from positions (k = 32): 2D {knn_pos['2d']:.2f} ms (same as the quad-tree: "
            f"{knn_pos['2d_equals_quadtree']}), 3D {knn_pos['3d']:.2f} ms, 2D with two species (1.1e6) "
            f"{knn_pos['2d_two_species']:.2f} ms")

        # forward + adjoint on the lens-fitting workload: 1e5 particles, 1e5 rays,
        # L = sum |x - alpha - beta*|^2 (step = build + alpha walk + adjoint walk)
        lens5 = synth.nfw_halo(100_000, synth.BASE_SEED + 5)
        r5x, r5y = synth.uniform_points(100_000, synth.BASE_SEED + 6)
        x5, y5, m5, s5, rx5, ry5 = (d(a) for a in (lens5.x, lens5.y, lens5.m, lens5.s, r5x, r5y))
        bx5 = rx5 - 0.1 * rx5  # fixed target source positions (only the data flow matters for timing)
        by5 = ry5 - 0.1 * ry5  # (the 1e6 step above uses the fitting recipe's beta*)
        tree5 = g.Tree().build(x5, y5, m5, s5, theta=THETA, q=lens5.q, leaf_size=LEAF, order=ORDER)
        ws5 = torch.empty(g.adjoint_workspace_bytes(tree5, rx5.numel()), dtype=torch.uint8, device=dev)
        out5 = {k: torch.empty(rx5.numel(), dtype=torch.float32, device=dev) for k in ["a1", "a2"]}
        grads5 = [torch.zeros(lens5.n, dtype=torch.float64, device=dev) for _ in range(4)]

        def step5():
            tree5.build(x5, y5, m5, s5, theta=THETA, q=lens5.q, leaf_size=LEAF, order=ORDER)
            g.shoot(tree5, rx5, ry5, out=out5, workspace=ws5, alpha_only=True)
            ga1 = (-2.0 * (rx5 - out5["a1"] - bx5)).float()
            ga2 = (-2.0 * (ry5 - out5["a2"] - by5)).float()
            for t_ in grads5:
                t_.zero_()
            g.shoot_adjoint(tree5, rx5, ry5, ga1, ga2, *grads5, workspace=ws5)

        for _ in range(2):
            step5()
        torch.cuda.synchronize()
        t = time.perf_counter()
        n5 = max(3, args.steps)
        for _ in range(n5):
            step5()
        torch.cuda.synchronize()
        fa5_ms = 1e3 * (time.perf_counter() - t) / n5
        log(f"fwd+adjoint (1e5 particles, 1e5 rays): {fa5_ms:.3f} ms -> {rx5.numel() / (fa5_ms * 1e-3):.4e} rays/s")

        # the same with kappa and gamma in the loss: L += sum (kappa - 1/2)^2 + |gamma|^2
        out5k = {k: torch.empty(rx5.numel(), dtype=torch.float32, device=dev) for k in ["a1", "a2", "kappa", "g1", "g2"]}

        def step5kg():
            tree5.build(x5, y5, m5, s5, theta=THETA, q=lens5.q, leaf_size=LEAF, order=ORDER)
            g.shoot(tree5, rx5, ry5, out=out5k, workspace=ws5)
            ga1 = (-2.0 * (rx5 - out5k["a1"] - bx5)).float()
            ga2 = (-2.0 * (ry5 - out5k["a2"] - by5)).float()
            for t_ in grads5:
                t_.zero_()
            g.shoot_adjoint(tree5, rx5, ry5, ga1, ga2, *grads5, workspace=ws5, gk=2.0 * (out5k["kappa"] - 0.5),
                            gg1=2.0 * out5k["g1"], gg2=2.0 * out5k["g2"])

        for _ in range(2):
            step5kg()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n5):
            step5kg()
        torch.cuda.synchronize()
        fak_ms = 1e3 * (time.perf_counter() - t) / n5
        log(f"fwd+adjoint with kappa and gamma in the loss: {fak_ms:.3f} ms -> {rx5.numel() / (fak_ms * 1e-3):.4e} rays/s")

        # microlensing refinement: halo + 1e5 stars, 256^2 base cells over the star
        # patch, 6 rounds refining the top 10% by 3x3, all rounds in one HIP graph
        lens3, cx3, cy3, side3 = synth.workload_microlensing()
        x3, y3, m3, s3 = d(lens3.x), d(lens3.y), d(lens3.m), d(lens3.s)
        tree3 = g.Tree().build(x3, y3, m3, s3, theta=THETA, q=lens3.q, leaf_size=LEAF, order=ORDER)
        run3 = g.RefinementRun(tree3, d(cx3), d(cy3), d(side3), g.refine_schedule(cx3.size))
        n3 = run3.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            run3.run()
        torch.cuda.synchronize()
        eager3 = (time.perf_counter() - t) / 3
        graph3 = run3.capture()
        graph3.replay()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            graph3.replay()
        torch.cuda.synchronize()
        graph3_s = (time.perf_counter() - t) / 3
        log(f"refinement (6 rounds, {n3} rays): graph {1e3 * graph3_s:.2f} ms, eager {1e3 * eager3:.2f} ms "
            f"-> {n3 / graph3_s:.4e} rays/s")

        # refinement with the interpolation shortcut on a smooth patch of the 1e6 halo
        # (0.0002 square at (0.3, 0.05), 256^2 base cells, 6 rounds): plain vs interpolated
        pa, pc = 0.0002, (0.3, 0.05)
        ix6, iy6 = synth.ray_grid(256, 0.0, pa)
        run6 = g.RefinementRun(tree3, d(ix6 + pc[0] - pa / 2), d(iy6 + pc[1] - pa / 2),
                               d(np.full(ix6.size, pa / 256)), g.refine_schedule(ix6.size))
        for _ in range(2):
            n6 = run6.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            run6.run()
        torch.cuda.synchronize()
        plain6 = (time.perf_counter() - t) / 3
        run6.run_interp(pc[0] - pa / 2, pc[1] - pa / 2, pa / 256, 256, tol=1e-4)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            _, walked6 = run6.run_interp(pc[0] - pa / 2, pc[1] - pa / 2, pa / 256, 256, tol=1e-4)
        torch.cuda.synchronize()
        interp6 = (time.perf_counter() - t) / 3
        log(f"refinement of a smooth patch ({n6} cells): plain {1e3 * plain6:.2f} ms, with interpolation "
            f"{1e3 * interp6:.2f} ms, walking {walked6} rays")

        # 64 independent lenses in one persistent launch, autotuned: one order for the
        # batch, theta and leaf size per lens, each accepted on 16,384 random rays plus
        # the 4,096 nearest its densest point against the FP64 direct sum
        lenses4 = synth.workload_batched_lenses(64)
        dl4 = [(d(l4.x), d(l4.y), d(l4.m), d(l4.s), d(r4x), d(r4y)) for l4, r4x, r4y in lenses4]
        t = time.perf_counter()
        order4, picks4, _ = g.autotune_batch(dl4, q=lenses4[0][0].q)
        tune4_s = time.perf_counter() - t
        trees4 = [g.Tree().build(x4, y4, m4, s4, theta=p4["theta"], q=l4.q, leaf_size=p4["leaf_size"], order=order4)
                  for (x4, y4, m4, s4, _, _), p4, (l4, _, _) in zip(dl4, picks4, lenses4)]
        rays4 = [(r4x, r4y) for (_, _, _, _, r4x, r4y) in dl4]
        R4 = sum(r[0].numel() for r in rays4)
        outs4 = [{k: torch.empty(r[0].numel(), dtype=torch.float32, device=dev) for k in ["a1", "a2", "kappa", "g1", "g2"]}
                 for r in rays4]
        ws4 = torch.empty(g.batch.batched_workspace_bytes([r[0].numel() for r in rays4]), dtype=torch.uint8, device=dev)
        g.shoot_batched(trees4, rays4, outs=outs4, workspace=ws4)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            g.shoot_batched(trees4, rays4, outs=outs4, workspace=ws4)
        torch.cuda.synchronize()
        b4 = (time.perf_counter() - t) / 3
        ws4b = torch.empty(g.workspace_bytes(max(r[0].numel() for r in rays4)), dtype=torch.uint8, device=dev)
        t = time.perf_counter()
        for _ in range(3):
            for tr, (r4x, r4y), o4 in zip(trees4, rays4, outs4):
                g.shoot(tr, r4x, r4y, out=o4, workspace=ws4b)
        torch.cuda.synchronize()
        l4 = (time.perf_counter() - t) / 3
        # every lens's error over all its rays against the FP64 direct sum (the bar's definition)
        g.shoot_batched(trees4, rays4, outs=outs4, workspace=ws4)
        lens4_err = []
        for (x4, y4, m4, s4, r4x, r4y), o4, l4_ in zip(dl4, outs4, lenses4):
            f4 = g.shoot_direct(x4, y4, m4, s4, l4_[0].q, r4x, r4y, fp64=True)
            lens4_err.append(max(g.batch._errors(o4, f4)))
        log(f"64 lenses ({R4} rays), autotuned in {tune4_s:.1f} s: order {order4}, (theta, leaf) "
            f"{sorted(set((p4['theta'], p4['leaf_size']) for p4 in picks4))}; one persistent launch {1e3 * b4:.2f} ms "
            f"({R4 / b4:.4e} rays/s), per-lens launches {1e3 * l4:.2f} ms; worst lens error over all its rays "
            f"{max(lens4_err):.2e}")
        # the same lenses at one fixed setting (theta 0.3, order 8, leaf 16): its time, and how many
        # lenses it leaves above the bar over all their rays
        trees4f = [g.Tree().build(x4, y4, m4, s4, theta=THETA, q=l4.q, leaf_size=LEAF, order=ORDER)
                   for (x4, y4, m4, s4, _, _), (l4, _, _) in zip(dl4, lenses4)]
        g.shoot_batched(trees4f, rays4, outs=outs4, workspace=ws4)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            g.shoot_batched(trees4f, rays4, outs=outs4, workspace=ws4)
        torch.cuda.synchronize()
        b4f = (time.perf_counter() - t) / 3
        fixed_err = []
        for (x4, y4, m4, s4, r4x, r4y), o4, l4_ in zip(dl4, outs4, lenses4):
            f4 = g.shoot_direct(x4, y4, m4, s4, l4_[0].q, r4x, r4y, fp64=True)
            fixed_err.append(max(g.batch._errors(o4, f4)))
        del trees4f
        log(f"64 lenses at fixed theta {THETA}, order {ORDER}, leaf {LEAF}: {1e3 * b4f:.2f} ms; "
            f"{sum(e > 1e-4 for e in fixed_err)} lenses above the bar (worst {max(fixed_err):.2e})")
        batched4 = {"lenses": len(lenses4), "rays": R4, "ms": 1e3 * b4, "rays_per_s": R4 / b4,
                    "fixed_setting": {"theta": THETA, "order": ORDER, "leaf_size": LEAF, "ms": 1e3 * b4f,
                                      "lenses_above_1e-4": int(sum(e > 1e-4 for e in fixed_err)),
                                      "max_err": max(fixed_err)},
                    "per_lens_launches_ms": 1e3 * l4, "order": order4, "tune_s": tune4_s,
                    "theta_leaf_per_lens": [(p4["theta"], p4["leaf_size"]) for p4 in picks4],
                    "max_err_per_lens_vs_gpu_fp64_direct_all_rays": lens4_err}
        del trees4, rays4, outs4, ws4, ws4b, dl4

        # truncated NFW halos as particles: the halo convergence test's field (1e4 halos
        # in the unit disk, sizes U(0, 0.3), dN/dm ~ m^-2 on [1e-3, 1], c = 3) under a
        # 2048^2 grid over [-1, 1]^2; tree at the headline theta / order / leaf size
        lh, ch = synth.nfw_halo_field(10_000, synth.BASE_SEED + 7)
        xh, yh, mh, sh = d(lh.x), d(lh.y), d(lh.m), d(lh.s)
        hx, hy = synth.ray_grid_tiled(2048, -1.0, 1.0)
        hxd, hyd = d(hx), d(hy)
        treeh = g.Tree()

        def steph():
            treeh.build(xh, yh, mh, sh, theta=THETA, q=ch, leaf_size=LEAF, order=ORDER, nfw=True)
            g.shoot(treeh, hxd, hyd, out=out, workspace=ws)

        for _ in range(2):
            steph()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            steph()
        torch.cuda.synchronize()
        nfw_ms = 1e3 * (time.perf_counter() - t) / 5
        ev0.record(stream)
        for _ in range(5):
            g.shoot(treeh, hxd, hyd, out=out, ordered=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        nfw_walk_ms = ev0.elapsed_time(ev1) / 5
        cnth = g.shoot(treeh, hxd, hyd, counts=True, ordered=True)["counts"].cpu().numpy().astype(np.float64)
        g.shoot(treeh, hxd, hyd, out=out, workspace=ws)
        resh = {}
        for fp64 in (False, True):
            g.shoot_direct(xh, yh, mh, sh, ch, hxd[:256], hyd[:256], fp64=fp64, nfw=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            fullh = g.shoot_direct(xh, yh, mh, sh, ch, hxd, hyd, fp64=fp64, nfw=True)
            torch.cuda.synchronize()
            resh[fp64] = R / (time.perf_counter() - t)
        ref_a = torch.stack([fullh["a1"], fullh["a2"]], 1)
        ref_g = torch.stack([fullh["g1"], fullh["g2"]], 1)
        e_a = (torch.stack([out["a1"], out["a2"]], 1).double() - ref_a).norm(dim=1) / ref_a.norm(dim=1)
        e_g = (torch.stack([out["g1"], out["g2"]], 1).double() - ref_g).norm(dim=1) / ref_g.norm(dim=1)
        inside = fullh["kappa"] > 0
        e_k = (out["kappa"].double() - fullh["kappa"]).abs()[inside] / fullh["kappa"][inside]
        gnorm = ref_g.norm(dim=1)
        worst = int(e_g.argmax())
        nfw_err = {"alpha_max": float(e_a.max()), "alpha_median": float(e_a.median()),
                   "kappa_max": float(e_k.max()), "gamma_max": float(e_g.max()),
                   "gamma_p999": float(torch.quantile(e_g.float(), 0.999)),
                   "gamma_rays_above_1e-4": int((e_g > 1e-4).sum()),
                   "gamma_worst_ray_abs_over_median_abs": float(gnorm[worst] / gnorm.median()),
                   "kappa_zero_outside_exact": bool((out["kappa"][~inside] == 0).all())}
        # the bar's definition: rays whose reference is under 1e-3 of the median are measured against the median
        ebar = g.batch._errors(out, fullh)
        nfw_err["max_err_bar_definition"] = max(ebar)
        gbar = g.batch._rel_errors((torch.stack([out["g1"], out["g2"]], 1).double() - ref_g).norm(dim=1),
                                   ref_g.norm(dim=1))
        nfw_err["gamma_rays_above_1e-4_bar_definition"] = int((gbar > 1e-4).sum())
        nfw_err["passes_1e-4_bar_definition"] = max(ebar) <= 1e-4
        # the same field at theta 0.2, order 12 (leaf 16): its time and errors
        TH2, P2 = 0.2, 12

        def steph2():
            treeh.build(xh, yh, mh, sh, theta=TH2, q=ch, leaf_size=LEAF, order=P2, nfw=True)
            g.shoot(treeh, hxd, hyd, out=out, workspace=ws)

        for _ in range(2):
            steph2()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            steph2()
        torch.cuda.synchronize()
        nfw2_ms = 1e3 * (time.perf_counter() - t) / 5
        ebar2 = g.batch._errors(out, fullh)
        gbar2 = g.batch._rel_errors((torch.stack([out["g1"], out["g2"]], 1).double() - ref_g).norm(dim=1),
                                    ref_g.norm(dim=1))
        inside2 = fullh["kappa"] > 0
        nfw_tight = {"theta": TH2, "order": P2, "leaf_size": LEAF, "step_ms": nfw2_ms, "rays_per_s": R / (nfw2_ms * 1e-3),
                     "max_err_bar_definition": max(ebar2), "err_alpha_kappa_gamma_bar_definition": list(ebar2),
                     "gamma_rays_above_1e-4_bar_definition": int((gbar2 > 1e-4).sum()),
                     "kappa_zero_outside_exact": bool((out["kappa"][~inside2] == 0).all()),
                     "passes_1e-4_bar_definition": max(ebar2) <= 1e-4}
        log(f"NFW halo field at theta {TH2}, order {P2}: build + shoot {nfw2_ms:.2f} ms "
            f"({R / (nfw2_ms * 1e-3):.4e} rays/s); max error under the bar's definition {max(ebar2):.2e}, "
            f"{nfw_tight['gamma_rays_above_1e-4_bar_definition']} rays with gamma above 1e-4")
        del fullh, ref_a, ref_g, e_a, e_g, e_k, gnorm, gbar, gbar2, inside2
        log(f"NFW halo field under the bar's definition: max error {max(ebar):.2e}, "
            f"{nfw_err['gamma_rays_above_1e-4_bar_definition']} rays with gamma above 1e-4")
        extras = {"direct_fp32_rays_per_s": res[False], "direct_fp64_rays_per_s": res[True],
                  "potential_walk_ms": pot_ms, "potential_walk_rays_per_s": R / (pot_ms * 1e-3),
                  "knn_smoothing_1e6_ms": knn_ms, "knn_max_rel_diff_vs_host_kdtree": knn_diff,
                  "knn_from_positions_ms": knn_pos,
                  "fwd_adjoint_1e5_rays_per_s": rx5.numel() / (fa5_ms * 1e-3), "fwd_adjoint_1e5_ms": fa5_ms,
                  "fwd_adjoint_1e5_workload": "nfw_1e5_particles_1e5_uniform_rays, L = sum |x - alpha - beta*|^2",
                  "fwd_adjoint_kappa_gamma_ms": fak_ms,
                  "fwd_adjoint_kappa_gamma_rays_per_s": rx5.numel() / (fak_ms * 1e-3),
                  "refinement_rays": n3, "refinement_graph_ms": 1e3 * graph3_s, "refinement_eager_ms": 1e3 * eager3,
                  "refinement_rays_per_s": n3 / graph3_s,
                  "refinement_workload": "nfw_1e6 + 1e5 Salpeter stars, 256^2 base, 6 rounds top-10% 3x3",
                  "interp_refinement_cells": n6, "interp_refinement_walked": walked6,
                  "interp_refinement_plain_ms": 1e3 * plain6, "interp_refinement_ms": 1e3 * interp6,
                  "interp_refinement_workload": "nfw_1e6 + stars tree, smooth 0.0002 patch at (0.3, 0.05), "
                                                "256^2 base, 6 rounds, tol 1e-4",
                  "batched_64_lenses": batched4,
                  "nfw_halos": {"workload": "1e4 truncated NFW halos (unit disk, sizes U(0, 0.3), dN/dm ~ m^-2 "
                                            "on [1e-3, 1], c = 3), 2048^2 grid over [-1, 1]^2",
                                "note": "this field fails the 1e-4 bar on the shear of a few rays where |gamma| is "
                                        "about 1e-3 to 2e-2 of the median (many halos' shears cancel there). At "
                                        "theta 0.3, order 8 the FP64 oracle tree misses there too (truncation); at "
                                        "theta 0.2, order 12 it passes, and the FP32 terms of the walk leave a few "
                                        "rays at about 1.6e-4; see err_vs_gpu_fp64_direct and tighter_setting",
                                "step_ms": nfw_ms, "rays_per_s": R / (nfw_ms * 1e-3), "walk_ms": nfw_walk_ms,
                                "direct_fp32_rays_per_s": resh[False], "direct_fp64_rays_per_s": resh[True],
                                "err_vs_gpu_fp64_direct": nfw_err, "tighter_setting": nfw_tight,
                                "counts_per_ray": dict(zip(["visited", "accepted", "leaf", "list_hits"],
                                                           cnth.mean(0).tolist()))}}

    # counter calibration: a plain device copy of 1 GiB (reads 1 GiB, writes 1 GiB)
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    line = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "nfw_1e6_particles_grid2048", "particles": lens.n, "rays": R, "theta": THETA,
                   "order": ORDER, "leaf_size": LEAF, "q": lens.q, "step": "build_tree + shoot (alpha, kappa, gamma); the ray staging runs on a second stream "
                                           "beside the build"},
        "ms_per_step_one_stream": ms_step_one_stream,
        "roofline": {"bound": "alu", "kernel": "k_walk", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(),
                     "kernel_ms": walk_ms, "flop_per_launch": flop, "lane_use": lane_use,
                     "search_overhead_flop_per_launch": scan_flop, **issued_valu(flop)},
        "fwd_adjoint": fwd_adjoint,
        "full_grid_err_vs_gpu_fp64_direct": full_err,
        "extras": {"build_ms": build_ms, "walk_only_rays_per_s": R / (walk_ms * 1e-3),
                   "fwd_adjoint_1e6_rays_per_s": fwd_adjoint["value"],
                   "ncells": info["ncells"], "nlisted": info["nlisted"],
                   "counts_per_ray": dict(zip(["visited", "accepted", "leaf", "list_hits"], cnt.mean(0).tolist())),
                   **extras},
    }

    if not args.no_cpu:
        import oracle

        oracle.build(force=False)
        nt = cpu_threads()
        gen = synth.rng(synth.BASE_SEED + 99)
        # oracle A (FP64 brute force): a probe sizes a sample of ~12 s on all threads
        probe = gen.choice(R, 256, replace=False)
        t = time.perf_counter()
        oracle.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx_t[probe], ry_t[probe], threads=nt)
        per_ray = (time.perf_counter() - t) / probe.size
        k = int(min(R, max(256, 12.0 / per_ray)))
        idx = np.sort(gen.choice(R, k, replace=False))
        t = time.perf_counter()
        ref = oracle.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx_t[idx], ry_t[idx], threads=nt)
        cpu_el = time.perf_counter() - t
        # ... and on one thread, over the sample's first k1 rays (~6 s)
        k1 = int(max(16, min(k, 6.0 / (cpu_el / k * nt))))
        t = time.perf_counter()
        oracle.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx_t[idx[:k1]], ry_t[idx[:k1]], threads=1)
        cpu1_el = time.perf_counter() - t
        g.shoot(tree, rx, ry, out=out, workspace=ws)
        got = np.stack([out[kk].double().cpu().numpy()[idx] for kk in ["a1", "a2", "kappa", "g1", "g2"]], axis=1)
        ea = np.linalg.norm(got[:, :2] - ref[:, :2], axis=1) / np.linalg.norm(ref[:, :2], axis=1)
        ek = np.abs(got[:, 2] - ref[:, 2]) / np.abs(ref[:, 2])
        eg = np.linalg.norm(got[:, 3:] - ref[:, 3:], axis=1) / np.linalg.norm(ref[:, 3:], axis=1)
        # oracle B (FP64 reference tree, the CPU analogue of the paper's threaded tree
        # solver) at the same theta, order and leaf size: build, then a sample of ~4 s
        t = time.perf_counter()
        T = oracle.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, THETA, LEAF, ORDER)
        treeB_build = time.perf_counter() - t
        t = time.perf_counter()
        T.shoot(rx_t[idx], ry_t[idx], threads=nt)
        per_rayB = (time.perf_counter() - t) / idx.size
        kB = int(min(R, max(idx.size, 4.0 / per_rayB)))
        idxB = np.sort(gen.choice(R, kB, replace=False))
        t = time.perf_counter()
        T.shoot(rx_t[idxB], ry_t[idxB], threads=nt)
        treeB_el = time.perf_counter() - t
        kB1 = int(max(64, min(kB, 4.0 / (treeB_el / kB * nt))))
        t = time.perf_counter()
        T.shoot(rx_t[idxB[:kB1]], ry_t[idxB[:kB1]], threads=1)
        treeB1_el = time.perf_counter() - t
        del T
        line["cpu_baseline"] = {
            "value": k / cpu_el, "unit": "rays/s", "cores": nt, "kind": "oracle",
            "sample": f"{k} random rays of the 2048^2 grid, FP64 brute force (oracle A) over all {lens.n} "
                      f"particles ({cpu_el:.1f} s on {nt} threads; {k1} of them on 1 thread, {cpu1_el:.1f} s)",
            "value_1_thread": k1 / cpu1_el, "cpu_model": cpu_model(),
            "tree": {"kind": "oracle", "value": kB / treeB_el, "value_1_thread": kB1 / treeB1_el, "cores": nt,
                     "build_s": treeB_build,
                     "sample": f"FP64 reference tree (oracle B), theta {THETA}, order {ORDER}, leaf {LEAF}: "
                               f"{kB} random rays of the grid on {nt} threads ({treeB_el:.1f} s), {kB1} on 1 thread "
                               f"({treeB1_el:.1f} s); the single-threaded build of the 1e6-particle tree "
                               f"({treeB_build:.1f} s) is not in the rate"}}
        line["parity_vs_fp64_sample"] = {"rays": k, "alpha_max": float(ea.max()), "kappa_max": float(ek.max()),
                                         "gamma_max": float(eg.max())}
        log(f"cpu oracle A: {k / cpu_el:.1f} rays/s on {nt} threads, {k1 / cpu1_el:.1f} on 1; oracle B tree: "
            f"{kB / treeB_el:.1f} rays/s on {nt} threads, {kB1 / treeB1_el:.1f} on 1 (build {treeB_build:.1f} s); "
            f"sample max rel err alpha {ea.max():.2e} kappa {ek.max():.2e} gamma {eg.max():.2e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
