"""Batched walks, device-side refinement rounds (graph-capturable) and the
parameter autotuner.  Argument marshalling over the C ABI; the work runs in
the library's kernels."""
from __future__ import annotations

import ctypes
import math
import time

import torch

from . import _capi
from ._capi import GLM_ALPHA_ONLY, GLM_INTERP_DEFLECTIONS, GlmLensRays


def _ptr(t):
    return t.data_ptr() if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def batched_workspace_bytes(nrays) -> int:
    lib = _capi.load()
    arr = (ctypes.c_int64 * len(nrays))(*[int(n) for n in nrays])
    b = ctypes.c_size_t(0)
    _capi.check(lib.glm_shoot_batched_workspace_bytes(arr, len(nrays), ctypes.byref(b)))
    return int(b.value)


def shoot_batched(trees, rays, alpha_only: bool = False, outs=None, workspace=None):
    """Walk len(trees) lenses in one persistent launch.  rays: list of (rx, ry)
    float64 CUDA tensors.  Returns a list of output dicts (float32)."""
    n = len(trees)
    assert len(rays) == n and n > 0
    dev = rays[0][0].device
    names = ["a1", "a2"] if alpha_only else ["a1", "a2", "kappa", "g1", "g2"]
    if outs is None:
        outs = [{k: torch.empty(r[0].numel(), dtype=torch.float32, device=dev) for k in names} for r in rays]
    ents = (GlmLensRays * n)()
    for i, (t, (rx, ry), o) in enumerate(zip(trees, rays, outs)):
        assert rx.dtype == torch.float64 and rx.is_contiguous() and ry.is_contiguous()
        ents[i] = GlmLensRays(t.handle.value, _ptr(rx), _ptr(ry), rx.numel(), _ptr(o["a1"]), _ptr(o["a2"]),
                              _ptr(o.get("kappa")), _ptr(o.get("g1")), _ptr(o.get("g2")))
    if workspace is None:
        workspace = torch.empty(max(batched_workspace_bytes([r[0].numel() for r in rays]), 1), dtype=torch.uint8,
                                device=dev)
    lib = _capi.load()
    _capi.check(lib.glm_shoot_batched(ents, n, GLM_ALPHA_ONLY if alpha_only else 0, ctypes.c_void_p(_ptr(workspace)),
                                      workspace.numel(), _stream()))
    return outs


def refine_workspace_bytes(ncells: int) -> int:
    lib = _capi.load()
    b = ctypes.c_size_t(0)
    _capi.check(lib.glm_refine_workspace_bytes(int(ncells), ctypes.byref(b)))
    return int(b.value)


def refine_round(cx, cy, side, kappa, g1, g2, ncells: int, nrefine: int, refined=None, workspace=None):
    """One 3x3 refinement round of the nrefine highest-ranked cells (in place;
    8 new cells appended at [ncells, ncells + 8 nrefine))."""
    if workspace is None:
        workspace = torch.empty(max(refine_workspace_bytes(ncells), 1), dtype=torch.uint8, device=cx.device)
    lib = _capi.load()
    _capi.check(lib.glm_refine_round(ctypes.c_void_p(_ptr(cx)), ctypes.c_void_p(_ptr(cy)), ctypes.c_void_p(_ptr(side)),
                                     ctypes.c_void_p(_ptr(kappa)), ctypes.c_void_p(_ptr(g1)), ctypes.c_void_p(_ptr(g2)),
                                     int(ncells), int(nrefine), ctypes.c_void_p(_ptr(refined)),
                                     ctypes.c_void_p(_ptr(workspace)), workspace.numel(), _stream()))


def _size(fn, *args) -> int:
    b = ctypes.c_size_t(0)
    _capi.check(fn(*args, ctypes.byref(b)))
    return int(b.value)


def interp_init(cx, cy, ncells: int, x0: float, y0: float, h0: float, capacity: int, state):
    """Index the base grid (nbase x nbase cells of side h0, lower-left corner
    (x0, y0)) for the interpolation shortcut; state: uint8 CUDA tensor."""
    lib = _capi.load()
    _capi.check(lib.glm_interp_init(ctypes.c_void_p(_ptr(cx)), ctypes.c_void_p(_ptr(cy)), int(ncells), float(x0),
                                    float(y0), float(h0), int(capacity), ctypes.c_void_p(_ptr(state)), state.numel(),
                                    _stream()))


def refine_interp_round(cx, cy, side, out, ncells: int, nrefine: int, nbase: int, tol: float, capacity: int, state,
                        shoot_idx, shoot_count, refined=None, workspace=None, deflections: bool = False):
    """One refinement round with the interpolation shortcut (Sec. 3.4): new
    cells of uniform cells are filled in `out`, the others are listed in
    shoot_idx with their number in shoot_count (device).  deflections: the
    uniformity test and the fill use the three-point magnification matrix
    from deflections (App. A) instead of kappa and gamma."""
    lib = _capi.load()
    if workspace is None:
        workspace = torch.empty(_size(lib.glm_interp_round_workspace_bytes, int(ncells), int(nrefine)),
                                dtype=torch.uint8, device=cx.device)
    v = lambda t: ctypes.c_void_p(_ptr(t))
    _capi.check(lib.glm_refine_interp_round(v(cx), v(cy), v(side), v(out["a1"]), v(out["a2"]), v(out["kappa"]),
                                            v(out["g1"]), v(out["g2"]), int(ncells), int(nrefine), int(nbase),
                                            float(tol), GLM_INTERP_DEFLECTIONS if deflections else 0, v(refined),
                                            v(shoot_idx), v(shoot_count), int(capacity), v(state), state.numel(),
                                            v(workspace), workspace.numel(), _stream()))


def interp_estimate(cx, cy, out, nbase: int, capacity: int, state, idx=None, count=None, max_count: int = 0):
    """kappa, g1, g2 in `out` of the cells idx[:count] (device count; idx None:
    cells 0 .. max_count - 1) from their three-point magnification matrix (App. A)."""
    lib = _capi.load()
    v = lambda t: ctypes.c_void_p(_ptr(t))
    _capi.check(lib.glm_interp_estimate(v(cx), v(cy), v(out["a1"]), v(out["a2"]), v(out["kappa"]), v(out["g1"]),
                                        v(out["g2"]), v(idx), v(count), int(max_count), int(nbase), int(capacity),
                                        v(state), state.numel(), _stream()))


def shoot_indexed(tree, cx, cy, idx, count: int, out, workspace=None, alpha_only: bool = False):
    """Walk the rays (cx[idx[t]], cy[idx[t]]), t < count, writing out[...][idx[t]]."""
    lib = _capi.load()
    if workspace is None:
        workspace = torch.empty(max(_size(lib.glm_shoot_indexed_workspace_bytes, int(count)), 1), dtype=torch.uint8,
                                device=cx.device)
    v = lambda t: ctypes.c_void_p(_ptr(t))
    _capi.check(lib.glm_shoot_indexed(tree.handle.value, v(cx), v(cy), v(idx), int(count), v(out["a1"]), v(out["a2"]),
                                      v(out.get("kappa")), v(out.get("g1")), v(out.get("g2")),
                                      GLM_ALPHA_ONLY if alpha_only else 0, v(workspace), workspace.numel(), _stream()))


def refine_schedule(n0: int, rounds: int = 6, frac: float = 0.1, max_new_rays: int = 600_000):
    """Cells refined per round: floor(frac * cells), with 8 new rays per refined
    cell capped at max_new_rays."""
    out, n = [], n0
    for _ in range(rounds):
        k = min(int(math.floor(frac * n)), max_new_rays // 8)
        out.append(k)
        n += 8 * k
    return out


class RefinementRun:
    """A base grid of square cells on one tree, then refinement rounds, each
    shooting its 8 new rays per refined cell.  Buffers have fixed capacity, so
    run() can be captured once in a HIP graph (capture()) and replayed."""

    def __init__(self, tree, cx0, cy0, side0, schedule):
        from . import shoot, workspace_bytes

        self._shoot = shoot
        self.tree = tree
        self.schedule = list(schedule)
        self.n0 = cx0.numel()
        self.cap = self.n0 + 8 * sum(self.schedule)
        dev = cx0.device
        f64 = dict(dtype=torch.float64, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        self.cx = torch.zeros(self.cap, **f64)
        self.cy = torch.zeros(self.cap, **f64)
        self.side = torch.zeros(self.cap, **f64)
        self.base = (cx0.clone(), cy0.clone(), side0.clone())
        self.out = {k: torch.zeros(self.cap, **f32) for k in ["a1", "a2", "kappa", "g1", "g2"]}
        self.refined = torch.zeros(max(self.schedule + [1]), dtype=torch.int32, device=dev)
        ws = max(workspace_bytes(n) for n in [self.n0] + [8 * k for k in self.schedule])
        self.ws_shoot = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.ws_refine = torch.empty(max(refine_workspace_bytes(self.cap), 1), dtype=torch.uint8, device=dev)
        self.sizes = [self.n0] + [8 * k for k in self.schedule]

    def _shoot_range(self, a, b):
        o = {k: v[a:b] for k, v in self.out.items()}
        self._shoot(self.tree, self.cx[a:b], self.cy[a:b], out=o, workspace=self.ws_shoot)

    def run(self):
        bx, by, bs = self.base
        self.cx[: self.n0].copy_(bx)
        self.cy[: self.n0].copy_(by)
        self.side[: self.n0].copy_(bs)
        self._shoot_range(0, self.n0)
        n = self.n0
        for k in self.schedule:
            refine_round(self.cx, self.cy, self.side, self.out["kappa"], self.out["g1"], self.out["g2"], n, k,
                         refined=self.refined, workspace=self.ws_refine)
            self._shoot_range(n, n + 8 * k)
            n += 8 * k
        return n

    def run_interp(self, x0: float, y0: float, h0: float, nbase: int, tol: float = 1e-4, alpha_only: bool = False):
        """The same schedule with the interpolation shortcut (Sec. 3.4): the
        base cells (an nbase x nbase grid of side h0 from (x0, y0)) are shot,
        then each round fills the new cells of uniform cells by the linear lens
        equation and walks only the others.  alpha_only: the walks compute
        deflections only, and the magnification matrix (for the ranking, the
        uniformity test and the fill) comes from deflections at three points
        (App. A).  Reads the number of rays to walk once per round (a host
        synchronisation), so it is not graph-captured.  Returns (cells, rays walked)."""
        lib = _capi.load()
        dev = self.cx.device
        if not hasattr(self, "_interp"):
            self._interp = dict(
                state=torch.empty(_size(lib.glm_interp_state_bytes, self.cap), dtype=torch.uint8, device=dev),
                idx=torch.zeros(max(8 * max(self.schedule + [1]), 1), dtype=torch.int32, device=dev),
                count=torch.zeros(1, dtype=torch.int32, device=dev),
                ws_round=torch.empty(max(_size(lib.glm_interp_round_workspace_bytes, n, max(k, 1))
                                         for n, k in self._rounds()), dtype=torch.uint8, device=dev),
                ws_idx=torch.empty(_size(lib.glm_shoot_indexed_workspace_bytes, 8 * max(self.schedule + [1])),
                                   dtype=torch.uint8, device=dev))
        it = self._interp
        bx, by, bs = self.base
        self.cx[: self.n0].copy_(bx)
        self.cy[: self.n0].copy_(by)
        self.side[: self.n0].copy_(bs)
        interp_init(self.cx, self.cy, self.n0, x0, y0, h0, self.cap, it["state"])
        if alpha_only:
            shoot_indexed(self.tree, self.cx, self.cy, torch.arange(self.n0, dtype=torch.int32, device=dev), self.n0,
                          self.out, alpha_only=True)
            interp_estimate(self.cx, self.cy, self.out, nbase, self.cap, it["state"], max_count=self.n0)
        else:
            self._shoot_range(0, self.n0)
        n, walked = self.n0, self.n0
        for k in self.schedule:
            if k > 0:
                refine_interp_round(self.cx, self.cy, self.side, self.out, n, k, nbase, tol, self.cap, it["state"],
                                    it["idx"], it["count"], refined=self.refined, workspace=it["ws_round"],
                                    deflections=alpha_only)
                cnt = int(it["count"].item())
                shoot_indexed(self.tree, self.cx, self.cy, it["idx"], cnt, self.out, workspace=it["ws_idx"],
                              alpha_only=alpha_only)
                if alpha_only:
                    interp_estimate(self.cx, self.cy, self.out, nbase, self.cap, it["state"], idx=it["idx"],
                                    count=it["count"], max_count=8 * k)
                walked += cnt
            n += 8 * k
        return n, walked

    def _rounds(self):
        n = self.n0
        for k in self.schedule:
            yield n, k
            n += 8 * k

    def capture(self):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        return g


def validation_rays(x, y, s, rx, ry, sample: int = 16384, dense: int = 4096, seed: int = 0):
    """Indices of the rays an autotuned configuration must pass on: `sample`
    seeded random rays plus the `dense` rays nearest the densest point (the
    particle with the smallest smoothing length, or the centre of mass of
    equal point masses), where the walk opens the most boxes and the shear is
    the smallest difference of large terms.  All rays if there are fewer."""
    R = rx.numel()
    if sample + dense >= R:
        return torch.arange(R, device=rx.device)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    pick = torch.randperm(R, generator=gen)[:sample].to(rx.device)
    if s is not None and bool((s > 0).any()):
        sp = torch.where(s > 0, s, torch.full_like(s, float("inf")))
        j = int(torch.argmin(sp))
        cx, cy = x[j], y[j]
    else:
        cx, cy = x.mean(), y.mean()
    near = torch.argsort((rx - cx) ** 2 + (ry - cy) ** 2)[:dense]
    return torch.unique(torch.cat([pick, near]))


def _rel_errors(err, mag):
    """Per-ray error over the reference magnitude; rays whose reference is under
    1e-3 of the median magnitude are measured against the median instead (the
    error definition of the accuracy bar: a near-zero reference has no
    meaningful relative error)."""
    med = mag.median()
    return err / torch.where(mag >= 1e-3 * med, mag, med)


def _errors(o, ref):
    ra = torch.stack([ref["a1"], ref["a2"]], 1)
    rg = torch.stack([ref["g1"], ref["g2"]], 1)
    rk = ref["kappa"]
    ea = _rel_errors((torch.stack([o["a1"], o["a2"]], 1).double() - ra).norm(dim=1), ra.norm(dim=1)).max().item()
    eg = _rel_errors((torch.stack([o["g1"], o["g2"]], 1).double() - rg).norm(dim=1), rg.norm(dim=1)).max().item()
    nz = rk != 0
    ek = _rel_errors((o["kappa"].double() - rk).abs()[nz], rk.abs()[nz]).max().item() if bool(nz.any()) else 0.0
    # kappa must vanish exactly where no particle holds the ray
    if bool((~nz).any()) and bool((o["kappa"][~nz] != 0).any()):
        ek = float("inf")
    return ea, ek, eg


def autotune(x, y, m, s, rx, ry, q: float = 3.0, tol: float = 1e-4, thetas=(0.2, 0.3, 0.4, 0.5),
             orders=(4, 6, 8, 10, 12), leaves=(8, 16, 24), sample: int = 16384, dense: int = 4096, reps: int = 3,
             seed: int = 0, nfw: bool = False, every_order: bool = False):
    """Pick (theta, order, leaf size) for one lens: the fastest build + walk of
    all rays rx, ry whose max fractional errors of alpha, kappa and gamma stay
    within `tol` against the library's FP64 direct sum on the validation rays
    (validation_rays: `sample` random rays plus the `dense` nearest the densest
    point; every ray when sample + dense covers them).  For each (leaf size,
    theta) only the smallest passing order is timed (a larger order costs more
    and is no more needed), unless every_order is set: then every order is
    checked and timed (a batch needs each lens's best setting at one order).  The walk group is one wavefront (64 rays) by
    construction.  Errors are per ray relative to the reference magnitude,
    except on rays whose reference is under 1e-3 of the median magnitude, which
    are measured against the median.  Returns (best, table); best is None when nothing passes,
    table has a row per evaluated (theta, order, leaf size) with its errors,
    whether it passed, and its time (NaN unless timed)."""
    from . import Tree, shoot, shoot_direct, workspace_bytes

    R = rx.numel()
    idx = validation_rays(x, y, s, rx, ry, sample, dense, seed)
    sx, sy = rx[idx].contiguous(), ry[idx].contiguous()
    ref = shoot_direct(x, y, m, s, q, sx, sy, fp64=True, nfw=nfw)
    ws = torch.empty(workspace_bytes(R), dtype=torch.uint8, device=rx.device)
    out = {k: torch.empty(R, dtype=torch.float32, device=rx.device) for k in ["a1", "a2", "kappa", "g1", "g2"]}
    table = []
    best = None
    tree = Tree()
    for L in leaves:
        for th in thetas:
            for p in sorted(orders):
                tree.build(x, y, m, s, theta=th, q=q, leaf_size=L, order=p, nfw=nfw)
                ea, ek, eg = _errors(shoot(tree, sx, sy), ref)
                ok = max(ea, eg, ek) <= tol
                ms = float("nan")
                if ok:
                    torch.cuda.synchronize()
                    ts = []
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        tree.build(x, y, m, s, theta=th, q=q, leaf_size=L, order=p, nfw=nfw)
                        shoot(tree, rx, ry, out=out, workspace=ws)
                        torch.cuda.synchronize()
                        ts.append(time.perf_counter() - t0)
                    ms = 1e3 * sorted(ts)[len(ts) // 2]
                    if best is None or ms < best["ms"]:
                        best = dict(theta=th, order=p, leaf_size=L, ms=ms, err=max(ea, eg, ek),
                                    err_alpha=ea, err_kappa=ek, err_gamma=eg, rays_checked=int(idx.numel()))
                table.append(dict(theta=th, order=p, leaf_size=L, err_alpha=ea, err_kappa=ek, err_gamma=eg, ok=ok,
                                  ms=ms))
                if ok and not every_order:
                    break  # larger orders at this (leaf size, theta) only cost more
    return best, table


def autotune_batch(lenses, q: float = 3.0, tol: float = 1e-4, thetas=(0.2, 0.3, 0.4), orders=(6, 8, 10, 12),
                   leaves=(8, 16, 24), sample: int = 16384, dense: int = 4096, reps: int = 3, seed: int = 0):
    """Tune a batch of lenses for one persistent launch: every tree of a batch
    has the same order, while theta and the leaf size may differ per lens.
    lenses: list of (x, y, m, s, rx, ry) CUDA float64 tensors.  Each lens is
    tuned by `autotune` over the orders (accepted on its validation rays);
    then, for every order that passes on all lenses, the trees are built at
    each lens's fastest passing (theta, leaf size) for that order and the
    batched launch is timed; the order of the fastest launch wins.  Returns
    (order, [per-lens dict(theta, leaf_size, ms, err...)], batched ms) or
    (None, [], nan) when no order passes on every lens."""
    from . import Tree

    per_order = {p: [] for p in orders}
    for li, (x, y, m, s, rx, ry) in enumerate(lenses):
        _, table = autotune(x, y, m, s, rx, ry, q=q, tol=tol, thetas=thetas, orders=orders, leaves=leaves,
                            sample=sample, dense=dense, reps=reps, seed=seed + li, every_order=True)
        for p in orders:
            rows = [t for t in table if t["ok"] and t["order"] == p]
            per_order[p].append(min(rows, key=lambda t: t["ms"]) if rows else None)
    feasible = [p for p, rows in per_order.items() if all(r is not None for r in rows)]
    if not feasible:
        return None, [], float("nan")
    rays = [(rx, ry) for (_, _, _, _, rx, ry) in lenses]
    dev = rays[0][0].device
    outs = [{k: torch.empty(r[0].numel(), dtype=torch.float32, device=dev) for k in ["a1", "a2", "kappa", "g1", "g2"]}
            for r in rays]
    ws = torch.empty(batched_workspace_bytes([r[0].numel() for r in rays]), dtype=torch.uint8, device=dev)
    best = (None, float("inf"))
    for p in feasible:
        trees = [Tree().build(x, y, m, s, theta=r["theta"], q=q, leaf_size=r["leaf_size"], order=p)
                 for (x, y, m, s, _, _), r in zip(lenses, per_order[p])]
        shoot_batched(trees, rays, outs=outs, workspace=ws)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            shoot_batched(trees, rays, outs=outs, workspace=ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = 1e3 * sorted(ts)[len(ts) // 2]
        if ms < best[1]:
            best = (p, ms)
        del trees
    return best[0], per_order[best[0]], best[1]
