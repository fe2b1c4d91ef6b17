"""MI355X (gfx950) tree ray-shooting for one lens plane (GLAMER, Sec. 3).

Thin Python binding over libglamer.so (include/glamer.h).  PyTorch supplies
device memory and streams; every step of the computation runs in the HIP
kernels of the library.  Inputs are CUDA (HIP) float64 tensors.

    tree = Tree().build(x, y, m, s, theta=0.3, q=3.0, leaf_size=8, order=8)
    out = shoot(tree, rx, ry)           # dict of float32 tensors a1 a2 kappa g1 g2
"""
from __future__ import annotations

import ctypes

import torch

from . import _capi
from ._capi import (GLM_ALPHA_ONLY, GLM_NFW_HALOS, GLM_FP32_ALPHA, GLM_RAYS_ORDERED, GLM_RAYS_STAGED, GlamerError,  # noqa: F401
                    GlmParams, GlmTreeInfo)

__all__ = ["Tree", "shoot", "shoot_direct", "shoot_adjoint", "ShootFn", "GlamerError", "GLM_ALPHA_ONLY",
           "GLM_NFW_HALOS", "GLM_FP32_ALPHA", "GLM_RAYS_ORDERED", "workspace_bytes", "shoot_batched", "refine_round",
           "refine_schedule", "RefinementRun", "autotune", "autotune_batch", "smoothing_lengths", "interp_init",
           "refine_interp_round", "shoot_indexed", "shoot_potential", "knn", "knn_workspace_bytes",
           "tree_workspace_bytes", "adjoint_workspace_bytes", "shoot_noalloc", "stage_rays"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _f64(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return t.contiguous()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace_bytes(nrays: int) -> int:
    lib = _capi.load()
    b = ctypes.c_size_t(0)
    _capi.check(lib.glm_shoot_workspace_bytes(int(nrays), ctypes.byref(b)))
    return int(b.value)


def tree_workspace_bytes(n: int, params) -> int:
    """Upper bound of the tree workspace for n particles (params: GlmParams)."""
    b = ctypes.c_size_t(0)
    _capi.check(_capi.load().glm_tree_workspace_bytes(int(n), ctypes.byref(params), ctypes.byref(b)))
    return int(b.value)


def adjoint_workspace_bytes(tree, nrays: int) -> int:
    b = ctypes.c_size_t(0)
    _capi.check(_capi.load().glm_adjoint_workspace_bytes(tree.handle, int(nrays), ctypes.byref(b)))
    return int(b.value)


class Tree:
    """Handle of a tree built on the GPU (glm_tree)."""

    def __init__(self):
        self._lib = _capi.load()
        h = ctypes.c_void_p()
        _capi.check(self._lib.glm_tree_create(ctypes.byref(h)))
        self._h = h
        self.params = None
        self.n = 0
        self.workspace = None  # uint8 CUDA tensor holding the tree's device arrays

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.glm_tree_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def build(self, x, y, m, s=None, theta=0.3, q=3.0, leaf_size=8, order=8, flags=0, nfw: bool = False,
              workspace=None):
        """nfw: the particles are truncated NFW halos of sizes s and concentration q.
        workspace: uint8 CUDA tensor for the tree's device arrays; by default the
        handle keeps one of glm_tree_workspace_bytes (reused while large enough)."""
        if nfw:
            flags |= GLM_NFW_HALOS
        x, y, m = _f64(x, "x"), _f64(y, "y"), _f64(m, "m")
        s = _f64(s, "s") if s is not None else None
        n = x.shape[0]
        if y.shape[0] != n or m.shape[0] != n or (s is not None and s.shape[0] != n):
            raise ValueError("x, y, m, s must have the same length")
        p = GlmParams(float(theta), float(q), int(leaf_size), int(order), int(flags))
        if workspace is None:
            need = tree_workspace_bytes(n, p)
            workspace = self.workspace
            if workspace is None or workspace.numel() < need or workspace.device != x.device:
                self.workspace = None
                workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
        self.workspace = workspace
        _capi.check(self._lib.glm_build_tree(self._h, _ptr(x), _ptr(y), _ptr(m), _ptr(s), n,
                                             ctypes.byref(p), _ptr(workspace), workspace.numel(), _stream()))
        self.params = p
        self.n = n
        return self

    def required_bytes(self) -> int:
        """Exact workspace bytes the last build needed."""
        b = ctypes.c_size_t(0)
        _capi.check(self._lib.glm_tree_required_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def info(self) -> dict:
        inf = GlmTreeInfo()
        _capi.check(self._lib.glm_tree_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in GlmTreeInfo._fields_}

    def knn(self, k: int = 32, out=None):
        """Smoothing lengths (Sec. 3.1) of the tree's particles: float64 tensor of
        the distance from each particle to its k-th nearest other particle."""
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _capi.check(self._lib.glm_tree_knn(self._h, int(k), _ptr(out), _stream()))
        return out

    def export(self) -> dict:
        """Host copy of the boxes (preorder), the Morton order and the lists."""
        import numpy as np

        inf = self.info()
        nc, n, nl, P = inf["ncells"], inf["n"], inf["nlisted"], inf["order"] + 1
        out = dict(level=np.zeros(nc, np.int32), ix=np.zeros(nc, np.uint32), iy=np.zeros(nc, np.uint32),
                   beg=np.zeros(nc, np.int32), end=np.zeros(nc, np.int32), next=np.zeros(nc, np.int32),
                   leaf=np.zeros(nc, np.int32), lbeg=np.zeros(nc, np.int32), lend=np.zeros(nc, np.int32),
                   M=np.zeros(nc), cx=np.zeros(nc), cy=np.zeros(nc), rcut2=np.zeros(nc),
                   Q=np.zeros((nc, P, 2)), perm=np.zeros(n, np.int32), key=np.zeros(n, np.uint64),
                   list_idx=np.zeros(max(nl, 1), np.int32))
        order = ["level", "ix", "iy", "beg", "end", "next", "leaf", "lbeg", "lend", "M", "cx", "cy", "rcut2", "Q",
                 "perm", "key", "list_idx"]
        _capi.check(self._lib.glm_tree_export(self._h, *[ctypes.c_void_p(out[k].ctypes.data) for k in order]))
        out["Q"] = out["Q"][..., 0] + 1j * out["Q"][..., 1]
        out["list_idx"] = out["list_idx"][:nl]
        out.update(inf)
        return out


def stage_rays(rx, ry, workspace, stream=None):
    """glm_stage_rays: the ray staging of shoot() into `workspace` (at least
    workspace_bytes(R) bytes), on `stream` (a torch.cuda.Stream; default the
    current one), so that it can overlap the tree build; then
    shoot(..., staged=True, workspace=workspace) on the build's stream, after
    an event recorded here, walks the staged rays."""
    rx, ry = _f64(rx, "rx"), _f64(ry, "ry")
    s = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    _capi.check(_capi.load().glm_stage_rays(_ptr(rx), _ptr(ry), rx.shape[0], _ptr(workspace), workspace.numel(), s))


def shoot(tree: Tree, rx, ry, counts: bool = False, alpha_only: bool = False, fp32_alpha: bool = False,
          ordered: bool = False, out=None, workspace=None, staged: bool = False):
    """Forward walk: returns a dict of float32 tensors a1, a2 (and kappa, g1, g2
    unless alpha_only), plus counts [R, 8] int32 if requested: per ray boxes
    visited, accepted, leaf particles, list hits; per wavefront list entries
    tested, boxes accepted, leaf particles and list candidates evaluated.
    staged: the workspace holds these rays as stage_rays() left them."""
    rx, ry = _f64(rx, "rx"), _f64(ry, "ry")
    R = rx.shape[0]
    dev = rx.device
    if staged and workspace is None:
        raise ValueError("staged=True needs the workspace stage_rays() wrote")
    flags = (GLM_ALPHA_ONLY if alpha_only else 0) | (GLM_FP32_ALPHA if fp32_alpha else 0) | \
            (GLM_RAYS_ORDERED if ordered else 0) | (GLM_RAYS_STAGED if staged else 0)
    if out is None:
        names = ["a1", "a2"] if alpha_only else ["a1", "a2", "kappa", "g1", "g2"]
        out = {k: torch.empty(R, dtype=torch.float32, device=dev) for k in names}
    cnt = torch.empty((R, _capi.GLM_COUNTS), dtype=torch.int32, device=dev) if counts else None
    if workspace is None:
        workspace = torch.empty(max(workspace_bytes(R), 1), dtype=torch.uint8, device=dev)
    ws_bytes = workspace.numel() if workspace is not None else 0
    lib = _capi.load()
    _capi.check(lib.glm_shoot(tree.handle, _ptr(rx), _ptr(ry), R, _ptr(out["a1"]), _ptr(out["a2"]),
                              _ptr(out.get("kappa")), _ptr(out.get("g1")), _ptr(out.get("g2")), _ptr(cnt), flags,
                              _ptr(workspace), ws_bytes, _stream()))
    if counts:
        out["counts"] = cnt
    return out


def shoot_noalloc(tree: Tree, rx, ry, out, counts=None, alpha_only: bool = False, ordered: bool = False):
    """glm_shoot_noalloc: the forward walk with the library's static ray
    workspace (no device allocation in the call; at most GLM_NOALLOC_MAX_RAYS
    rays).  out: dict of float32 tensors a1, a2 (kappa, g1, g2 unless
    alpha_only); counts: int32 [R, 8] tensor or None."""
    rx, ry = _f64(rx, "rx"), _f64(ry, "ry")
    flags = (GLM_ALPHA_ONLY if alpha_only else 0) | (GLM_RAYS_ORDERED if ordered else 0)
    lib = _capi.load()
    _capi.check(lib.glm_shoot_noalloc(tree.handle, _ptr(rx), _ptr(ry), rx.shape[0], _ptr(out["a1"]),
                                      _ptr(out["a2"]), _ptr(out.get("kappa")), _ptr(out.get("g1")),
                                      _ptr(out.get("g2")), _ptr(counts), flags, _stream()))
    return out


def shoot_potential(tree: Tree, rx, ry, ordered: bool = False, workspace=None):
    """Deflection, lensing potential and time delay (Sec. 3.2) in one walk:
    dict of float32 tensors a1, a2, psi, tdelay (|alpha|^2 / 2 - psi)."""
    rx, ry = _f64(rx, "rx"), _f64(ry, "ry")
    R = rx.shape[0]
    out = {k: torch.empty(R, dtype=torch.float32, device=rx.device) for k in ["a1", "a2", "psi", "tdelay"]}
    if workspace is None:
        workspace = torch.empty(max(workspace_bytes(R), 1), dtype=torch.uint8, device=rx.device)
    lib = _capi.load()
    _capi.check(lib.glm_shoot_potential(tree.handle, _ptr(rx), _ptr(ry), R, _ptr(out["a1"]), _ptr(out["a2"]),
                                        _ptr(out["psi"]), _ptr(out["tdelay"]), GLM_RAYS_ORDERED if ordered else 0,
                                        _ptr(workspace), workspace.numel(), _stream()))
    return out


def smoothing_lengths(x, y, k: int = 32, leaf_size: int = 16, z=None, species=None, workspace=None):
    """Smoothing lengths of particles at (x, y) (float64 CUDA tensors): the
    distance from each to its k-th nearest other particle (Sec. 3.1).  In 2D
    without species, on a quad-tree built from the positions alone; with z
    (3D smoothing) or species (int32 ids, each species smoothed on its own),
    on the bounding-box hierarchy of glm_knn."""
    x, y = _f64(x, "x"), _f64(y, "y")
    if z is None and species is None:
        tree = Tree().build(x, y, torch.ones_like(x), None, theta=0.5, q=3.0, leaf_size=leaf_size, order=0)
        return tree.knn(k)
    return knn(x, y, k, z=z, species=species, workspace=workspace)


def knn_workspace_bytes(n: int, species: bool = False) -> int:
    nb = ctypes.c_size_t()
    _capi.check(_capi.load().glm_knn_workspace_bytes(int(n), 1 if species else 0, ctypes.byref(nb)))
    return nb.value


def knn(x, y, k: int = 32, z=None, species=None, out=None, workspace=None):
    """glm_knn: k-th nearest-neighbour distances from raw positions, 2D or 3D
    (z), optionally per species (int32 ids)."""
    x, y = _f64(x, "x"), _f64(y, "y")
    z = _f64(z, "z") if z is not None else None
    if species is not None:
        assert species.dtype == torch.int32 and species.is_contiguous() and species.is_cuda
    n = x.shape[0]
    lib = _capi.load()
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=x.device)
    if workspace is None:
        workspace = torch.empty(max(knn_workspace_bytes(n, species is not None), 1), dtype=torch.uint8,
                                device=x.device)
    _capi.check(lib.glm_knn(_ptr(x), _ptr(y), _ptr(z), _ptr(species), n, int(k), _ptr(out), _ptr(workspace),
                            workspace.numel(), _stream()))
    return out


def shoot_direct(x, y, m, s, q, rx, ry, fp64: bool = False, alpha_only: bool = False, nfw: bool = False):
    """Plain direct sum over all particles on the GPU (nfw: truncated NFW halos
    of sizes s and concentration q)."""
    if nfw and s is None:
        raise ValueError("NFW halos need their sizes s")
    x, y, m = _f64(x, "x"), _f64(y, "y"), _f64(m, "m")
    s = _f64(s, "s") if s is not None else None
    rx, ry = _f64(rx, "rx"), _f64(ry, "ry")
    R = rx.shape[0]
    dt = torch.float64 if fp64 else torch.float32
    names = ["a1", "a2"] if alpha_only else ["a1", "a2", "kappa", "g1", "g2"]
    out = {k: torch.empty(R, dtype=dt, device=rx.device) for k in names}
    arr = (ctypes.c_void_p * 5)(*[out[k].data_ptr() if k in out else None
                                  for k in ["a1", "a2", "kappa", "g1", "g2"]])
    lib = _capi.load()
    fn = lib.glm_shoot_direct_nfw if nfw else lib.glm_shoot_direct
    _capi.check(fn(_ptr(x), _ptr(y), _ptr(m), _ptr(s), x.shape[0], float(q), _ptr(rx), _ptr(ry),
                   R, 1 if fp64 else 0, arr, _stream()))
    return out


def shoot_adjoint(tree: Tree, rx, ry, ga1, ga2, dm=None, dx=None, dy=None, ds=None, ordered: bool = False,
                  workspace=None, gk=None, gg1=None, gg2=None, staged: bool = False):
    """Adjoint walk: accumulates dL/d(m, x, y, s) (float64, original particle
    order) for cotangents ga = dL/dalpha and optionally gk = dL/dkappa,
    gg = dL/dgamma (float32; any may be None).  Returns (dm, dx, dy, ds).
    staged: stage_rays() staged these rays into the start of `workspace`."""
    if staged and workspace is None:
        raise ValueError("staged=True needs the workspace stage_rays() wrote")
    rx, ry = _f64(rx, "rx"), _f64(ry, "ry")
    R = rx.shape[0]
    dev = rx.device
    f32 = lambda t: t.to(torch.float32).contiguous() if t is not None else None
    ga1, ga2, gk, gg1, gg2 = f32(ga1), f32(ga2), f32(gk), f32(gg1), f32(gg2)
    n = tree.n
    dm = torch.zeros(n, dtype=torch.float64, device=dev) if dm is None else dm
    dx = torch.zeros(n, dtype=torch.float64, device=dev) if dx is None else dx
    dy = torch.zeros(n, dtype=torch.float64, device=dev) if dy is None else dy
    ds = torch.zeros(n, dtype=torch.float64, device=dev) if ds is None else ds
    if workspace is None:
        workspace = torch.empty(max(adjoint_workspace_bytes(tree, R), 1), dtype=torch.uint8, device=dev)
    ws_bytes = workspace.numel()
    flags = (GLM_RAYS_ORDERED if ordered else 0) | (GLM_RAYS_STAGED if staged else 0)
    lib = _capi.load()
    _capi.check(lib.glm_shoot_adjoint(tree.handle, _ptr(rx), _ptr(ry), R, _ptr(ga1), _ptr(ga2), _ptr(gk), _ptr(gg1),
                                      _ptr(gg2), _ptr(dm), _ptr(dx), _ptr(dy), _ptr(ds), flags, _ptr(workspace),
                                      ws_bytes, _stream()))
    return dm, dx, dy, ds


class ShootFn(torch.autograd.Function):
    """alpha(rays; m, x, y, s) through the tree -- or (a1, a2, kappa, g1, g2)
    with lensing=True -- differentiable in the particle masses, positions and
    smoothing lengths (the tree topology and every walk decision are those of
    the forward call)."""

    @staticmethod
    def forward(ctx, rx, ry, m, x, y, s, params: dict, lensing: bool = False):
        tree = Tree().build(x.detach(), y.detach(), m.detach(), s.detach() if s is not None else None, **params)
        out = shoot(tree, rx, ry, alpha_only=not lensing)
        ctx.tree = tree
        ctx.save_for_backward(rx, ry)
        ctx.has_s = s is not None
        ctx.lensing = lensing
        if lensing:
            return out["a1"], out["a2"], out["kappa"], out["g1"], out["g2"]
        return out["a1"], out["a2"]

    @staticmethod
    def backward(ctx, g1, g2, gk=None, gg1=None, gg2=None):
        rx, ry = ctx.saved_tensors
        dm, dx, dy, ds = shoot_adjoint(ctx.tree, rx, ry, g1, g2, gk=gk, gg1=gg1, gg2=gg2)
        return None, None, dm, dx, dy, (ds if ctx.has_s else None), None, None


from .batch import (RefinementRun, autotune, autotune_batch, interp_estimate, interp_init, refine_interp_round, refine_round,  # noqa: E402
                    refine_schedule, shoot_batched, shoot_indexed)
