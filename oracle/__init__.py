"""CPU oracle for the lensing hot path -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes) to the plain FP64 C implementations in this folder:

* oracle A (``direct``, ``direct_grad``): brute-force superposition of every
  particle, the theta_force = 0 limit of Sec. 5.1;
* oracle B (``Tree``): the modified quad-tree solver of Sec. 3.2, recursive and
  in FP64, with per-ray interaction counts and a decision tape for frozen-walk
  finite differences;
* ``knn``: smoothing lengths (Sec. 3.1), the distance to the k-th nearest
  other particle, by brute force.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ["direct.c", "tree.c", "knn.c", "nfw.c"]

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, no FP contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    d = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    vp = ctypes.c_void_p
    lib.ora_direct.argtypes = [d, d, d, d, i64, ctypes.c_double, d, d, i64, d, d, d, d, d, ctypes.c_int]
    lib.ora_direct_grad.argtypes = [d, d, d, d, i64, ctypes.c_double, d, d, i64, d, d, d, d, d, d,
                                    ctypes.c_int]
    lib.ora_unit_terms.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, d]
    lib.ora_kernel_norm.argtypes = [ctypes.c_double]
    lib.ora_kernel_norm.restype = ctypes.c_double
    lib.ora_knn.argtypes = [d, d, i64, ctypes.c_int, d, ctypes.c_int]
    for fn in ("ora_nfw_F", "ora_nfw_f", "ora_nfw_g"):
        getattr(lib, fn).argtypes = [ctypes.c_double]
        getattr(lib, fn).restype = ctypes.c_double
    lib.ora_nfw_terms.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, d]
    lib.ora_direct_nfw.argtypes = [d, d, d, d, i64, ctypes.c_double, d, d, i64, d, d, d, d, d, ctypes.c_int]
    lib.ora_tree_build_nfw.argtypes = [d, d, d, d, i64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int]
    lib.ora_tree_build_nfw.restype = vp
    lib.ora_tree_shoot_psi.restype = ctypes.c_int
    lib.ora_unit_psi.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int]
    lib.ora_nfw_df.argtypes = [ctypes.c_double]
    lib.ora_nfw_df.restype = ctypes.c_double
    lib.ora_nfw_dterms.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, d]
    lib.ora_nfw_H.argtypes = [ctypes.c_double]
    lib.ora_nfw_H.restype = ctypes.c_double
    lib.ora_nfw_psi.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int]
    lib.ora_nfw_psi.restype = ctypes.c_double
    lib.ora_direct_nfw_psi.argtypes = [d, d, d, d, i64, ctypes.c_double, d, d, i64, d, ctypes.c_int]
    lib.ora_unit_psi.restype = ctypes.c_double
    lib.ora_ein.argtypes = [ctypes.c_double]
    lib.ora_ein.restype = ctypes.c_double
    lib.ora_direct_psi.argtypes = [d, d, d, d, i64, ctypes.c_double, d, d, i64, d, ctypes.c_int]
    lib.ora_tree_shoot_psi.argtypes = [vp, d, d, i64, d, ctypes.c_int]
    lib.ora_knn_at.argtypes = [d, d, i64, ctypes.c_int, vp, i64, d, ctypes.c_int]
    lib.ora_knn_ex.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int, vp, i64, d, ctypes.c_int]
    lib.ora_tree_build.argtypes = [d, d, d, d, i64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int]
    lib.ora_tree_build.restype = vp
    lib.ora_tree_free.argtypes = [vp]
    lib.ora_tree_ncells.argtypes = [vp]
    lib.ora_tree_ncells.restype = i64
    lib.ora_tree_root.argtypes = [vp, d]
    lib.ora_tree_export.argtypes = [vp] + [vp] * 12
    lib.ora_tree_members.argtypes = [vp, i64, vp]
    lib.ora_tree_members.restype = i64
    lib.ora_tree_list.argtypes = [vp, i64, vp]
    lib.ora_tree_list.restype = i64
    lib.ora_tree_shoot.argtypes = [vp, d, d, i64, d, d, d, d, d, vp, ctypes.c_int]
    lib.ora_tree_record.argtypes = [vp, d, d, i64]
    lib.ora_tree_set_particles.argtypes = [vp, d, d, d, d]
    lib.ora_tree_shoot_frozen.argtypes = [vp, d, d, i64, d, d, d, d, d]
    lib.ora_tree_shoot_frozen.restype = ctypes.c_int
    lib.ora_tree_grad.argtypes = [vp, d, d, i64, d, d, d, d, d, d]
    lib.ora_tree_grad_kg.argtypes = [vp, d, d, i64, d, d, d, d, d, d, d, d, d]
    lib.ora_tree_grad_kg.restype = ctypes.c_int
    lib.ora_direct_grad_kg.argtypes = [d, d, d, d, i64, ctypes.c_double, d, d, i64, d, d, d, d, d, d, d, d, d,
                                       ctypes.c_int]
    lib.ora_unit_dterms.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, d]
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def kernel_norm(q: float) -> float:
    return _load().ora_kernel_norm(q)


def unit_terms(d1: float, d2: float, s: float, q: float, inside: bool) -> np.ndarray:
    out = np.zeros(7)
    _load().ora_unit_terms(d1, d2, s, q, int(inside), _p(out))
    return out


def direct(x, y, m, s, q, rx, ry, threads: int | None = None) -> np.ndarray:
    """Oracle A.  Returns an (R, 5) array: alpha1, alpha2, kappa, gamma1, gamma2."""
    lib = _load()
    x, y, m = _f64(x), _f64(y), _f64(m)
    s = _f64(s) if s is not None else np.zeros_like(x)
    rx, ry = _f64(rx), _f64(ry)
    nr = rx.shape[0]
    out = [np.zeros(nr) for _ in range(5)]
    lib.ora_direct(_p(x), _p(y), _p(m), _p(s), x.shape[0], float(q), _p(rx), _p(ry), nr,
                   *[_p(o) for o in out], threads or default_threads())
    return np.stack(out, axis=1)


def nfw_F(x: float) -> float:
    return _load().ora_nfw_F(x)


def nfw_f(x: float) -> float:
    return _load().ora_nfw_f(x)


def nfw_g(x: float) -> float:
    return _load().ora_nfw_g(x)


def nfw_terms(d1: float, d2: float, R: float, c: float, inside: bool) -> np.ndarray:
    out = np.zeros(7)
    _load().ora_nfw_terms(d1, d2, R, c, int(inside), _p(out))
    return out


def direct_nfw(x, y, m, R, c, rx, ry, threads: int | None = None) -> np.ndarray:
    """Oracle A for truncated NFW halos (size R, concentration c)."""
    lib = _load()
    x, y, m, R = _f64(x), _f64(y), _f64(m), _f64(R)
    rx, ry = _f64(rx), _f64(ry)
    nr = rx.shape[0]
    out = [np.zeros(nr) for _ in range(5)]
    lib.ora_direct_nfw(_p(x), _p(y), _p(m), _p(R), x.shape[0], float(c), _p(rx), _p(ry), nr,
                       *[_p(o) for o in out], threads or default_threads())
    return np.stack(out, axis=1)


def unit_psi(d1: float, d2: float, s: float, q: float, inside: bool) -> float:
    return _load().ora_unit_psi(d1, d2, s, q, int(inside))


def ein(z: float) -> float:
    return _load().ora_ein(z)


def nfw_df(x: float) -> float:
    return _load().ora_nfw_df(x)


def nfw_dterms(d1: float, d2: float, R: float, c: float, inside: bool) -> np.ndarray:
    out = np.zeros(9)
    _load().ora_nfw_dterms(float(d1), float(d2), float(R), float(c), int(inside), _p(out))
    return out


def nfw_H(x: float) -> float:
    return _load().ora_nfw_H(x)


def nfw_psi(d1: float, d2: float, R: float, c: float, inside: bool) -> float:
    return _load().ora_nfw_psi(d1, d2, R, c, int(inside))


def direct_nfw_psi(x, y, m, R, c, rx, ry, threads: int | None = None) -> np.ndarray:
    """Oracle A for the potential of truncated NFW halos (sizes R, concentration c)."""
    lib = _load()
    x, y, m, R = _f64(x), _f64(y), _f64(m), _f64(R)
    rx, ry = _f64(rx), _f64(ry)
    out = np.zeros(rx.shape[0])
    lib.ora_direct_nfw_psi(_p(x), _p(y), _p(m), _p(R), x.shape[0], float(c), _p(rx), _p(ry), rx.shape[0], _p(out),
                           threads or default_threads())
    return out


def direct_psi(x, y, m, s, q, rx, ry, threads: int | None = None) -> np.ndarray:
    """Oracle A for the lensing potential psi (alpha = grad psi)."""
    lib = _load()
    x, y, m = _f64(x), _f64(y), _f64(m)
    s = _f64(s) if s is not None else np.zeros_like(x)
    rx, ry = _f64(rx), _f64(ry)
    out = np.zeros(rx.shape[0])
    lib.ora_direct_psi(_p(x), _p(y), _p(m), _p(s), x.shape[0], float(q), _p(rx), _p(ry), rx.shape[0], _p(out),
                       threads or default_threads())
    return out


def knn(x, y, k: int = 32, at=None, threads: int | None = None, z=None, species=None) -> np.ndarray:
    """Smoothing lengths: distance from each particle (or from the particles
    listed in ``at``) to its k-th nearest other particle; in 3D when z is
    given, and among the particle's own species when species is given."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    zz = _f64(z) if z is not None else None
    sp = np.ascontiguousarray(species, dtype=np.int32) if species is not None else None
    q = np.ascontiguousarray(at, dtype=np.int64) if at is not None else None
    out = np.zeros(q.shape[0] if q is not None else x.shape[0])
    rc = lib.ora_knn_ex(_p(x), _p(y), _p(zz) if zz is not None else None,
                        sp.ctypes.data if sp is not None else None, x.shape[0], int(k),
                        q.ctypes.data if q is not None else None, out.shape[0], _p(out),
                        threads or default_threads())
    if rc != 0:
        raise ValueError("need 1 <= k <= n - 1 and at least k + 1 particles of every queried species")
    return out


def _cot(gk, gg):
    """kappa and gamma cotangents as (gk, gg1, gg2) arrays or None."""
    k = _f64(gk) if gk is not None else None
    if gg is None:
        return k, None, None
    gg = np.ascontiguousarray(gg, dtype=np.float64)
    return k, _f64(gg[:, 0]), _f64(gg[:, 1])


def _pn(a):
    return _p(a) if a is not None else None


def direct_grad(x, y, m, s, q, rx, ry, ga, threads: int | None = None, gk=None, gg=None):
    """Oracle A adjoint for L = sum_r ga_r . alpha_r (+ gk_r kappa_r + gg_r . gamma_r
    when gk [nr] / gg [nr, 2] are given).  Returns (dm, dx, dy, ds)."""
    lib = _load()
    x, y, m = _f64(x), _f64(y), _f64(m)
    s = _f64(s) if s is not None else np.zeros_like(x)
    rx, ry = _f64(rx), _f64(ry)
    ga = np.ascontiguousarray(ga, dtype=np.float64)
    g1, g2 = _f64(ga[:, 0]), _f64(ga[:, 1])
    k, h1, h2 = _cot(gk, gg)
    n = x.shape[0]
    out = [np.zeros(n) for _ in range(4)]
    lib.ora_direct_grad_kg(_p(x), _p(y), _p(m), _p(s), n, float(q), _p(rx), _p(ry), rx.shape[0],
                           _p(g1), _p(g2), _pn(k), _pn(h1), _pn(h2), *[_p(o) for o in out],
                           threads or default_threads())
    return tuple(out)


def unit_dterms(d1: float, d2: float, s: float, q: float, inside: bool) -> np.ndarray:
    """Per unit mass: d(kappa, gamma1, gamma2) / d(d1, d2) and / d s."""
    out = np.zeros(9)
    _load().ora_unit_dterms(float(d1), float(d2), float(s), float(q), int(inside), _p(out))
    return out


class Tree:
    """Oracle B: FP64 reference quad-tree (Sec. 3.2)."""

    def __init__(self, x, y, m, s, q=3.0, theta=0.5, leaf_size=8, order=2, nfw: bool = False):
        """nfw: the particles are truncated NFW halos, s their sizes and q
        their concentration."""
        lib = _load()
        self._keep = [_f64(x), _f64(y), _f64(m),
                      _f64(s) if s is not None else np.zeros(np.asarray(x).shape[0])]
        self.n = self._keep[0].shape[0]
        self.q, self.theta, self.leaf_size, self.order = float(q), float(theta), int(leaf_size), int(order)
        build = lib.ora_tree_build_nfw if nfw else lib.ora_tree_build
        self._h = build(*[_p(a) for a in self._keep], self.n, self.q, self.theta, self.leaf_size, self.order)
        if not self._h:
            raise ValueError("oracle tree build rejected its arguments")
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_tree_free(h)
            self._h = None

    @property
    def ncells(self) -> int:
        return int(self._lib.ora_tree_ncells(self._h))

    def root(self):
        out = np.zeros(3)
        self._lib.ora_tree_root(self._h, _p(out))
        return out

    def export(self) -> dict:
        nc, P = self.ncells, self.order + 1
        arr = dict(level=np.zeros(nc, np.int32), ix=np.zeros(nc, np.uint32), iy=np.zeros(nc, np.uint32),
                   np=np.zeros(nc, np.int32), leaf=np.zeros(nc, np.int32), nl=np.zeros(nc, np.int32),
                   next=np.zeros(nc, np.int64), M=np.zeros(nc), cx=np.zeros(nc), cy=np.zeros(nc),
                   rcut2=np.zeros(nc), Q=np.zeros((nc, P, 2)))
        order = ["level", "ix", "iy", "np", "leaf", "nl", "next", "M", "cx", "cy", "rcut2", "Q"]
        self._lib.ora_tree_export(self._h, *[arr[k].ctypes.data for k in order])
        arr["Q"] = arr["Q"][..., 0] + 1j * arr["Q"][..., 1]
        return arr

    def members(self, cell: int) -> np.ndarray:
        out = np.zeros(self.n, np.int32)
        k = self._lib.ora_tree_members(self._h, int(cell), out.ctypes.data)
        return out[:k].copy()

    def list_of(self, cell: int) -> np.ndarray:
        out = np.zeros(self.n, np.int32)
        k = self._lib.ora_tree_list(self._h, int(cell), out.ctypes.data)
        return out[:k].copy()

    def shoot(self, rx, ry, counts: bool = False, threads: int | None = None):
        rx, ry = _f64(rx), _f64(ry)
        nr = rx.shape[0]
        out = [np.zeros(nr) for _ in range(5)]
        cnt = np.zeros((nr, 5), np.int64) if counts else None
        self._lib.ora_tree_shoot(self._h, _p(rx), _p(ry), nr, *[_p(o) for o in out],
                                 cnt.ctypes.data if counts else None, threads or default_threads())
        res = np.stack(out, axis=1)
        return (res, cnt) if counts else res

    def shoot_psi(self, rx, ry, threads: int | None = None):
        """The potential psi along the same walk."""
        rx, ry = _f64(rx), _f64(ry)
        out = np.zeros(rx.shape[0])
        self._lib.ora_tree_shoot_psi(self._h, _p(rx), _p(ry), rx.shape[0], _p(out), threads or default_threads())
        return out

    def record(self, rx, ry):
        rx, ry = _f64(rx), _f64(ry)
        self._lib.ora_tree_record(self._h, _p(rx), _p(ry), rx.shape[0])

    def set_particles(self, x, y, m, s):
        self._keep = [_f64(x), _f64(y), _f64(m), _f64(s)]
        self._lib.ora_tree_set_particles(self._h, *[_p(a) for a in self._keep])

    def shoot_frozen(self, rx, ry):
        rx, ry = _f64(rx), _f64(ry)
        nr = rx.shape[0]
        out = [np.zeros(nr) for _ in range(5)]
        rc = self._lib.ora_tree_shoot_frozen(self._h, _p(rx), _p(ry), nr, *[_p(o) for o in out])
        if rc != 0:
            raise ValueError("record() the same rays first")
        return np.stack(out, axis=1)

    def grad(self, rx, ry, ga, gk=None, gg=None):
        rx, ry = _f64(rx), _f64(ry)
        ga = np.ascontiguousarray(ga, dtype=np.float64)
        g1, g2 = _f64(ga[:, 0]), _f64(ga[:, 1])
        k, h1, h2 = _cot(gk, gg)
        out = [np.zeros(self.n) for _ in range(4)]
        rc = self._lib.ora_tree_grad_kg(self._h, _p(rx), _p(ry), rx.shape[0], _p(g1), _p(g2), _pn(k), _pn(h1),
                                        _pn(h2), *[_p(o) for o in out])
        if rc != 0:
            raise ValueError("bad arguments")
        return tuple(out)
