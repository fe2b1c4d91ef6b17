"""Shared helpers of the GPU parity tests (the GPU side goes through the C ABI
via the package's ctypes binding; the reference side is the CPU oracle)."""
import sys

import numpy as np


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def build(lens, theta, leaf, order, flags=0):
    import paper_1312_1128_amd as g

    return g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), theta=theta, q=lens.q,
                          leaf_size=leaf, order=order, flags=flags)


def shoot(tree, rx, ry, counts=False, **kw):
    import paper_1312_1128_amd as g
    import torch

    out = g.shoot(tree, dev(rx), dev(ry), counts=counts, **kw)
    torch.cuda.synchronize()
    names = [k for k in ["a1", "a2", "kappa", "g1", "g2"] if k in out]
    res = np.stack([out[k].double().cpu().numpy() for k in names], axis=1)
    if counts:
        return res, out["counts"].cpu().numpy()
    return res


def rel_err(got, ref):
    """Per-ray fractional errors of alpha, kappa, gamma (the paper's measure:
    |delta alpha| / |alpha|)."""
    ea = np.linalg.norm(got[:, 0:2] - ref[:, 0:2], axis=1) / np.linalg.norm(ref[:, 0:2], axis=1)
    ek = np.abs(got[:, 2] - ref[:, 2]) / np.abs(ref[:, 2])
    eg = np.linalg.norm(got[:, 3:5] - ref[:, 3:5], axis=1) / np.linalg.norm(ref[:, 3:5], axis=1)
    return ea, ek, eg


def stats(name, e):
    e = e[np.isfinite(e)]
    say(f"  {name}: median {np.median(e):.3e}  p99.9 {np.quantile(e, 0.999):.3e}  max {e.max():.3e}")
