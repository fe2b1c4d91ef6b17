"""GPU direct sum (FP64 and FP32) against oracle A, element by element."""
import numpy as np
import pytest

import synth
from gpu_helpers import dev, rel_err, say, stats

pytestmark = pytest.mark.gpu


def run_direct(lens, rx, ry, fp64):
    import paper_1312_1128_amd as g
    import torch

    out = g.shoot_direct(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), lens.q, dev(rx), dev(ry), fp64=fp64)
    torch.cuda.synchronize()
    return np.stack([out[k].double().cpu().numpy() for k in ["a1", "a2", "kappa", "g1", "g2"]], axis=1)


@pytest.mark.parametrize("which", ["point_masses_1k", "blobs_3k", "nfw_50k"])
def test_direct_matches_oracle(ora, which):
    if which == "point_masses_1k":
        lens, rx, ry = synth.workload_point_masses_1k()
    elif which == "blobs_3k":
        lens = synth.gaussian_blobs(3000, 61, s_lo=0.001, s_hi=0.2)
        lens.s[::4] = 0.0
        rx, ry = synth.uniform_points(3001, 62)
    else:
        lens = synth.nfw_halo(50000, 63)
        rx, ry = synth.ray_grid(50)
    say(f"[gpu] direct {which}: n={lens.n} rays={rx.size}")
    ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry)
    d64 = run_direct(lens, rx, ry, True)
    ea, ek, eg = rel_err(d64, ref)
    stats("fp64 alpha", ea)
    assert ea.max() <= 1e-10 and eg.max() <= 1e-10
    if lens.s.max() > 0:
        ok = ref[:, 2] != 0
        assert np.all(ek[ok] <= 1e-10)
    d32 = run_direct(lens, rx, ry, False)
    ea, ek, eg = rel_err(d32, ref)
    stats("fp32 alpha", ea)
    stats("fp32 gamma", eg)
    assert np.quantile(ea, 0.999) < 1e-5
