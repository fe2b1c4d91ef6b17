"""glm_shoot_noalloc (the walk with the library's static ray workspace) against
glm_shoot with a caller workspace, through the C ABI: identical outputs and
counts on calls in a row with shrinking ray sets (the static array keeps the
previous call's contents), and sizes beyond GLM_NOALLOC_MAX_RAYS refused."""
import numpy as np
import pytest

import synth
from gpu_helpers import dev, say

pytestmark = pytest.mark.gpu

NAMES = ["a1", "a2", "kappa", "g1", "g2"]


def test_noalloc_matches_shoot_on_shrinking_calls():
    import paper_1312_1128_amd as g
    import torch
    from paper_1312_1128_amd import _capi

    lens = synth.nfw_halo(20000, 771)
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), theta=0.3, q=lens.q, leaf_size=8,
                          order=6)
    big_x, big_y = synth.uniform_points(_capi.GLM_NOALLOC_MAX_RAYS, 773)
    for nr in (_capi.GLM_NOALLOC_MAX_RAYS, 300_001, 4_999):
        say(f"[gpu] noalloc walk, {nr} rays")
        rx, ry = dev(big_x[:nr]), dev(big_y[:nr])
        out = {k: torch.full((nr,), float("nan"), dtype=torch.float32, device="cuda") for k in NAMES}
        cnt = torch.full((nr, _capi.GLM_COUNTS), -1, dtype=torch.int32, device="cuda")
        g.shoot_noalloc(tree, rx, ry, out, counts=cnt)
        ref = g.shoot(tree, rx, ry, counts=True)
        torch.cuda.synchronize()
        for k in NAMES:
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=k)
        np.testing.assert_array_equal(cnt.cpu().numpy(), ref["counts"].cpu().numpy())
        # alpha only, without counts
        oa = {k: torch.empty(nr, dtype=torch.float32, device="cuda") for k in ["a1", "a2"]}
        g.shoot_noalloc(tree, rx, ry, oa, alpha_only=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(oa["a1"].cpu().numpy(), ref["a1"].cpu().numpy())
        del rx, ry, out, cnt, ref, oa


def test_noalloc_rejects_oversize_and_bad_arguments():
    import paper_1312_1128_amd as g
    import torch
    from paper_1312_1128_amd import _capi

    lib = _capi.load()
    lens = synth.point_masses(500, 775)
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), None, theta=0.5, leaf_size=8, order=2)
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    o = torch.zeros(4, dtype=torch.float32, device="cuda")
    p = lambda t: t.data_ptr()
    rc = lib.glm_shoot_noalloc(tree.handle, p(x), p(x), _capi.GLM_NOALLOC_MAX_RAYS + 1, p(o), p(o), p(o), p(o),
                               p(o), None, 0, None)
    assert rc == _capi.GLM_EINVAL and b"GLM_NOALLOC_MAX_RAYS" in lib.glm_last_error()
    assert lib.glm_shoot_noalloc(tree.handle, p(x), p(x), -1, p(o), p(o), p(o), p(o), p(o), None, 0,
                                 None) == _capi.GLM_EINVAL
    unbuilt = g.Tree()
    assert lib.glm_shoot_noalloc(unbuilt.handle, p(x), p(x), 4, p(o), p(o), p(o), p(o), p(o), None, 0,
                                 None) == _capi.GLM_ESTATE
    # zero rays: nothing to do
    assert lib.glm_shoot_noalloc(tree.handle, p(x), p(x), 0, p(o), p(o), p(o), p(o), p(o), None, 0, None) == 0
