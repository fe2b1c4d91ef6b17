"""glm_stage_rays on a second stream, then glm_shoot with GLM_RAYS_STAGED on the
build's stream, against glm_shoot staging its own rays: identical outputs and
counts, for a ray set large enough for one wavefront per 64-ray group and for
one small enough for the split walk (several wavefronts per group, which also
reads the staged rays' bounding box); and the flag's misuses refused."""
import numpy as np
import pytest

import synth
from gpu_helpers import dev, say

pytestmark = pytest.mark.gpu

NAMES = ["a1", "a2", "kappa", "g1", "g2"]


def test_staged_rays_on_a_second_stream_match_shoot():
    import paper_1312_1128_amd as g
    import torch

    lens = synth.nfw_halo(50000, 881)
    x, y, m, s = dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s)
    px, py = synth.uniform_points(1_500_000, 883)
    side = torch.cuda.Stream()
    tree = g.Tree()
    for nr in (1_500_000, 3_001):
        say(f"[gpu] staged rays on a side stream, {nr} rays")
        rx, ry = dev(px[:nr]), dev(py[:nr])
        ws = torch.empty(g.workspace_bytes(nr), dtype=torch.uint8, device="cuda")
        main = torch.cuda.current_stream()
        side.wait_stream(main)  # inputs and workspace ready
        with torch.cuda.stream(side):
            g.stage_rays(rx, ry, ws, stream=side)
            staged = torch.cuda.Event()
            staged.record(side)
        tree.build(x, y, m, s, theta=0.3, q=lens.q, leaf_size=16, order=8)  # on the main stream meanwhile
        main.wait_event(staged)
        got = g.shoot(tree, rx, ry, counts=True, workspace=ws, staged=True)
        ref = g.shoot(tree, rx, ry, counts=True)
        torch.cuda.synchronize()
        for k in NAMES:
            np.testing.assert_array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=k)
        np.testing.assert_array_equal(got["counts"].cpu().numpy(), ref["counts"].cpu().numpy())


def test_staged_flag_misuse_refused():
    import ctypes

    import paper_1312_1128_amd as g
    import torch
    from paper_1312_1128_amd import _capi

    lens = synth.nfw_halo(2000, 887)
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), theta=0.3, q=lens.q, leaf_size=8,
                          order=4)
    rx, ry = dev(np.linspace(-0.2, 0.2, 500)), dev(np.zeros(500))
    ws = torch.empty(g.workspace_bytes(500), dtype=torch.uint8, device="cuda")
    out = {k: torch.empty(500, dtype=torch.float32, device="cuda") for k in NAMES}
    lib = _capi.load()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [tree.handle, p(rx), p(ry), 500] + [p(out[k]) for k in NAMES] + [None]
    assert lib.glm_shoot(*args, _capi.GLM_RAYS_STAGED | _capi.GLM_RAYS_ORDERED, p(ws), ws.numel(), st) == \
        _capi.GLM_EINVAL
    assert lib.glm_stage_rays(p(rx), p(ry), 500, p(ws), 16, st) == _capi.GLM_ENOMEM
    assert lib.glm_stage_rays(None, p(ry), 500, p(ws), ws.numel(), st) == _capi.GLM_EINVAL
    assert lib.glm_shoot_noalloc(*args, _capi.GLM_RAYS_STAGED, st) == _capi.GLM_EINVAL
    assert lib.glm_stage_rays(p(rx), p(ry), 0, None, 0, st) == _capi.GLM_OK
    with pytest.raises(ValueError):
        g.shoot(tree, rx, ry, staged=True)


def test_adjoint_with_staged_rays_matches():
    """The forward alpha walk and the adjoint on rays staged once into the
    adjoint's workspace equal the calls that stage their own (the adjoint to
    FP64 rounding: its atomics add in no fixed order)."""
    import paper_1312_1128_amd as g
    import torch

    lens = synth.nfw_halo(30000, 891)
    x, y, m, s = dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s)
    tree = g.Tree().build(x, y, m, s, theta=0.3, q=lens.q, leaf_size=16, order=8)
    px, py = synth.uniform_points(200_000, 893)
    rx, ry = dev(px), dev(py)
    gen = torch.Generator(device="cpu").manual_seed(5)
    ga1 = torch.randn(rx.numel(), generator=gen).float().cuda()
    ga2 = torch.randn(rx.numel(), generator=gen).float().cuda()
    wsa = torch.empty(g.adjoint_workspace_bytes(tree, rx.numel()), dtype=torch.uint8, device="cuda")
    g.stage_rays(rx, ry, wsa)
    fa = g.shoot(tree, rx, ry, alpha_only=True, workspace=wsa, staged=True)
    fr = g.shoot(tree, rx, ry, alpha_only=True)
    got = g.shoot_adjoint(tree, rx, ry, ga1, ga2, workspace=wsa, staged=True)
    ref = g.shoot_adjoint(tree, rx, ry, ga1, ga2)
    torch.cuda.synchronize()
    for k in ("a1", "a2"):
        np.testing.assert_array_equal(fa[k].cpu().numpy(), fr[k].cpu().numpy(), err_msg=k)
    for a, b, name in zip(got, ref, "mxys"):
        # the bound of the repeated-adjoint test: FP64 sums in a different order
        np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-9,
                                   atol=1e-12 * float(b.abs().max()), err_msg=name)
