"""The full-size workloads on the GPU, in the launch configurations bench.py times.

The multispectral 10240 x 10240 solve (16-band guide, T = 10) is checked three ways:
- against one full FP64 oracle run of the same solve (about two minutes of host time);
- against the oracle on a two-iteration, one-step solve of the same full-size inputs,
  which isolates the first passes: the fused distance pass over 16 bands, the 40-chunk
  column pass, the streaming row pass and the update epilogue;
- by a property at the full T = 10 configuration: a constant target with uniform
  confidence is a fixed point.
The 8 x 1024^2 batch (T = 15) runs whole on the GPU; two of its images are compared with
the oracle's forward solve.
The 8 x 1024^2 forward + backward (T = 15) is checked two ways: all three gradients of
one full image against the oracle's FP64 adjoint, element by element; and directional
derivatives of the loss sum((z - r)^2) over the whole batch.  The solve is linear in the
target, so along a target direction the loss is quadratic and a central difference is
exact up to rounding; along confidence and guide directions a small step bounds the
truncation error (the distances are smooth in the guide since d >= 1).
"""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu


def note(*what):
    print("STEP", *what, flush=True)


@pytest.fixture(scope="module")
def multispectral_10240():
    note("generating the 10240 x 10240 x 16 workload")
    return dts_inputs.multispectral_10240()


def test_multispectral_10240_full_solve_matches_oracle(multispectral_10240):
    c = multispectral_10240
    note("GPU solve N=3 T=10")
    g, t, cf = (torch.from_numpy(c[k]).cuda() for k in ("guide", "target", "conf"))
    got = dts.solve(g, t, cf, c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"]).cpu().numpy()
    del g, t, cf
    torch.cuda.empty_cache()
    note("oracle solve N=3 T=10 (about two minutes)")
    ref = oracle.solve(c["guide"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], c["filter_iters"],
                       c["solver_iters"])
    err = float(np.abs(got - ref).max())
    note("max abs err", err)
    assert err <= 1e-4


def test_multispectral_10240_two_passes_match_oracle(multispectral_10240):
    c = multispectral_10240
    N, T = 2, 1
    note("GPU solve N=2 T=1")
    g, t, cf = (torch.from_numpy(c[k]).cuda() for k in ("guide", "target", "conf"))
    got = dts.solve(g, t, cf, c["sigma_s"], c["sigma_r"], N, T).cpu().numpy()
    del g, t, cf
    torch.cuda.empty_cache()
    note("oracle solve N=2 T=1")
    ref = oracle.solve(c["guide"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], N, T)
    err = float(np.abs(got - ref).max())
    note("max abs err", err)
    assert err <= 1e-4


def test_multispectral_10240_constant_target_is_a_fixed_point(multispectral_10240):
    c = multispectral_10240
    note("GPU solve N=3 T=10, constant target")
    g = torch.from_numpy(c["guide"]).cuda()
    t = torch.full((1,) + c["guide"].shape[1:], 0.37, dtype=torch.float32, device="cuda")
    cf = torch.from_numpy(c["conf"]).cuda()
    z = dts.solve(g, t, cf, c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"])
    dev = float((z - 0.37).abs().max())
    note("max deviation", dev)
    assert dev <= 1e-6


def test_rgb_batch_8x1024_forward_matches_oracle():
    c = dts_inputs.rgb_batch_8x1024()
    note("8 x 1024^2 forward, T=15")
    g, t, cf = (torch.from_numpy(c[k]).cuda() for k in ("guide", "target", "conf"))
    got = dts.solve(g, t, cf, c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"]).cpu().numpy()
    for b in (0, 7):
        note("oracle forward of image", b)
        ref = oracle.solve(c["guide"][b], c["target"][b], c["conf"][b], c["sigma_s"], c["sigma_r"],
                           c["filter_iters"], c["solver_iters"])
        err = float(np.abs(got[b] - ref).max())
        note("image", b, "max abs err", err)
        assert err <= 1e-4


def _loss(z, r):
    return float(((z.double() - r.double()) ** 2).sum())


def test_rgb_batch_8x1024_gradients_match_directional_derivatives():
    c = dts_inputs.rgb_batch_8x1024()
    note("8 x 1024^2 forward + backward")
    g, t, cf, r = (torch.from_numpy(c[k]).cuda() for k in ("guide", "target", "conf", "ref"))
    ss, sr, N, T = c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"]
    z, ck = dts.solve(g, t, cf, ss, sr, N, T, checkpoints=True)
    gt, gc, gg = dts.solve_backward(g, t, cf, ck, (2.0 * (z - r)).contiguous(), ss, sr, N, T)
    gen = torch.Generator(device="cuda").manual_seed(5)
    # target: exact central difference (the loss is quadratic in t)
    v = torch.randn(t.shape, generator=gen, device="cuda")
    eps = 1e-2
    fd = (_loss(dts.solve(g, t + eps * v, cf, ss, sr, N, T), r)
          - _loss(dts.solve(g, t - eps * v, cf, ss, sr, N, T), r)) / (2 * eps)
    an = float((gt.double() * v.double()).sum())
    note("target: adjoint", an, "central difference", fd)
    assert abs(an - fd) <= 1e-3 * abs(fd)
    # confidence: a small step keeps c inside [0.1, 1] and the truncation error small
    # (measured at this step: 4e-5 relative; smaller steps are dominated by the fp32
    # rounding of the forward solves)
    v = torch.rand(cf.shape, generator=gen, device="cuda") - 0.5
    eps = 3e-3
    fd = (_loss(dts.solve(g, t, cf + eps * v, ss, sr, N, T), r)
          - _loss(dts.solve(g, t, cf - eps * v, ss, sr, N, T), r)) / (2 * eps)
    an = float((gc.double() * v.double()).sum())
    note("confidence: adjoint", an, "central difference", fd)
    assert abs(an - fd) <= 1e-3 * abs(fd)
    # guide: the loss is smooth in the guide (d >= 1).  Truncation grows above this step
    # and the forward's fp32 rounding below it, so the best central difference agrees to
    # about 9e-4 (measured); the element-wise FP64 comparison above is the 1e-3 check.
    v = torch.rand(g.shape, generator=gen, device="cuda") - 0.5
    eps = 1e-3
    fd = (_loss(dts.solve(g + eps * v, t, cf, ss, sr, N, T), r)
          - _loss(dts.solve(g - eps * v, t, cf, ss, sr, N, T), r)) / (2 * eps)
    an = float((gg.double() * v.double()).sum())
    note("guide: adjoint", an, "central difference", fd)
    assert abs(an - fd) <= 2e-3 * abs(fd)


def test_rgb_batch_8x1024_tape_path_matches_the_recomputing_one():
    """The forward + backward the benchmark times (pass outputs kept in a tape, no
    recomputation) against the recomputing path at full size, bit for bit; the
    recomputing path is checked against the oracle below."""
    c = dts_inputs.rgb_batch_8x1024()
    ss, sr, N, T = c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"]
    note("8 x 1024^2 forward + backward, tape against recomputation")
    g, t, cf, r = (torch.from_numpy(c[k]).cuda() for k in ("guide", "target", "conf", "ref"))
    z, ck, tp = dts.solve(g, t, cf, ss, sr, N, T, tape=True)
    go = (2.0 * (z - r)).contiguous()
    got = dts.solve_backward(g, t, cf, ck, go, ss, sr, N, T, tape=tp)
    del tp
    ref = dts.solve_backward(g, t, cf, ck, go, ss, sr, N, T)
    for name, a, b in zip(("target", "conf", "guide"), got, ref):
        assert torch.equal(a, b), name


def test_rgb_batch_8x1024_gradients_match_oracle_on_one_image():
    c = dts_inputs.rgb_batch_8x1024()
    ss, sr, N, T = c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"]
    note("8 x 1024^2 forward + backward on the GPU")
    g, t, cf, r = (torch.from_numpy(c[k]).cuda() for k in ("guide", "target", "conf", "ref"))
    z, ck = dts.solve(g, t, cf, ss, sr, N, T, checkpoints=True)
    gt, gc, gg = dts.solve_backward(g, t, cf, ck, (2.0 * (z - r)).contiguous(), ss, sr, N, T)
    got = {k: v[3].double().cpu().numpy() for k, v in (("target", gt), ("conf", gc), ("guide", gg))}
    del z, ck, gt, gc, gg
    b = 3
    note("oracle forward + adjoint of image", b, "(about a minute)")
    zr = oracle.solve(c["guide"][b], c["target"][b], c["conf"][b], ss, sr, N, T)
    rt, rc, rg = oracle.solve_backward(c["guide"][b], c["target"][b], c["conf"][b], ss, sr,
                                       2.0 * (zr - c["ref"][b]), N, T)
    for name, ref in (("target", rt), ("conf", rc), ("guide", rg)):
        err = got[name] - ref
        rel = float(np.linalg.norm(err) / np.linalg.norm(ref))
        elem = float(np.abs(err).max())
        floor = 1e-3 * float(np.abs(ref).max())
        note(name, "rel L2", rel, "max abs", elem, "floor", floor)
        assert rel <= 1e-3, (name, rel)
        assert elem <= floor, (name, elem, floor)
