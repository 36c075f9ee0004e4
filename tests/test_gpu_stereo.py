"""Stereo refinement (Eq. (11)) on the GPU against the FP64 oracle.

Where the iteration is contractive (the Charbonnier target term's curvature 1/eps times
step * c stays below 2, here eps = 2 px), GPU and oracle agree to 1e-4 of the disparity
range.  With the paper's eps = 0.001 the descent step on that term is about 990 times
its curvature limit: at pixels where |z - t| < eps the iteration amplifies any rounding
difference until the Charbonnier derivative saturates, so two correct implementations
with different rounding part ways there.  For that setting the tests check one exact
step (T = 1) tightly and bound the share of diverging pixels over the full 20 steps."""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu

CASES = [
    # H, W, Cg, d_max, T, eps, batch
    (40, 64, 3, 8.0, 5, 2.0, 1),
    (1, 300, 3, 16.0, 5, 2.0, 1),
    (97, 131, 1, 12.0, 4, 2.0, 2),
    (200, 90, 3, 20.0, 5, 2.0, 1),
    (33, 1, 3, 4.0, 3, 2.0, 1),
    (64, 257, 3, 16.0, 1, 0.001, 1),   # one step at the paper's epsilon
    (97, 131, 3, 12.0, 1, 0.001, 2),
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_Cg{c[2]}_d{c[3]:g}_T{c[4]}_eps{c[5]:g}_B{c[6]}" for c in CASES])
def test_stereo_matches_oracle(case):
    H, W, Cg, d_max, T, eps, B = case
    print("CASE stereo", case, flush=True)
    cs = [dts_inputs.stereo_case(500 + 7 * b + H, H, W, Cg, d_max=d_max, T=T, eps=eps) for b in range(B)]
    stack = lambda key: np.stack([c[key] for c in cs])
    c0 = cs[0]
    got = dts.solve_stereo(dev(stack("left")), dev(stack("right")), dev(stack("target")), dev(stack("conf")),
                           c0["sigma_s"], c0["sigma_r"], 3, T, gamma=c0["gamma"], eps=eps)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    for b, c in enumerate(cs):
        ref = oracle.solve_stereo(c["left"], c["right"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"],
                                  3, T, gamma=c["gamma"], eps=eps)
        err = np.abs(got[b] - ref).max()
        assert err <= 1e-4 * d_max, (case, b, err)


def test_zero_iterations_copy_the_target():
    c = dts_inputs.stereo_case(3, 20, 30)
    out = dts.solve_stereo(dev(c["left"]), dev(c["right"]), dev(c["target"]), dev(c["conf"]), 8.0, 0.2, 3, 0)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), c["target"])


def test_full_size_contractive():
    c = dts_inputs.stereo_pair_1920x1080()
    print("CASE stereo 1920x1080, T=20, eps=2", flush=True)
    got = dts.solve_stereo(dev(c["left"]), dev(c["right"]), dev(c["target"]), dev(c["conf"]), c["sigma_s"],
                           c["sigma_r"], 3, c["solver_iters"], gamma=c["gamma"], eps=2.0)
    torch.cuda.synchronize()
    ref = oracle.solve_stereo(c["left"], c["right"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], 3,
                              c["solver_iters"], gamma=c["gamma"], eps=2.0)
    assert np.abs(got.cpu().numpy() - ref).max() <= 1e-4 * c["value_range"]


def test_full_size_paper_parameters_diverge_only_locally():
    c = dts_inputs.stereo_pair_1920x1080()
    print("CASE stereo 1920x1080, T=20, eps=0.001", flush=True)
    got = dts.solve_stereo(dev(c["left"]), dev(c["right"]), dev(c["target"]), dev(c["conf"]), c["sigma_s"],
                           c["sigma_r"], 3, c["solver_iters"], gamma=c["gamma"], eps=c["eps"])
    torch.cuda.synchronize()
    ref = oracle.solve_stereo(c["left"], c["right"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], 3,
                              c["solver_iters"], gamma=c["gamma"], eps=c["eps"])
    err = np.abs(got.cpu().numpy() - ref)
    tol = 1e-4 * c["value_range"]
    assert (err > tol).mean() <= 1e-3, (err > tol).mean()
    assert np.percentile(err, 99.9) <= tol


def test_full_size_paper_parameters_every_step():
    # A complete check at the paper's eps = gamma = 0.001: each of the 20 GPU steps is
    # taken from the oracle's own iterate z^k (passed as the initial iterate) and compared
    # with the oracle's z^{k+1} on every pixel.  A single step is well conditioned, so the
    # bar is the same as for the contractive setting.
    c = dts_inputs.stereo_pair_1920x1080()
    T = c["solver_iters"]
    print("CASE stereo 1920x1080, every step at eps=0.001", flush=True)
    _, its = oracle.solve_stereo(c["left"], c["right"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], 3, T,
                                 gamma=c["gamma"], eps=c["eps"], return_iterates=True)
    L, R, t, cf = (dev(c[k]) for k in ("left", "right", "target", "conf"))
    tol = 1e-4 * c["value_range"]
    worst = 0.0
    for k in range(T):
        z1 = dts.solve_stereo(L, R, t, cf, c["sigma_s"], c["sigma_r"], 3, 1, gamma=c["gamma"], eps=c["eps"],
                              init=dev(its[k]))
        torch.cuda.synchronize()
        err = float(np.abs(z1.cpu().numpy() - its[k + 1]).max())
        worst = max(worst, err)
        assert err <= tol, (k, err)
    print("worst single-step error", worst, flush=True)
