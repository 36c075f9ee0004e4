"""GPU adjoint (dts_solve_backward) against the FP64 oracle's gradient, through the C ABI.

Bar: relative L2 error <= 1e-3 per gradient, plus an elementwise check with an absolute
floor of 1e-3 * max |reference|.  The oracle's adjoint is itself pinned to central finite
differences and to the dense Jacobian in the CPU tests.
"""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu

REL = 1e-3


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def check(name, got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
    floor = 1e-3 * np.abs(ref).max()
    elem = np.abs(got - ref).max()
    print(f"  {name}: rel L2 {rel:.2e}  max abs {elem:.2e}  floor {floor:.2e}", flush=True)
    assert rel <= REL, (name, rel)
    assert elem <= max(floor, 1e-7), (name, elem, floor)


def run_case(case, seed=7):
    print("CASE adjoint", case["name"], flush=True)
    T = case["solver_iters"]
    rng = np.random.default_rng(seed)
    ref_r = rng.uniform(size=case["target"].shape).astype(np.float32)
    g, t, c = dev(case["guide"]), dev(case["target"]), dev(case["conf"])
    z, ck = dts.solve(g, t, c, case["sigma_s"], case["sigma_r"], case["filter_iters"], T,
                      checkpoints=True)
    go = 2.0 * (z - dev(ref_r))
    gt, gc, gg = dts.solve_backward(g, t, c, ck, go.contiguous(), case["sigma_s"],
                                    case["sigma_r"], case["filter_iters"], T)
    zr = oracle.solve(case["guide"], case["target"], case["conf"], case["sigma_s"],
                      case["sigma_r"], case["filter_iters"], T)
    rt, rc, rg = oracle.solve_backward(case["guide"], case["target"], case["conf"],
                                       case["sigma_s"], case["sigma_r"], 2.0 * (zr - ref_r),
                                       case["filter_iters"], T)
    check("grad_target", host(gt), rt)
    check("grad_conf", host(gc), rc)
    check("grad_guide", host(gg), rg)


SHAPES = [
    # H, W, Cg, Ct, Cc, T
    (1, 1, 1, 1, 1, 2),
    (12, 10, 2, 2, 2, 3),
    (37, 70, 3, 1, 1, 4),
    (64, 64, 3, 3, 3, 3),
    (45, 130, 2, 3, 1, 2),
    (300, 67, 1, 2, 2, 2),
    (130, 257, 8, 1, 1, 2),
    (6, 5001, 2, 2, 1, 2),  # a width that is not a multiple of 4, 8 pixels per lane
]


@pytest.mark.parametrize("H,W,Cg,Ct,Cc,T", SHAPES)
def test_backward_matches_oracle(H, W, Cg, Ct, Cc, T):
    case = dts_inputs.random_case(6000 + H * W + Ct, H, W, Cg, Ct, Cc=Cc, sigma_s=6.0,
                                  sigma_r=0.3, T=T)
    run_case(case)


def test_backward_zero_iterations():
    case = dts_inputs.random_case(61, 20, 30, 3, 2, T=0)
    g, t, c = dev(case["guide"]), dev(case["target"]), dev(case["conf"])
    go = torch.randn_like(t)
    ck = torch.empty((0, 1) + tuple(t.shape), dtype=torch.float32, device="cuda")
    gt, gc, gg = dts.solve_backward(g, t, c, ck, go, 6.0, 0.25, 3, 0)
    assert torch.equal(gt, go)
    assert float(gc.abs().max()) == 0.0 and float(gg.abs().max()) == 0.0


def test_autograd_function_matches_backward():
    case = dts_inputs.random_case(62, 40, 90, 3, 2, Cc=1, T=3)
    p = dts.Params(case["sigma_s"], case["sigma_r"], 3, 3)
    g = dev(case["guide"]).requires_grad_(True)
    t = dev(case["target"]).requires_grad_(True)
    c = dev(case["conf"]).requires_grad_(True)
    r = dev(np.random.default_rng(1).uniform(size=case["target"].shape).astype(np.float32))
    z = dts.DTSFunction.apply(g, t, c, p)
    loss = ((z - r) ** 2).sum()
    loss.backward()
    zr = oracle.solve(case["guide"], case["target"], case["conf"], case["sigma_s"],
                      case["sigma_r"], 3, 3)
    rt, rc, rg = oracle.solve_backward(case["guide"], case["target"], case["conf"],
                                       case["sigma_s"], case["sigma_r"],
                                       2.0 * (zr - r.cpu().numpy()), 3, 3)
    check("autograd target", host(t.grad), rt)
    check("autograd conf", host(c.grad), rc)
    check("autograd guide", host(g.grad), rg)
