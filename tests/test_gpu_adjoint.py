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


@pytest.mark.parametrize("H,W,Cg,Ct,Cc,T,N", [(37, 70, 3, 1, 1, 4, 3), (300, 67, 1, 2, 2, 2, 2),
                                              (45, 130, 2, 3, 1, 2, 1), (700, 90, 3, 2, 1, 3, 3)])
def test_tape_gives_the_recomputed_gradients_bit_for_bit(H, W, Cg, Ct, Cc, T, N):
    """dts_solve_tape + dts_solve_backward_tape against dts_solve + dts_solve_backward: the
    same z^T, checkpoints and gradients bit for bit (the tape holds exactly the pass outputs
    the backward would recompute), and the tape's first slot is the first row pass of
    z^0 = target."""
    case = dts_inputs.random_case(6100 + H + W + Ct, H, W, Cg, Ct, Cc=Cc, sigma_s=6.0, sigma_r=0.3, T=T)
    print("CASE tape", H, W, Cg, Ct, Cc, T, N, flush=True)
    g, t, c = dev(case["guide"]), dev(case["target"]), dev(case["conf"])
    ss, sr = case["sigma_s"], case["sigma_r"]
    z0, ck0 = dts.solve(g, t, c, ss, sr, N, T, checkpoints=True)
    z1, ck1, tp = dts.solve(g, t, c, ss, sr, N, T, tape=True)
    torch.cuda.synchronize()
    assert tp.shape == (T, 2 * N - 1, 1) + tuple(t.shape)  # a 3-D target is a batch of one
    assert torch.equal(z0, z1) and torch.equal(ck0, ck1)
    dx, _ = dts.distances(g, ss, sr)
    assert torch.equal(tp[0, 0], dts.row_pass(t, dx, ss, 1, N))
    go = (2.0 * (z0 - dev(np.random.default_rng(3).uniform(size=case["target"].shape).astype(np.float32))))
    go = go.contiguous()
    ref = dts.solve_backward(g, t, c, ck0, go, ss, sr, N, T)
    got = dts.solve_backward(g, t, c, ck1, go, ss, sr, N, T, tape=tp)
    for name, a, b in zip(("target", "conf", "guide"), got, ref):
        assert torch.equal(a, b), name


def test_autograd_function_with_tape_matches_without():
    case = dts_inputs.random_case(63, 50, 80, 3, 2, Cc=2, T=3)
    p = dts.Params(case["sigma_s"], case["sigma_r"], 3, 3)
    r = dev(np.random.default_rng(2).uniform(size=case["target"].shape).astype(np.float32))
    grads = []
    for tape in (False, True):
        g = dev(case["guide"]).requires_grad_(True)
        t = dev(case["target"]).requires_grad_(True)
        c = dev(case["conf"]).requires_grad_(True)
        z = dts.DTSFunction.apply(g, t, c, p, True, tape)
        ((z - r) ** 2).sum().backward()
        grads.append((g.grad, t.grad, c.grad))
    for a, b in zip(*grads):
        assert torch.equal(a, b)


def test_tape_entry_points_refuse_a_missing_tape():
    case = dts_inputs.random_case(64, 20, 30, 2, 1, T=2)
    g, t, c = dev(case["guide"]), dev(case["target"]), dev(case["conf"])
    z, ck = dts.solve(g, t, c, 6.0, 0.3, 3, 2, checkpoints=True)
    with pytest.raises(ValueError):
        dts.solve_backward(g, t, c, ck, torch.ones_like(t), 6.0, 0.3, 3, 2,
                           tape=torch.zeros((2, 4, 1) + tuple(t.shape), device="cuda"))
