"""The Python binding's argument checks (wrong shapes, devices and batch layouts are
refused before any pointer reaches the library) and the device-status path: when the
host makes every bounded wait of the carry exchange give up (dts_tune_spin_limit with a
negative count), every call still completes and the failure reaches the caller as
DTSError(DTS_EDEVICE) through solve, solve_backward, DTSFunction and BatchedSolver."""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(H=600, W=150, Cg=3, Ct=2, Cc=2, T=2, seed=31):
    c = dts_inputs.random_case(seed, H, W, Cg, Ct, Cc=Cc, sigma_s=10.0, sigma_r=0.2, T=T)
    return c, dev(c["guide"])[None], dev(c["target"])[None], dev(c["conf"])[None]


def test_solve_refuses_mismatched_tensors():
    print("CASE binding solve checks", flush=True)
    c, g, t, cf = _case()
    args = (10.0, 0.2, 3, 2)
    with pytest.raises(ValueError):
        dts.solve(g, t, cf, *args, out=torch.empty((1, 2, 600, 149), device="cuda"))
    with pytest.raises(ValueError):
        dts.solve(g[:, :, :599], t, cf, *args)
    with pytest.raises(ValueError):
        dts.solve(g, t, torch.ones((1, 3, 600, 150), device="cuda"), *args)
    with pytest.raises(ValueError):
        dts.solve(torch.cat([g, g]), t, cf, *args)
    with pytest.raises(ValueError):
        dts.filter(g, t, 10.0, 0.2, out=torch.empty((1, 1, 600, 150), device="cuda"))
    with pytest.raises(ValueError):
        dts.col_pass(t, torch.ones((1, 600, 150), device="cuda"), 10.0, 1, out=torch.empty(5, device="cuda"))


def test_solve_backward_refuses_mismatched_tensors():
    print("CASE binding backward checks", flush=True)
    c, g, t, cf = _case()
    z, ck = dts.solve(g, t, cf, 10.0, 0.2, 3, 2, checkpoints=True)
    args = (10.0, 0.2, 3, 2)
    with pytest.raises(ValueError):
        dts.solve_backward(g, t, cf, ck, z[:, :1].contiguous(), *args)
    with pytest.raises(ValueError):
        dts.solve_backward(g[:, :, :, :100].contiguous(), t, cf, ck, z, *args)
    with pytest.raises(ValueError):
        dts.solve_backward(g, t, cf[:, :, :300].contiguous(), ck, z, *args)
    with pytest.raises(ValueError):
        dts.solve_backward(g, t, cf, ck[:1].contiguous(), z, *args)
    gt, gc, gg = dts.solve_backward(g, t, cf, ck, z, *args)  # well-formed call still works
    assert gt.shape == t.shape and gc.shape == cf.shape and gg.shape == g.shape


def test_batched_solver_refuses_a_batch_of_images():
    print("CASE binding batched checks", flush=True)
    c, g, t, cf = _case(H=100, W=120)
    q = dict(guide=torch.cat([g, g]), target=torch.cat([t, t]), conf=torch.cat([cf, cf]), sigma_s=8.0,
             sigma_r=0.2)
    with pytest.raises(ValueError):
        dts.BatchedSolver([q], variant=0)


def test_timed_out_waits_reach_the_caller():
    print("CASE binding timed-out waits", flush=True)
    c, g, t, cf = _case(H=700, W=200, T=2)
    args = (10.0, 0.2, 3, 2)
    dts.tune_spin_limit(-1)
    try:
        with pytest.raises(dts.DTSError) as e:
            dts.solve(g, t, cf, *args)
        assert e.value.code == dts.DTS_EDEVICE
        z, ck = dts.solve(g, t, cf, *args, checkpoints=True, check=False)  # asynchronous: no error
        with pytest.raises(dts.DTSError) as e:
            dts.solve_backward(g, t, cf, ck, z, *args)
        assert e.value.code == dts.DTS_EDEVICE
        p = dts.Params(*args)
        with pytest.raises(dts.DTSError) as e:
            dts.DTSFunction.apply(g, t, cf, p)
        assert e.value.code == dts.DTS_EDEVICE
        probs = [dict(guide=g[0], target=t[0], conf=cf[0], sigma_s=10.0, sigma_r=0.2, solver_iters=2)]
        bs = dts.BatchedSolver(probs, variant=0)
        with pytest.raises(dts.DTSError) as e:
            bs.run(check=True)
        assert e.value.code == dts.DTS_EDEVICE
    finally:
        dts.tune_spin_limit(0)
    # with the default bound the same calls are clean and right
    z = dts.solve(g, t, cf, *args)
    ref = oracle.solve(c["guide"], c["target"], c["conf"], 10.0, 0.2, 3, 2)
    assert np.abs(z[0].cpu().numpy() - ref).max() <= 1e-4
    bs.run(check=True)
    assert np.abs(bs.outputs[0].cpu().numpy() - ref).max() <= 1e-4
