"""dts_solve captured into a HIP graph (SolveGraph): every replay against the eager solve,
bit for bit, with other eager work between the replays, and replays after new inputs are
copied in."""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("which", ["polygon_256", "disparity_1920x1080"])
def test_graph_replays_match_eager(which):
    c = getattr(dts_inputs, which)()
    print("CASE graph", c["name"], flush=True)
    args = (c["sigma_s"], c["sigma_r"], c["filter_iters"], c["solver_iters"])
    g, t, cf = dev(c["guide"]), dev(c["target"]), dev(c["conf"])
    eager = dts.solve(g, t, cf, *args)
    sg = dts.SolveGraph(g, t, cf, *args)
    for rep in range(3):
        got = sg.replay()[0].clone()
        torch.cuda.synchronize()
        assert torch.equal(got, eager), rep
        # eager work of another shape and input between the replays
        dts.solve(g[:, :100, :120].contiguous(), (0.5 * t[:, :100, :120]).contiguous(),
                  cf[:, :100, :120].contiguous(), *args)
        torch.cuda.synchronize()
    # new inputs copied into the graph's buffers
    t2 = (t.flip(-1) * 0.9).contiguous()
    sg.target.copy_(t2[None])
    got = sg.replay()[0].clone()
    eager2 = dts.solve(g, t2, cf, *args)
    assert torch.equal(got, eager2)
    if which == "polygon_256":
        ref = oracle.solve(c["guide"], t2.cpu().numpy(), c["conf"], *args)
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-4
