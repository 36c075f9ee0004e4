"""Variance-based confidence (Eq. (7)) on the GPU against the FP64 oracle."""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu

TOL = 1e-4  # max abs on confidences in [0, 1] from [0, 1]-valued inputs

CASES = [
    # H, W, Cg, C, N, batch, sigma_s, sigma_r, sigma_c
    (1, 1, 1, 1, 3, 1, 8.0, 0.2, 0.1),
    (1, 300, 3, 1, 3, 1, 8.0, 0.2, 0.1),
    (67, 129, 3, 1, 3, 2, 6.0, 0.25, 0.08),
    (200, 300, 8, 2, 2, 1, 12.0, 0.15, 0.1),
    (37, 1500, 1, 3, 3, 1, 20.0, 0.3, 0.2),
    (1500, 37, 3, 1, 3, 1, 20.0, 0.1, 0.1),
    (33, 17, 16, 8, 1, 1, 4.0, 0.2, 0.05),
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_Cg{c[2]}_C{c[3]}_N{c[4]}_B{c[5]}" for c in CASES])
def test_variance_confidence_matches_oracle(case):
    H, W, Cg, C, N, B, ss, sr, sc = case
    print("CASE variance confidence", case, flush=True)
    rng = np.random.default_rng(H * 7919 + W * 31 + Cg + C)
    guides, zs = [], []
    for b in range(B):
        c = dts_inputs.random_case(int(rng.integers(1 << 30)), H, W, Cg, C, Cc=1, sigma_s=ss, sigma_r=sr, T=1)
        guides.append(c["guide"])
        zs.append(c["target"])
    g = np.stack(guides)
    z = np.stack(zs)
    got = dts.variance_confidence(dev(g), dev(z), ss, sr, sc, filter_iters=N)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    for b in range(B):
        ref, _ = oracle.variance_confidence(g[b], z[b], ss, sr, sc, filter_iters=N)
        err = np.abs(got[b] - ref).max()
        assert err <= TOL, (case, b, err)


def test_constant_input_gives_unit_confidence():
    rng = np.random.default_rng(3)
    g = dev(rng.random((3, 300, 257)))
    z = dev(np.stack([np.full((300, 257), 0.25), np.full((300, 257), 0.75)]))
    c = dts.variance_confidence(g, z, 10.0, 0.2, 0.05)
    torch.cuda.synchronize()
    assert (c - 1.0).abs().max().item() <= TOL


def test_output_may_alias_input():
    case = dts_inputs.random_case(41, 90, 133, 3, 2, Cc=1, sigma_s=8.0, sigma_r=0.2, T=1)
    z = dev(case["target"])
    ref = dts.variance_confidence(dev(case["guide"]), z, 8.0, 0.2, 0.1)
    out = dts.variance_confidence(dev(case["guide"]), z, 8.0, 0.2, 0.1, out=z)
    torch.cuda.synchronize()
    assert out.data_ptr() == z.data_ptr()
    assert torch.equal(out, ref)


def test_full_size_stereo_shape():
    c = dts_inputs.disparity_1920x1080()
    print("CASE variance confidence 1920x1080", flush=True)
    z = c["target"] / np.float32(c["value_range"])  # disparities scaled to [0, 1)
    got = dts.variance_confidence(dev(c["guide"]), dev(z), c["sigma_s"], c["sigma_r"], 0.05)
    torch.cuda.synchronize()
    ref, _ = oracle.variance_confidence(c["guide"], z, c["sigma_s"], c["sigma_r"], 0.05)
    assert np.abs(got.cpu().numpy() - ref).max() <= TOL
