"""Box form of the edge-aware mean (Sec. 3.2, Eq. (10) as written; readings B1-B4) on the
GPU against the FP64 oracle, through the C ABI: the integer codes bit for bit, the filter
and the solver element by element."""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu

# one pass is a mean whose sum carries the float32 rounding of its own additions (the
# column pass keeps a float32 prefix within 32-row blocks): ~32 ulp of the signal range at
# most per pass, ~2e-6 on [0, 1]; six passes of a filter stay below 1e-5
FILTER_TOL = 1e-5
SOLVE_TOL = 1e-4  # x signal range, as for the recursive solve


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


CODE_CASES = [
    # H, W, Cg, sigma_s, sigma_r, guide scale
    (1, 1, 1, 8.0, 0.2, 1.0),
    (37, 53, 3, 8.0, 0.2, 1.0),
    (64, 300, 16, 32.0, 0.15, 1.0),
    (200, 129, 1, 4.0, 0.05, 1.0),
    (50, 60, 3, 16.0, 0.1, 50.0),   # huge distances: codes reach the cap
]


@pytest.mark.parametrize("case", CODE_CASES, ids=[f"{c[0]}x{c[1]}_Cg{c[2]}_s{c[3]}" for c in CODE_CASES])
def test_codes_are_bit_exact(case):
    H, W, Cg, ss, sr, scale = case
    print("CASE box codes", case, flush=True)
    rng = np.random.default_rng(H * 31 + W + Cg)
    g = (rng.random((2, Cg, H, W)) * scale).astype(np.float32)
    # smooth parts too, so that many codes sit near 256
    g[1] = np.cumsum(rng.normal(0, 0.002, (Cg, H, W)), axis=2).astype(np.float32)
    qx, qy = dts.box_codes(dev(g), ss, sr)
    qx = qx.cpu().numpy().view(np.uint32).astype(np.int64)
    qy = qy.cpu().numpy().view(np.uint32).astype(np.int64)
    for b in range(2):
        rx, ry = oracle.box_codes(g[b], ss, sr)
        rx, ry = np.minimum(rx, 65536), np.minimum(ry, 65536)
        assert np.array_equal(qx[b], rx), (case, b, int((qx[b] != rx).sum()))
        assert np.array_equal(qy[b], ry), (case, b, int((qy[b] != ry).sum()))


FILTER_CASES = [
    # H, W, Cg, C, N, batch, sigma_s, sigma_r
    (1, 1, 1, 1, 3, 1, 8.0, 0.2),
    (1, 300, 3, 1, 3, 1, 8.0, 0.2),
    (300, 1, 3, 1, 3, 1, 8.0, 0.2),
    (67, 129, 3, 2, 3, 2, 6.0, 0.25),
    (33, 2500, 3, 1, 3, 1, 16.0, 0.1),     # three row segments
    (3000, 65, 3, 1, 3, 1, 32.0, 0.15),    # many column segments, a ragged strip
    (90, 140, 16, 3, 1, 1, 40.0, 0.2),     # one iteration, wide boxes
    (45, 70, 1, 1, 2, 1, 2.0, 0.3),        # boxes of a few pixels
]


@pytest.mark.parametrize("case", FILTER_CASES, ids=[f"{c[0]}x{c[1]}_Cg{c[2]}_C{c[3]}_N{c[4]}_B{c[5]}" for c in FILTER_CASES])
def test_filter_box_matches_oracle(case):
    H, W, Cg, C, N, B, ss, sr = case
    print("CASE box filter", case, flush=True)
    rng = np.random.default_rng(H * 7919 + W * 31 + Cg + C)
    cs = [dts_inputs.random_case(int(rng.integers(1 << 30)), H, W, Cg, C, sigma_s=ss, sigma_r=sr, T=1)
          for _ in range(B)]
    g = np.stack([c["guide"] for c in cs])
    x = np.stack([c["target"] for c in cs])
    got = dts.filter_box(dev(g), dev(x), ss, sr, N).cpu().numpy()
    for b in range(B):
        qx, qy = oracle.box_codes(g[b], ss, sr)
        ref = oracle.box_filter(x[b], qx, qy, ss, N)
        assert np.abs(got[b] - ref).max() <= FILTER_TOL, (case, b, float(np.abs(got[b] - ref).max()))


# Column passes with h <= 64 run as one kernel over a window of rows in LDS (128 output
# rows per tile, 64 columns); wider ones take the block-prefix and ring kernels.  These
# shapes sit on the window's edges, and each runs both ways against the oracle.
WINDOW_CASES = [
    # H, W, Cg, C, N, batch, sigma_s, sigma_r
    (1000, 70, 3, 1, 1, 1, 37.0, 0.2),     # h = 64, the widest window; ragged tiles and strip
    (100, 130, 3, 2, 3, 2, 20.0, 0.15),    # one tile per strip, shorter than its halo span
    (50, 1, 1, 1, 3, 1, 30.0, 0.2),        # one column (63 idle lanes), image shorter than h
    (300, 200, 3, 1, 1, 1, 0.5, 0.2),      # h = 0: one-pixel boxes
    (257, 64, 16, 1, 3, 1, 37.0, 0.1),     # a last tile of one row
    (400, 90, 3, 1, 1, 1, 37.6, 0.2),      # h = 65: the wide-box kernels either way
]


@pytest.mark.parametrize("window", [1, 0], ids=["window", "wide"])
@pytest.mark.parametrize("case", WINDOW_CASES, ids=[f"{c[0]}x{c[1]}_C{c[3]}_N{c[4]}_s{c[6]}" for c in WINDOW_CASES])
def test_filter_box_column_kernels_match_oracle(case, window):
    H, W, Cg, C, N, B, ss, sr = case
    print("CASE box window", case, window, flush=True)
    rng = np.random.default_rng(H * 613 + W * 17 + C)
    cs = [dts_inputs.random_case(int(rng.integers(1 << 30)), H, W, Cg, C, sigma_s=ss, sigma_r=sr, T=1)
          for _ in range(B)]
    g = np.stack([c["guide"] for c in cs])
    x = np.stack([c["target"] for c in cs])
    dts.tune_box_window(window)
    try:
        got = dts.filter_box(dev(g), dev(x), ss, sr, N).cpu().numpy()
    finally:
        dts.tune_box_window(1)
    for b in range(B):
        qx, qy = oracle.box_codes(g[b], ss, sr)
        ref = oracle.box_filter(x[b], qx, qy, ss, N)
        assert np.abs(got[b] - ref).max() <= FILTER_TOL, (case, b, float(np.abs(got[b] - ref).max()))


@pytest.mark.parametrize("window", [1, 0], ids=["window", "wide"])
def test_solve_box_column_kernels_match_oracle(window):
    # the update epilogue of the last column pass, in place over z^k after the first step
    H, W, Cg, Ct, Cc, N, T, ss, sr = 300, 150, 3, 2, 1, 3, 3, 30.0, 0.2
    print("CASE box window solve", window, flush=True)
    c = dts_inputs.random_case(77, H, W, Cg, Ct, Cc=Cc, sigma_s=ss, sigma_r=sr, T=T)
    dts.tune_box_window(window)
    try:
        got = dts.solve_box(dev(c["guide"])[None], dev(c["target"])[None], dev(c["conf"])[None], ss, sr, N,
                            T).cpu().numpy()[0]
    finally:
        dts.tune_box_window(1)
    ref = oracle.solve_box(c["guide"], c["target"], c["conf"], ss, sr, N, T)
    assert np.abs(got - ref).max() <= SOLVE_TOL, float(np.abs(got - ref).max())


# More window tiles than resident workgroups (800 and 720 against 512 on an MI355X): the
# plain column pass's workgroups then take several tiles each, the next one's window
# loaded while the current one is summed.
PERSISTENT_CASES = [(2560, 2560, 8.0, 3), (2304, 2560, 37.0, 1)]


@pytest.mark.parametrize("case", PERSISTENT_CASES, ids=["2560x2560_N3", "2304x2560_h64"])
def test_filter_box_several_tiles_per_workgroup_matches_oracle(case):
    H, W, ss, N = case
    print("CASE box persistent", case, flush=True)
    c = dts_inputs.random_case(11 + H, H, W, 3, 1, sigma_s=ss, sigma_r=0.2, T=1)
    got = dts.filter_box(dev(c["guide"][None]), dev(c["target"][None]), ss, 0.2, N).cpu().numpy()[0]
    qx, qy = oracle.box_codes(c["guide"], ss, 0.2)
    ref = oracle.box_filter(c["target"], qx, qy, ss, N)
    assert np.abs(got - ref).max() <= FILTER_TOL, (case, float(np.abs(got - ref).max()))


SOLVE_CASES = [
    # H, W, Cg, Ct, Cc, N, T, batch, sigma_s, sigma_r
    (1, 1, 1, 1, 1, 3, 3, 1, 8.0, 0.2),
    (67, 129, 3, 1, 1, 3, 5, 2, 6.0, 0.25),
    (40, 1100, 3, 2, 2, 3, 4, 1, 12.0, 0.2),
    (700, 50, 8, 3, 1, 2, 3, 1, 20.0, 0.15),
]


@pytest.mark.parametrize("case", SOLVE_CASES, ids=[f"{c[0]}x{c[1]}_Ct{c[3]}_Cc{c[4]}_T{c[6]}_B{c[7]}" for c in SOLVE_CASES])
def test_solve_box_matches_oracle(case):
    H, W, Cg, Ct, Cc, N, T, B, ss, sr = case
    print("CASE box solve", case, flush=True)
    rng = np.random.default_rng(H * 131 + W * 7 + Ct)
    cs = [dts_inputs.random_case(int(rng.integers(1 << 30)), H, W, Cg, Ct, Cc=Cc, sigma_s=ss, sigma_r=sr, T=T)
          for _ in range(B)]
    g, t, c = (np.stack([q[k] for q in cs]) for k in ("guide", "target", "conf"))
    got = dts.solve_box(dev(g), dev(t), dev(c), ss, sr, N, T).cpu().numpy()
    for b in range(B):
        ref = oracle.solve_box(g[b], t[b], c[b], ss, sr, N, T)
        assert np.abs(got[b] - ref).max() <= SOLVE_TOL, (case, b, float(np.abs(got[b] - ref).max()))


def test_solve_box_zero_iterations_copies_the_target():
    c = dts_inputs.random_case(3, 20, 30, 3, 1, T=0)
    got = dts.solve_box(dev(c["guide"]), dev(c["target"]), dev(c["conf"]), 6.0, 0.25, 3, 0).cpu().numpy()
    assert np.array_equal(got, c["target"])


def test_solve_box_full_stereo_shape():
    # the 1920 x 1080 disparity workload (sigma_s = 16, sigma_r = 0.1, T = 20); the
    # disparities lie in [0, 256) and are compared at 1e-4 of that range
    c = dts_inputs.disparity_1920x1080(seed=1)
    print("CASE box solve 1920x1080 T=20", flush=True)
    got = dts.solve_box(dev(c["guide"]), dev(c["target"]), dev(c["conf"]), c["sigma_s"], c["sigma_r"],
                        c["filter_iters"], c["solver_iters"]).cpu().numpy()
    ref = oracle.solve_box(c["guide"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], c["filter_iters"],
                           c["solver_iters"])
    assert np.abs(got - ref).max() <= SOLVE_TOL * c["value_range"]


def test_box_calls_leave_a_clean_status():
    # a workspace holding garbage reads DTS_OK after a call: every call clears the status
    c = dts_inputs.random_case(9, 40, 60, 3, 1, T=2)
    lib = dts.library()
    ws = torch.full((lib.dts_box_workspace_bytes(1, 40, 60, 1, 3),), 255, dtype=torch.uint8, device="cuda")
    dts.solve_box(dev(c["guide"]), dev(c["target"]), dev(c["conf"]), 6.0, 0.25, 3, 2, workspace=ws)
    assert dts.workspace_status(ws) == dts.DTS_OK
    ws.fill_(255)
    dts.filter_box(dev(c["guide"]), dev(c["target"]), 6.0, 0.25, 3, workspace=ws)
    assert dts.workspace_status(ws) == dts.DTS_OK
