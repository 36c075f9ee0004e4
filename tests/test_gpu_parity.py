"""GPU parity of libdts against the FP64 oracle, through the C ABI.

Tolerance (max abs error): 1e-4 on [0,1]-valued signals for the solve, scaled by the
signal range for the [0,256) disparity workload; 1e-5 for a single filter call.  Inputs
are the seeded synthetic scenes of dts_inputs; expected values come from oracle/ only.
"""
import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-4
FILTER_TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def announce(*what):
    print("CASE", *what, flush=True)


def oracle_filter(guide, src, ss, sr, N):
    dx, dy = oracle.distances(guide, ss, sr)
    return oracle.dt_filter(src, dx, dy, ss, N)


STEP_SHAPES = [
    # H, W, Cg, C
    (1, 1, 1, 1),
    (3, 257, 3, 2),
    (255, 9, 2, 1),
    (1000, 70, 3, 1),
    (513, 600, 16, 3),
    (61, 4096, 1, 4),
    (33, 1000, 3, 6),
    (3000, 65, 2, 2),
    (4099, 3, 1, 1),
    (1500, 130, 3, 3),
    (700, 200, 2, 4),
    # widths not a multiple of 4 at 8 and 16 pixels per lane: rows start off 16-byte
    # alignment and still move as 16-byte accesses
    (5, 6001, 2, 2),
    (3, 9999, 1, 1),
]


@pytest.mark.parametrize("H,W,Cg,C", STEP_SHAPES)
def test_distances_match_oracle(H, W, Cg, C):
    announce("distances", H, W, Cg)
    case = dts_inputs.random_case(4000 + H + W, H, W, Cg, 1)
    dx, dy = dts.distances(dev(case["guide"]), 6.0, 0.05)
    rdx, rdy = oracle.distances(case["guide"], 6.0, 0.05)
    np.testing.assert_allclose(host(dx)[0], rdx, rtol=2e-6, atol=0)
    np.testing.assert_allclose(host(dy)[0], rdy, rtol=2e-6, atol=0)


@pytest.mark.parametrize("H,W,Cg,C", STEP_SHAPES)
@pytest.mark.parametrize("it", [1, 3])
def test_single_passes_match_oracle(H, W, Cg, C, it):
    announce("passes", H, W, Cg, C, it)
    case = dts_inputs.random_case(5000 + H + W, H, W, Cg, C, sigma_s=10.0, sigma_r=0.2)
    rdx, rdy = oracle.distances(case["guide"], 10.0, 0.2)
    a = oracle.feedback_coefficients(10.0, 3)[it - 1]
    f = case["target"].astype(np.float64)
    # rows: recursion along axis -1 of every channel; columns: along axis -2
    ref_row = np.moveaxis(oracle.rf1d_lines(np.moveaxis(f, -1, 0), np.moveaxis(a ** rdx, -1, 0)[:, None, :]), 0, -1)
    ref_col = np.moveaxis(oracle.rf1d_lines(np.moveaxis(f, -2, 0), (a ** rdy)[:, None, :]), 0, -2)
    dx = dev(rdx.astype(np.float32)[None])
    dy = dev(rdy.astype(np.float32)[None])
    x = dev(case["target"])
    got_row = host(dts.row_pass(x, dx, 10.0, it, 3))
    got_col = host(dts.col_pass(x, dy, 10.0, it, 3))
    assert np.abs(got_row - ref_row).max() <= 2e-6
    assert np.abs(got_col - ref_col).max() <= 2e-6


FILTER_SHAPES = [
    # H, W, Cg, Cs
    (1, 1, 1, 1),
    (1, 300, 3, 1),
    (300, 1, 3, 1),
    (2, 2, 2, 2),
    (37, 300, 3, 1),
    (70, 257, 2, 2),
    (33, 515, 16, 3),
    (45, 64, 1, 5),
    (129, 1025, 3, 1),
    (65, 4100, 3, 1),
    (97, 63, 8, 4),
    (9, 6001, 3, 2),
    (4, 10001, 2, 1),
]


@pytest.mark.parametrize("H,W,Cg,Cs", FILTER_SHAPES)
def test_filter_matches_oracle(H, W, Cg, Cs):
    announce("filter", H, W, Cg, Cs)
    case = dts_inputs.random_case(1000 + H + W, H, W, Cg, Cs, sigma_s=7.0, sigma_r=0.3)
    src = case["target"]
    got = host(dts.filter(dev(case["guide"]), dev(src), 7.0, 0.3, 3))
    ref = oracle_filter(case["guide"], src, 7.0, 0.3, 3)
    err = np.abs(got - ref).max()
    assert err <= FILTER_TOL, err


@pytest.mark.parametrize("N", [1, 2, 5])
def test_filter_iteration_counts(N):
    announce("filter N", N)
    case = dts_inputs.random_case(77, 50, 333, 3, 1, sigma_s=12.0, sigma_r=0.1)
    got = host(dts.filter(dev(case["guide"]), dev(case["target"]), 12.0, 0.1, N))
    ref = oracle_filter(case["guide"], case["target"], 12.0, 0.1, N)
    assert np.abs(got - ref).max() <= FILTER_TOL


def test_filter_batched_and_in_place():
    announce("filter batched in-place")
    cases = [dts_inputs.random_case(200 + i, 40, 130, 3, 2) for i in range(3)]
    g = np.stack([c["guide"] for c in cases])
    x = np.stack([c["target"] for c in cases])
    xd = dev(x)
    out = dts.filter(dev(g), xd, 6.0, 0.25, 3, out=xd)
    got = host(out)
    for i, c in enumerate(cases):
        ref = oracle_filter(c["guide"], c["target"], 6.0, 0.25, 3)
        assert np.abs(got[i] - ref).max() <= FILTER_TOL


def test_filter_preserves_constants_and_is_deterministic():
    announce("filter constants")
    case = dts_inputs.random_case(5, 200, 700, 3, 1)
    c = np.full_like(case["target"], 0.625)
    got = host(dts.filter(dev(case["guide"]), dev(c), 9.0, 0.15, 3))
    assert np.abs(got - 0.625).max() <= 2e-6
    g, t = dev(case["guide"]), dev(case["target"])
    a = host(dts.filter(g, t, 9.0, 0.15, 3))
    b = host(dts.filter(g, t, 9.0, 0.15, 3))
    assert np.array_equal(a, b)


def oracle_solve(case, T=None):
    return oracle.solve(case["guide"], case["target"], case["conf"], case["sigma_s"],
                        case["sigma_r"], case["filter_iters"],
                        case["solver_iters"] if T is None else T, case["lam"], case["step"])


def gpu_solve(case, **kw):
    return dts.solve(dev(case["guide"]), dev(case["target"]), dev(case["conf"]), case["sigma_s"],
                     case["sigma_r"], case["filter_iters"], kw.pop("T", case["solver_iters"]),
                     case["lam"], case["step"], **kw)


SOLVE_CASES = [
    # H, W, Cg, Ct, Cc, T
    (1, 1, 1, 1, 1, 3),
    (9, 700, 3, 1, 1, 4),
    (64, 64, 1, 2, 1, 5),
    (81, 290, 3, 3, 3, 6),
    (130, 77, 8, 2, 2, 3),
    (47, 517, 16, 1, 1, 5),
    (33, 100, 2, 5, 1, 2),
]


@pytest.mark.parametrize("H,W,Cg,Ct,Cc,T", SOLVE_CASES)
def test_solve_matches_oracle(H, W, Cg, Ct, Cc, T):
    announce("solve", H, W, Cg, Ct, Cc, T)
    case = dts_inputs.random_case(3000 + H * W, H, W, Cg, Ct, Cc=Cc, sigma_s=8.0, sigma_r=0.2, T=T)
    got = host(gpu_solve(case))
    ref = oracle_solve(case)
    err = np.abs(got - ref).max()
    assert err <= SOLVE_TOL, err


def test_solve_polygon_256_full():
    case = dts_inputs.polygon_256()
    announce(case["name"])
    got = host(gpu_solve(case))
    ref = oracle_solve(case)
    err = np.abs(got - ref).max()
    print("polygon 256x256 max abs err", err, flush=True)
    assert err <= SOLVE_TOL


def test_solve_disparity_1920x1080_full():
    case = dts_inputs.disparity_1920x1080()
    announce(case["name"])
    got = host(gpu_solve(case))
    ref = oracle_solve(case)
    err = np.abs(got - ref).max() / case["value_range"]
    print("disparity 1920x1080 max abs err / range", err, flush=True)
    assert err <= SOLVE_TOL


def test_solve_zero_iterations_and_constant_target():
    announce("solve T=0 / constant")
    case = dts_inputs.random_case(11, 40, 90, 3, 2)
    got = host(gpu_solve(case, T=0))
    assert np.array_equal(got, case["target"].astype(np.float64))
    case["target"] = np.full_like(case["target"], 0.3)
    got = host(gpu_solve(case, T=7))
    assert np.abs(got - 0.3).max() <= 1e-6


def test_solve_checkpoints_hold_iterates():
    announce("solve checkpoints")
    case = dts_inputs.random_case(12, 60, 150, 3, 2, Cc=1, T=4)
    z, ck = gpu_solve(case, checkpoints=True)
    z, ck = host(z), host(ck)
    _, its = oracle.solve(case["guide"], case["target"], case["conf"], case["sigma_s"],
                          case["sigma_r"], 3, 4, return_iterates=True)
    assert ck.shape == (4, 1, 2, 60, 150)
    for k in range(4):
        assert np.abs(ck[k, 0] - its[k]).max() <= SOLVE_TOL, k
    assert z.shape == its[4].shape
    assert np.abs(z - its[4]).max() <= SOLVE_TOL
    z2 = host(gpu_solve(case))
    assert np.array_equal(z, z2)


def test_solve_batch_equals_single():
    announce("solve batch")
    cases = [dts_inputs.random_case(300 + i, 50, 210, 3, 2, Cc=2, sigma_s=8.0, sigma_r=0.2, T=3)
             for i in range(3)]
    g = dev(np.stack([c["guide"] for c in cases]))
    t = dev(np.stack([c["target"] for c in cases]))
    c = dev(np.stack([c["conf"] for c in cases]))
    zb = host(dts.solve(g, t, c, 8.0, 0.2, 3, 3))
    for i, cs in enumerate(cases):
        zi = host(gpu_solve(cs))
        assert np.array_equal(zb[i], zi)
        assert np.abs(zi - oracle_solve(cs)).max() <= SOLVE_TOL


def test_workspace_status_is_clean():
    announce("status")
    case = dts_inputs.random_case(13, 300, 300, 3, 1, T=2)
    p = dts.Params(8.0, 0.2, 3, 2)
    lib = dts.library()
    import ctypes
    ws = torch.empty(lib.dts_solve_workspace_bytes(1, 300, 300, 1, ctypes.byref(p.c())),
                     dtype=torch.uint8, device="cuda")
    dts.solve(dev(case["guide"]), dev(case["target"]), dev(case["conf"]), 8.0, 0.2, 3, 2,
              workspace=ws)
    assert dts.workspace_status(ws) == 0


def _variant_cases():
    # every column-pass variant, pinned in turn: 2.5 chunks per strip plus a ragged row
    # tail, three strips with a ragged column tail, and for four-channel groups a second,
    # partial channel group
    return [(v, ct, R, nw) for v, ct, R, nw in dts.col_variants()]


@pytest.mark.parametrize("v,ct,R,nw", _variant_cases())
def test_every_column_variant_matches_oracle(v, ct, R, nw):
    H, W = int(2.5 * R * nw) + 3, 130
    C = ct if ct < 4 else 5
    announce("column variant", v, ct, R, nw, H, W, C)
    case = dts_inputs.random_case(6100 + v, H, W, 3, C, Cc=1, sigma_s=12.0, sigma_r=0.2, T=2)
    rdx, rdy = oracle.distances(case["guide"], 12.0, 0.2)
    a = oracle.feedback_coefficients(12.0, 3)[0]
    f = case["target"].astype(np.float64)
    ref_col = np.moveaxis(oracle.rf1d_lines(np.moveaxis(f, -2, 0), (a ** rdy)[:, None, :]), 0, -2)
    ref_solve = oracle_solve(case)
    dts.tune_col_variant(ct, v)
    try:
        got_col = host(dts.col_pass(dev(case["target"]), dev(rdy.astype(np.float32)[None]), 12.0, 1, 3))
        got_solve = host(gpu_solve(case))
    finally:
        dts.tune_col_variant(ct, -1)
    assert np.abs(got_col[0] - ref_col).max() <= FILTER_TOL
    assert np.abs(got_solve - ref_solve).max() <= SOLVE_TOL


@pytest.mark.parametrize("v,ct,R,nw", _variant_cases())
def test_every_column_variant_on_long_strips(v, ct, R, nw):
    # about 20 chunks per strip, so each look-back and look-ahead takes several round
    # trips of NWV neighbours; two strips, the second ragged
    H, W = int(19.5 * R * nw) + 5, 77
    C = ct if ct < 4 else 5
    announce("column variant, long strips", v, ct, R, nw, H, W, C)
    case = dts_inputs.random_case(6200 + v, H, W, 2, C, Cc=1, sigma_s=40.0, sigma_r=0.3, T=1)
    rdx, rdy = oracle.distances(case["guide"], 40.0, 0.3)
    a = oracle.feedback_coefficients(40.0, 3)[0]
    f = case["target"].astype(np.float64)
    ref_col = np.moveaxis(oracle.rf1d_lines(np.moveaxis(f, -2, 0), (a ** rdy)[:, None, :]), 0, -2)
    dts.tune_col_variant(ct, v)
    try:
        got_col = host(dts.col_pass(dev(case["target"]), dev(rdy.astype(np.float32)[None]), 40.0, 1, 3))
    finally:
        dts.tune_col_variant(ct, -1)
    assert np.abs(got_col[0] - ref_col).max() <= FILTER_TOL


def test_column_carries_without_truncation():
    # A nearly flat guide and a very wide kernel (sigma_s = 2000) keep every product of
    # weights along a strip above the point where a carry walk may stop early, so each
    # chunk composes the aggregates of every other chunk of its strip: 32 chunks, eight
    # round trips of the exchange each way.
    H, W = 10240, 70
    announce("column pass, untruncated walks", H, W)
    rng = np.random.default_rng(17)
    guide = (0.5 + 1e-6 * rng.standard_normal((1, H, W))).astype(np.float32)
    f = rng.uniform(size=(1, H, W)).astype(np.float32)
    rdx, rdy = oracle.distances(guide, 2000.0, 0.5)
    a = oracle.feedback_coefficients(2000.0, 3)[0]
    assert a ** (rdy.max() * H) > 2.0 ** -30  # no walk may stop before the strip's end
    ref = np.moveaxis(oracle.rf1d_lines(np.moveaxis(f.astype(np.float64), -2, 0), (a ** rdy)[:, None, :]), 0, -2)
    dy = dev(rdy.astype(np.float32)[None])
    x = dev(f)
    got = host(dts.col_pass(x, dy, 2000.0, 1, 3))
    assert np.abs(got[0] - ref).max() <= FILTER_TOL
    again = host(dts.col_pass(x, dy, 2000.0, 1, 3))
    assert np.array_equal(got, again)


@pytest.mark.parametrize("H,W,Ct", [(1500, 300, 1), (2600, 130, 3), (10240, 64, 1)])
def test_multi_chunk_solve_is_bitwise_reproducible(H, W, Ct):
    # Which neighbours a chunk composes, and in which order, depends on the data only, so
    # repeated solves agree bit for bit however the chunks' workgroups are timed; other
    # work runs between the calls.
    announce("bitwise reproducible", H, W, Ct)
    case = dts_inputs.random_case(8100 + H, H, W, 3, Ct, Cc=1, sigma_s=24.0, sigma_r=0.2, T=3)
    g, t, c = dev(case["guide"]), dev(case["target"]), dev(case["conf"])
    first = host(dts.solve(g, t, c, 24.0, 0.2, 3, 3))
    for rep in range(3):
        dts.solve(g[:, :, :200 + rep].contiguous(), t[:, :, :200 + rep].contiguous(),
                  c[:, :, :200 + rep].contiguous(), 24.0, 0.2, 3, 2)
        assert np.array_equal(host(dts.solve(g, t, c, 24.0, 0.2, 3, 3)), first), rep
    if H <= 2600:
        assert np.abs(first - oracle_solve(case)).max() <= SOLVE_TOL


def test_column_chunk_placement_does_not_change_results():
    # Chunks of a strip kept on one XCD (the default) or dealt round-robin: the carries a
    # chunk composes are the same, so the column pass and the adjoint agree bit for bit.
    H, W = 2600, 300
    announce("column chunk placement", H, W)
    case = dts_inputs.random_case(8300, H, W, 3, 2, Cc=2, sigma_s=20.0, sigma_r=0.2, T=2)
    rdx, rdy = oracle.distances(case["guide"], 20.0, 0.2)
    x, dy = dev(case["target"]), dev(rdy.astype(np.float32)[None])
    g, t, c = dev(case["guide"]), dev(case["target"]), dev(case["conf"])
    got = {}
    try:
        for on in (0, 1):
            dts.tune_col_xcd(on)
            z, ck = dts.solve(g, t, c, 20.0, 0.2, 3, 2, checkpoints=True)
            grads = dts.solve_backward(g, t, c, ck, z, 20.0, 0.2, 3, 2)
            got[on] = [host(dts.col_pass(x, dy, 20.0, 1, 3)), host(z)] + [host(q) for q in grads]
    finally:
        dts.tune_col_xcd(1)
    for a, b in zip(got[0], got[1]):
        assert np.array_equal(a, b)
    a = oracle.feedback_coefficients(20.0, 3)[0]
    ref = np.moveaxis(oracle.rf1d_lines(np.moveaxis(case["target"].astype(np.float64), -2, 0),
                                        (a ** rdy)[:, None, :]), 0, -2)
    assert np.abs(got[1][0][0] - ref).max() <= FILTER_TOL
