"""Batched persistent solve (dts_solve_batched) against the oracle and the single solve,
graph capture and replay, and the autotuner."""
import os

import numpy as np
import pytest
import torch

import dts_inputs
import oracle
import paper_1805_04590_amd as dts

pytestmark = pytest.mark.gpu

N_BATCH_VARIANTS = 5  # also checked against the library by a CPU test


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def small_set(seed0=900, n=6, T=3):
    rng = np.random.default_rng(seed0)
    cases = []
    for i in range(n):
        H = int(rng.integers(20, 300))
        W = int(rng.integers(30, 700))
        Cg = int(rng.choice([1, 3, 8, 16]))
        Ct = int(rng.integers(1, 4))
        Cc = int(rng.choice([1, Ct]))
        case = dts_inputs.random_case(seed0 + 10 + i, H, W, Cg, Ct, Cc=Cc,
                                      sigma_s=float(rng.uniform(4, 32)),
                                      sigma_r=float(rng.uniform(0.05, 0.3)), T=T)
        cases.append(case)
    return cases


def problems_of(cases):
    return [dict(guide=dev(c["guide"]), target=dev(c["target"]), conf=dev(c["conf"]),
                 sigma_s=c["sigma_s"], sigma_r=c["sigma_r"], filter_iters=3,
                 solver_iters=c["solver_iters"]) for c in cases]


@pytest.mark.parametrize("variant", range(N_BATCH_VARIANTS))
def test_batched_matches_oracle_and_single(variant):
    cases = small_set()
    print("CASE batched variant", variant, [c["name"] for c in cases], flush=True)
    probs = problems_of(cases)
    bs = dts.BatchedSolver(probs, variant=variant)
    outs = bs.run()
    torch.cuda.synchronize()
    bs.status()
    for c, q, o in zip(cases, probs, outs):
        single = dts.solve(q["guide"], q["target"], q["conf"], c["sigma_s"], c["sigma_r"], 3,
                           c["solver_iters"])
        ref = oracle.solve(c["guide"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], 3,
                           c["solver_iters"])
        got = o.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-4, c["name"]
        assert np.abs(got - single.cpu().numpy()).max() <= 1e-5, c["name"]


@pytest.mark.parametrize("variant", range(N_BATCH_VARIANTS))
def test_batched_wide_rows(variant):
    """Rows filtered by one wave, by one wave in two sections (1024 < W <= 2048, widths
    that are and are not multiples of 4, one to three channels), by all four waves of a
    workgroup, the widest accepted row, a 1-row and a 1-column image, next to each other in
    one launch."""
    shapes = [(9, 1100, 3, 1), (6, 2500, 1, 2), (5, 4096, 8, 1), (3, 2048, 2, 1), (1, 300, 3, 1),
              (70, 1, 1, 2), (33, 100, 16, 3), (12, 1024, 1, 1), (7, 513, 3, 2), (5, 1025, 2, 3),
              (11, 1999, 3, 2), (2, 2049, 1, 1), (6, 1536, 16, 3)]
    cases = [dts_inputs.random_case(1200 + k, H, W, Cg, Ct, Cc=1, sigma_s=12.0, sigma_r=0.2, T=2)
             for k, (H, W, Cg, Ct) in enumerate(shapes)]
    print("CASE batched wide rows", variant, shapes, flush=True)
    probs = problems_of(cases)
    bs = dts.BatchedSolver(probs, variant=variant)
    outs = bs.run()
    torch.cuda.synchronize()
    bs.status()
    for c, o in zip(cases, outs):
        ref = oracle.solve(c["guide"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], 3, 2)
        assert np.abs(o.cpu().numpy() - ref).max() <= 1e-4, c["name"]


def test_graph_replays_match_eager():
    cases = small_set(seed0=950, n=5, T=2)
    print("CASE batched graph", flush=True)
    probs = problems_of(cases)
    bs = dts.BatchedSolver(probs, variant=0)
    eager = [o.clone() for o in bs.run()]
    torch.cuda.synchronize()
    graph = bs.capture()
    for rep in range(4):
        for o in bs.outputs:
            o.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        bs.status()
        for e, o in zip(eager, bs.outputs):
            assert torch.equal(e, o), rep


def test_autotuner_picks_and_caches(tmp_path):
    os.environ["DTS_TUNE_CACHE"] = str(tmp_path / "tune.json")
    try:
        cases = small_set(seed0=970, n=4, T=2)
        probs = problems_of(cases)
        bs = dts.BatchedSolver(probs)  # variant=None -> autotune
        assert 0 <= bs.variant < len(dts.batched_variants())
        assert (tmp_path / "tune.json").exists()
        bs2 = dts.BatchedSolver(probs)
        assert bs2.variant == bs.variant
        ref = oracle.solve(cases[0]["guide"], cases[0]["target"], cases[0]["conf"],
                           cases[0]["sigma_s"], cases[0]["sigma_r"], 3, 2)
        out = bs2.run()[0]
        torch.cuda.synchronize()
        assert np.abs(out.cpu().numpy() - ref).max() <= 1e-4
    finally:
        del os.environ["DTS_TUNE_CACHE"]


@pytest.fixture(scope="module")
def uneven_batch_64():
    """The 64-instance workload, and the FP64 oracle's solves of 12 of its instances: the
    smallest one of every (guide channels, target channels) pair, Cg in {1, 3, 8, 16} and
    Ct in {1, 2, 3}."""
    cases = dts_inputs.uneven_batch_64()
    pick = {}
    for i, c in enumerate(cases):
        key = (c["guide"].shape[0], c["target"].shape[0])
        px = c["target"].shape[1] * c["target"].shape[2]
        if key not in pick or px < pick[key][0]:
            pick[key] = (px, i)
    assert len(pick) == 12
    refs = {}
    for key in sorted(pick):
        i = pick[key][1]
        c = cases[i]
        print("STEP oracle solve of instance", i, "Cg, Ct =", key, flush=True)
        refs[i] = oracle.solve(c["guide"], c["target"], c["conf"], c["sigma_s"], c["sigma_r"], 3, 10)
    return cases, refs


@pytest.mark.parametrize("variant", range(N_BATCH_VARIANTS))
def test_uneven_batch_64_matches_single_solves_and_oracle(variant, uneven_batch_64):
    cases, refs = uneven_batch_64
    print("CASE 64 uneven solves, variant", variant, flush=True)
    probs = problems_of(cases)
    bs = dts.BatchedSolver(probs, variant=variant)
    outs = bs.run(check=True)
    for i, (c, q, o) in enumerate(zip(cases, probs, outs)):
        single = dts.solve(q["guide"], q["target"], q["conf"], c["sigma_s"], c["sigma_r"], 3, 10)
        assert (o - single).abs().max().item() <= 1e-5, c["name"]
    worst = 0.0
    for i, ref in refs.items():
        err = float(np.abs(outs[i].cpu().numpy() - ref).max())
        worst = max(worst, err)
        assert err <= 1e-4, (cases[i]["name"], err)
    print("worst oracle error over the 12 instances", worst, flush=True)
