"""GPU: schedule invariance. Every launch schedule the library can pick (small levels in LDS or
as half-sweep launches; level entries fused into one launch or separate) gives the same matches,
compacted inliers and evaluation counts, equal to the oracle's, for a lone pair and a batch."""
import sys

import numpy as np
import pytest

import oracle
import paper_1704_03217_amd as pgm
import synth
from conftest import CONFIG_PARAMS, base_params

pytestmark = pytest.mark.gpu

SCHEDULES = [pgm.SCHED_AUTO, pgm.SCHED_LEVEL_LDS, pgm.SCHED_LEVEL_LAUNCHES, pgm.SCHED_SEPARATE,
             pgm.SCHED_LEVEL_LDS | pgm.SCHED_SEPARATE, pgm.SCHED_LEVEL_LAUNCHES | pgm.SCHED_SEPARATE]


@pytest.fixture(scope="module")
def matcher():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = pgm.Matcher(0, 1 << 30)
    yield m
    pgm.pgm_schedule(m.ctx, pgm.SCHED_AUTO)
    m.close()


def outputs(m, o, n_pairs):
    n = o["n"]
    return (m.to_numpy(o["fwd"]).reshape(n_pairs, n), m.to_numpy(o["bwd"]).reshape(n_pairs, n),
            m.to_numpy(o["compact"]).reshape(n_pairs, n), o["n_inliers"].cpu().numpy(), int(o["n_evals"].item()))


@pytest.mark.parametrize("name,params,make", [
    ("config1", CONFIG_PARAMS[1], lambda: synth.config_pair(1)),
    ("config2", CONFIG_PARAMS[2], lambda: synth.config_pair(2)),
    ("refine_gray", base_params(refine_rounds=2, color=1, rng_seed=31), lambda: synth.config_pair(1)),
])
def test_every_schedule_gives_the_oracle_result(matcher, name, params, make):
    torch = matcher.torch
    pair = make()
    h, w = pair.img1.shape[:2]
    r = oracle.match(params, pair.img1, pair.img2, trace=False)
    a = torch.from_numpy(pair.img1).cuda()
    b = torch.from_numpy(pair.img2).cuda()
    for sched in SCHEDULES:
        print(f"[gpu schedule] {name} schedule {sched}", file=sys.stderr, flush=True)
        pgm.pgm_schedule(matcher.ctx, sched)
        o = matcher.outputs(params, w, h)
        matcher.match_into(params, a, b, o)
        torch.cuda.synchronize()
        fwd, bwd, comp, nin, nev = outputs(matcher, o, 1)
        assert np.array_equal(fwd[0], r["fwd"]) and np.array_equal(bwd[0], r["bwd"]), sched
        assert nin[0] == r["n_inliers"] and np.array_equal(comp[0, : nin[0]], r["compact"]), sched
        assert nev == r["n_evals"], sched
    pgm.pgm_schedule(matcher.ctx, pgm.SCHED_AUTO)


def test_every_schedule_gives_the_same_batch(matcher):
    torch = matcher.torch
    prs = [synth.config_pair(1, 40 + k) for k in range(4)]
    p = CONFIG_PARAMS[1]
    a = torch.from_numpy(np.stack([q.img1 for q in prs])).cuda()
    b = torch.from_numpy(np.stack([q.img2 for q in prs])).cuda()
    ref = [oracle.match(p, q.img1, q.img2, trace=False) for q in prs]
    for sched in SCHEDULES:
        print(f"[gpu schedule] batch schedule {sched}", file=sys.stderr, flush=True)
        pgm.pgm_schedule(matcher.ctx, sched)
        o = matcher.outputs_batch(p, 256, 192, len(prs))
        matcher.match_batch_into(p, a, b, o)
        torch.cuda.synchronize()
        fwd, bwd, comp, nin, nev = outputs(matcher, o, len(prs))
        for k, r in enumerate(ref):
            assert np.array_equal(fwd[k], r["fwd"]) and np.array_equal(bwd[k], r["bwd"]), (sched, k)
            assert nin[k] == r["n_inliers"] and np.array_equal(comp[k, : nin[k]], r["compact"]), (sched, k)
        assert nev == sum(r["n_evals"] for r in ref), sched
    pgm.pgm_schedule(matcher.ctx, pgm.SCHED_AUTO)


def test_tune_picks_a_schedule_and_keeps_the_oracle_result(matcher):
    torch = matcher.torch
    prs = [synth.config_pair(1, 60 + k) for k in range(2)]
    p = CONFIG_PARAMS[1]
    a = torch.from_numpy(np.stack([q.img1 for q in prs])).cuda()
    b = torch.from_numpy(np.stack([q.img2 for q in prs])).cuda()
    ref = [oracle.match(p, q.img1, q.img2, trace=False) for q in prs]
    print("[gpu schedule] tune two config-1 pairs", file=sys.stderr, flush=True)
    o = matcher.outputs_batch(p, 256, 192, len(prs))
    flags = matcher.tune(p, a, b, o, repeats=2)
    assert flags in SCHEDULES
    for out in (o, matcher.match_batch_into(p, a, b, matcher.outputs_batch(p, 256, 192, len(prs)))):
        torch.cuda.synchronize()
        fwd, bwd, comp, nin, _ = outputs(matcher, out, len(prs))
        for k, r in enumerate(ref):
            assert np.array_equal(fwd[k], r["fwd"]) and np.array_equal(bwd[k], r["bwd"]), (flags, k)
            assert nin[k] == r["n_inliers"] and np.array_equal(comp[k, : nin[k]], r["compact"]), (flags, k)
    pgm.pgm_schedule(matcher.ctx, pgm.SCHED_AUTO)
