"""GPU: the launch configurations that bench.py times, at their full sizes, against the oracle.

- The uniform batch: 32 resident 1024x436 pairs (two distinct pairs, alternating) in one
  pgm_match_batch call with the configuration-2 parameters; every pair must equal the oracle's
  result for its distinct pair.
- The uneven batch: pairs of the four batch sizes with preset 4 (configuration-2 matching,
  |d| <= ceil(w / 5)), grouped by size into one pgm_match_groups call, run eagerly and then
  replayed from its HIP graph; every pair of every run must equal the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1704_03217_amd as pgm
import synth

pytestmark = pytest.mark.gpu

BATCH_SIZES = [(320, 240), (640, 480), (1024, 436), (1242, 375)]


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def oracle_dict(p):
    """The binding's parameter struct as the oracle's parameter dictionary."""
    return pgm.params_dict(p)


def test_uniform_batch_of_32_config2_pairs(torch):
    print("[gpu bench config] uniform batch 32 x 1024x436", file=sys.stderr, flush=True)
    p = pgm.pgm_default_params(pgm.PRESET_CONFIG2)
    distinct = [synth.config_pair(2, i) for i in range(2)]
    B = 32
    q = pgm.pgm_query(p, 1024, 436)
    m = pgm.Matcher(0, q.workspace_shared_bytes + B * q.workspace_pair_bytes + (1 << 20))
    try:
        a = torch.from_numpy(np.stack([distinct[k % 2].img1 for k in range(B)])).cuda()
        b = torch.from_numpy(np.stack([distinct[k % 2].img2 for k in range(B)])).cuda()
        o = m.outputs_batch(p, 1024, 436, B)
        m.match_batch_into(p, a, b, o)
        torch.cuda.synchronize()
        n = o["n"]
        fwd = m.to_numpy(o["fwd"]).reshape(B, n)
        bwd = m.to_numpy(o["bwd"]).reshape(B, n)
        comp = m.to_numpy(o["compact"]).reshape(B, n)
        nin = o["n_inliers"].cpu().numpy()
        ref = [oracle.match(oracle_dict(p), d.img1, d.img2, trace=False) for d in distinct]
        for k in range(B):
            r = ref[k % 2]
            assert np.array_equal(fwd[k], r["fwd"]) and np.array_equal(bwd[k], r["bwd"]), f"pair {k}"
            assert nin[k] == r["n_inliers"] and np.array_equal(comp[k, : nin[k]], r["compact"]), f"pair {k}"
        assert int(o["n_evals"].item()) == 16 * (ref[0]["n_evals"] + ref[1]["n_evals"])
    finally:
        m.close()


def test_uneven_groups_bench_config_with_graph_replays(torch):
    print("[gpu bench config] uneven groups, graph replays", file=sys.stderr, flush=True)
    per_size = 2
    groups, pairs, params = [], [], []
    need = 0
    for (w, h) in BATCH_SIZES:
        p = pgm.pgm_default_params(pgm.PRESET_CONFIG4)    # the benchmark's uneven-batch parameters
        q = pgm.pgm_query(p, w, h)
        need += (q.workspace_shared_bytes + per_size * q.workspace_pair_bytes + 255) // 256 * 256
        params.append(p)
    m = pgm.Matcher(0, need + (1 << 20))
    try:
        for (w, h), p in zip(BATCH_SIZES, params):
            prs = [synth.config_pair(4, 1000 * w + k, (w, h)) for k in range(per_size)]
            a = torch.from_numpy(np.stack([x.img1 for x in prs])).cuda()
            b = torch.from_numpy(np.stack([x.img2 for x in prs])).cuda()
            groups.append((p, a, b, m.outputs_batch(p, w, h, per_size, count_evals=False)))
            pairs.append(prs)
        refs = [[oracle.match(oracle_dict(p), x.img1, x.img2, trace=False) for x in prs]
                for p, prs in zip(params, pairs)]
        for run, graph in enumerate([False, True, True, True]):
            for *_, o in groups:
                o["fwd"].zero_(); o["bwd"].zero_(); o["compact"].zero_(); o["n_inliers"].zero_()
            torch.cuda.synchronize()
            m.match_groups_into(groups, use_graph=graph)
            torch.cuda.synchronize()
            for (p, _, _, o), rs in zip(groups, refs):
                n = o["n"]
                fwd = m.to_numpy(o["fwd"]).reshape(per_size, n)
                bwd = m.to_numpy(o["bwd"]).reshape(per_size, n)
                comp = m.to_numpy(o["compact"]).reshape(per_size, n)
                nin = o["n_inliers"].cpu().numpy()
                for k, r in enumerate(rs):
                    assert np.array_equal(fwd[k], r["fwd"]) and np.array_equal(bwd[k], r["bwd"]), f"run {run}"
                    assert nin[k] == r["n_inliers"] and np.array_equal(comp[k, : nin[k]], r["compact"]), f"run {run}"
    finally:
        m.close()
