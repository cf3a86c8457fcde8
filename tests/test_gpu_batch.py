"""GPU: pgm_match_batch. Every pair of a batch must give exactly what pgm_match gives for that
pair alone, which is exactly the oracle's synchronous schedule."""
import sys

import numpy as np
import pytest

import oracle
import paper_1704_03217_amd as pgm
import synth
from conftest import CONFIG_PARAMS, base_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def matcher():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = pgm.Matcher(0, 1536 << 20)
    yield m
    m.close()


def run_batch(m, params, pairs):
    torch = m.torch
    a = torch.from_numpy(np.stack([p.img1 for p in pairs])).cuda()
    b = torch.from_numpy(np.stack([p.img2 for p in pairs])).cuda()
    o = m.match_batch(params, a, b)
    torch.cuda.synchronize()
    n = o["n"]
    fwd = m.to_numpy(o["fwd"]).reshape(len(pairs), n)
    bwd = m.to_numpy(o["bwd"]).reshape(len(pairs), n)
    comp = m.to_numpy(o["compact"]).reshape(len(pairs), n)
    nin = o["n_inliers"].cpu().numpy()
    return fwd, bwd, comp, nin, int(o["n_evals"].item())


@pytest.mark.parametrize("case", ["config1_x3", "patch5_11_gray_x4", "refine_x2", "direction_x2", "regions_x3"])
def test_batch_equals_oracle_per_pair(matcher, case):
    if case == "config1_x3":
        pairs = [synth.config_pair(1, i) for i in range(3)]
        params = CONFIG_PARAMS[1]
    elif case == "patch5_11_gray_x4":
        pairs = [synth.rect_pair(50 + i, 120, 160, dmax=12) for i in range(4)]
        params = base_params(patch_fwd=5, patch_bwd=11, color=1, max_disp=12, rng_seed=31)
    elif case == "refine_x2":
        pairs = [synth.config_pair(1, i) for i in range(2)]
        params = base_params(refine_rounds=2, rng_seed=32)
    elif case == "regions_x3":
        pairs = [synth.config_pair(1, i) for i in range(3)]
        params = base_params(min_region_px=45, region_link_px=1, rng_seed=34)
    else:
        pairs = [synth.config_pair(1, i) for i in range(2)]
        params = base_params(feature=1, rng_seed=33)
    print(f"[gpu batch] {case}", file=sys.stderr, flush=True)
    fwd, bwd, comp, nin, nev = run_batch(matcher, params, pairs)
    total = 0
    for k, pr in enumerate(pairs):
        r = oracle.match(params, pr.img1, pr.img2, trace=False)
        assert np.array_equal(fwd[k], r["fwd"]), f"pair {k} fwd"
        assert np.array_equal(bwd[k], r["bwd"]), f"pair {k} bwd"
        assert nin[k] == r["n_inliers"], f"pair {k} inliers"
        assert np.array_equal(comp[k, : nin[k]], r["compact"]), f"pair {k} compact"
        total += r["n_evals"]
    assert nev == total


def test_batch_config2_size(matcher):
    pairs = [synth.config_pair(2, i) for i in range(2)]
    print("[gpu batch] config2_x2", file=sys.stderr, flush=True)
    fwd, bwd, comp, nin, nev = run_batch(matcher, CONFIG_PARAMS[2], pairs)
    for k, pr in enumerate(pairs):
        r = oracle.match(CONFIG_PARAMS[2], pr.img1, pr.img2, trace=False)
        assert np.array_equal(fwd[k], r["fwd"]) and np.array_equal(bwd[k], r["bwd"])
        assert nin[k] == r["n_inliers"]


def test_batch_too_large_is_enomem(matcher):
    torch = matcher.torch
    s = pgm.pgm_query(CONFIG_PARAMS[1], 256, 192)
    small = pgm.Matcher(0, s.workspace_shared_bytes + 2 * s.workspace_pair_bytes)
    try:
        img = torch.zeros((3, 192, 256, 3), dtype=torch.uint8, device="cuda")
        with pytest.raises(pgm.PGMError) as e:
            small.match_batch(CONFIG_PARAMS[1], img, img)
        assert e.value.status == pgm.PGM_ENOMEM
        ok = small.match_batch(CONFIG_PARAMS[1], img[:2], img[:2])   # exactly fits
        torch.cuda.synchronize()
        assert ok["n_inliers"].shape[0] == 2
    finally:
        small.close()


def _check_pairs(params, pairs, fwd, bwd, comp, nin, nev, tag):
    total = 0
    for k, pr in enumerate(pairs):
        r = oracle.match(params, pr.img1, pr.img2, trace=False)
        assert np.array_equal(fwd[k], r["fwd"]), f"{tag}: pair {k} fwd"
        assert np.array_equal(bwd[k], r["bwd"]), f"{tag}: pair {k} bwd"
        assert nin[k] == r["n_inliers"], f"{tag}: pair {k} inliers"
        assert np.array_equal(comp[k, : nin[k]], r["compact"]), f"{tag}: pair {k} compact"
        total += r["n_evals"]
    assert nev == total, tag


def test_batch_padded_pitch_and_image_stride(matcher):
    """Pairs cut out of larger frames: rows longer than the image and a gap between images."""
    torch = matcher.torch
    pairs = [synth.config_pair(1, 20 + i) for i in range(3)]
    params = CONFIG_PARAMS[1]
    h, w = pairs[0].img1.shape[:2]
    print("[gpu batch] padded pitch and image stride", file=sys.stderr, flush=True)
    big = [np.full((3, h + 3, w + 5, 3), 77, np.uint8) for _ in range(2)]
    for k, pr in enumerate(pairs):
        big[0][k, :h, :w] = pr.img1
        big[1][k, :h, :w] = pr.img2
    a = torch.from_numpy(big[0]).cuda()[:, :h, :w]
    b = torch.from_numpy(big[1]).cuda()[:, :h, :w]
    assert a.stride(1) == (w + 5) * 3 and a.stride(0) == (h + 3) * (w + 5) * 3
    o = matcher.match_batch(params, a, b)
    torch.cuda.synchronize()
    n = o["n"]
    fwd = matcher.to_numpy(o["fwd"]).reshape(len(pairs), n)
    bwd = matcher.to_numpy(o["bwd"]).reshape(len(pairs), n)
    comp = matcher.to_numpy(o["compact"]).reshape(len(pairs), n)
    _check_pairs(params, pairs, fwd, bwd, comp, o["n_inliers"].cpu().numpy(), int(o["n_evals"].item()), "padded")


@pytest.mark.parametrize("name,params,hw", [
    ("direction_patch11_9", base_params(feature=1, patch_fwd=11, patch_bwd=9, max_disp=6, rng_seed=41), (48, 64)),
    ("gray_patch13", base_params(color=1, patch_fwd=13, patch_bwd=13, max_disp=6, rng_seed=42), (48, 64)),
    ("ssd_patch8", base_params(metric=1, max_disp=6, rng_seed=43), (48, 64)),
    # odd seed counts at every level (247, 63, 15): the 8-byte distances of the squared metric
    # sit after an odd number of 4-byte displacements in LDS
    ("ssd_patch8_odd_grids", base_params(metric=1, max_disp=6, rng_seed=45), (40, 56)),
    ("sign_patch16", base_params(feature=2, patch_fwd=16, patch_bwd=16, max_disp=6, rng_seed=44), (48, 64)),
])
def test_batch16_small_levels_in_lds(matcher, name, params, hw):
    """Sixteen small pairs: at 16 pairs or more every level that fits in LDS runs in one
    work-group per pair and direction, here with 16-lane patches, gray, float direction
    features, signs and squared differences."""
    pairs = [synth.rect_pair(60 + i, hw[0], hw[1], n_rect=2, dmax=6) for i in range(16)]
    print(f"[gpu batch] batch16 {name}", file=sys.stderr, flush=True)
    pgm.pgm_profile(matcher.ctx, True)
    try:
        fwd, bwd, comp, nin, nev = run_batch(matcher, params, pairs)
        launches, _, _ = pgm.pgm_profile_read(matcher.ctx, pgm.K_LEVEL)
    finally:
        pgm.pgm_profile(matcher.ctx, False)
    assert launches > 0, "no level ran in LDS"
    _check_pairs(params, pairs, fwd, bwd, comp, nin, nev, name)
