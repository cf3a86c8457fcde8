"""GPU parity: libpgm (HIP, gfx950) against the CPU oracle's synchronous schedule.

The integer path must agree bit for bit in every level's displacements, distances and
flags, in the level-0 outputs, the compacted inliers and the number of distance
evaluations. The direction-only float path computes its patch distances exactly (see the
kernels), so it is held to the same bar.
"""
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
    m = pgm.Matcher(0, 768 << 20)
    yield m
    m.close()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(m, params, img1, img2):
    torch = m.torch
    t1 = torch.from_numpy(np.ascontiguousarray(img1)).cuda()
    t2 = torch.from_numpy(np.ascontiguousarray(img2)).cuda()
    o = m.match(params, t1, t2)
    torch.cuda.synchronize()
    n_in = int(o["n_inliers"].item())
    return dict(fwd=m.to_numpy(o["fwd"]), bwd=m.to_numpy(o["bwd"]), n_inliers=n_in,
                compact=m.to_numpy(o["compact"], n_in), n_evals=int(o["n_evals"].item()), sizes=o["sizes"])


def compare(m, params, img1, img2, name, levels=True, features=True):
    _say(f"[gpu parity] {name} {img1.shape[1]}x{img1.shape[0]} params={params}")
    g = gpu_run(m, params, img1, img2)
    r = oracle.match(params, img1, img2, schedule=oracle.SYNC)
    L = params["levels"]
    if features:
        check_features(m, params, img1, img2, name)
    if levels:
        problems = []
        for l in reversed(range(L)):          # coarse to fine: the first divergence comes first
            for d in range(2):
                got = m.dump_level(l, d)
                exp = r["levels"][d][l]
                if not np.array_equal(got, exp):
                    bad = np.nonzero((got != exp).any(axis=1))[0]
                    problems.append(f"level {l} dir {d}: {len(bad)} of {len(exp)} seeds differ; first {bad[:5]}: "
                                    f"gpu {got[bad[:3]].tolist()} oracle {exp[bad[:3]].tolist()}")
        assert not problems, f"{name}: " + " | ".join(problems)
    for key in ("fwd", "bwd"):
        assert np.array_equal(g[key], r[key]), f"{name}: {key} output differs"
    assert g["n_inliers"] == r["n_inliers"]
    assert np.array_equal(g["compact"], r["compact"])
    assert g["n_evals"] == r["n_evals"], (g["n_evals"], r["n_evals"])
    return g, r


def check_features(m, params, img1, img2, name):
    """Pyramid (Sec. III-D) and gradient image (Eq. 1-2) of every level, bit-exact, in the
    colour space of each direction's pyramid (Table II)."""
    L = params["levels"]
    f32 = params["feature"] == 1
    ch = 1 if params["color"] == 1 else 3
    sf = params.get("space_fwd", [0] * L)
    sb = params.get("space_bwd", [0] * L)
    ims = [np.ascontiguousarray(img1), np.ascontiguousarray(img2)]
    problems = []
    for l in range(L):
        if l > 0:
            ims = [oracle.pyr_down(x) for x in ims]
        for k in range(2):
            gp = m.dump_pyramid(l, k)
            if not np.array_equal(gp, ims[k]):
                problems.append(f"pyramid level {l} image {k}: {(gp != ims[k]).sum()} values differ")
        for slot in range(4):
            k = slot % 2
            space = sf[l] if slot < 2 else sb[l]
            src = oracle.gray(ims[k]) if ch == 1 else oracle.convert(ims[k], space)
            G = oracle.gradient_image(src, params["sobel_ksize"])
            if f32:
                G = oracle.direction(G)
            elif params["feature"] == 2:
                G = oracle.sign(G)
            got = m.dump_gradient(l, slot, 2 * ch, f32)
            a, b = (got.view(np.uint32), G.view(np.uint32)) if f32 else (got, G)
            if not np.array_equal(a, b):
                bad = np.argwhere(a != b)
                problems.append(f"gradient level {l} slot {slot}: {len(bad)} values differ, first {bad[:3].tolist()} "
                                f"gpu {[got[tuple(i)] for i in bad[:3]]} oracle {[G[tuple(i)] for i in bad[:3]]}")
    assert not problems, f"{name}: " + " | ".join(problems)


def tie_pair(kind, h=40, w=56):
    """Degenerate inputs whose candidate costs tie: flat images (all gradients zero) and
    vertical stripes of period 4."""
    if kind == "flat":
        img = np.full((h, w, 3), 100, np.uint8)
    else:
        col = np.array([30, 90, 200, 140], np.uint8)[np.arange(w) % 4]
        img = np.repeat(np.repeat(col[None, :, None], h, axis=0), 3, axis=2)
    return synth.Pair(img, img.copy(), np.zeros((h, w, 2), np.float32), np.ones((h, w), bool))


CASES = {
    "config1": (lambda: synth.config_pair(1), CONFIG_PARAMS[1]),
    "config1_s3_patch5_11": (lambda: synth.config_pair(1), base_params(sobel_ksize=3, patch_fwd=5, patch_bwd=11, rng_seed=7)),
    "config1_gray": (lambda: synth.config_pair(1), base_params(color=1, rng_seed=8)),
    "config1_refine2": (lambda: synth.config_pair(1), base_params(refine_rounds=2, rng_seed=9)),
    "config1_patch16_tau0": (lambda: synth.config_pair(1), base_params(patch_fwd=16, patch_bwd=16, consistency_px=0, rng_seed=10)),
    "config1_patch1_nofb": (lambda: synth.config_pair(1), base_params(patch_fwd=1, patch_bwd=1, fwd_bwd=0, rng_seed=11)),
    "config1_patch15_paper_like": (lambda: synth.config_pair(1), base_params(patch_fwd=15, patch_bwd=11, iters=[6, 4, 4], refine_rounds=2, rng_seed=12)),
    "dense_stride1": (lambda: synth.rect_pair(5, 48, 64, dmax=6), base_params(seed_stride=1, max_disp=6, rng_seed=13)),
    "stride2_even": (lambda: synth.rect_pair(6, 50, 70, dmax=8), base_params(seed_stride=2, max_disp=8, rng_seed=14)),
    "exhaustive": (lambda: synth.rect_pair(3, 32, 40, dmax=4), base_params(levels=2, iters=[3, 3], init_mode=1, max_disp=6, rng_seed=15)),
    "exhaustive_whole_image": (lambda: synth.rect_pair(4, 20, 24, n_rect=2, dmax=4), base_params(levels=1, iters=[2], init_mode=1, max_disp=0)),
    "tiny_1x1": (lambda: synth.rect_pair(1, 1, 1, n_rect=0, dmax=1), base_params(levels=1, iters=[2])),
    "tiny_3x2": (lambda: synth.rect_pair(1, 2, 3, n_rect=0, dmax=1), base_params(levels=2, iters=[2, 2], max_disp=2)),
    "ragged_17x9": (lambda: synth.rect_pair(2, 9, 17, n_rect=1, dmax=3), base_params(levels=3, iters=[3, 3, 3], max_disp=4)),
    "ragged_101x67": (lambda: synth.rect_pair(3, 67, 101, dmax=10), base_params(levels=4, iters=[2, 3, 4, 5], max_disp=12)),
    "wide_16384x12": (lambda: synth.rect_pair(9, 12, 16384, n_rect=2, dmax=20), base_params(levels=2, iters=[2, 2], max_disp=20, seed_stride=5)),
    "tall_12x16384": (lambda: synth.rect_pair(10, 16384, 12, n_rect=2, dmax=20), base_params(levels=2, iters=[2, 2], max_disp=20, seed_stride=5)),
    "translation": (lambda: synth.translate_pair(3, 72, 96, 10, -6), base_params(levels=2, iters=[8, 8], max_disp=16)),
    "identical": (lambda: (lambda p: synth.Pair(p.img1, p.img1, p.flow, p.valid))(synth.config_pair(1)), base_params(rng_seed=3)),
    # small-region removal (Sec. III-E): the paper's 9 px / 12 px on a dense field, and a
    # stride-3 grid where regions under 9 seeds of equal displacement go
    # "G./|G|" read element-wise (literal signs, Sec. III-F), colour and gray
    "sign_feature": (lambda: synth.config_pair(1), base_params(feature=2, rng_seed=18)),
    "sign_feature_gray_dense": (lambda: synth.rect_pair(22, 48, 64, dmax=6), base_params(feature=2, color=1, seed_stride=1, max_disp=6, rng_seed=19)),
    # the colour spaces of Table II (forward RGB, CIELab, YCrCb; backward CIELab, YCrCb, RGB),
    # the same with direction features, and one space shared by both pyramids
    "spaces_table2": (lambda: synth.config_pair(1), base_params(space_fwd=[0, 2, 1], space_bwd=[2, 1, 0], rng_seed=20)),
    "spaces_table2_direction": (lambda: synth.config_pair(1), base_params(feature=1, space_fwd=[0, 2, 1], space_bwd=[2, 1, 0], rng_seed=21)),
    "spaces_shared_lab": (lambda: synth.rect_pair(23, 96, 128, dmax=10), base_params(levels=2, iters=[3, 3], max_disp=10, space_fwd=[2, 2], space_bwd=[2, 2], rng_seed=22)),
    "regions_dense": (lambda: synth.rect_pair(21, 72, 96, dmax=8), base_params(seed_stride=1, levels=2, iters=[3, 3], max_disp=8, min_region_px=9, region_link_px=12, rng_seed=16)),
    "regions_stride3": (lambda: synth.config_pair(1), base_params(min_region_px=81, region_link_px=1, rng_seed=17)),
    # Eq. 3 as printed: squared differences, 64-bit sums (colour, 16-wide patches, signs,
    # gray dense with the exhaustive start)
    "ssd": (lambda: synth.config_pair(1), base_params(metric=1, rng_seed=23)),
    "ssd_patch16_s3": (lambda: synth.config_pair(1), base_params(metric=1, patch_fwd=16, patch_bwd=13, sobel_ksize=3, rng_seed=24)),
    "ssd_sign": (lambda: synth.config_pair(1), base_params(metric=1, feature=2, rng_seed=25)),
    "ssd_gray_dense_exhaustive": (lambda: synth.rect_pair(24, 40, 56, dmax=5), base_params(metric=1, color=1, seed_stride=1, levels=2, iters=[3, 3], init_mode=1, max_disp=6, rng_seed=26)),
    # one random-search candidate at the initial level (R_top = 1), and a level without
    # iterations between two with them (entered, checked and left without a sweep)
    "init_radius1": (lambda: synth.rect_pair(25, 60, 80, dmax=2), base_params(levels=2, iters=[3, 3], max_disp=2, rng_seed=27)),
    "level_without_iterations": (lambda: synth.rect_pair(26, 90, 120, dmax=8), base_params(levels=3, iters=[3, 0, 2], max_disp=8, rng_seed=28)),
    # ties everywhere: flat images (zero gradients) and periodic stripes, with the exhaustive
    # start (first minimum in scan order) and with random starts and the full pyramid
    "flat_exhaustive": (lambda: tie_pair("flat"), base_params(levels=2, iters=[2, 2], init_mode=1, max_disp=6, rng_seed=35)),
    "flat_random": (lambda: tie_pair("flat"), base_params(levels=3, iters=[3, 3, 3], max_disp=8, rng_seed=36)),
    "stripes_exhaustive": (lambda: tie_pair("stripes"), base_params(levels=2, iters=[2, 2], init_mode=1, max_disp=6, patch_fwd=5, patch_bwd=5, rng_seed=37)),
    "stripes_random": (lambda: tie_pair("stripes"), base_params(levels=3, iters=[3, 3, 3], max_disp=8, rng_seed=38)),
    # the symmetric reading of the random-search offsets (uniform in [-w_i, w_i]), with a
    # large top radius and the refinement
    "rs_symmetric": (lambda: synth.config_pair(1), base_params(rs_mode=1, rng_seed=46)),
    "rs_symmetric_refine_ssd": (lambda: synth.rect_pair(28, 120, 160, dmax=16), base_params(rs_mode=1, metric=1, refine_rounds=1, max_disp=16, rng_seed=47)),
    # the batched/served presets' scaled bound (max_disp = -5: ceil(w / 5))
    "scaled_max_disp": (lambda: synth.rect_pair(29, 120, 200, dmax=40), base_params(levels=4, iters=[3] * 4, max_disp=-5, rng_seed=48)),
    # the deepest pyramid (8 levels: 300x260 down to 3x3)
    "levels8": (lambda: synth.rect_pair(27, 260, 300, dmax=12), base_params(levels=8, iters=[2] * 8, max_disp=12, rng_seed=29)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pipeline_bit_exact(matcher, name):
    make, params = CASES[name]
    pair = make()
    compare(matcher, params, pair.img1, pair.img2, name)


def test_config2_full_size_bit_exact(matcher):
    pair = synth.config_pair(2)
    g, r = compare(matcher, CONFIG_PARAMS[2], pair.img1, pair.img2, "config2")
    assert g["fwd"].shape[0] == 49445


def test_paper_preset_at_benchmark_size(matcher):
    """The paper's own parameters as the benchmark runs them: a dense stride-1 field of
    446,464 seeds per direction at 1024x436, patches 15 / 11, refinement N = 2, the colour
    spaces of Table II and small-region removal (Sec. III-E) at full resolution."""
    pair = synth.config_pair(2)
    p = pgm.params_dict(pgm.pgm_default_params(pgm.PRESET_PAPER))
    g, r = compare(matcher, p, pair.img1, pair.img2, "paper_preset_1024x436")
    assert g["fwd"].shape[0] == 1024 * 436


def test_config3_direction_full_size(matcher):
    pair = synth.config_pair(3)
    compare(matcher, CONFIG_PARAMS[3], pair.img1, pair.img2, "config3")


def test_direction_small_variants(matcher):
    pair = synth.config_pair(1)
    compare(matcher, base_params(feature=1, rng_seed=21), pair.img1, pair.img2, "dir_rgb")
    compare(matcher, base_params(feature=1, color=1, patch_fwd=11, patch_bwd=7, rng_seed=22), pair.img1, pair.img2, "dir_gray")


def test_repeatable_and_context_reuse(matcher):
    a = synth.config_pair(1)
    b = synth.rect_pair(77, 100, 150, dmax=12)
    p = CONFIG_PARAMS[1]
    g1 = gpu_run(matcher, p, a.img1, a.img2)
    gpu_run(matcher, base_params(levels=2, iters=[3, 3], rng_seed=5), b.img1, b.img2)
    g2 = gpu_run(matcher, p, a.img1, a.img2)
    assert np.array_equal(g1["fwd"], g2["fwd"]) and np.array_equal(g1["bwd"], g2["bwd"])
    assert g1["n_evals"] == g2["n_evals"]


def test_pitched_input(matcher):
    torch = matcher.torch
    pair = synth.config_pair(1)
    h, w = pair.img1.shape[:2]
    big1 = torch.zeros((h, w + 13, 3), dtype=torch.uint8, device="cuda")
    big2 = torch.zeros((h, w + 13, 3), dtype=torch.uint8, device="cuda")
    big1[:, :w] = torch.from_numpy(pair.img1).cuda()
    big2[:, :w] = torch.from_numpy(pair.img2).cuda()
    o = matcher.match(CONFIG_PARAMS[1], big1[:, :w], big2[:, :w])
    torch.cuda.synchronize()
    r = oracle.match(CONFIG_PARAMS[1], pair.img1, pair.img2)
    assert np.array_equal(matcher.to_numpy(o["fwd"]), r["fwd"])


def test_workspace_too_small_is_enomem(matcher):
    torch = matcher.torch
    small = pgm.Matcher(0, 1 << 16)
    try:
        img = torch.zeros((64, 64, 3), dtype=torch.uint8, device="cuda")
        with pytest.raises(pgm.PGMError) as e:
            small.match(base_params(), img, img)
        assert e.value.status == pgm.PGM_ENOMEM
    finally:
        small.close()


def test_image_span_of_2_31_bytes_is_einval(matcher):
    """The image kernels address an image's bytes with 32-bit offsets, so a pitch that makes one
    image span 2^31 bytes or more is refused before any launch (the images here are small; the
    pitch alone is checked)."""
    torch = matcher.torch
    img = torch.zeros((64, 64, 3), dtype=torch.uint8, device="cuda")
    o = matcher.outputs(base_params(), 64, 64)
    stream = torch.cuda.current_stream().cuda_stream
    pitch = (2**31 - 3 * 64 - 4) // 63 + 1   # 63 * pitch + 3 * 64 + 4 > 2^31 - 1
    with pytest.raises(pgm.PGMError) as e:
        pgm.pgm_match(matcher.ctx, base_params(), img.data_ptr(), img.data_ptr(), 64, 64, pitch,
                      o["fwd"].data_ptr(), None, None, None, None, stream)
    assert e.value.status == pgm.PGM_EINVAL
    assert "2^31" in pgm.pgm_last_error(matcher.ctx)
    torch.cuda.synchronize()


@pytest.mark.parametrize("size", [(160, 118), (240, 200), (330, 250)], ids=["160x118", "240x200", "330x250"])
@pytest.mark.parametrize("iters", [[1, 2, 3, 5], [4, 6, 7, 1], [2, 5, 8, 3]], ids=["1-2-3-5", "4-6-7-1", "2-5-8-3"])
def test_multi_half_sweeps_every_count(matcher, iters, size):
    """Smaller levels run several half-sweeps per launch, each launch reading the field from one
    buffer and writing it whole to the other, the level's entry writing the second buffer when
    the number of such launches is odd: up to four per launch on levels of at most 8192 seeds
    (every level of the 160x118 and 240x200 pairs, 80x67 seeds at level 0 of the latter), two
    on 6x8 tiles with a last odd one in place at most 16384 (level 0 of the 330x250 pair,
    110x84 seeds). Per-level iteration counts 1-8, with and without the first half-sweep fused
    into the level's entry, on seed grids whose tiles are cut by every border, against the
    oracle bit for bit; and the same under PGM_SCHED_SEPARATE (one launch per half-sweep)."""
    pair = synth.config_pair(1, 21, size)
    img1, img2 = pair.img1, pair.img2
    params = base_params(levels=4, iters=iters, seed_stride=3, radius=3, max_disp=24, rng_seed=4242)
    compare(matcher, params, img1, img2, f"multi iters {iters}", features=False)
    pgm.pgm_schedule(matcher.ctx, pgm.SCHED_SEPARATE)
    try:
        compare(matcher, params, img1, img2, f"separate iters {iters}", features=False)
    finally:
        pgm.pgm_schedule(matcher.ctx, pgm.SCHED_AUTO)
