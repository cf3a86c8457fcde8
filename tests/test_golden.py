"""Stored fixtures under tests/golden/: the settings the paper states (Sec. IV, Sec. III-E,
Table II, Sec. III-G), the Sobel kernels of Eq. 1-2 as the oracle's impulse response, and
frozen CPU-oracle runs (written by tests/golden/make_golden.py) that the oracle must still
reproduce and the HIP library must equal (the GPU test)."""
import glob
import math
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1704_03217_amd as pgm
from conftest import CONFIG_PARAMS, ROOT

GOLDEN = os.path.join(ROOT, "tests", "golden")
sys.path.insert(0, GOLDEN)
import make_golden  # noqa: E402

TINY = sorted(glob.glob(os.path.join(GOLDEN, "tiny_*.txt")))
SPACES = {"RGB": pgm.SPACE_RGB, "CIELab": pgm.SPACE_LAB, "YCrCb": pgm.SPACE_YCRCB}


def paper_settings():
    out = {}
    for ln in open(os.path.join(GOLDEN, "paper_settings.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        body, where = ln.split("|")
        name, *vals = body.split()
        assert where.strip()
        out[name] = vals
    return out


def sobel_kernels():
    ks, cur = {}, None
    for ln in open(os.path.join(GOLDEN, "sobel_kernels.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        if ln.startswith("S "):
            cur = int(ln.split()[1])
            ks[cur] = []
        else:
            ks[cur].append([int(v) for v in ln.split()])
    return {S: np.array(k, np.int64) for S, k in ks.items()}


def as_rows(m):
    return np.stack([m[k].astype(np.int64) for k in m.dtype.names], axis=1)


def test_paper_preset_is_the_papers_settings():
    s = paper_settings()
    d = pgm.params_dict(pgm.pgm_default_params(pgm.PRESET_PAPER))
    L = int(s["L"][0])
    assert d["radius"] == int(s["W"][0])
    assert d["sobel_ksize"] == int(s["S"][0])
    assert d["levels"] == L and d["levels"] - 1 == int(s["m"][0])
    assert d["refine_rounds"] == int(s["N"][0])
    assert d["iters"] == [int(s["iters_full"][0])] + [int(s["iters_other"][0])] * (L - 1)
    assert d["patch_fwd"] == 2 * int(s["r_fwd"][0]) + 1 and d["patch_bwd"] == 2 * int(s["r_bwd"][0]) + 1
    assert d["min_region_px"] == int(s["min_region_px"][0])
    assert d["space_fwd"] == [SPACES[v] for v in s["space_fwd"]]
    assert d["space_bwd"] == [SPACES[v] for v in s["space_bwd"]]
    # Table II: the two pyramids differ at every level, and each uses every space once
    assert all(a != b for a, b in zip(d["space_fwd"], d["space_bwd"]))
    assert sorted(d["space_fwd"]) == sorted(d["space_bwd"]) == sorted(SPACES.values())


def test_pyramid_scale_and_grid_spacing():
    s = paper_settings()
    scale = float(s["s"][0])
    d = pgm.params_dict(pgm.pgm_default_params(pgm.PRESET_PAPER))
    for w, h in ((1024, 436), (1242, 375), (33, 17)):
        geo = oracle.geometry(d, w, h)
        for l, (lw, lh, nx, ny) in enumerate(geo):
            assert (lw, lh) == (math.ceil(w * scale ** l), math.ceil(h * scale ** l))
            assert (nx, ny) == (lw, lh)          # dense field: one seed per pixel
    # the grid workloads match on the paper's output grid
    for cfg in CONFIG_PARAMS.values():
        assert cfg["seed_stride"] == int(s["grid_spacing"][0])


@pytest.mark.parametrize("S", [3, 5])
def test_oracle_impulse_response_is_the_sobel_kernel(S):
    K = sobel_kernels()[S]
    assert K.shape == (S, S)
    h, w, y0, x0, v = 15, 17, 7, 8, 3
    img = np.zeros((h, w, 3), np.uint8)
    img[y0, x0, 1] = v
    G = oracle.gradient_image(img, S).astype(np.int64)
    k = S // 2
    win = G[y0 - k:y0 + k + 1, x0 - k:x0 + k + 1]
    # correlation with an impulse gives the kernel turned half a turn
    np.testing.assert_array_equal(win[::-1, ::-1, 1], v * K)
    np.testing.assert_array_equal(win[::-1, ::-1, 4], v * K.T)
    assert not G[..., [0, 2, 3, 5]].any()
    # nothing outside the kernel's footprint
    G[y0 - k:y0 + k + 1, x0 - k:x0 + k + 1] = 0
    assert not G.any()


@pytest.mark.parametrize("path", TINY, ids=[os.path.basename(p)[:-4] for p in TINY])
def test_oracle_reproduces_frozen_run(path):
    p, img1, img2, fwd, bwd, nin, nev = make_golden.read(path)
    r = oracle.match(p, img1, img2, trace=False)
    np.testing.assert_array_equal(as_rows(r["fwd"]), fwd)
    np.testing.assert_array_equal(as_rows(r["bwd"]), bwd)
    assert (r["n_inliers"], r["n_evals"]) == (nin, nev)
    assert nin == int(((fwd[:, 5] & pgm.FLAG_INLIER) != 0).sum())


def test_frozen_runs_cover_the_cases():
    assert {os.path.basename(p)[:-4] for p in TINY} == set(make_golden.CASES)


@pytest.fixture(scope="module")
def matcher():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = pgm.Matcher(0, 256 << 20)
    yield m
    m.close()


@pytest.mark.gpu
@pytest.mark.parametrize("path", TINY, ids=[os.path.basename(p)[:-4] for p in TINY])
def test_library_equals_frozen_run(matcher, path):
    torch = matcher.torch
    p, img1, img2, fwd, bwd, nin, nev = make_golden.read(path)
    print(f"[gpu golden] {os.path.basename(path)}", file=sys.stderr, flush=True)
    h, w = img1.shape[:2]
    o = matcher.outputs(p, w, h)
    matcher.match_into(p, torch.from_numpy(img1).cuda(), torch.from_numpy(img2).cuda(), o)
    torch.cuda.synchronize()
    n = o["n"]
    got_f = matcher.to_numpy(o["fwd"])[:n]
    got_b = matcher.to_numpy(o["bwd"])[:n]
    np.testing.assert_array_equal(as_rows(got_f), fwd)
    np.testing.assert_array_equal(as_rows(got_b), bwd)
    assert int(o["n_inliers"].cpu()[0]) == nin and int(o["n_evals"].item()) == nev
    comp = as_rows(matcher.to_numpy(o["compact"])[:nin])
    np.testing.assert_array_equal(comp, fwd[(fwd[:, 5] & pgm.FLAG_INLIER) != 0])
