"""CPU: the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host
code only) runs the whole method on small cases of every kind of parameter without a
report, and gives the same results as the ordinary build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from conftest import ROOT, base_params

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    "config1": (lambda: synth.config_pair(1), base_params(rng_seed=1000)),
    "refine_gray": (lambda: synth.rect_pair(5, 60, 80, dmax=6), base_params(color=1, refine_rounds=2, max_disp=6)),
    "dense_regions_spaces": (lambda: synth.rect_pair(6, 30, 40, dmax=4),
                             base_params(seed_stride=1, patch_fwd=15, patch_bwd=11, min_region_px=9, max_disp=4,
                                         space_fwd=[0, 2, 1], space_bwd=[2, 1, 0])),
    "direction": (lambda: synth.rect_pair(7, 48, 64, dmax=6), base_params(feature=1, max_disp=6)),
    "ssd_sign_exhaustive": (lambda: synth.rect_pair(8, 24, 32, dmax=3),
                            base_params(metric=1, feature=2, init_mode=1, levels=2, iters=[2, 2], max_disp=4)),
    "symmetric_scaled": (lambda: synth.rect_pair(9, 50, 90, dmax=18), base_params(rs_mode=1, max_disp=-5)),
    "tiny_1x1": (lambda: synth.rect_pair(1, 1, 1, n_rect=0, dmax=1), base_params(levels=1, iters=[2])),
    "ragged_17x9_patch16": (lambda: synth.rect_pair(2, 9, 17, n_rect=1, dmax=3),
                            base_params(patch_fwd=16, patch_bwd=1, max_disp=4)),
}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "oracle_asan")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "oracle"),
                           os.path.join(HERE, "oracle_asan_driver.c"), os.path.join(ROOT, "oracle", "pgm_oracle.c"),
                           "-o", exe, "-lm"])
    return exe


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_clean_under_sanitizers(driver, tmp_path, name):
    make, params = CASES[name]
    pair = make()
    h, w = pair.img1.shape[:2]
    p = oracle.make_params(params)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        f.write(bytes(p))
        f.write(np.array([w, h], np.int32).tobytes())
        f.write(np.ascontiguousarray(pair.img1).tobytes())
        f.write(np.ascontiguousarray(pair.img2).tobytes())
    out = tmp_path / "out.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([driver, str(inp), str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    raw = out.read_bytes()
    _, _, nx, ny = oracle.geometry(params, w, h)[0]
    n = nx * ny
    off = 0
    for schedule in (oracle.SYNC, oracle.SCAN):
        nev = int(np.frombuffer(raw, np.uint64, 1, off)[0]); off += 8
        nin = int(np.frombuffer(raw, np.int32, 1, off)[0]); off += 4
        fwd = np.frombuffer(raw, oracle.MATCH_DTYPE, n, off); off += 24 * n
        bwd = np.frombuffer(raw, oracle.MATCH_DTYPE, n, off); off += 24 * n
        ref = oracle.match(params, pair.img1, pair.img2, schedule=schedule, trace=False)
        assert nev == ref["n_evals"] and nin == ref["n_inliers"]
        assert np.array_equal(fwd, ref["fwd"]) and np.array_equal(bwd, ref["bwd"])
    assert off == len(raw)
