"""Host-only checks of the C ABI: the library loads, exports every declared entry point, its
struct layouts agree with the binding, presets and sizes agree with the oracle's geometry,
and invalid arguments are rejected without device work."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import paper_1704_03217_amd as pgm
from conftest import CONFIG_PARAMS, ROOT, base_params

HEADER = os.path.join(ROOT, "include", "pgm.h")


def declared_functions():
    src = open(HEADER).read()
    return re.findall(r"PGM_API\s+[\w\s\*]+?\b(pgm_\w+)\s*\(", src)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(pgm.EXPORTS)
    L = pgm.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", pgm.LIB_PATH]).decode()
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_struct_layout_matches_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "pgm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(pgm_params), offsetof(pgm_params, iters),
         offsetof(pgm_params, rng_seed), sizeof(pgm_match_t), sizeof(pgm_sizes),
         offsetof(pgm_sizes, workspace_bytes), offsetof(pgm_sizes, workspace_pair_bytes),
         sizeof(pgm_group), offsetof(pgm_group, image_stride_bytes), offsetof(pgm_group, out_compact));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    exp = [C.sizeof(pgm.pgm_params), pgm.pgm_params.iters.offset, pgm.pgm_params.rng_seed.offset,
           pgm.MATCH_BYTES, C.sizeof(pgm.pgm_sizes), pgm.pgm_sizes.workspace_bytes.offset,
           pgm.pgm_sizes.workspace_pair_bytes.offset, C.sizeof(pgm.pgm_group),
           pgm.pgm_group.image_stride_bytes.offset, pgm.pgm_group.out_compact.offset]
    assert got == exp
    assert pgm.MATCH_DTYPE.itemsize == pgm.MATCH_BYTES


@pytest.mark.parametrize("preset,cfg", [(pgm.PRESET_CONFIG1, 1), (pgm.PRESET_CONFIG2, 2), (pgm.PRESET_CONFIG3, 3)])
def test_presets_match_workload_parameters(preset, cfg):
    d = pgm.params_dict(pgm.pgm_default_params(preset))
    assert d == CONFIG_PARAMS[cfg]


def test_paper_preset():
    d = pgm.params_dict(pgm.pgm_default_params(pgm.PRESET_PAPER))
    # Sec. IV: W=2, S=5, L=3, N=2, 6 iterations at full resolution and 4 elsewhere; r = 7 / 5
    assert (d["radius"], d["sobel_ksize"], d["levels"], d["refine_rounds"]) == (2, 5, 3, 2)
    assert d["iters"] == [6, 4, 4]
    assert (d["patch_fwd"], d["patch_bwd"]) == (15, 11)
    assert d["seed_stride"] == 1
    assert (d["min_region_px"], d["region_link_px"]) == (9, 12)   # Sec. III-E
    assert d["space_fwd"] == [pgm.SPACE_RGB, pgm.SPACE_LAB, pgm.SPACE_YCRCB]   # Table II
    assert d["space_bwd"] == [pgm.SPACE_LAB, pgm.SPACE_YCRCB, pgm.SPACE_RGB]


@pytest.mark.parametrize("w,h,L,stride", [(1024, 436, 5, 3), (1242, 375, 5, 3), (256, 192, 3, 3),
                                          (1, 1, 1, 3), (17, 9, 3, 2), (640, 480, 8, 1), (16384, 12, 2, 5)])
def test_query_geometry_matches_oracle(w, h, L, stride):
    p = base_params(levels=L, seed_stride=stride, iters=[2] * L)
    s = pgm.pgm_query(p, w, h)
    geo = oracle.geometry(p, w, h)
    assert s.levels == L
    for l, (lw, lh, nx, ny) in enumerate(geo):
        assert (s.level_w[l], s.level_h[l], s.level_nx[l], s.level_ny[l]) == (lw, lh, nx, ny)
    assert (s.nx, s.ny) == geo[0][2:]
    assert s.workspace_bytes > 0
    assert s.workspace_bytes == s.workspace_shared_bytes + s.workspace_pair_bytes


def test_query_workspace_of_config2_is_modest():
    s = pgm.pgm_query(CONFIG_PARAMS[2], 1024, 436)
    assert s.nx * s.ny == 49445
    assert s.workspace_bytes < 64 << 20


@pytest.mark.parametrize("bad", [dict(levels=0), dict(levels=9), dict(seed_stride=0), dict(patch_fwd=0),
                                 dict(patch_bwd=17), dict(iters=[256, 1, 1]), dict(radius=0),
                                 dict(sobel_ksize=7), dict(feature=3), dict(color=3), dict(fwd_bwd=2),
                                 dict(consistency_px=-1), dict(init_mode=2), dict(refine_rounds=17),
                                 dict(levels=1, iters=[1], refine_rounds=1), dict(max_disp=-1025),
                                 dict(min_region_px=-1), dict(min_region_px=9, region_link_px=0),
                                 dict(min_region_px=9, region_link_px=65536), dict(space_fwd=[3, 0, 0]),
                                 dict(space_bwd=[0, -1, 0]), dict(color=1, space_fwd=[1, 0, 0]),
                                 dict(metric=2), dict(metric=-1), dict(metric=1, feature=1), dict(rs_mode=2)])
def test_query_rejects_invalid_parameters(bad):
    with pytest.raises(pgm.PGMError) as e:
        pgm.pgm_query(base_params(**bad), 64, 64)
    assert e.value.status == pgm.PGM_EINVAL


@pytest.mark.parametrize("w,h", [(0, 10), (10, 0), (16385, 10), (10, 16385)])
def test_query_rejects_bad_sizes(w, h):
    with pytest.raises(pgm.PGMError):
        pgm.pgm_query(base_params(), w, h)


def test_null_arguments_rejected_without_device_work():
    L = pgm.lib()
    assert L.pgm_default_params(None, 1) == pgm.PGM_EINVAL
    assert L.pgm_default_params(C.byref(pgm.pgm_params()), 99) == pgm.PGM_EINVAL
    assert L.pgm_query(None, 10, 10, C.byref(pgm.pgm_sizes())) == pgm.PGM_EINVAL
    assert L.pgm_query(C.byref(pgm.params(base_params())), 10, 10, None) == pgm.PGM_EINVAL
    assert L.pgm_create(0, 0, None) == pgm.PGM_EINVAL
    p = pgm.params(base_params())
    assert L.pgm_match(None, C.byref(p), None, None, 10, 10, 30, None, None, None, None, None, None) == pgm.PGM_EINVAL
    assert L.pgm_match_batch(None, C.byref(p), 2, None, None, 10, 10, 30, 300, None, None, None, None, None,
                             None) == pgm.PGM_EINVAL
    assert L.pgm_match_groups(None, 1, None, None, 0, None) == pgm.PGM_EINVAL
    assert L.pgm_server_create(0, 1 << 20, 0, 0, 0, C.byref(C.c_void_p())) == pgm.PGM_EINVAL
    assert L.pgm_server_create(0, 1 << 20, 1, -1, 0, C.byref(C.c_void_p())) == pgm.PGM_EINVAL
    assert L.pgm_server_create(0, 1 << 20, 1, 0, 17, C.byref(C.c_void_p())) == pgm.PGM_EINVAL
    assert L.pgm_server_create(0, 1 << 20, 1, 0, 0, None) == pgm.PGM_EINVAL
    assert L.pgm_server_stats(None, None, None, None) == pgm.PGM_EINVAL
    assert L.pgm_server_submit(None, C.byref(p), None, None, 10, 10, 30, None, None, None, None, None, 0,
                               None) == pgm.PGM_EINVAL
    assert L.pgm_server_poll(None, None, None, 0) == pgm.PGM_EINVAL
    assert L.pgm_server_drain(None) == pgm.PGM_EINVAL
    L.pgm_server_destroy(None)
    assert L.pgm_dump_level(None, 0, 0, None) == pgm.PGM_EINVAL
    L.pgm_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pgm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pgm, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        pgm.lib()


def test_format_matches_epicflow_lines(tmp_path):
    """Host-only formatting of grid matches as "x1 y1 x2 y2" lines, all or inliers only."""
    rng = np.random.default_rng(3)
    m = np.zeros(50, pgm.MATCH_DTYPE)
    for k in ("x1", "y1", "x2", "y2"):
        m[k] = rng.integers(-5, 2000, 50)
    m["dist"] = rng.integers(0, 10**6, 50)
    m["flags"] = rng.integers(0, 8, 50)
    text_all = pgm.pgm_format_matches(m, inliers_only=False)
    assert text_all == "".join(f"{a} {b} {c} {d}\n" for a, b, c, d in zip(m["x1"], m["y1"], m["x2"], m["y2"]))
    inl = m[(m["flags"] & pgm.FLAG_INLIER) != 0]
    path = tmp_path / "matches.txt"
    n = pgm.write_epicflow_matches(str(path), m)
    assert n == len(inl)
    back = np.loadtxt(path, dtype=np.int64, ndmin=2)
    assert np.array_equal(back, np.stack([inl["x1"], inl["y1"], inl["x2"], inl["y2"]], 1))
    assert pgm.pgm_format_matches(m[:0]) == ""
    L = pgm.lib()
    small = C.create_string_buffer(4)
    need = C.c_uint64()
    assert L.pgm_format_matches(m.ctypes.data, 50, 0, small, 4, C.byref(need)) == pgm.PGM_ENOMEM
    assert need.value == len(text_all)
    assert L.pgm_format_matches(None, 5, 0, None, 0, C.byref(need)) == pgm.PGM_EINVAL


def test_schedule_needs_a_context():
    assert pgm.lib().pgm_schedule(None, 0) == pgm.PGM_EINVAL


def test_tune_rejects_bad_arguments_without_device_work():
    L = pgm.lib()
    p = pgm.pgm_default_params(pgm.PRESET_CONFIG1)
    f = C.c_int32(-1)
    # no context
    assert L.pgm_tune(None, C.byref(p), 1, None, None, 64, 64, 192, 0, None, None, None, None, 1, None,
                      C.byref(f)) == pgm.PGM_EINVAL
    assert f.value == -1


@pytest.mark.parametrize("preset", [pgm.PRESET_CONFIG4, pgm.PRESET_CONFIG5])
def test_batch_and_served_presets(preset):
    """Configurations 4 and 5: configuration 2's matching with |d| <= ceil(w / 5) per pair."""
    d = pgm.params_dict(pgm.pgm_default_params(preset))
    exp = dict(CONFIG_PARAMS[2], max_disp=-5, rng_seed=1000 * preset)
    assert d == exp


@pytest.mark.parametrize("w,h", [(320, 240), (640, 480), (1024, 436), (1242, 375), (2048, 834), (333, 241)])
def test_scaled_max_disp_sets_the_top_radius_as_the_oracle(w, h):
    """max_disp = -k bounds |d| by ceil(w / k): the top radius equals the oracle's and that of
    the explicit bound ceil(w / 5)."""
    p = pgm.pgm_default_params(pgm.PRESET_CONFIG4)
    d = pgm.params_dict(p)
    explicit = dict(d, max_disp=-(-w // 5))
    assert oracle.top_radius(d, w, h) == oracle.top_radius(explicit, w, h)
    m = d["levels"] - 1
    assert oracle.top_radius(d, w, h) == -(-(-(-w // 5)) // (1 << m))
    # the library's workspace (random-number table sized by the top radius) agrees too
    q1 = pgm.pgm_query(p, w, h)
    q2 = pgm.pgm_query(pgm.params(explicit), w, h)
    assert q1.workspace_bytes == q2.workspace_bytes


def test_rs_mode_and_max_disp_are_validated():
    ok = base_params()
    pgm.pgm_query(ok, 256, 192)
    pgm.pgm_query(dict(ok, rs_mode=pgm.RS_SYMMETRIC), 256, 192)
    pgm.pgm_query(dict(ok, max_disp=-1024), 256, 192)
    for bad in (dict(ok, rs_mode=2), dict(ok, rs_mode=-1), dict(ok, max_disp=-1025)):
        with pytest.raises(pgm.PGMError) as e:
            pgm.pgm_query(bad, 256, 192)
        assert e.value.status == pgm.PGM_EINVAL


def test_status_codes_match_header():
    src = open(HEADER).read()
    for name in ("PGM_OK", "PGM_EINVAL", "PGM_ENOMEM", "PGM_EDEVICE", "PGM_EBUSY", "PGM_EUNSUPPORTED"):
        v = int(re.search(rf"\b{name}\s*=\s*(-?\d+)", src).group(1))
        assert getattr(pgm, name) == v, name


def test_pgm_log_reports_failures_on_stderr():
    """PGM_LOG=1 prints failures: here pgm_create refused on a machine without a usable device
    (or for a device index out of range)."""
    import sys
    code = ("import sys; sys.path.insert(0, %r); import paper_1704_03217_amd as pgm\n"
            "try:\n    pgm.pgm_create(999, 1 << 20)\nexcept pgm.PGMError as e:\n    print('status', e.status)\n"
            % ROOT)
    env = dict(os.environ, PGM_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert "status" in r.stdout
    assert "[pgm] error" in r.stderr
    env["PGM_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert "[pgm]" not in r.stderr


def test_division_multipliers_are_exact(tmp_path):
    """The kernels divide seed and work-group indices by launch-uniform values with host-
    computed multipliers (DivM, fdiv); the same code, built for the host, must give n / d for
    every divisor and dividend tried (all divisors up to 70000, powers of two and their
    neighbours, random 32-bit divisors; edge and random dividends)."""
    exe = tmp_path / "divm_check"
    src = os.path.join(ROOT, "tests", "divm_check.hip")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950",
                           "-I", os.path.join(ROOT, "paper_1704_03217_amd", "csrc"), src, "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert int(out.stdout.split()[-1]) > 10_000_000
