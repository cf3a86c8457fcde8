"""GPU: pgm_match_static, the entry point for callers that cannot allocate device memory
(its workspace is a fixed array inside the library), against pgm_match on the same pairs:
two calls in a row, the second on a smaller pair, every output bit for bit; a pair larger
than the array is refused with PGM_ENOMEM before any device work."""
import sys

import numpy as np
import pytest

import paper_1704_03217_amd as pgm
import synth

pytestmark = pytest.mark.gpu


def _outputs(torch, n):
    dev = torch.device("cuda", 0)
    return dict(fwd=torch.empty(n * 6, dtype=torch.int32, device=dev),
                bwd=torch.empty(n * 6, dtype=torch.int32, device=dev),
                n_inliers=torch.zeros(1, dtype=torch.int32, device=dev),
                compact=torch.zeros(n * 6, dtype=torch.int32, device=dev),
                n_evals=torch.zeros(1, dtype=torch.int64, device=dev))


def _static(torch, p, a, b, o):
    h, w = a.shape[:2]
    stream = torch.cuda.current_stream(0).cuda_stream
    pgm.pgm_match_static(p, a.data_ptr(), b.data_ptr(), w, h, a.stride(0), o["fwd"].data_ptr(), o["bwd"].data_ptr(),
                         o["n_inliers"].data_ptr(), o["compact"].data_ptr(), o["n_evals"].data_ptr(), stream)


def _host(o, nin=None):
    n_in = int(o["n_inliers"].item())
    return dict(fwd=o["fwd"].cpu().numpy(), bwd=o["bwd"].cpu().numpy(), n_inliers=n_in,
                compact=o["compact"].cpu().numpy().reshape(-1, 6)[:n_in], n_evals=int(o["n_evals"].item()))


def test_static_entry_point_equals_pgm_match_twice_then_smaller():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cases = [(pgm.PRESET_CONFIG2, synth.config_pair(2, 3)), (pgm.PRESET_CONFIG1, synth.config_pair(1, 4))]
    m = pgm.Matcher(0, 64 << 20)
    try:
        for k, (preset, pair) in enumerate(cases):
            h, w = pair.img1.shape[:2]
            print(f"[gpu no-alloc] call {k}: {w}x{h} preset {preset}", file=sys.stderr, flush=True)
            p = pgm.pgm_default_params(preset)
            a = torch.from_numpy(pair.img1).cuda()
            b = torch.from_numpy(pair.img2).cuda()
            q = pgm.pgm_query(p, w, h)
            assert q.workspace_bytes <= pgm.STATIC_SCRATCH_BYTES
            n = q.nx * q.ny
            os_ = _outputs(torch, n)
            _static(torch, p, a, b, os_)
            ref = m.match(p, a, b)
            torch.cuda.synchronize()
            got, exp = _host(os_), _host(ref)
            for key in ("fwd", "bwd", "compact"):
                assert np.array_equal(got[key], exp[key]), (k, key)
            assert got["n_inliers"] == exp["n_inliers"] and got["n_evals"] == exp["n_evals"], k
            assert got["n_evals"] > 0 and got["n_inliers"] > 0
    finally:
        m.close()


def test_static_entry_point_refuses_pairs_beyond_its_array():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = pgm.pgm_default_params(pgm.PRESET_CONFIG5)
    w, h = 2048, 1024
    assert pgm.pgm_query(p, w, h).workspace_bytes > pgm.STATIC_SCRATCH_BYTES
    img = torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda")
    o = _outputs(torch, pgm.pgm_query(p, w, h).nx * pgm.pgm_query(p, w, h).ny)
    with pytest.raises(pgm.PGMError) as e:
        _static(torch, p, img, img, o)
    assert e.value.status == pgm.PGM_ENOMEM
    assert "fixed array" in pgm.pgm_last_error(None)
