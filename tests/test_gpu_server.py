"""GPU: the request server. Requests of mixed sizes submitted together (and through a pool too
small for all of them, so that some wait) must each give exactly what the oracle gives for
that pair alone."""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1704_03217_amd as pgm
import synth
from conftest import base_params

pytestmark = pytest.mark.gpu

SIZES = [(320, 240), (200, 150), (256, 192), (330, 250), (160, 120), (288, 200)]


def requests(torch):
    out = []
    for k, (w, h) in enumerate(SIZES):
        pr = synth.config_pair(5, 50 + k, (w, h))
        p = base_params(max_disp=max(1, -(-w // 5)), rng_seed=5000 + k)
        out.append((p, pr, torch.from_numpy(pr.img1).cuda(), torch.from_numpy(pr.img2).cuda()))
    return out


def run_all(server, reqs, torch, timeout_s=60.0):
    tags = {server.submit(p, a, b): k for k, (p, _, a, b) in enumerate(reqs)}
    done, t0, max_queued = {}, time.time(), 0
    while len(done) < len(reqs):
        q, r, f = server.pending()
        max_queued = max(max_queued, q)
        for tag, o in server.poll():
            done[tags[tag]] = o
        assert time.time() - t0 < timeout_s, "requests did not finish"
    torch.cuda.synchronize()
    return done, max_queued


def check(done, reqs):
    for k, (p, pr, _, _) in enumerate(reqs):
        o = done[k]
        r = oracle.match(p, pr.img1, pr.img2, trace=False)
        fwd = o["fwd"].cpu().numpy().view(pgm.MATCH_DTYPE)
        bwd = o["bwd"].cpu().numpy().view(pgm.MATCH_DTYPE)
        assert np.array_equal(fwd, r["fwd"]) and np.array_equal(bwd, r["bwd"]), f"request {k}"
        nin = int(o["n_inliers"].item())
        assert nin == r["n_inliers"]
        assert np.array_equal(o["compact"].cpu().numpy().view(pgm.MATCH_DTYPE)[:nin], r["compact"])


def test_server_mixed_sizes_equal_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu server] mixed sizes, large pool", file=sys.stderr, flush=True)
    reqs = requests(torch)
    srv = pgm.Server(0, 256 << 20, 3)
    try:
        done, _ = run_all(srv, reqs, torch)
        check(done, reqs)
    finally:
        srv.close()


def test_server_small_pool_queues_and_stays_exact():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu server] small pool", file=sys.stderr, flush=True)
    reqs = requests(torch)
    need = max((pgm.pgm_query(p, pr.img1.shape[1], pr.img1.shape[0]).workspace_bytes + 255) // 256 * 256
               for p, pr, _, _ in reqs)
    srv = pgm.Server(0, need + need // 2, 4)
    try:
        done, max_queued = run_all(srv, reqs, torch)
        assert max_queued > 0      # the pool held back some requests
        check(done, reqs)
    finally:
        srv.close()


def test_server_rejects_request_larger_than_pool():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    srv = pgm.Server(0, 1 << 20, 1)
    try:
        img = torch.zeros((192, 256, 3), dtype=torch.uint8, device="cuda")
        with pytest.raises(pgm.PGMError) as e:
            srv.submit(base_params(), img, img)
        assert e.value.status == pgm.PGM_ENOMEM
        assert srv.pending() == (0, 0, 0)
    finally:
        srv.close()
