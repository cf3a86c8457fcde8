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
        if o["n_evals"] is not None:
            assert int(o["n_evals"].item()) == r["n_evals"], f"request {k}: evaluations"
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


# sizes the benchmark's served stream reaches (log-uniform area up to 2048x1024)
LARGE_SIZES = [(2048, 834), (1024, 436), (640, 480), (1500, 700), (320, 240)]


def test_server_large_served_sizes_equal_oracle():
    """Requests as large as the served benchmark's (a 2048-wide pair among them), with the
    served preset (configuration 2's matching, |d| <= ceil(w / 5)), each bit-exact with the
    oracle on that pair alone."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu server] large served sizes", file=sys.stderr, flush=True)
    reqs = []
    for k, (w, h) in enumerate(LARGE_SIZES):
        pr = synth.config_pair(5, 80 + k, (w, h))
        p = pgm.params_dict(pgm.pgm_default_params(pgm.PRESET_CONFIG5))
        p["rng_seed"] = 5100 + k
        reqs.append((p, pr, torch.from_numpy(pr.img1).cuda(), torch.from_numpy(pr.img2).cuda()))
    need = sum((pgm.pgm_query(p, pr.img1.shape[1], pr.img1.shape[0]).workspace_bytes + 255) // 256 * 256
               for p, pr, _, _ in reqs)
    srv = pgm.Server(0, need // 2, 4)     # the pool holds about half of them at once
    try:
        done, max_queued = run_all(srv, reqs, torch, timeout_s=120.0)
        assert max_queued > 0
        check(done, reqs)
    finally:
        srv.close()


def test_server_waits_for_the_callers_stream():
    """Images written by torch on the current stream just before submit (behind a long
    kernel) are the ones matched: the request's launches wait for the caller's stream."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu server] ordering after the caller's stream", file=sys.stderr, flush=True)
    src = requests(torch)
    srv = pgm.Server(0, 256 << 20, 4)
    try:
        reqs, tags = [], {}
        for k, (p, pr, a, b) in enumerate(src):
            img1 = torch.zeros_like(a)
            img2 = torch.zeros_like(b)
            torch.cuda._sleep(20_000_000)       # ~10 ms of GPU time on the current stream
            img1.copy_(a)
            img2.copy_(b)
            reqs.append((p, pr, img1, img2))
            tags[srv.submit(p, img1, img2)] = k
        done = {}
        t0 = time.time()
        while len(done) < len(reqs):
            for tag, o in srv.poll():
                done[tags[tag]] = o
            assert time.time() - t0 < 60.0
        torch.cuda.synchronize()
        check(done, reqs)
    finally:
        srv.close()


def test_server_full_queue_is_ebusy():
    """With max_queued = 1 and a pool for one request, a third request submitted while the
    first waits for the caller's stream and the second waits for memory is refused with
    PGM_EBUSY (nothing queued); after the queue drains it is accepted, and all three results
    equal the oracle's."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu server] full queue", file=sys.stderr, flush=True)
    reqs = requests(torch)[:3]
    need = max((pgm.pgm_query(p, pr.img1.shape[1], pr.img1.shape[0]).workspace_bytes + 255) // 256 * 256
               for p, pr, _, _ in reqs)
    srv = pgm.Server(0, need, 2, max_queued=1)
    try:
        tags = {}
        torch.cuda._sleep(200_000_000)          # holds the first request's start (~0.1 s)
        p, _, a, b = reqs[0]
        tags[srv.submit(p, a, b)] = 0
        p, _, a, b = reqs[1]
        tags[srv.submit(p, a, b)] = 1
        assert srv.pending()[0] == 1            # the second waits for memory
        p, _, a, b = reqs[2]
        with pytest.raises(pgm.PGMError) as e:
            srv.submit(p, a, b)
        assert e.value.status == pgm.PGM_EBUSY
        assert srv.pending()[0] == 1
        done, t0 = {}, time.time()
        while len(done) < 2:
            for tag, o in srv.poll():
                done[tags[tag]] = o
            assert time.time() - t0 < 60.0
        tags[srv.submit(p, a, b)] = 2
        while len(done) < 3:
            for tag, o in srv.poll():
                done[tags[tag]] = o
            assert time.time() - t0 < 60.0
        torch.cuda.synchronize()
        check(done, reqs)
    finally:
        srv.close()


def test_server_same_shape_requests_share_launches():
    """Requests of three shapes (different images, one parameter set per shape) queue behind a
    long kernel on the caller's stream; once memory frees, queued requests of the head's
    shape start together as one batch (fewer launch sequences than requests). Every result,
    the evaluation count included, equals the oracle's on that pair alone."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu server] same-shape requests batched", file=sys.stderr, flush=True)
    shapes = [(320, 240), (256, 192), (330, 250)]
    reqs = []
    for k in range(12):
        w, h = shapes[k % 3]
        pr = synth.config_pair(5, 300 + k, (w, h))
        p = base_params(max_disp=max(1, -(-w // 5)), rng_seed=5200 + k % 3)
        reqs.append((p, pr, torch.from_numpy(pr.img1).cuda(), torch.from_numpy(pr.img2).cuda()))
    need = max((pgm.pgm_query(p, pr.img1.shape[1], pr.img1.shape[0]).workspace_bytes + 255) // 256 * 256
               for p, pr, _, _ in reqs)
    srv = pgm.Server(0, 16 * need, 2)         # at most 4 launch sequences in flight
    try:
        tags = {}
        torch.cuda._sleep(100_000_000)          # the first requests wait; the rest queue up
        for k, (p, _, a, b) in enumerate(reqs):
            tags[srv.submit(p, a, b, count_evals=True)] = k
        assert srv.pending()[0] > 0
        done, t0 = {}, time.time()
        while len(done) < len(reqs):
            for tag, o in srv.poll():
                done[tags[tag]] = o
            assert time.time() - t0 < 60.0
        torch.cuda.synchronize()
        sequences, started, in_use = srv.stats()
        assert started == len(reqs) and sequences < len(reqs), (sequences, started)
        assert in_use == 0          # every sequence finished and gave its memory back
        check(done, reqs)
    finally:
        srv.close()


def test_server_logs_requests_with_pgm_log():
    """PGM_LOG=2: the server logs its creation, each started launch sequence with the pool bytes
    in use, and each finished request with its latency (in a child process, stderr captured)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import os
    import subprocess
    from conftest import ROOT
    code = f"""
import sys, time
sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})
import torch
import paper_1704_03217_amd as pgm
import synth
from conftest import base_params
srv = pgm.Server(0, 64 << 20, 1)
pr = synth.config_pair(5, 1, (160, 120))
a, b = torch.from_numpy(pr.img1).cuda(), torch.from_numpy(pr.img2).cuda()
for k in range(2):
    srv.submit(base_params(max_disp=32), a, b)
done, t0 = 0, time.time()
while done < 2 and time.time() - t0 < 60:
    done += len(srv.poll())
print("done", done, srv.stats())
srv.close()
"""
    env = dict(os.environ, PGM_LOG="2")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=180)
    assert "done 2" in r.stdout, r.stdout + r.stderr[-2000:]
    assert "[pgm] server on device 0" in r.stderr
    assert r.stderr.count("server: started") >= 1 and "pool in use" in r.stderr
    assert r.stderr.count("finished, status 0") == 2
