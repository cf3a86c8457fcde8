"""Pins of the CPU oracle against things other than itself: library routines (numpy, scipy,
PyTorch's Philox engine, exact rational arithmetic), closed forms, brute force on tiny
inputs and invariants that follow from the paper's definitions (Li, arXiv:1704.03217)."""
import math
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from conftest import base_params

RNG = np.random.default_rng(12345)


# --------------------------------------------------------------------------------------
# borders, pyramid, gradient image (Sec. III-A, III-D)
# --------------------------------------------------------------------------------------

def test_reflect101_is_numpy_reflect():
    for n in range(1, 8):
        pad = 3 * n + 12
        ext = np.pad(np.arange(n), pad, mode="reflect")
        for i in range(-pad, n + pad):
            assert oracle.reflect101(i, n) == ext[i + pad], (i, n)


def _binomial(k):
    """binomial taps of length k from repeated [1, 1] convolutions (library routine)"""
    t = np.array([1])
    for _ in range(k - 1):
        t = np.convolve(t, [1, 1])
    return t


@pytest.mark.parametrize("shape", [(9, 11, 3), (16, 16, 3), (7, 13, 1), (31, 20, 3)])
def test_pyr_down_is_binomial_filter_and_decimation(shape):
    img = RNG.integers(0, 256, shape, dtype=np.uint8)
    got = oracle.pyr_down(img[..., 0] if shape[2] == 1 else img)
    b5 = _binomial(5)
    k = np.outer(b5, b5)
    assert k.sum() == 256
    chans = [img[..., c].astype(np.int64) for c in range(shape[2])]
    exp = [((ndimage.correlate(c, k, mode="mirror") + 128) >> 8)[::2, ::2] for c in chans]
    exp = np.stack(exp, -1).astype(np.uint8)
    assert got.reshape(exp.shape).shape == ((shape[0] + 1) // 2, (shape[1] + 1) // 2, shape[2])
    np.testing.assert_array_equal(got.reshape(exp.shape), exp)


def test_pyr_down_keeps_constants():
    for v in (0, 1, 127, 255):
        img = np.full((13, 21, 3), v, np.uint8)
        assert (oracle.pyr_down(img) == v).all()


def test_gray_keeps_gray_inputs():
    v = np.arange(256, dtype=np.uint8)
    img = np.repeat(v[None, :, None], 3, axis=2)
    np.testing.assert_array_equal(oracle.gray(img)[0], v)


def test_gray_is_bt601_luma():
    """PGM-G's gray image (Sec. III-F, reading: integer BT.601 luma) stays within 1 of the
    real-valued 0.299 R + 0.587 G + 0.114 B on random colours and on the three primaries."""
    img = RNG.integers(0, 256, (16, 24, 3), dtype=np.uint8)
    img[0, 0], img[0, 1], img[0, 2] = (255, 0, 0), (0, 255, 0), (0, 0, 255)
    real = img.astype(np.float64) @ np.array([0.299, 0.587, 0.114])
    got = oracle.gray(img).astype(np.float64)
    assert np.abs(got - real).max() <= 1.0
    assert (got[0, 0], got[0, 1], got[0, 2]) == (77, 149, 29)


@pytest.mark.parametrize("shape", [(12, 17, 3), (8, 9, 1), (25, 6, 3)])
def test_gradient_s3_is_scipy_sobel(shape):
    img = RNG.integers(0, 256, shape, dtype=np.uint8)
    G = oracle.gradient_image(img[..., 0] if shape[2] == 1 else img, 3)
    ch = shape[2]
    for c in range(ch):
        I = img[..., c].astype(np.int64)
        np.testing.assert_array_equal(G[..., c], ndimage.sobel(I, axis=1, mode="mirror"))
        np.testing.assert_array_equal(G[..., ch + c], ndimage.sobel(I, axis=0, mode="mirror"))


@pytest.mark.parametrize("shape", [(12, 17, 3), (9, 9, 1), (20, 31, 3)])
def test_gradient_s5_is_s3_of_binomial_smoothed(shape):
    """S=5 Sobel = S=3 Sobel after one more [1 2 1] x [1 2 1] smoothing; with mirror borders
    the identity also holds at the border (the even extension commutes with both)."""
    img = RNG.integers(0, 256, shape, dtype=np.uint8)
    G = oracle.gradient_image(img[..., 0] if shape[2] == 1 else img, 5)
    ch = shape[2]
    b3 = _binomial(3)
    for c in range(ch):
        I = img[..., c].astype(np.int64)
        S = ndimage.correlate(I, np.outer(b3, b3), mode="mirror")
        np.testing.assert_array_equal(G[..., c], ndimage.sobel(S, axis=1, mode="mirror"))
        np.testing.assert_array_equal(G[..., ch + c], ndimage.sobel(S, axis=0, mode="mirror"))


@pytest.mark.parametrize("ksize,gain", [(3, 8), (5, 128)])
def test_gradient_ramp_closed_form(ksize, gain):
    """On I = a x + b y the interior gradient is (gain a, gain b) with gain = 8 (S=3) or 128
    (S=5); the sign is positive where intensity rises."""
    h, w = 20, 24
    for a, b in ((1, 0), (0, 2), (3, -2), (-4, 5), (-2, -3)):
        yy, xx = np.mgrid[0:h, 0:w]
        I = 120 + a * xx + b * yy
        assert I.min() >= 0 and I.max() <= 255
        img = np.repeat(I[..., None], 3, axis=2).astype(np.uint8)
        G = oracle.gradient_image(img, ksize)
        k = ksize // 2
        inner = G[k:h - k, k:w - k]
        assert (inner[..., 0:3] == gain * a).all() and (inner[..., 3:6] == gain * b).all()


def test_gradient_bounds():
    img = np.zeros((12, 12, 3), np.uint8)
    img[:, 6:] = 255
    G = oracle.gradient_image(img, 5)
    assert np.abs(G).max() == 48 * 255


def test_direction_unit_vectors():
    G = RNG.integers(-12240, 12241, (40, 40, 6)).astype(np.int16)
    G[::3, ::5] = 0
    G[1, 1, 0] = 1
    G[1, 1, 3] = 12240
    U = oracle.direction(G)
    assert U.dtype == np.float32
    for c in range(3):
        gx = G[..., c].astype(np.float64)
        gy = G[..., 3 + c].astype(np.float64)
        ux = U[..., c].astype(np.float64)
        uy = U[..., 3 + c].astype(np.float64)
        nz = (gx != 0) | (gy != 0)
        assert (ux[~nz] == 0).all() and (uy[~nz] == 0).all()
        np.testing.assert_allclose(ux[nz] ** 2 + uy[nz] ** 2, 1.0, atol=3e-7)
        ang = np.arctan2(gy[nz], gx[nz])
        np.testing.assert_allclose(np.arctan2(uy[nz], ux[nz]), ang, atol=1e-6)
        # nonzero components are at least 2^-14 in magnitude (used by the exact distance)
        comp = np.abs(np.concatenate([ux[nz], uy[nz]]))
        assert comp[comp > 0].min() >= 2.0 ** -14


# --------------------------------------------------------------------------------------
# patch distance (Eq. 3, absolute-difference reading)
# --------------------------------------------------------------------------------------

def _brute_dist(Ga, Gb, P, xa, ya, xb, yb):
    h, w = Ga.shape[:2]
    o = np.arange(-(P // 2), (P + 1) // 2)
    ya_i = np.clip(ya + o, 0, h - 1)[:, None]
    xa_i = np.clip(xa + o, 0, w - 1)[None, :]
    yb_i = np.clip(yb + o, 0, h - 1)[:, None]
    xb_i = np.clip(xb + o, 0, w - 1)[None, :]
    return Ga[ya_i, xa_i].astype(np.float64), Gb[yb_i, xb_i].astype(np.float64)


@pytest.mark.parametrize("P", [1, 4, 5, 8, 11, 15, 16])
def test_dist_i16_brute_force(P):
    h, w = 19, 23
    Ga = RNG.integers(-12240, 12241, (h, w, 6)).astype(np.int16)
    Gb = RNG.integers(-12240, 12241, (h, w, 6)).astype(np.int16)
    pts = [(0, 0), (w - 1, h - 1), (3, 17), (22, 0)] + [tuple(RNG.integers(0, (w, h))) for _ in range(20)]
    for (xa, ya) in pts:
        xb, yb = int(RNG.integers(0, w)), int(RNG.integers(0, h))
        A, B = _brute_dist(Ga, Gb, P, int(xa), int(ya), xb, yb)
        assert oracle.dist(Ga, Gb, P, int(xa), int(ya), xb, yb) == int(np.abs(A - B).sum())
        # symmetric in its arguments, zero on identical patches
        assert oracle.dist(Gb, Ga, P, xb, yb, int(xa), int(ya)) == oracle.dist(Ga, Gb, P, int(xa), int(ya), xb, yb)
        assert oracle.dist(Ga, Ga, P, int(xa), int(ya), int(xa), int(ya)) == 0


def test_dist_f32_is_exact_sum_rounded_once():
    h, w = 17, 21
    G1 = RNG.integers(-12240, 12241, (h, w, 6)).astype(np.int16)
    G2 = RNG.integers(-12240, 12241, (h, w, 6)).astype(np.int16)
    G1[::4] = 0
    U1, U2 = oracle.direction(G1), oracle.direction(G2)
    for _ in range(40):
        xa, ya, xb, yb = (int(v) for v in RNG.integers(0, [w, h, w, h]))
        P = int(RNG.choice([3, 8, 16]))
        A, B = _brute_dist(U1, U2, P, xa, ya, xb, yb)
        exact = math.fsum(abs(Fraction(float(a)) - Fraction(float(b))) for a, b in zip(A.ravel(), B.ravel()))
        assert oracle.dist(U1, U2, P, xa, ya, xb, yb) == np.float32(exact)


# --------------------------------------------------------------------------------------
# random numbers (Eq. 5 needs uniform R_i; Philox4x32-10 supplies them)
# --------------------------------------------------------------------------------------

PHILOX_HARNESS = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    at::philox_engine e(strtoull(argv[a], 0, 0), strtoull(argv[a + 1], 0, 0), strtoull(argv[a + 2], 0, 0));
    for (int i = 0; i < 4; i++) printf("%u ", e());
    printf("\n");
  }
}
"""


def _torch_include():
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) else None


@pytest.mark.skipif(_torch_include() is None, reason="PyTorch headers not installed")
def test_philox_matches_pytorch_engine():
    """PyTorch's header-only philox_engine(seed, subsequence, offset) produces Philox4x32-10
    of counter {offset lo, offset hi, subsequence lo, subsequence hi} under key {seed lo,
    seed hi}."""
    cases = [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**64 - 1)]
    cases += [tuple(int(v) for v in RNG.integers(0, 2**64, 3, dtype=np.uint64)) for _ in range(30)]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(src, "w").write(PHILOX_HARNESS)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", _torch_include(), src, "-o", exe])
        outs = subprocess.check_output([exe] + [str(v) for c in cases for v in c]).decode().split("\n")
    for (seed, sub, off), line in zip(cases, outs):
        ref = [int(v) for v in line.split()]
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert list(oracle.philox(ctr, key)) == ref


def _search_exact(u, W, i):
    R = Fraction(2 * u + 1, 2**32) - 1
    return math.floor(R * W / 2**i)


def test_search_offset_is_exact_floor():
    us = [0, 1, 2, 2**30 - 1, 2**30, 2**31 - 1, 2**31, 2**31 + 1, 3 * 2**30, 2**32 - 2, 2**32 - 1]
    us += [int(v) for v in RNG.integers(0, 2**32, 300, dtype=np.int64)]
    for W in (1, 2, 3, 5, 13, 16, 100, 1023):
        nI = int(math.floor(math.log2(W))) + 1
        for i in range(nI):
            vals = set()
            for u in us:
                v = oracle.search_offset(u, W, i)
                assert v == _search_exact(u, W, i), (u, W, i)
                vals.add(v)
            lim = math.ceil(W / 2**i)
            assert min(vals) >= -lim and max(vals) <= lim - 1
    # W = 2: {-2..1} for i = 0 and {-1, 0} for i = 1, equally likely
    assert {oracle.search_offset(u, 2, 0) for u in (0, 2**30, 2**31, 3 * 2**30)} == {-2, -1, 0, 1}
    assert {oracle.search_offset(u, 2, 1) for u in (0, 2**31)} == {-1, 0}


@pytest.mark.parametrize("W,expected", [(1, 150.0), (2, 337.5), (13, 775.0)])
def test_random_search_takes_floor_log2_W_plus_one_candidates(W, expected):
    """Eq. 5: the limited random search tries i = 0 .. floor(log2 W), one candidate each. A
    lone seed (no neighbours to propagate from) on flat gradients (every cost ties, so the
    match never moves) evaluates every candidate whose offset is not (0, 0); over 200
    iterations the count is near 200 * sum_i (1 - P(offset_i = 0)^2), which one candidate
    more or fewer would move by more than 18%."""
    h, w = 41, 41
    G = np.zeros((h, w, 6), np.int16)
    p = base_params(levels=1, seed_stride=w, max_disp=0, rng_seed=97)
    st = dict(dx=[0], dy=[0], dist=[0], init=[1])
    out, nev = oracle.sweep(p, G, G, st, W=W, t0=0, n_iter=200)
    assert (out["dx"][0], out["dy"][0]) == (0, 0)
    assert abs(nev - expected) <= 0.1 * expected, (W, nev, expected)


def test_init_offset_is_exact_and_uniform():
    for R in (0, 1, 5, 13, 16, 300):
        for u in [0, 2**32 - 1] + [int(v) for v in RNG.integers(0, 2**32, 200, dtype=np.int64)]:
            exp = math.floor(Fraction(u, 2**32) * (2 * R + 1)) - R
            assert oracle.init_offset(u, R) == exp
    # chi-square over Philox draws
    R = 5
    words = np.concatenate([oracle.philox([i, 7, 0, 0], [99, 0]) for i in range(3000)])
    vals = np.array([oracle.init_offset(int(u), R) for u in words])
    cnt = np.bincount(vals + R, minlength=2 * R + 1)
    exp = len(vals) / (2 * R + 1)
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 35.0   # 10 dof, p ~ 1e-4


# --------------------------------------------------------------------------------------
# seed grid
# --------------------------------------------------------------------------------------

def test_grid_nearest_brute_force():
    for stride in range(1, 6):
        for n in range(1, 25):
            cnt = oracle.grid_count(n, stride)
            pos = [oracle.grid_pos(i, n, stride) for i in range(cnt)]
            assert all(0 <= p < n for p in pos) and pos == sorted(set(pos))
            assert pos[0] == min(stride // 2, n - 1)
            if cnt > 1:
                assert all(b - a == stride for a, b in zip(pos, pos[1:]))
                assert n - 1 - pos[-1] < stride
            for x in range(n):
                d = [abs(x - p) for p in pos]
                best = min(d)
                exp = max(i for i in range(cnt) if d[i] == best)
                assert oracle.grid_nearest(x, cnt, stride) == exp, (stride, n, x)


# --------------------------------------------------------------------------------------
# the whole method on small inputs
# --------------------------------------------------------------------------------------

def _features(img, ksize=5):
    return oracle.gradient_image(img, ksize)


def _cost_volume(Ga, Gb, P, pts):
    """D(p, q) for every seed p in pts and every pixel q of Gb (numpy brute force)."""
    h, w = Gb.shape[:2]
    o = np.arange(-(P // 2), (P + 1) // 2)
    yy, xx = np.mgrid[0:h, 0:w]
    # patches of every q: (h, w, P, P, C)
    qy = np.clip(yy[..., None, None] + o[:, None], 0, h - 1)
    qx = np.clip(xx[..., None, None] + o[None, :], 0, w - 1)
    PB = Gb[qy, qx].astype(np.int64)
    out = []
    for (x, y) in pts:
        A = Ga[np.clip(y + o, 0, h - 1)[:, None], np.clip(x + o, 0, w - 1)[None, :]].astype(np.int64)
        out.append(np.abs(PB - A).sum(axis=(2, 3, 4)))
    return np.array(out)


def _seed_pts(w, h, stride):
    nx, ny = oracle.grid_count(w, stride), oracle.grid_count(h, stride)
    return [(oracle.grid_pos(i, w, stride), oracle.grid_pos(j, h, stride)) for j in range(ny) for i in range(nx)]


def _tie_pair(kind):
    """Image pairs whose window costs tie: flat images (every candidate costs 0) and vertical
    stripes of period 4 (candidates tie along every column shift by 4 and every row shift)."""
    h, w = 20, 24
    if kind == "flat":
        img = np.full((h, w, 3), 100, np.uint8)
    else:
        col = np.array([30, 90, 200, 140], np.uint8)[np.arange(w) % 4]
        img = np.repeat(np.repeat(col[None, :, None], h, axis=0), 3, axis=2)
    return synth.Pair(img, img.copy(), np.zeros((h, w, 2), np.float32), np.ones((h, w), bool))


@pytest.mark.parametrize("seed,P", [(1, 8), (2, 5), (3, 1), ("flat", 8), ("stripes", 5)])
def test_exhaustive_init_is_brute_force_argmin(seed, P):
    """The exhaustive start is the window's argmin, scanning dy outer and dx inner and keeping
    the first minimum (strictly smaller wins), which the tie cases pin."""
    pair = synth.rect_pair(seed, 20, 24, n_rect=2, dmax=4) if isinstance(seed, int) else _tie_pair(seed)
    p = base_params(levels=1, iters=[0], init_mode=1, max_disp=0, patch_fwd=P, patch_bwd=P)
    r = oracle.match(p, pair.img1, pair.img2)
    G1, G2 = _features(pair.img1), _features(pair.img2)
    h, w = G1.shape[:2]
    pts = _seed_pts(w, h, 3)
    for d, (Ga, Gb) in enumerate(((G1, G2), (G2, G1))):
        vol = _cost_volume(Ga, Gb, P, pts)
        st = r["levels"][d][0]
        for s, (x, y) in enumerate(pts):
            flat = vol[s].ravel()            # row-major over (qy, qx): dy outer, dx inner
            k = int(np.argmin(flat))         # first minimum
            qy, qx = divmod(k, w)
            assert (st[s, 0], st[s, 1]) == (qx - x, qy - y)
            assert st[s, 2] == flat[k]
    # every window position inside the image is evaluated exactly once per seed
    assert r["n_evals"] == 2 * len(pts) * w * h


def test_patchmatch_never_beats_brute_force():
    pair = synth.rect_pair(7, 24, 32, n_rect=2, dmax=5)
    p = base_params(levels=1, iters=[8], max_disp=0, rng_seed=77)
    r = oracle.match(p, pair.img1, pair.img2)
    G1, G2 = _features(pair.img1), _features(pair.img2)
    h, w = G1.shape[:2]
    pts = _seed_pts(w, h, 3)
    vol = _cost_volume(G1, G2, 8, pts)
    st = r["levels"][0][0]
    hits = 0
    for s, (x, y) in enumerate(pts):
        assert st[s, 3] & oracle.F_INIT
        dx, dy = st[s, 0], st[s, 1]
        assert 0 <= x + dx < w and 0 <= y + dy < h
        assert st[s, 2] == vol[s, y + dy, x + dx]        # stored distance is D(p, p + d)
        assert st[s, 2] >= vol[s].min()
        hits += st[s, 2] == vol[s].min()
    assert hits >= 0.8 * len(pts)


def test_distance_non_increasing_over_iterations():
    pair = synth.config_pair(1)
    prev = None
    for k in range(0, 5):
        p = base_params(levels=1, iters=[k], max_disp=8, rng_seed=5)
        r = oracle.match(p, pair.img1[:96, :128], pair.img2[:96, :128])
        st = r["levels"][0][0]
        if prev is not None:
            assert (st[:, 2] <= prev[:, 2]).all()
            assert (st[:, 2] < prev[:, 2]).any() or k > 3
        prev = st


def _interior(pts, w, h, d, margin):
    out = []
    for s, (x, y) in enumerate(pts):
        if margin <= x < w - margin and margin <= y < h - margin and \
           margin <= x + d[0] < w - margin and margin <= y + d[1] < h - margin:
            out.append(s)
    return out


@pytest.mark.parametrize("dx,dy,L,init_mode,N", [(5, -3, 1, 1, 0), (-7, 2, 1, 0, 0), (10, -6, 2, 0, 0),
                                                  (12, 8, 3, 0, 0), (0, 0, 2, 0, 0), (0, 0, 1, 1, 0),
                                                  (12, 8, 3, 0, 2), (-8, 4, 3, 1, 1), (4, -6, 2, 0, 3)])
def test_translation_recovered_exactly(dx, dy, L, init_mode, N):
    """An integer translation is recovered exactly at interior seeds (distance 0, inlier) and
    the backward field is its negative. Below the top level the translation must be divisible
    by 2^level for the coarser images to be exact translations too. With N refinement rounds
    (Sec. III-D) the result must be the same (the lift itself is pinned separately: a uniform
    translation heals a wrong lift at the finer levels)."""
    h, w = 72, 96
    pair = synth.translate_pair(11 + dx, h, w, dx, dy)
    p = base_params(levels=L, iters=[8] * L, max_disp=16, init_mode=init_mode, refine_rounds=N, rng_seed=3)
    r = oracle.match(p, pair.img1, pair.img2)
    pts = _seed_pts(w, h, 3)
    margin = 4 + 3 + 1
    st_f, st_b = r["levels"][0][0], r["levels"][1][0]
    fin = _interior(pts, w, h, (dx, dy), margin)
    bin_ = _interior(pts, w, h, (-dx, -dy), margin)
    assert len(fin) > 100
    for s in fin:
        assert (st_f[s, 0], st_f[s, 1], st_f[s, 2]) == (dx, dy, 0)
        assert st_f[s, 3] & oracle.F_INLIER
    for s in bin_:
        assert (st_b[s, 0], st_b[s, 1], st_b[s, 2]) == (-dx, -dy, 0)


def test_ties_keep_the_current_match():
    """Sec. III-B reading: a candidate replaces the match only if strictly better. On flat
    images every patch distance is 0, so propagation and random search only meet ties and the
    iterated field must equal the random start."""
    pair = _tie_pair("flat")
    base = dict(levels=1, max_disp=6, fwd_bwd=0, rng_seed=21)
    r0 = oracle.match(base_params(iters=[0], **base), pair.img1, pair.img2)
    r3 = oracle.match(base_params(iters=[3], **base), pair.img1, pair.img2)
    for d in range(2):
        a, b = r0["levels"][d][0], r3["levels"][d][0]
        np.testing.assert_array_equal(a[:, :3], b[:, :3])
    assert r3["n_evals"] > r0["n_evals"]        # the ties were evaluated, not skipped


def test_exact_cancellation_is_consistent_at_tau_zero():
    """The check accepts displacements that cancel within tau pixels, tau included (the reading
    of Sec. III-C/E): at tau = 0 a pure translation, whose forward and backward fields cancel
    exactly, must leave its interior seeds inliers at every level."""
    h, w, dx, dy = 72, 96, 8, -4
    pair = synth.translate_pair(17, h, w, dx, dy)
    p = base_params(levels=2, iters=[8, 8], max_disp=16, consistency_px=0, rng_seed=4)
    r = oracle.match(p, pair.img1, pair.img2)
    pts = _seed_pts(w, h, 3)
    fin = _interior(pts, w, h, (dx, dy), 4 + 3 + 1)
    assert len(fin) > 100
    st = r["levels"][0][0]
    for s in fin:
        assert (st[s, 0], st[s, 1]) == (dx, dy) and st[s, 3] & oracle.F_INLIER, (s, st[s].tolist())


def test_lift_rounds_the_halved_mean_of_inlier_children():
    """The lift toward the coarser level (Sec. III-D, Eq. 6 with k = j+1) on a hand-made field:
    a 12x12 grid (stride 3, seeds at 1, 4, 7, 10) under a 6x6 one (seeds at 1, 4), so every
    coarse seed has the 2x2 finer seeds nearest to twice its position as children. The coarse
    displacement is the mean of the inlier children's displacements halved, rounded to the
    nearest integer with halves away from zero (reading), and a coarse seed without inlier
    children stays uninitialised."""
    fdx = np.zeros(16, np.int32); fdy = np.zeros(16, np.int32); inl = np.zeros(16, np.uint8)
    def put(children, dxs, dys, flags):
        for c, x, y, f in zip(children, dxs, dys, flags):
            fdx[c], fdy[c], inl[c] = x, y, f
    put([0, 1, 4, 5], [4, 6, 4, 6], [-2, -2, -2, -4], [1, 1, 1, 1])     # dx 20/8 = 2.5, dy -10/8
    put([2, 3, 6, 7], [-4, -5, 100, 100], [5, 6, 100, 100], [1, 1, 0, 0])  # -9/4, 11/4; outliers ignored
    put([8, 9, 12, 13], [2, 2, 2, 2], [2, 2, 2, 2], [0, 0, 0, 0])        # no inlier child
    put([10, 11, 14, 15], [0, 0, 0, 2], [-4, -6, -4, -6], [1, 1, 1, 1])   # 2/8, -20/8 = -2.5
    cdx, cdy, cinit = oracle.lift(12, 12, 6, 6, 3, fdx, fdy, inl)
    assert cinit.tolist() == [1, 1, 0, 1]
    assert (cdx[0], cdy[0]) == (3, -1)
    assert (cdx[1], cdy[1]) == (-2, 3)
    assert (cdx[3], cdy[3]) == (0, -3)


def test_refinement_lift_halves_the_mean_of_inlier_children():
    """Refinement (Sec. III-D, Eq. 6 toward the coarser level): with the coarsest level never
    iterated, its final field is the lift of the finer level's inliers. Under a translation d
    divisible by 4, the exhaustive start finds d/4 at level 2, level 1 holds d/2 and keeps it
    (distance 0 cannot be beaten), so the lift must give d/4 back at every interior seed that
    has an inlier child; without the halving it would give d/2."""
    h, w, dx, dy = 144, 192, 8, -4
    pair = synth.translate_pair(31, h, w, dx, dy)
    p = base_params(levels=3, iters=[4, 4, 0], max_disp=16, init_mode=1, refine_rounds=1, rng_seed=5)
    r = oracle.match(p, pair.img1, pair.img2)
    lw, lh, nx, ny = r["geometry"][2]
    st = r["levels"][0][2]
    checked = 0
    for j in range(ny):
        for i in range(nx):
            x, y = oracle.grid_pos(i, lw, 3), oracle.grid_pos(j, lh, 3)
            if not (6 <= x < lw - 6 and 6 <= y < lh - 6):
                continue
            s = j * nx + i
            if st[s, 3] & oracle.F_INIT:
                assert (st[s, 0], st[s, 1]) == (dx // 4, dy // 4), (i, j, st[s].tolist())
                checked += 1
    assert checked >= 40


def _nearest_idx(x, n, stride):
    pos = np.array([oracle.grid_pos(i, 10**9, stride) for i in range(n)])
    d = np.abs(pos[None, :] - np.asarray(x)[:, None])
    # ties toward the larger index
    return (d.shape[1] - 1 - np.argmin(d[:, ::-1], axis=1))


def _geom(r, l):
    return r["geometry"][l]


@pytest.mark.parametrize("tau", [1, 3, 10**6])
def test_consistency_and_record_invariants(tau):
    """Re-derive Step 2-3 (check + Eq. 7) and Eq. 8 from the oracle's own per-level output."""
    pair = synth.config_pair(1)
    p = base_params(levels=4, iters=[3, 3, 3, 3], max_disp=20, consistency_px=tau, rng_seed=9)
    r = oracle.match(p, pair.img1, pair.img2)
    L = p["levels"]
    for l in range(L):
        lw, lh, nx, ny = _geom(r, l)
        xs = np.array([oracle.grid_pos(i, lw, 3) for i in range(nx)])
        ys = np.array([oracle.grid_pos(j, lh, 3) for j in range(ny)])
        px = np.tile(xs, ny)
        py = np.repeat(ys, nx)
        carried = l <= L - 3                      # record carried into levels below m-1
        for d in range(2):
            a, b = r["levels"][d][l], r["levels"][1 - d][l]
            init = (a[:, 3] & oracle.F_INIT) > 0
            qx, qy = px + a[:, 0], py + a[:, 1]
            oi = _nearest_idx(qx, nx, 3)
            oj = _nearest_idx(qy, ny, 3)
            os_ = oj * nx + oi
            binit = (b[os_, 3] & oracle.F_INIT) > 0
            ex = a[:, 0] + b[os_, 0]
            ey = a[:, 1] + b[os_, 1]
            cons = init & binit & (ex.astype(np.int64) ** 2 + ey.astype(np.int64) ** 2 <= tau * tau)
            rec = (a[:, 3] & oracle.F_RECORD) > 0
            inl = (a[:, 3] & oracle.F_INLIER) > 0
            exp = cons & rec if carried else cons
            np.testing.assert_array_equal(inl, exp)
            if not carried:
                assert not rec.any()
            else:
                # Eq. 8 toward the finer level: record = parent's inlier state
                pw, ph, pnx, pny = _geom(r, l + 1)
                pi = _nearest_idx(px // 2, pnx, 3)
                pj = _nearest_idx(py // 2, pny, 3)
                par_inl = (r["levels"][d][l + 1][pj * pnx + pi, 3] & oracle.F_INLIER) > 0
                np.testing.assert_array_equal(rec, par_inl)
            if tau >= 10**6:
                np.testing.assert_array_equal(inl, init & binit & (rec if carried else True))


@pytest.mark.parametrize("cfg_index,levels", [(0, 4), (1, 5)])
def test_outlier_record_is_monotone(cfg_index, levels):
    """Sec. III-C/D: a seed judged an outlier stays one at the following levels, so wherever the
    record is carried (the levels below m-1), a seed can only be an inlier if the coarser seed
    it descends from was one; the data must also contain seeds under outlier parents, or the
    pin would test nothing. Level m-1 receives the field without the record."""
    pair = synth.config_pair(1, cfg_index)
    p = base_params(levels=levels, iters=[3] * levels, max_disp=20, rng_seed=11 + cfg_index)
    r = oracle.match(p, pair.img1, pair.img2)
    blocked = 0
    for l in range(levels - 2):                   # levels carrying the record: below m - 1
        lw, lh, nx, ny = _geom(r, l)
        pw, ph, pnx, pny = _geom(r, l + 1)
        px = np.tile([oracle.grid_pos(i, lw, 3) for i in range(nx)], ny)
        py = np.repeat([oracle.grid_pos(j, lh, 3) for j in range(ny)], nx)
        parent = _nearest_idx(py // 2, pny, 3) * pnx + _nearest_idx(px // 2, pnx, 3)
        for d in range(2):
            child_in = (r["levels"][d][l][:, 3] & oracle.F_INLIER) > 0
            par_in = (r["levels"][d][l + 1][parent, 3] & oracle.F_INLIER) > 0
            assert not (child_in & ~par_in).any(), (l, d, int((child_in & ~par_in).sum()))
            blocked += int((~par_in & ((r["levels"][d][l][:, 3] & oracle.F_INIT) > 0)).sum())
    assert blocked > 0
    # the field enters level m-1 without the record of level m (the one link of Sec. III-D that
    # carries the field only), so there some inliers descend from outliers
    l = levels - 2
    lw, lh, nx, ny = _geom(r, l)
    pw, ph, pnx, pny = _geom(r, l + 1)
    px = np.tile([oracle.grid_pos(i, lw, 3) for i in range(nx)], ny)
    py = np.repeat([oracle.grid_pos(j, lh, 3) for j in range(ny)], nx)
    parent = _nearest_idx(py // 2, pny, 3) * pnx + _nearest_idx(px // 2, pnx, 3)
    freed = 0
    for d in range(2):
        child_in = (r["levels"][d][l][:, 3] & oracle.F_INLIER) > 0
        par_in = (r["levels"][d][l + 1][parent, 3] & oracle.F_INLIER) > 0
        freed += int((child_in & ~par_in).sum())
    assert freed > 0


def test_level_down_transition():
    """With no iterations at the finer level, its field is exactly Eq. 6 toward k = j-1:
    twice the parent's displacement (clamped) where the parent is an inlier, else
    uninitialised; the stored distance is D(p, p+d)."""
    pair = synth.config_pair(1)
    p = base_params(levels=3, iters=[0, 0, 4], max_disp=20, rng_seed=4)
    r = oracle.match(p, pair.img1, pair.img2)
    for l in (1, 0):
        lw, lh, nx, ny = _geom(r, l)
        pw, ph, pnx, pny = _geom(r, l + 1)
        img1 = pair.img1
        img2 = pair.img2
        for _ in range(l):
            img1, img2 = oracle.pyr_down(img1), oracle.pyr_down(img2)
        G = [_features(img1), _features(img2)]
        for d in range(2):
            st = r["levels"][d][l]
            par = r["levels"][d][l + 1]
            for s in range(nx * ny):
                i, j = s % nx, s // nx
                x, y = oracle.grid_pos(i, lw, 3), oracle.grid_pos(j, lh, 3)
                ps = oracle.grid_nearest(y // 2, pny, 3) * pnx + oracle.grid_nearest(x // 2, pnx, 3)
                if par[ps, 3] & oracle.F_INLIER:
                    ex = min(max(x + 2 * par[ps, 0], 0), lw - 1) - x
                    ey = min(max(y + 2 * par[ps, 1], 0), lh - 1) - y
                    assert st[s, 3] & oracle.F_INIT
                    assert (st[s, 0], st[s, 1]) == (ex, ey)
                    A, B = _brute_dist(G[d], G[1 - d], 8, x, y, x + ex, y + ey)
                    assert st[s, 2] == int(np.abs(A - B).sum())
                else:
                    assert not st[s, 3] & oracle.F_INIT


@pytest.mark.parametrize("t", [0, 1, 2, 3])
def test_propagation_direction_order(t):
    """Eq. 4 with the FlowFields order of (Delta_x, Delta_y): starting from a single
    initialised seed, one synchronous iteration spreads it two grid steps along -Delta
    (first the opposite colour, then the seed's own colour), and a raster pass along the
    same direction fills the whole quadrant."""
    h, w = 60, 60
    img = synth.texture(np.random.default_rng(1), h, w)
    G = _features(img)
    nx = ny = oracle.grid_count(w, 3)
    i0, j0 = 10, 9
    st = dict(dx=np.zeros(nx * ny), dy=np.zeros(nx * ny), dist=np.zeros(nx * ny),
              init=np.zeros(nx * ny))
    st["init"][j0 * nx + i0] = 1
    p = base_params(levels=1)
    sx, sy = [(1, 1), (-1, -1), (-1, 1), (1, -1)][t]   # direction of spreading = Delta
    out, _ = oracle.sweep(p, G, G, st, W=1, t0=t, n_iter=1)
    got = {(s % nx, s // nx) for s in np.nonzero(out["init"])[0]}
    exp = {(i0, j0), (i0 + sx, j0), (i0, j0 + sy), (i0 + 2 * sx, j0), (i0 + sx, j0 + sy), (i0, j0 + 2 * sy)}
    assert got == exp
    out, _ = oracle.sweep(p, G, G, st, W=1, t0=t, n_iter=1, schedule=oracle.SCAN)
    got = {(s % nx, s // nx) for s in np.nonzero(out["init"])[0]}
    exp = {(i, j) for i in range(nx) for j in range(ny) if (i - i0) * sx >= 0 and (j - j0) * sy >= 0}
    assert got == exp


def test_scan_and_sync_schedules_agree_statistically():
    pair = synth.config_pair(1)
    p = base_params(levels=3, iters=[4, 4, 4], max_disp=20, rng_seed=1000)
    a = oracle.match(p, pair.img1, pair.img2, schedule=oracle.SYNC)["fwd"]
    b = oracle.match(p, pair.img1, pair.img2, schedule=oracle.SCAN)["fwd"]
    ia, ib = (a["flags"] & 2) > 0, (b["flags"] & 2) > 0
    assert abs(ia.mean() - ib.mean()) < 0.05
    both = ia & ib
    same = (a["x2"] == b["x2"]) & (a["y2"] == b["y2"])
    assert same[both].mean() > 0.95


def test_output_and_compaction():
    pair = synth.config_pair(1)
    p = base_params(rng_seed=1000)
    r = oracle.match(p, pair.img1, pair.img2)
    f = r["fwd"]
    inl = (f["flags"] & 2) > 0
    assert r["n_inliers"] == inl.sum()
    np.testing.assert_array_equal(r["compact"], f[inl])
    lv = r["levels"][0][0]
    init = (lv[:, 3] & 1) > 0
    np.testing.assert_array_equal(f["x2"] - f["x1"], np.where(init, lv[:, 0], 0))
    np.testing.assert_array_equal(f["dist"], lv[:, 2])
    assert (f["dist"][~init] == 0x7FFFFFFF).all()
    # quality on the synthetic pair: most inliers within 1 px of the ground truth
    gt = pair.flow[f["y1"], f["x1"]]
    err = np.hypot(f["x2"] - f["x1"] - gt[:, 0], f["y2"] - f["y1"] - gt[:, 1])
    assert inl.mean() > 0.7 and (err[inl] < 1).mean() > 0.95


def test_direction_variant_runs_and_matches_translation():
    h, w = 60, 72
    pair = synth.translate_pair(4, h, w, 6, -2)
    p = base_params(levels=2, iters=[4, 4], max_disp=12, feature=1, rng_seed=8)
    r = oracle.match(p, pair.img1, pair.img2)
    pts = _seed_pts(w, h, 3)
    st = r["levels"][0][0]
    for s in _interior(pts, w, h, (6, -2), 8):
        assert (st[s, 0], st[s, 1]) == (6, -2)
        assert np.int32(st[s, 2]).view(np.float32) == 0.0


def test_invalid_parameters_rejected():
    img = np.zeros((20, 20, 3), np.uint8)
    for bad in (dict(levels=0), dict(levels=9), dict(seed_stride=0), dict(patch_fwd=17),
                dict(sobel_ksize=7), dict(radius=0), dict(feature=5), dict(iters=[300, 4, 4]),
                dict(rs_mode=2), dict(max_disp=-1025)):
        with pytest.raises(ValueError):
            oracle.match(base_params(**bad), img, img)


# ---- small-region removal (Sec. III-E) ----

def _regions_by_csgraph(dx, dy, inl, stride, min_px, link_px):
    """Expected result from scipy's connected components of the linked-inlier graph."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    ny, nx = inl.shape
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols = [], []
    for a_sl, b_sl in (((slice(None), slice(0, nx - 1)), (slice(None), slice(1, nx))),
                       ((slice(0, ny - 1), slice(None)), (slice(1, ny), slice(None)))):
        ok = inl[a_sl] & inl[b_sl]
        d2 = (dx[a_sl].astype(np.int64) - dx[b_sl]) ** 2 + (dy[a_sl].astype(np.int64) - dy[b_sl]) ** 2
        ok &= d2 < link_px * link_px
        rows.append(idx[a_sl][ok]); cols.append(idx[b_sl][ok])
    r = np.concatenate(rows); c = np.concatenate(cols)
    g = coo_matrix((np.ones(len(r)), (r, c)), shape=(nx * ny, nx * ny))
    _, lab = connected_components(g, directed=False)
    lab = lab.reshape(ny, nx)
    sizes = np.bincount(lab[inl], minlength=lab.max() + 1)
    keep = inl.copy()
    keep[inl] = sizes[lab[inl]] * stride * stride >= min_px
    return keep


@pytest.mark.parametrize("seed,stride,min_px,link", [(0, 1, 9, 12), (1, 3, 27, 3), (2, 2, 12, 2), (3, 1, 30, 5)])
def test_region_removal_matches_scipy_components(oracle_lib, seed, stride, min_px, link):
    rng = np.random.default_rng(seed)
    ny, nx = 23, 31
    dx = rng.integers(-6, 7, (ny, nx)).astype(np.int32)
    dy = rng.integers(-6, 7, (ny, nx)).astype(np.int32)
    inl = rng.random((ny, nx)) < 0.7
    got = oracle.remove_small_regions(dx, dy, inl, stride, min_px, link)
    want = _regions_by_csgraph(dx, dy, inl, stride, min_px, link)
    assert np.array_equal(got, want)
    assert not np.any(got & ~inl)          # never creates inliers


def test_region_removal_piecewise_constant_matches_ndimage_label(oracle_lib):
    """Regions of constant displacement, neighbours of different regions far apart: the
    segments are exactly the 4-connected components of each constant region."""
    from scipy import ndimage
    rng = np.random.default_rng(7)
    ny, nx = 40, 50
    lab = rng.integers(0, 6, (ny // 4, nx // 5)).repeat(4, 0).repeat(5, 1)
    lab[rng.random((ny, nx)) < 0.05] = 6 + rng.integers(0, 4)    # speckle
    dx = (lab * 30).astype(np.int32)
    dy = (-lab * 20).astype(np.int32)
    inl = rng.random((ny, nx)) < 0.9
    want = np.zeros_like(inl)
    for v in np.unique(lab):
        comp, n = ndimage.label((lab == v) & inl)   # 4-connectivity
        sizes = np.bincount(comp.ravel())
        want |= (comp > 0) & (sizes[comp] >= 9)
    got = oracle.remove_small_regions(dx, dy, inl, 1, 9, 12)
    assert np.array_equal(got, want)


def test_region_removal_special_cases(oracle_lib):
    ny, nx = 9, 11
    z = np.zeros((ny, nx), np.int32)
    inl = np.zeros((ny, nx), bool)
    inl[::2, ::2] = True                      # isolated single inliers
    assert not oracle.remove_small_regions(z, z, inl, 1, 9, 12).any()       # 1 px < 9
    assert np.array_equal(oracle.remove_small_regions(z, z, inl, 3, 9, 12), inl)   # 9 px each
    full = np.ones((ny, nx), bool)
    assert oracle.remove_small_regions(z, z, full, 1, 9, 12).all()          # one big region
    # two seeds linked only when their displacements differ by less than link
    inl2 = np.zeros((ny, nx), bool); inl2[4, 4:6] = True
    dxs = z.copy(); dxs[4, 5] = 3
    assert oracle.remove_small_regions(dxs, z, inl2, 3, 18, 4).sum() == 2   # |3| < 4: 18 px kept
    assert oracle.remove_small_regions(dxs, z, inl2, 3, 18, 3).sum() == 0   # |3| = 3: split


def test_region_removal_in_the_pipeline_only_clears_forward_inliers(oracle_lib):
    pr = synth.config_pair(1, 0)
    p0 = base_params(seed_stride=1, levels=2, iters=[2, 2], rng_seed=77)
    a = oracle.match(p0, pr.img1, pr.img2, trace=False)
    b = oracle.match(dict(p0, min_region_px=9, region_link_px=12), pr.img1, pr.img2, trace=False)
    for k in ("x1", "y1", "x2", "y2", "dist"):
        assert np.array_equal(a["fwd"][k], b["fwd"][k])
    assert np.array_equal(a["bwd"], b["bwd"])
    ia = (a["fwd"]["flags"] & 2) != 0
    ib = (b["fwd"]["flags"] & 2) != 0
    assert not np.any(ib & ~ia) and ib.sum() < ia.sum()
    assert b["n_inliers"] == ib.sum()
    ny, nx = pr.img1.shape[0], pr.img1.shape[1]
    want = oracle.remove_small_regions((a["fwd"]["x2"] - a["fwd"]["x1"]).reshape(ny, nx),
                                       (a["fwd"]["y2"] - a["fwd"]["y1"]).reshape(ny, nx),
                                       ia.reshape(ny, nx), 1, 9, 12)
    assert np.array_equal(ib.reshape(ny, nx), want)


# ---- literal-sign direction variant (Sec. III-F, "G./|G|" element-wise) ----

def test_sign_feature_is_numpy_sign(oracle_lib):
    rng = np.random.default_rng(5)
    G = rng.integers(-30000, 30000, 5000).astype(np.int16)
    G[::7] = 0
    assert np.array_equal(oracle.sign(G), np.sign(G).astype(np.int16))


def test_sign_feature_distance_counts_sign_disagreements(oracle_lib):
    """On sign features the patch distance is the sum of |s_a - s_b|: 2 for opposite signs,
    1 where exactly one side is zero (checked by brute force on a gradient image)."""
    pair = synth.config_pair(1)
    G1 = oracle.sign(oracle.gradient_image(pair.img1, 5))
    G2 = oracle.sign(oracle.gradient_image(pair.img2, 5))
    h, w, C2 = G1.shape
    for (xa, ya, xb, yb) in [(40, 30, 43, 28), (0, 0, 5, 1), (w - 1, h - 1, w - 3, h - 2)]:
        a = G1[np.clip(ya + np.arange(-4, 4), 0, h - 1)][:, np.clip(xa + np.arange(-4, 4), 0, w - 1)]
        b = G2[np.clip(yb + np.arange(-4, 4), 0, h - 1)][:, np.clip(xb + np.arange(-4, 4), 0, w - 1)]
        want = int((a.astype(int) != b).sum() + ((a.astype(int) * b) < 0).sum())
        assert oracle.dist(G1, G2, 8, xa, ya, xb, yb) == want


@pytest.mark.parametrize("dx,dy", [(6, -2), (-4, 4)])
def test_sign_feature_recovers_translation(oracle_lib, dx, dy):
    h, w = 72, 96
    pair = synth.translate_pair(31 + dx, h, w, dx, dy)
    p = base_params(levels=2, iters=[8, 8], max_disp=16, feature=2, rng_seed=5)
    r = oracle.match(p, pair.img1, pair.img2)
    st = r["levels"][0][0]
    fin = _interior(_seed_pts(w, h, 3), w, h, (dx, dy), 8)
    assert len(fin) > 100
    ok = sum((st[s, 0], st[s, 1], st[s, 2]) == (dx, dy, 0) for s in fin)
    assert ok >= 0.98 * len(fin)     # sign patches can tie; almost every seed is exact


# ---- colour spaces of the two gradient pyramids (Sec. III-E, Table II) ----

def _all_colours(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.integers(0, 256, (n, 1, 3)).astype(np.uint8)
    extremes = np.array([[0, 0, 0], [255, 255, 255], [255, 0, 0], [0, 255, 0], [0, 0, 255],
                         [255, 255, 0], [0, 255, 255], [255, 0, 255]], np.uint8)[:, None, :]
    return np.concatenate([extremes, c])


def test_ycrcb_close_to_bt601_and_exact_on_greys(oracle_lib):
    c = _all_colours(200000, 1)
    out = oracle.convert(c, oracle.SPACE_YCRCB).astype(float)
    R, G, B = (c[..., k].astype(float) for k in range(3))
    Y = 0.299 * R + 0.587 * G + 0.114 * B
    ref = np.stack([Y, 128 + 0.713 * (R - Y), 128 + 0.564 * (B - Y)], -1).clip(0, 255)
    assert np.abs(out - ref).max() <= 2.0          # the integer approximation's error bound
    g = np.repeat(np.arange(256, dtype=np.uint8)[:, None, None], 3, axis=2)
    og = oracle.convert(g, oracle.SPACE_YCRCB)
    assert np.array_equal(og[..., 0, 0], np.arange(256)) and (og[..., 1:] == 128).all()


def test_lab_matches_the_standard_formula(oracle_lib):
    """The fixed-iteration powers agree with numpy's power / cbrt after rounding to 8 bits;
    white, black and greys land on their closed forms."""
    c = _all_colours(200000, 2)
    out = oracle.convert(c, oracle.SPACE_LAB).astype(int)
    v = c.astype(float) / 255.0
    lin = np.where(v <= 0.04045, v / 12.92, ((v + 0.055) / 1.055) ** 2.4)
    M = np.array([[0.4124564, 0.3575761, 0.1804375], [0.2126729, 0.7151522, 0.0721750],
                  [0.0193339, 0.1191920, 0.9503041]])
    XYZ = lin @ M.T / np.array([0.95047, 1.0, 1.08883])
    e = (6 / 29) ** 3
    f = np.where(XYZ > e, np.cbrt(XYZ), XYZ / (3 * (6 / 29) ** 2) + 4 / 29)
    L = 116 * f[..., 1] - 16
    ref = np.stack([L * 2.55, 500 * (f[..., 0] - f[..., 1]) + 128, 200 * (f[..., 1] - f[..., 2]) + 128], -1)
    ref = np.clip(np.floor(ref + 0.5), 0, 255).astype(int)
    diff = np.abs(out - ref)
    assert diff.max() <= 1 and (diff == 0).mean() > 0.99999
    assert oracle.convert(np.array([[[255, 255, 255]]], np.uint8), oracle.SPACE_LAB).tolist() == [[[255, 128, 128]]]
    assert oracle.convert(np.array([[[0, 0, 0]]], np.uint8), oracle.SPACE_LAB).tolist() == [[[0, 128, 128]]]
    g = np.repeat(np.arange(256, dtype=np.uint8)[:, None, None], 3, axis=2)
    og = oracle.convert(g, oracle.SPACE_LAB).astype(int)
    assert (np.abs(og[..., 1:] - 128) <= 1).all() and (np.diff(og[:, 0, 0]) >= 0).all()


def test_colour_spaces_in_the_pipeline(oracle_lib):
    """Table II's spaces change the features of each direction: identical pairs still give
    zero flow, and with every level in RGB the result equals the plain run."""
    pr = synth.config_pair(1, 0)
    p0 = base_params(rng_seed=61)
    paper = dict(p0, space_fwd=[0, 2, 1], space_bwd=[2, 1, 0])
    plain = oracle.match(p0, pr.img1, pr.img2, trace=False)
    same = oracle.match(dict(p0, space_fwd=[0, 0, 0], space_bwd=[0, 0, 0]), pr.img1, pr.img2, trace=False)
    assert np.array_equal(plain["fwd"], same["fwd"]) and np.array_equal(plain["bwd"], same["bwd"])
    r = oracle.match(paper, pr.img1, pr.img1, trace=False)
    init = (r["fwd"]["flags"] & 1) != 0
    assert np.all(r["fwd"]["x2"][init] == r["fwd"]["x1"][init])
    assert np.all(r["fwd"]["dist"][init] == 0)
    d = oracle.match(paper, pr.img1, pr.img2, trace=False)
    assert not np.array_equal(d["bwd"], plain["bwd"])      # the backward field sees other features


# ---- Eq. 3 as printed: the squared metric ----

@pytest.mark.parametrize("P", [1, 5, 8, 16])
def test_ssd_matches_numpy_brute_force(oracle_lib, P):
    rng = np.random.default_rng(P)
    h, w = 23, 29
    Ga = rng.integers(-24480, 24481, (h, w, 6)).astype(np.int16)
    Gb = rng.integers(-24480, 24481, (h, w, 6)).astype(np.int16)
    lo, hi = -(P // 2), (P + 1) // 2 - 1
    for (xa, ya, xb, yb) in [(10, 10, 12, 9), (0, 0, w - 1, h - 1), (3, h - 2, 1, 2)]:
        ys_a = np.clip(ya + np.arange(lo, hi + 1), 0, h - 1); xs_a = np.clip(xa + np.arange(lo, hi + 1), 0, w - 1)
        ys_b = np.clip(yb + np.arange(lo, hi + 1), 0, h - 1); xs_b = np.clip(xb + np.arange(lo, hi + 1), 0, w - 1)
        a = Ga[ys_a][:, xs_a].astype(np.int64); b = Gb[ys_b][:, xs_b].astype(np.int64)
        assert oracle.ssd(Ga, Gb, P, xa, ya, xb, yb) == int(((a - b) ** 2).sum())


def test_ssd_exact_beyond_32_bits(oracle_lib):
    h, w = 20, 20
    Ga = np.full((h, w, 6), 24480, np.int16)
    Gb = np.full((h, w, 6), -24480, np.int16)
    assert oracle.ssd(Ga, Gb, 16, 10, 10, 10, 10) == 16 * 16 * 6 * 48960 ** 2   # ~3.7e12


def test_ssd_pipeline_translation_and_output_clamp(oracle_lib):
    h, w = 72, 96
    pair = synth.translate_pair(41, h, w, 6, -4)
    p = base_params(levels=2, iters=[8, 8], max_disp=16, metric=1, rng_seed=7)
    r = oracle.match(p, pair.img1, pair.img2)
    st = r["levels"][0][0]
    fin = _interior(_seed_pts(w, h, 3), w, h, (6, -4), 8)
    assert len(fin) > 100
    for s in fin:
        assert (st[s, 0], st[s, 1], st[s, 2]) == (6, -4, 0)
    init = (r["fwd"]["flags"] & 1) != 0
    assert r["fwd"]["dist"][init].max() <= 0x7FFFFFFE            # clamped output


# --------------------------------------------------------------------------------------
# limited random search read symmetrically (an option of Eq. 5, Sec. III-B)
# --------------------------------------------------------------------------------------

def test_search_offset_sym_is_exact_with_full_range_and_uniform():
    """PGM_RS_SYMMETRIC: the i-th offset is floor(u (2 w_i + 1) / 2^32) - w_i with
    w_i = floor(W / 2^i): exact against rational arithmetic, exactly the integers of
    [-w_i, w_i] (both ends reached, nothing outside), and uniform (chi-square)."""
    us = [0, 1, 2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1]
    us += [int(v) for v in RNG.integers(0, 2**32, 300, dtype=np.int64)]
    for W in (1, 2, 3, 5, 13, 16, 100, 1023):
        nI = int(math.floor(math.log2(W))) + 1
        for i in range(nI):
            wi = W // 2**i
            for u in us:
                exp = math.floor(Fraction(u, 2**32) * (2 * wi + 1)) - wi
                assert oracle.search_offset_sym(u, W, i) == exp, (u, W, i)
            # the ends: the smallest draw gives -w_i, the largest +w_i
            assert oracle.search_offset_sym(0, W, i) == -wi
            assert oracle.search_offset_sym(2**32 - 1, W, i) == wi
            # every integer of the range has a draw: the first u of each cell
            for v in range(-wi, wi + 1):
                u = -(-((v + wi) * 2**32) // (2 * wi + 1))
                assert oracle.search_offset_sym(u, W, i) == v
                if u > 0:
                    assert oracle.search_offset_sym(u - 1, W, i) == v - 1
    W = 13
    words = np.concatenate([oracle.philox([i, 3, 0, 0], [77, 1]) for i in range(3000)])
    for i in range(4):
        wi = W >> i
        vals = np.array([oracle.search_offset_sym(int(u), W, i) for u in words])
        cnt = np.bincount(vals + wi, minlength=2 * wi + 1)
        exp = len(vals) / (2 * wi + 1)
        chi2 = ((cnt - exp) ** 2 / exp).sum()
        dof = 2 * wi
        assert chi2 < dof + 6 * math.sqrt(2 * dof), (i, chi2)


def test_symmetric_search_candidate_count_on_flat_gradients():
    """A lone seed on flat gradients (every cost ties, so the match never moves) evaluates
    exactly the candidates whose offset is not (0, 0): with the symmetric reading at W = 2 the
    expected count per iteration is (1 - 1/25) + (1 - 1/9) = 1.849 (i = 0 over [-2, 2]^2,
    i = 1 over [-1, 1]^2), against 1.6875 for the floor reading. The count is also recomputed
    exactly from the draws (Philox and the offset function, both pinned above)."""
    h, w = 41, 41
    G = np.zeros((h, w, 6), np.int16)
    n_iter = 250
    for rs_mode, per_iter in ((oracle.RS_SYMMETRIC, 1.849), (oracle.RS_FLOOR, 1.6875)):
        p = base_params(levels=1, seed_stride=w, max_disp=0, rng_seed=97, rs_mode=rs_mode)
        st = dict(dx=[0], dy=[0], dist=[0], init=[1])
        out, nev = oracle.sweep(p, G, G, st, W=2, t0=0, n_iter=n_iter)
        assert (out["dx"][0], out["dy"][0]) == (0, 0)
        assert abs(nev - per_iter * n_iter) <= 0.04 * per_iter * n_iter, (rs_mode, nev)
        off = oracle.search_offset_sym if rs_mode == oracle.RS_SYMMETRIC else oracle.search_offset
        exact = 0
        for t in range(n_iter):
            u = oracle.philox([0, t | (1 << 24), 0, 0], [97, 0])
            for i in range(2):
                exact += (off(int(u[2 * i]), 2, i), off(int(u[2 * i + 1]), 2, i)) != (0, 0)
        assert nev == exact


def test_symmetric_search_recovers_translation():
    pair = synth.translate_pair(5, 96, 128, 7, -4)
    p = base_params(levels=3, iters=[4, 4, 4], max_disp=12, rs_mode=oracle.RS_SYMMETRIC, rng_seed=31)
    f = oracle.match(p, pair.img1, pair.img2, trace=False)["fwd"]
    inner = (f["x1"] > 16) & (f["x1"] < 128 - 16) & (f["y1"] > 16) & (f["y1"] < 96 - 16)
    assert ((f["x2"] - f["x1"])[inner] == 7).all() and ((f["y2"] - f["y1"])[inner] == -4).all()
    assert (f["dist"][inner] == 0).all()


# --------------------------------------------------------------------------------------
# the sequential scan schedule (the paper's PatchMatch order, Sec. III-B)
# --------------------------------------------------------------------------------------

def test_scan_hand_worked_search_feeds_the_next_seed():
    """A hand-worked raster pass (t = 0: Delta_x = (1,0), Delta_y = (0,1), x and y ascending).
    Image 2 is image 1 moved one pixel right (left edge replicated, flat right margin), so
    d* = (1, 0) costs exactly 0 at every seed and nothing costs less. Only seed (0, 0) starts
    initialised, at (0, 0); the generator key is chosen so that its first random-search offset
    at t = 0 is (1, 0). In the sequential schedule seed (0, 0) finds d* by its search, and every
    later seed takes d* from an already updated neighbour before its own search (Eq. 4 then
    Eq. 5 per seed, in place): after one pass every seed holds d* at distance 0. The evaluation
    count is worked out from the draws: seed (0, 0) two (its two search candidates), every
    other seed one for the adopted neighbour plus one per search candidate that differs from
    d* after clamping.
    A scan in the wrong direction, a propagation pass before the search pass, or the
    synchronous schedule leaves most seeds uninitialised or away from d*. Which loop is outer
    cannot change the result: the draws are indexed by seed and iteration, and both nestings
    visit both propagation sources of a seed before the seed, so no pin can tell them apart."""
    h, w = 30, 48
    img = synth.texture(np.random.default_rng(3), h, w)
    G1 = _features(img).astype(np.int16)
    G1[:, 40:] = 0                               # flat right margin
    G2 = np.concatenate([G1[:, :1], G1[:, :-1]], axis=1)
    nx, ny = oracle.grid_count(w, 3), oracle.grid_count(h, 3)
    P = 8
    # a key whose first offset of seed 0 at t = 0 is (1, 0) (floor reading, W = 2)
    key = next(k for k in range(1, 5000)
               if (oracle.search_offset(int(oracle.philox([0, 1 << 24, 0, 0], [k, 0])[0]), 2, 0),
                   oracle.search_offset(int(oracle.philox([0, 1 << 24, 0, 0], [k, 0])[1]), 2, 0)) == (1, 0))
    p = base_params(levels=1, rng_seed=key)
    n = nx * ny
    st = dict(dx=np.zeros(n), dy=np.zeros(n), dist=np.zeros(n), init=np.zeros(n))
    st["init"][0] = 1
    st["dist"][0] = oracle.dist(G1, G2, P, 1, 1, 1, 1)
    assert st["dist"][0] > 0
    out, nev = oracle.sweep(p, G1, G2, st, W=2, t0=0, n_iter=1, schedule=oracle.SCAN)
    assert (out["init"] == 1).all()
    assert (out["dx"] == 1).all() and (out["dy"] == 0).all() and (out["dist"] == 0).all()
    # the evaluation count from the draws
    exp = 2
    for s in range(1, n):
        i, j = s % nx, s // nx
        px, py = oracle.grid_pos(i, w, 3), oracle.grid_pos(j, h, 3)
        u = oracle.philox([s, 1 << 24, 0, 0], [key, 0])
        exp += 1
        for c in range(2):
            ox, oy = oracle.search_offset(int(u[2 * c]), 2, c), oracle.search_offset(int(u[2 * c + 1]), 2, c)
            tx = min(max(px + 1 + ox, 0), w - 1) - px
            ty = min(max(py + oy, 0), h - 1) - py
            exp += (tx, ty) != (1, 0)
    assert nev == exp
    # the synchronous schedule spreads d* only to the two neighbours of seed (0, 0)
    sync, _ = oracle.sweep(p, G1, G2, st, W=2, t0=0, n_iter=1, schedule=oracle.SYNC)
    assert set(np.nonzero(sync["init"])[0]) == {0, 1, nx}
