"""Seeded synthetic image pairs shaped like the paper's workloads.

This module only draws input images (and, for reference, the ground-truth flow used to make
them). It contains none of the matching method's arithmetic, so both the GPU library's tests
and the CPU oracle's tests can take their inputs from here.

The paper evaluates on MPI Sintel (1024x436) and KITTI (1242x375) frames, which are not
available here; these generators stand in for them with the same shapes and with the
structure the method is sensitive to: multi-scale texture (so gradients are informative at
every pyramid level), piecewise motion with discontinuities and occlusions, large
displacements, sensor noise and a global gain change between the frames.

Every generator takes an explicit integer seed and is deterministic (numpy PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import ndimage

__all__ = [
    "Pair",
    "texture",
    "rect_pair",
    "layered_pair",
    "road_pair",
    "batch_sizes",
    "served_sizes",
    "config_pair",
    "translate_pair",
]


@dataclass
class Pair:
    img1: np.ndarray          # (h, w, 3) uint8, frame 1
    img2: np.ndarray          # (h, w, 3) uint8, frame 2
    flow: np.ndarray          # (h, w, 2) float32, frame-1 pixel -> frame-2 displacement (x, y)
    valid: np.ndarray         # (h, w) bool, frame-1 pixel visible in frame 2 (not occluded)
    name: str = ""


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def texture(rng: np.random.Generator, h: int, w: int, sigmas=(1.0, 4.0, 16.0)) -> np.ndarray:
    """Multi-scale texture: per channel, the sum over `sigmas` of Gaussian-blurred uniform
    noise, each octave standardised, mapped to uint8 as 128 + 40*z (clipped)."""
    out = np.empty((h, w, 3), np.float64)
    for c in range(3):
        acc = np.zeros((h, w), np.float64)
        for s in sigmas:
            f = ndimage.gaussian_filter(rng.random((h, w)), s, mode="reflect")
            sd = f.std()
            acc += (f - f.mean()) / (sd if sd > 0 else 1.0)
        acc /= math.sqrt(len(sigmas))
        out[..., c] = 128.0 + 40.0 * acc
    return np.clip(np.rint(out), 0, 255).astype(np.uint8)


def rect_pair(seed: int, h: int = 192, w: int = 256, n_rect: int = 4, dmax: int | None = None) -> Pair:
    """Static textured background plus `n_rect` axis-aligned textured rectangles, each moving
    by its own integer displacement with |d| <= dmax (default 20 px, or w/5 when w > 256).
    Frame 2 paints the rectangles at their moved positions in the same z-order."""
    rng = _rng(seed)
    if dmax is None:
        dmax = 20 if w <= 256 else max(1, w // 5)
    bg = texture(rng, h, w)
    img1 = bg.copy()
    img2 = bg.copy()
    flow = np.zeros((h, w, 2), np.float32)
    owner1 = np.full((h, w), -1, np.int32)
    owner2 = np.full((h, w), -1, np.int32)
    rects = []
    for k in range(n_rect):
        rw = int(rng.integers(max(2, w // 8), max(3, w // 2) + 1))
        rh = int(rng.integers(max(2, h // 8), max(3, h // 2) + 1))
        x0 = int(rng.integers(0, w - rw + 1))
        y0 = int(rng.integers(0, h - rh + 1))
        while True:
            dx = int(rng.integers(-dmax, dmax + 1))
            dy = int(rng.integers(-dmax, dmax + 1))
            if dx * dx + dy * dy <= dmax * dmax:
                break
        tex = texture(rng, rh, rw)
        rects.append((x0, y0, rw, rh, dx, dy, tex))
    for k, (x0, y0, rw, rh, dx, dy, tex) in enumerate(rects):
        img1[y0:y0 + rh, x0:x0 + rw] = tex
        flow[y0:y0 + rh, x0:x0 + rw] = (dx, dy)
        owner1[y0:y0 + rh, x0:x0 + rw] = k
        # frame 2: the rectangle moved by (dx, dy), clipped to the frame
        xa, ya = x0 + dx, y0 + dy
        sx0, sy0 = max(0, -xa), max(0, -ya)
        dx0, dy0 = max(0, xa), max(0, ya)
        cw = min(rw - sx0, w - dx0)
        ch = min(rh - sy0, h - dy0)
        if cw > 0 and ch > 0:
            img2[dy0:dy0 + ch, dx0:dx0 + cw] = tex[sy0:sy0 + ch, sx0:sx0 + cw]
            owner2[dy0:dy0 + ch, dx0:dx0 + cw] = k
    # visibility: the frame-1 owner of a pixel must own its target in frame 2
    yy, xx = np.mgrid[0:h, 0:w]
    tx = xx + flow[..., 0].astype(np.int64)
    ty = yy + flow[..., 1].astype(np.int64)
    inside = (tx >= 0) & (tx < w) & (ty >= 0) & (ty < h)
    valid = np.zeros((h, w), bool)
    valid[inside] = owner2[ty[inside], tx[inside]] == owner1[inside]
    return Pair(img1, img2, flow, valid, f"rect{seed}_{w}x{h}")


def _bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Bilinear sample of an (h, w, 3) image at float coordinates (clamped to the frame)."""
    h, w = img.shape[:2]
    x = np.clip(x, 0, w - 1.0)
    y = np.clip(y, 0, h - 1.0)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    fx = (x - x0)[..., None]
    fy = (y - y0)[..., None]
    f = img.astype(np.float64)
    top = f[y0, x0] * (1 - fx) + f[y0, x1] * fx
    bot = f[y1, x0] * (1 - fx) + f[y1, x1] * fx
    return top * (1 - fy) + bot * fy


def _finish(rng, f1: np.ndarray, f2: np.ndarray, noise: float, gain: tuple[float, float]):
    g = float(rng.uniform(*gain))
    n1 = rng.normal(0.0, noise, f1.shape)
    n2 = rng.normal(0.0, noise, f2.shape)
    a = np.clip(np.rint(f1 + n1), 0, 255).astype(np.uint8)
    b = np.clip(np.rint(f2 * g + n2), 0, 255).astype(np.uint8)
    return a, b


def layered_pair(seed: int, h: int = 436, w: int = 1024, n_layers: int = 6, dmax: float = 200.0,
                 noise: float = 2.0, gain=(0.9, 1.1)) -> Pair:
    """Sintel-shaped pair: a moving background plus `n_layers` textured regions (ellipses and
    convex polygons), each with its own affine motion whose displacement stays within dmax
    over the region. Regions occlude each other by z-order; frame 2 is rendered by inverse
    bilinear sampling of each layer's texture. Gaussian noise (sigma `noise`) on both frames
    and a global gain drawn from `gain` on frame 2."""
    rng = _rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)

    layers = []
    # layer 0: full-frame background with a small affine motion
    layers.append(dict(mask_fn=lambda X, Y: np.ones_like(X, bool), tex=texture(rng, h, w),
                       A=_affine(rng, w / 2, h / 2, min(dmax, 0.1 * dmax + 8), w, h)))
    for k in range(n_layers):
        cx = float(rng.uniform(0.1 * w, 0.9 * w))
        cy = float(rng.uniform(0.1 * h, 0.9 * h))
        rx = float(rng.uniform(0.06, 0.25) * w)
        ry = float(rng.uniform(0.08, 0.35) * h)
        if k % 2 == 0:
            th = float(rng.uniform(0, math.pi))
            mask_fn = _ellipse(cx, cy, rx, ry, th)
        else:
            mask_fn = _polygon(rng, cx, cy, rx, ry)
        layers.append(dict(mask_fn=mask_fn, tex=texture(rng, h, w), A=_affine(rng, cx, cy, dmax, rx, ry)))

    f1 = np.zeros((h, w, 3))
    f2 = np.zeros((h, w, 3))
    flow = np.zeros((h, w, 2), np.float32)
    own1 = np.full((h, w), -1, np.int32)
    own2 = np.full((h, w), -1, np.int32)
    for k, L in enumerate(layers):
        m1 = L["mask_fn"](xx, yy)
        f1[m1] = L["tex"][m1]
        own1[m1] = k
        fx, fy = _apply(L["A"], xx, yy)
        flow[m1, 0] = (fx - xx)[m1]
        flow[m1, 1] = (fy - yy)[m1]
        # frame 2: pixel X belongs to layer k if its preimage lies inside the layer's mask
        bx, by = _apply(_inverse(L["A"]), xx, yy)
        m2 = L["mask_fn"](bx, by) & (bx >= 0) & (bx <= w - 1) & (by >= 0) & (by <= h - 1)
        if k == 0:
            m2 = np.ones_like(m2)
        samp = _bilinear(L["tex"], bx, by)
        f2[m2] = samp[m2]
        own2[m2] = k
    tx = np.rint(xx + flow[..., 0]).astype(np.int64)
    ty = np.rint(yy + flow[..., 1]).astype(np.int64)
    inside = (tx >= 0) & (tx < w) & (ty >= 0) & (ty < h)
    valid = np.zeros((h, w), bool)
    valid[inside] = own2[ty[inside], tx[inside]] == own1[inside]
    a, b = _finish(rng, f1, f2, noise, gain)
    return Pair(a, b, flow, valid, f"layered{seed}_{w}x{h}")


def _affine(rng, cx, cy, dmax, rx, ry):
    """Affine map X -> X + t + M (X - c) with |displacement| <= dmax over a (rx, ry) region."""
    for _ in range(100):
        t = rng.uniform(-1, 1, 2) * dmax * 0.8
        M = rng.uniform(-0.08, 0.08, (2, 2))
        ext = np.abs(M) @ np.array([rx, ry])
        if np.hypot(abs(t[0]) + ext[0], abs(t[1]) + ext[1]) <= dmax:
            return (np.array([cx, cy]), t, M)
    return (np.array([cx, cy]), np.zeros(2), np.zeros((2, 2)))


def _apply(A, X, Y):
    c, t, M = A
    dx = X - c[0]
    dy = Y - c[1]
    return (X + t[0] + M[0, 0] * dx + M[0, 1] * dy, Y + t[1] + M[1, 0] * dx + M[1, 1] * dy)


def _inverse(A):
    c, t, M = A
    # Y = X + t + M (X - c)  =>  X = c + (I + M)^-1 (Y - c - t)
    Ainv = np.linalg.inv(np.eye(2) + M)
    # express as X = Y + t' + M' (Y - c') with c' = c + t
    c2 = c + t
    M2 = Ainv - np.eye(2)
    return (c2, c - c2, M2)


def _ellipse(cx, cy, rx, ry, th):
    ct, st = math.cos(th), math.sin(th)

    def f(X, Y):
        u = (X - cx) * ct + (Y - cy) * st
        v = -(X - cx) * st + (Y - cy) * ct
        return (u / rx) ** 2 + (v / ry) ** 2 <= 1.0
    return f


def _polygon(rng, cx, cy, rx, ry):
    n = int(rng.integers(3, 7))
    ang = np.sort(rng.uniform(0, 2 * math.pi, n))
    px = cx + rx * np.cos(ang)
    py = cy + ry * np.sin(ang)

    def f(X, Y):
        inside = np.ones_like(X, bool)
        for i in range(n):
            j = (i + 1) % n
            cross = (px[j] - px[i]) * (Y - py[i]) - (py[j] - py[i]) * (X - px[i])
            inside &= cross >= 0
        return inside
    return f


def road_pair(seed: int, h: int = 375, w: int = 1242, dmax: float = 250.0, n_boxes: int = 3,
              noise: float = 2.0, gain=(0.9, 1.1)) -> Pair:
    """KITTI-shaped pair: a textured ground plane over the lower 60% of the frame with
    forward-motion perspective flow (magnitude growing toward the bottom edge, up to dmax),
    a far background with small flow above it, and `n_boxes` textured boxes with their own
    translations. Frame 2 is rendered by backward bilinear warping."""
    rng = _rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    horizon = 0.4 * h
    ground_tex = texture(rng, h, w)
    sky_tex = texture(rng, h, w)
    f1 = np.where((yy >= horizon)[..., None], ground_tex, sky_tex).astype(np.float64)
    # forward motion: flow radiates from the focus of expansion at (w/2, horizon), its size
    # proportional to inverse depth (rows below the horizon)
    foe = np.array([w / 2, horizon])
    depth_inv = np.clip((yy - horizon) / (h - horizon), 0, 1)
    scale = dmax / max(np.hypot(w / 2, h - horizon), 1.0)
    flow = np.zeros((h, w, 2))
    g = yy >= horizon
    flow[..., 0] = np.where(g, (xx - foe[0]) * depth_inv * scale, rng.uniform(-2, 2))
    flow[..., 1] = np.where(g, (yy - foe[1]) * depth_inv * scale, rng.uniform(-1, 1))
    owner = np.where(g, 0, -1)
    for k in range(n_boxes):
        bw = int(rng.uniform(0.05, 0.15) * w)
        bh = int(rng.uniform(0.1, 0.3) * h)
        x0 = int(rng.integers(0, w - bw))
        y0 = int(rng.integers(int(0.2 * h), h - bh))
        t = rng.uniform(-1, 1, 2) * np.array([0.5 * dmax, 0.2 * dmax])
        f1[y0:y0 + bh, x0:x0 + bw] = texture(rng, bh, bw)
        flow[y0:y0 + bh, x0:x0 + bw] = t
        owner[y0:y0 + bh, x0:x0 + bw] = k + 1
    # frame 2 by backward warping with the flow splatted to the nearest target pixel (last
    # writer wins in z-order: ground < boxes); holes keep a plain warp of frame 1
    f2 = _bilinear(f1, xx - flow[..., 0], yy - flow[..., 1])
    tx = np.rint(xx + flow[..., 0]).astype(np.int64)
    ty = np.rint(yy + flow[..., 1]).astype(np.int64)
    inside = (tx >= 0) & (tx < w) & (ty >= 0) & (ty < h)
    own2 = np.full((h, w), -2, np.int64)
    order = np.argsort(owner[inside], kind="stable")
    src_y, src_x = np.nonzero(inside)
    src_y, src_x = src_y[order], src_x[order]
    f2[ty[src_y, src_x], tx[src_y, src_x]] = f1[src_y, src_x]
    own2[ty[src_y, src_x], tx[src_y, src_x]] = owner[src_y, src_x]
    valid = np.zeros((h, w), bool)
    valid[inside] = own2[ty[inside], tx[inside]] == owner[inside]
    a, b = _finish(rng, f1, f2, noise, gain)
    return Pair(a, b, flow.astype(np.float32), valid, f"road{seed}_{w}x{h}")


def translate_pair(seed: int, h: int, w: int, dx: int, dy: int) -> Pair:
    """Frame 2 = frame 1 shifted by an integer (dx, dy): I2(x + d) = I1(x). Pixels of frame 2
    with no source take fresh texture."""
    rng = _rng(seed)
    big = texture(rng, h + 2 * abs(dy) + 2, w + 2 * abs(dx) + 2)
    oy, ox = abs(dy) + 1, abs(dx) + 1
    img1 = np.ascontiguousarray(big[oy:oy + h, ox:ox + w])
    img2 = np.ascontiguousarray(big[oy - dy:oy - dy + h, ox - dx:ox - dx + w])
    flow = np.zeros((h, w, 2), np.float32)
    flow[..., 0] = dx
    flow[..., 1] = dy
    yy, xx = np.mgrid[0:h, 0:w]
    valid = (xx + dx >= 0) & (xx + dx < w) & (yy + dy >= 0) & (yy + dy < h)
    return Pair(img1, img2, flow, valid, f"translate{seed}_{dx}_{dy}")


BATCH_SHAPES = ((320, 240), (640, 480), (1024, 436), (1242, 375))


def batch_sizes(seed: int, n: int = 64):
    """Sizes (w, h) drawn uniformly from the four batch shapes."""
    rng = _rng(seed)
    idx = rng.integers(0, len(BATCH_SHAPES), n)
    return [BATCH_SHAPES[i] for i in idx]


def served_sizes(seed: int, n: int):
    """Request sizes: log-uniform area in [320*240, 2048*1024], aspect U[1.3, 3.3],
    clipped to [320, 2048] x [240, 1024]."""
    rng = _rng(seed)
    out = []
    for _ in range(n):
        area = math.exp(rng.uniform(math.log(320 * 240), math.log(2048 * 1024)))
        aspect = rng.uniform(1.3, 3.3)
        w = int(round(math.sqrt(area * aspect)))
        h = int(round(area / max(w, 1)))
        out.append((min(max(w, 320), 2048), min(max(h, 240), 1024)))
    return out


def config_pair(config: int, index: int = 0, size=None) -> Pair:
    """The seeded pair for workload `config` (1..5) and pair `index`."""
    seed = 1000 * config + index
    if config == 1:
        return rect_pair(seed, 192, 256)
    if config == 2:
        return layered_pair(seed, 436, 1024)
    if config == 3:
        return road_pair(seed, 375, 1242)
    if config in (4, 5):
        w, h = size
        return rect_pair(seed, h, w, dmax=max(1, w // 5))
    raise ValueError(f"unknown config {config}")
