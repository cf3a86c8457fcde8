"""ctypes front end of the CPU oracle (``libpgm_oracle.so``, built from ``pgm_oracle.c``).

TEST INFRASTRUCTURE ONLY. The oracle is a plain single-threaded C implementation of
pyramidal gradient matching (Li, arXiv:1704.03217, Sec. III) that the test-suite, the smoke
check and the benchmark's CPU-baseline leg compare the GPU library against. The GPU library
never imports this package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pgm_oracle.c")
LIB = os.path.join(HERE, "libpgm_oracle.so")

MAX_LEVELS = 8
SYNC, SCAN = 0, 1
F_INIT, F_INLIER, F_RECORD = 1, 2, 4
FEAT_INT16, FEAT_F32_DIR = 0, 1
RGB, GRAY = 0, 1
INIT_RANDOM, INIT_EXHAUSTIVE = 0, 1
RS_FLOOR, RS_SYMMETRIC = 0, 1


class Params(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("seed_stride", C.c_int32),
        ("patch_fwd", C.c_int32), ("patch_bwd", C.c_int32),
        ("iters", C.c_int32 * MAX_LEVELS),
        ("radius", C.c_int32), ("max_disp", C.c_int32), ("sobel_ksize", C.c_int32),
        ("feature", C.c_int32), ("color", C.c_int32), ("fwd_bwd", C.c_int32),
        ("consistency_px", C.c_int32), ("init_mode", C.c_int32), ("refine_rounds", C.c_int32),
        ("min_region_px", C.c_int32), ("region_link_px", C.c_int32),
        ("space_fwd", C.c_int32 * MAX_LEVELS), ("space_bwd", C.c_int32 * MAX_LEVELS),
        ("metric", C.c_int32), ("rs_mode", C.c_int32),
        ("rng_seed", C.c_uint64),
    ]


class Match(C.Structure):
    _fields_ = [("x1", C.c_int32), ("y1", C.c_int32), ("x2", C.c_int32), ("y2", C.c_int32),
                ("dist", C.c_int32), ("flags", C.c_uint32)]


MATCH_DTYPE = np.dtype([("x1", "<i4"), ("y1", "<i4"), ("x2", "<i4"), ("y2", "<i4"),
                        ("dist", "<i4"), ("flags", "<u4")])


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (plain C11, -O2, no intrinsics)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.pgmo_reflect101.argtypes = [C.c_int, C.c_int]
        L.pgmo_pyr_down.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, P]
        L.pgmo_gray.argtypes = [P, C.c_int, C.c_int, C.c_int, P]
        L.pgmo_gradient_image.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]
        L.pgmo_direction.argtypes = [P, C.c_int, C.c_int, P]
        L.pgmo_dist_i16.argtypes = [P, P] + [C.c_int] * 8
        L.pgmo_dist_i16.restype = C.c_int64
        L.pgmo_ssd_i16.argtypes = [P, P] + [C.c_int] * 8
        L.pgmo_ssd_i16.restype = C.c_int64
        L.pgmo_dist_f32.argtypes = [P, P] + [C.c_int] * 8
        L.pgmo_dist_f32.restype = C.c_float
        L.pgmo_philox4x32_10.argtypes = [P, P, P]
        L.pgmo_search_offset.argtypes = [C.c_uint32, C.c_int, C.c_int]
        L.pgmo_init_offset.argtypes = [C.c_uint32, C.c_int]
        L.pgmo_search_offset_sym.argtypes = [C.c_uint32, C.c_int, C.c_int]
        L.pgmo_grid_count.argtypes = [C.c_int, C.c_int]
        L.pgmo_grid_pos.argtypes = [C.c_int, C.c_int, C.c_int]
        L.pgmo_grid_nearest.argtypes = [C.c_int, C.c_int, C.c_int]
        L.pgmo_geometry.argtypes = [C.POINTER(Params), C.c_int, C.c_int, P, P, P, P]
        L.pgmo_top_radius.argtypes = [C.POINTER(Params), C.c_int, C.c_int]
        L.pgmo_convert.argtypes = [P, C.c_int, C.c_int, P]
        L.pgmo_convert.restype = None
        L.pgmo_sign.argtypes = [P, C.c_int]
        L.pgmo_sign.restype = None
        L.pgmo_remove_small_regions.argtypes = [P, P, P] + [C.c_int] * 5
        L.pgmo_remove_small_regions.restype = None
        L.pgmo_match.argtypes = [C.POINTER(Params), P, P, C.c_int, C.c_int, C.c_int, C.c_int,
                                 P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_params(d: dict) -> Params:
    p = Params()
    for k, v in d.items():
        if k in ("iters", "space_fwd", "space_bwd"):
            arr = (list(v) + [0] * MAX_LEVELS)[:MAX_LEVELS]
            setattr(p, k, (C.c_int32 * MAX_LEVELS)(*arr))
        else:
            setattr(p, k, v)
    return p


# ---- building blocks ----

SPACE_RGB, SPACE_YCRCB, SPACE_LAB = 0, 1, 2


def convert(img: np.ndarray, space: int) -> np.ndarray:
    """Colour conversion of an (h, w, 3) uint8 RGB image (Table II's spaces)."""
    img = np.ascontiguousarray(img, np.uint8)
    out = np.empty_like(img)
    lib().pgmo_convert(_p(img), img.size // 3, space, _p(out))
    return out


def sign(G: np.ndarray) -> np.ndarray:
    """Literal "G./|G|" of Sec. III-F: the sign of every gradient component (int16)."""
    out = np.ascontiguousarray(G, np.int16).copy()
    lib().pgmo_sign(_p(out), out.size)
    return out


def remove_small_regions(dx: np.ndarray, dy: np.ndarray, inl: np.ndarray, stride: int, min_px: int,
                         link_px: int) -> np.ndarray:
    """Small-region removal on an (ny, nx) grid field; returns the new inlier mask."""
    dx = np.ascontiguousarray(dx, np.int32)
    dy = np.ascontiguousarray(dy, np.int32)
    out = np.ascontiguousarray(inl, np.uint8).copy()
    ny, nx = out.shape
    lib().pgmo_remove_small_regions(_p(dx), _p(dy), _p(out), nx, ny, stride, min_px, link_px)
    return out.astype(bool)


def lift(fw: int, fh: int, cw: int, ch: int, stride: int, dx, dy, inl):
    """The lift toward the coarser level (Sec. III-D) of a finer field given as (nx*ny,) arrays;
    returns the coarse (dx, dy, init) arrays."""
    fdx = np.ascontiguousarray(dx, np.int32); fdy = np.ascontiguousarray(dy, np.int32)
    finl = np.ascontiguousarray(inl, np.uint8)
    n = grid_count(cw, stride) * grid_count(ch, stride)
    cdx = np.zeros(n, np.int32); cdy = np.zeros(n, np.int32); cinit = np.zeros(n, np.uint8)
    L = lib()
    L.pgmo_lift.argtypes = [C.c_int] * 5 + [C.c_void_p] * 6
    if L.pgmo_lift(fw, fh, cw, ch, stride, _p(fdx), _p(fdy), _p(finl), _p(cdx), _p(cdy), _p(cinit)) != 0:
        raise ValueError("oracle rejected the lift sizes")
    return cdx, cdy, cinit


def reflect101(i: int, n: int) -> int:
    return lib().pgmo_reflect101(i, n)


def pyr_down(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img)
    h, w = img.shape[:2]
    ch = 1 if img.ndim == 2 else img.shape[2]
    out = np.empty(((h + 1) // 2, (w + 1) // 2) + (() if img.ndim == 2 else (ch,)), np.uint8)
    lib().pgmo_pyr_down(_p(img), w, h, w * ch, ch, _p(out))
    return out


def gray(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img)
    h, w = img.shape[:2]
    out = np.empty((h, w), np.uint8)
    lib().pgmo_gray(_p(img), w, h, w * 3, _p(out))
    return out


def gradient_image(img: np.ndarray, ksize: int = 5) -> np.ndarray:
    """(h, w, 2*ch) int16 gradient image of an (h, w[, ch]) uint8 image."""
    img = np.ascontiguousarray(img)
    h, w = img.shape[:2]
    ch = 1 if img.ndim == 2 else img.shape[2]
    out = np.empty((h, w, 2 * ch), np.int16)
    lib().pgmo_gradient_image(_p(img), w, h, w * ch, ch, ksize, _p(out))
    return out


def direction(G: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(G, np.int16)
    ch = G.shape[-1] // 2
    out = np.empty(G.shape, np.float32)
    lib().pgmo_direction(_p(G), int(G.size // G.shape[-1]), ch, _p(out))
    return out


def dist(Ga: np.ndarray, Gb: np.ndarray, P: int, xa: int, ya: int, xb: int, yb: int):
    h, w, C2 = Ga.shape
    if Ga.dtype == np.int16:
        Ga = np.ascontiguousarray(Ga); Gb = np.ascontiguousarray(Gb)
        return lib().pgmo_dist_i16(_p(Ga), _p(Gb), w, h, C2, P, xa, ya, xb, yb)
    Ga = np.ascontiguousarray(Ga, np.float32); Gb = np.ascontiguousarray(Gb, np.float32)
    return lib().pgmo_dist_f32(_p(Ga), _p(Gb), w, h, C2, P, xa, ya, xb, yb)


def ssd(Ga: np.ndarray, Gb: np.ndarray, P: int, xa: int, ya: int, xb: int, yb: int) -> int:
    """Eq. 3 as printed (squared differences) on integer features, exact."""
    h, w, C2 = Ga.shape
    Ga = np.ascontiguousarray(Ga, np.int16); Gb = np.ascontiguousarray(Gb, np.int16)
    return lib().pgmo_ssd_i16(_p(Ga), _p(Gb), w, h, C2, P, xa, ya, xb, yb)


def philox(ctr, key) -> np.ndarray:
    c = np.array(ctr, np.uint32)
    k = np.array(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().pgmo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def search_offset(u: int, W: int, i: int) -> int:
    return lib().pgmo_search_offset(u, W, i)


def search_offset_sym(u: int, W: int, i: int) -> int:
    return lib().pgmo_search_offset_sym(u, W, i)


def init_offset(u: int, R: int) -> int:
    return lib().pgmo_init_offset(u, R)


def grid_count(n, stride):
    return lib().pgmo_grid_count(n, stride)


def grid_pos(i, n, stride):
    return lib().pgmo_grid_pos(i, n, stride)


def grid_nearest(x, nseeds, stride):
    return lib().pgmo_grid_nearest(x, nseeds, stride)


def geometry(params: dict, w: int, h: int):
    p = make_params(params)
    arrs = [np.zeros(MAX_LEVELS, np.int32) for _ in range(4)]
    rc = lib().pgmo_geometry(C.byref(p), w, h, *[_p(a) for a in arrs])
    if rc != 0:
        raise ValueError("invalid geometry")
    L = params["levels"]
    return [tuple(int(a[l]) for a in arrs) for l in range(L)]   # (w, h, nx, ny) per level


def top_radius(params: dict, w: int, h: int) -> int:
    p = make_params(params)
    return lib().pgmo_top_radius(C.byref(p), w, h)


# ---- the whole method ----

def match(params: dict, img1: np.ndarray, img2: np.ndarray, schedule: int = SYNC, trace: bool = True):
    """Run the oracle. Returns a dict with 'fwd', 'bwd' (structured match arrays of level 0),
    'compact', 'n_inliers', 'n_evals' and, with trace=True, 'levels': per dir a list over
    levels of (n, 4) int32 arrays {dx, dy, dist bits, flags}."""
    img1 = np.ascontiguousarray(img1, np.uint8)
    img2 = np.ascontiguousarray(img2, np.uint8)
    h, w = img1.shape[:2]
    assert img1.shape == (h, w, 3) and img2.shape == (h, w, 3)
    geo = geometry(params, w, h)
    n0 = geo[0][2] * geo[0][3]
    fwd = np.zeros(n0, MATCH_DTYPE)
    bwd = np.zeros(n0, MATCH_DTYPE)
    comp = np.zeros(n0, MATCH_DTYPE)
    ntot = sum(g[2] * g[3] for g in geo)
    tr = np.zeros(2 * ntot * 4, np.int32) if trace else None
    nin = np.zeros(1, np.int32)
    nev = np.zeros(1, np.uint64)
    p = make_params(params)
    rc = lib().pgmo_match(C.byref(p), _p(img1), _p(img2), w, h, w * 3, schedule, _p(fwd), _p(bwd),
                          _p(nin), _p(comp), _p(tr) if trace else None, _p(nev))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    out = dict(fwd=fwd, bwd=bwd, compact=comp[: int(nin[0])].copy(), n_inliers=int(nin[0]),
               n_evals=int(nev[0]), geometry=geo)
    if trace:
        levels = [[], []]
        off = 0
        for d in range(2):
            for (lw, lh, nx, ny) in geo:
                n = nx * ny
                levels[d].append(tr[off:off + 4 * n].reshape(n, 4).copy())
                off += 4 * n
        out["levels"] = levels
    return out


def sweep(params: dict, Ga: np.ndarray, Gb: np.ndarray, state: dict, *, W: int, t0: int = 0,
          n_iter: int = 1, level: int = 0, dir: int = 0, stage: int = 0, schedule: int = SYNC):
    """Run Step 1 (Eq. 4-5) alone on one field. `state` holds (nx*ny,) arrays dx, dy, dist
    (int32 / float bits) and init (uint8); returns the updated copy and the evaluation count."""
    h, w = Ga.shape[:2]
    Ga = np.ascontiguousarray(Ga); Gb = np.ascontiguousarray(Gb)
    st = {k: np.ascontiguousarray(np.array(state[k], dtype=dt)) for k, dt in
          (("dx", np.int32), ("dy", np.int32), ("dist", np.int32), ("init", np.uint8))}
    nev = np.zeros(1, np.uint64)
    p = make_params(params)
    L = lib()
    L.pgmo_sweep.argtypes = [C.POINTER(Params)] + [C.c_int] * 4 + [C.c_void_p, C.c_void_p] + \
        [C.c_int] * 5 + [C.c_void_p] * 5
    rc = L.pgmo_sweep(C.byref(p), level, dir, stage, W, _p(Ga), _p(Gb), w, h, t0, n_iter, schedule,
                      _p(st["dx"]), _p(st["dy"]), _p(st["dist"]), _p(st["init"]), _p(nev))
    if rc != 0:
        raise ValueError("oracle rejected the sweep arguments")
    return st, int(nev[0])
