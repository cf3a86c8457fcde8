"""Python binding of libpgm: pyramidal gradient matching (Li, arXiv:1704.03217) on MI355X.

The functions named pgm_* wrap the C entry points of ``include/pgm.h`` one to one (ctypes
argument marshalling only; every step of the method runs in the HIP kernels of libpgm.so).
PyTorch is used only to own device memory and streams: pass tensors' data pointers, or use
:class:`Matcher`, which allocates the outputs as torch tensors.

Importing this package does not need a GPU; loading the library does need it to be built
(``python -m paper_1704_03217_amd.build``) and a call that does device work needs a GPU.
There is no CPU fallback: without libpgm.so every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgm.so")

MAX_LEVELS = 8
PGM_OK, PGM_EINVAL, PGM_ENOMEM, PGM_EDEVICE, PGM_EBUSY, PGM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FEAT_INT16, FEAT_F32_DIR, FEAT_SIGN = 0, 1, 2
RGB, GRAY = 0, 1
SPACE_RGB, SPACE_YCRCB, SPACE_LAB = 0, 1, 2
INIT_RANDOM, INIT_EXHAUSTIVE = 0, 1
METRIC_SAD, METRIC_SSD = 0, 1
RS_FLOOR, RS_SYMMETRIC = 0, 1
FLAG_INIT, FLAG_INLIER, FLAG_RECORD = 1, 2, 4
PRESET_PAPER, PRESET_CONFIG1, PRESET_CONFIG2, PRESET_CONFIG3, PRESET_CONFIG4, PRESET_CONFIG5 = 0, 1, 2, 3, 4, 5


class pgm_params(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("seed_stride", C.c_int32),
        ("patch_fwd", C.c_int32), ("patch_bwd", C.c_int32),
        ("iters", C.c_int32 * MAX_LEVELS),
        ("radius", C.c_int32), ("max_disp", C.c_int32), ("sobel_ksize", C.c_int32),
        ("feature", C.c_int32), ("color", C.c_int32), ("fwd_bwd", C.c_int32),
        ("consistency_px", C.c_int32), ("init_mode", C.c_int32), ("refine_rounds", C.c_int32),
        ("min_region_px", C.c_int32), ("region_link_px", C.c_int32),
        ("space_fwd", C.c_int32 * MAX_LEVELS), ("space_bwd", C.c_int32 * MAX_LEVELS),
        ("metric", C.c_int32), ("rs_mode", C.c_int32), ("rng_seed", C.c_uint64),
    ]


class pgm_sizes(C.Structure):
    _fields_ = [
        ("levels", C.c_int32),
        ("level_w", C.c_int32 * MAX_LEVELS), ("level_h", C.c_int32 * MAX_LEVELS),
        ("level_nx", C.c_int32 * MAX_LEVELS), ("level_ny", C.c_int32 * MAX_LEVELS),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("workspace_bytes", C.c_uint64),
        ("workspace_shared_bytes", C.c_uint64),
        ("workspace_pair_bytes", C.c_uint64),
    ]


class pgm_group(C.Structure):
    _fields_ = [
        ("params", C.POINTER(pgm_params)),
        ("n_pairs", C.c_int32), ("w", C.c_int32), ("h", C.c_int32), ("pitch_bytes", C.c_int32),
        ("image_stride_bytes", C.c_int64),
        ("img1", C.c_void_p), ("img2", C.c_void_p),
        ("out_fwd", C.c_void_p), ("out_bwd", C.c_void_p),
        ("out_n_inliers", C.c_void_p), ("out_compact", C.c_void_p),
    ]


MATCH_DTYPE = np.dtype([("x1", "<i4"), ("y1", "<i4"), ("x2", "<i4"), ("y2", "<i4"),
                        ("dist", "<i4"), ("flags", "<u4")])
MATCH_BYTES = 24

EXPORTS = ("pgm_default_params", "pgm_query", "pgm_create", "pgm_match", "pgm_match_static", "pgm_match_batch",
           "pgm_match_groups",
           "pgm_server_create", "pgm_server_submit", "pgm_server_poll", "pgm_server_stats", "pgm_server_pending",
           "pgm_server_drain", "pgm_server_last_error", "pgm_server_destroy", "pgm_format_matches",
           "pgm_dump_level",
           "pgm_dump_gradient", "pgm_dump_pyramid", "pgm_schedule", "pgm_tune", "pgm_profile", "pgm_profile_read",
           "pgm_last_error", "pgm_destroy")

# kernel kinds of pgm_profile_read
K_PYRAMID, K_GRADIENT, K_PREP, K_INIT, K_DOWN, K_UP, K_SWEEP, K_CHECK, K_OUTPUT, K_COMPACT, K_LEVEL, K_REGION, \
    K_SWEEP_MULTI, K_SWEEP_PAIR = range(14)
KIND_NAMES = ("pyramid", "gradient", "prep", "init", "down", "up", "sweep", "check", "output", "compact", "level",
              "region", "sweep_multi", "sweep_pair")


class PGMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpgm status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libpgm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1704_03217_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        L.pgm_default_params.argtypes = [C.POINTER(pgm_params), C.c_int32]
        L.pgm_default_params.restype = C.c_int32
        L.pgm_query.argtypes = [C.POINTER(pgm_params), C.c_int32, C.c_int32, C.POINTER(pgm_sizes)]
        L.pgm_query.restype = C.c_int32
        L.pgm_create.argtypes = [C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]
        L.pgm_create.restype = C.c_int32
        L.pgm_match.argtypes = [V, C.POINTER(pgm_params), V, V, C.c_int32, C.c_int32, C.c_int32,
                                V, V, V, V, V, V]
        L.pgm_match.restype = C.c_int32
        L.pgm_match_static.argtypes = [C.POINTER(pgm_params), V, V, C.c_int32, C.c_int32, C.c_int32,
                                       V, V, V, V, V, V]
        L.pgm_match_static.restype = C.c_int32
        L.pgm_match_batch.argtypes = [V, C.POINTER(pgm_params), C.c_int32, V, V, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_int64, V, V, V, V, V, V]
        L.pgm_match_batch.restype = C.c_int32
        L.pgm_match_groups.argtypes = [V, C.c_int32, C.POINTER(pgm_group), V, C.c_int32, V]
        L.pgm_match_groups.restype = C.c_int32
        L.pgm_server_create.argtypes = [C.c_int32, C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_void_p)]
        L.pgm_server_create.restype = C.c_int32
        L.pgm_server_submit.argtypes = [V, C.POINTER(pgm_params), V, V, C.c_int32, C.c_int32, C.c_int32,
                                        V, V, V, V, V, C.c_uint64, V]
        L.pgm_server_submit.restype = C.c_int32
        L.pgm_server_poll.argtypes = [V, C.POINTER(C.c_uint64), C.POINTER(C.c_int32), C.c_int32]
        L.pgm_server_poll.restype = C.c_int32
        L.pgm_server_stats.argtypes = [V, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]
        L.pgm_server_stats.restype = C.c_int32
        L.pgm_server_pending.argtypes = [V, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.pgm_server_pending.restype = C.c_int32
        L.pgm_server_drain.argtypes = [V]
        L.pgm_server_drain.restype = C.c_int32
        L.pgm_server_last_error.argtypes = [V]
        L.pgm_server_last_error.restype = C.c_char_p
        L.pgm_server_destroy.argtypes = [V]
        L.pgm_server_destroy.restype = None
        L.pgm_format_matches.argtypes = [V, C.c_int64, C.c_int32, V, C.c_uint64, C.POINTER(C.c_uint64)]
        L.pgm_format_matches.restype = C.c_int32
        L.pgm_dump_level.argtypes = [V, C.c_int32, C.c_int32, V]
        L.pgm_dump_level.restype = C.c_int32
        L.pgm_dump_gradient.argtypes = [V, C.c_int32, C.c_int32, V]
        L.pgm_dump_gradient.restype = C.c_int32
        L.pgm_dump_pyramid.argtypes = [V, C.c_int32, C.c_int32, V]
        L.pgm_dump_pyramid.restype = C.c_int32
        L.pgm_schedule.argtypes = [V, C.c_int32]
        L.pgm_schedule.restype = C.c_int32
        L.pgm_tune.argtypes = [V, C.POINTER(pgm_params), C.c_int32, V, V, C.c_int32, C.c_int32, C.c_int32,
                               C.c_int64, V, V, V, V, C.c_int32, V, C.POINTER(C.c_int32)]
        L.pgm_tune.restype = C.c_int32
        L.pgm_profile.argtypes = [V, C.c_int32]
        L.pgm_profile.restype = C.c_int32
        L.pgm_profile_read.argtypes = [V, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_uint64)]
        L.pgm_profile_read.restype = C.c_int32
        L.pgm_last_error.argtypes = [V]
        L.pgm_last_error.restype = C.c_char_p
        L.pgm_destroy.argtypes = [V]
        L.pgm_destroy.restype = None
        _lib = L
    return _lib


def params(d: dict | None = None, preset: int | None = None, **kw) -> pgm_params:
    """Build a pgm_params from a preset and/or a dict of field values."""
    p = pgm_params()
    if preset is not None:
        _check(lib().pgm_default_params(C.byref(p), preset), None)
    for k, v in dict(d or {}, **kw).items():
        if k in ("iters", "space_fwd", "space_bwd"):
            vals = (list(v) + [0] * MAX_LEVELS)[:MAX_LEVELS]
            setattr(p, k, (C.c_int32 * MAX_LEVELS)(*vals))
        else:
            setattr(p, k, v)
    return p


def params_dict(p: pgm_params) -> dict:
    d = {name: getattr(p, name) for name, _ in pgm_params._fields_}
    d["iters"] = list(p.iters)[: p.levels]
    d["space_fwd"] = list(p.space_fwd)[: p.levels]
    d["space_bwd"] = list(p.space_bwd)[: p.levels]
    return d


def _check(status, ctx):
    if status != PGM_OK:
        msg = lib().pgm_last_error(ctx)
        raise PGMError(status, msg.decode() if msg else "")
    return status


# ---- one-to-one wrappers of the C entry points ----

def pgm_default_params(preset: int) -> pgm_params:
    p = pgm_params()
    _check(lib().pgm_default_params(C.byref(p), preset), None)
    return p


def pgm_query(p, w: int, h: int) -> pgm_sizes:
    s = pgm_sizes()
    st = lib().pgm_query(C.byref(_as_params(p)), w, h, C.byref(s))
    if st != PGM_OK:
        raise PGMError(st, "invalid parameters or image size")
    return s


def pgm_create(device: int = 0, workspace_bytes: int = 0):
    h = C.c_void_p()
    _check(lib().pgm_create(device, workspace_bytes, C.byref(h)), None)
    return h


def pgm_match(ctx, p, img1: int, img2: int, w: int, h: int, pitch_bytes: int, out_fwd: int,
              out_bwd: int | None = None, out_n_inliers: int | None = None,
              out_compact: int | None = None, out_n_evals: int | None = None, stream: int | None = None):
    """All pointer arguments are integer device addresses (or None)."""
    return _check(lib().pgm_match(ctx, C.byref(_as_params(p)), img1, img2, w, h, pitch_bytes, out_fwd,
                                  out_bwd, out_n_inliers, out_compact, out_n_evals, stream), ctx)


STATIC_SCRATCH_BYTES = 64 << 20


def pgm_match_static(p, img1: int, img2: int, w: int, h: int, pitch_bytes: int, out_fwd: int,
                     out_bwd: int | None = None, out_n_inliers: int | None = None,
                     out_compact: int | None = None, out_n_evals: int | None = None, stream: int | None = None):
    """pgm_match without a context (no device allocation); on the current HIP device."""
    return _check(lib().pgm_match_static(C.byref(_as_params(p)), img1, img2, w, h, pitch_bytes, out_fwd,
                                         out_bwd, out_n_inliers, out_compact, out_n_evals, stream), None)


def pgm_match_batch(ctx, p, n_pairs: int, img1: int, img2: int, w: int, h: int, pitch_bytes: int,
                    image_stride_bytes: int, out_fwd: int, out_bwd: int | None = None,
                    out_n_inliers: int | None = None, out_compact: int | None = None,
                    out_n_evals: int | None = None, stream: int | None = None):
    """All pointer arguments are integer device addresses (or None)."""
    return _check(lib().pgm_match_batch(ctx, C.byref(_as_params(p)), n_pairs, img1, img2, w, h, pitch_bytes,
                                        image_stride_bytes, out_fwd, out_bwd, out_n_inliers, out_compact,
                                        out_n_evals, stream), ctx)


def pgm_match_groups(ctx, groups, out_n_evals: int | None = None, use_graph: bool = False,
                     stream: int | None = None):
    """groups: a sequence of pgm_group (their params pointers must stay alive for the call)."""
    arr = (pgm_group * len(groups))(*groups)
    return _check(lib().pgm_match_groups(ctx, len(groups), arr, out_n_evals, 1 if use_graph else 0, stream), ctx)


def _check_server(status, server):
    if status < 0:
        msg = lib().pgm_server_last_error(server)
        raise PGMError(status, msg.decode() if msg else "")
    return status


def pgm_server_create(device: int, pool_bytes: int, n_streams: int, max_queued: int = 0, max_batch: int = 0):
    h = C.c_void_p()
    _check_server(lib().pgm_server_create(device, pool_bytes, n_streams, max_queued, max_batch, C.byref(h)), None)
    return h


def pgm_server_submit(server, p, img1: int, img2: int, w: int, h: int, pitch_bytes: int, out_fwd: int,
                      out_bwd: int | None, out_n_inliers: int | None, out_compact: int | None,
                      out_n_evals: int | None, tag: int, stream: int | None = None):
    return _check_server(lib().pgm_server_submit(server, C.byref(_as_params(p)), img1, img2, w, h, pitch_bytes,
                                                 out_fwd, out_bwd, out_n_inliers, out_compact, out_n_evals,
                                                 tag, stream), server)


def pgm_server_poll(server, max_tags: int = 256) -> list:
    """[(tag, status)] of the requests finished since the last poll."""
    buf = (C.c_uint64 * max(1, max_tags))()
    st = (C.c_int32 * max(1, max_tags))()
    n = _check_server(lib().pgm_server_poll(server, buf, st, max_tags), server)
    return [(buf[k], st[k]) for k in range(n)]


def pgm_server_stats(server):
    """(launch sequences started, requests started, pool bytes in use)."""
    a, b, u = C.c_int64(), C.c_int64(), C.c_uint64()
    _check_server(lib().pgm_server_stats(server, C.byref(a), C.byref(b), C.byref(u)), server)
    return a.value, b.value, u.value


def pgm_server_pending(server):
    q, r, f = C.c_int32(), C.c_int32(), C.c_int32()
    _check_server(lib().pgm_server_pending(server, C.byref(q), C.byref(r), C.byref(f)), server)
    return q.value, r.value, f.value


def pgm_server_last_error_text(server) -> str:
    m = lib().pgm_server_last_error(server)
    return m.decode() if m else ""


def pgm_server_drain(server) -> None:
    _check_server(lib().pgm_server_drain(server), server)


def pgm_server_destroy(server) -> None:
    lib().pgm_server_destroy(server)


def pgm_format_matches(matches: np.ndarray, inliers_only: bool = True) -> str:
    """EpicFlow-style "x1 y1 x2 y2" lines of host matches (a MATCH_DTYPE array)."""
    m = np.ascontiguousarray(matches).view(MATCH_DTYPE)
    n = C.c_uint64()
    ptr = m.ctypes.data if m.size else None
    st = lib().pgm_format_matches(ptr, m.size, 1 if inliers_only else 0, None, 0, C.byref(n))
    if st != PGM_OK:
        raise PGMError(st, "invalid arguments")
    buf = C.create_string_buffer(max(1, n.value))
    st = lib().pgm_format_matches(ptr, m.size, 1 if inliers_only else 0, buf, n.value, C.byref(n))
    if st != PGM_OK:
        raise PGMError(st, "formatting failed")
    return buf.raw[: n.value].decode()


def write_epicflow_matches(path: str, matches: np.ndarray, inliers_only: bool = True) -> int:
    """Write the matches to a text file for an external interpolator; returns the line count."""
    text = pgm_format_matches(matches, inliers_only)
    with open(path, "w") as f:
        f.write(text)
    return text.count("\n")


def pgm_dump_level(ctx, level: int, dir: int, n: int) -> np.ndarray:
    out = np.zeros((n, 4), np.int32)
    _check(lib().pgm_dump_level(ctx, level, dir, out.ctypes.data), ctx)
    return out


def pgm_dump_gradient(ctx, level: int, image: int, shape, f32: bool) -> np.ndarray:
    out = np.zeros(shape, np.float32 if f32 else np.int16)
    _check(lib().pgm_dump_gradient(ctx, level, image, out.ctypes.data), ctx)
    return out


def pgm_dump_pyramid(ctx, level: int, image: int, w: int, h: int) -> np.ndarray:
    out = np.zeros((h, w, 3), np.uint8)
    _check(lib().pgm_dump_pyramid(ctx, level, image, out.ctypes.data), ctx)
    return out


SCHED_AUTO, SCHED_LEVEL_LDS, SCHED_LEVEL_LAUNCHES, SCHED_SEPARATE = 0, 1, 2, 4


def pgm_schedule(ctx, flags: int) -> None:
    _check(lib().pgm_schedule(ctx, flags), ctx)


def pgm_tune(ctx, p, n_pairs: int, img1: int, img2: int, w: int, h: int, pitch_bytes: int, image_stride_bytes: int,
             out_fwd: int, out_bwd: int | None = None, out_n_inliers: int | None = None,
             out_compact: int | None = None, repeats: int = 3, stream: int | None = None) -> int:
    """All pointer arguments are integer device addresses (or None); returns the chosen flags."""
    flags = C.c_int32(0)
    _check(lib().pgm_tune(ctx, C.byref(_as_params(p)), n_pairs, img1, img2, w, h, pitch_bytes, image_stride_bytes,
                          out_fwd, out_bwd, out_n_inliers, out_compact, repeats, stream, C.byref(flags)), ctx)
    return flags.value


def pgm_profile(ctx, enable: bool) -> None:
    _check(lib().pgm_profile(ctx, 1 if enable else 0), ctx)


def pgm_profile_read(ctx, kind: int):
    """(launches, total milliseconds, distance evaluations) of one kernel kind."""
    n, ms, ev = C.c_int64(), C.c_double(), C.c_uint64()
    _check(lib().pgm_profile_read(ctx, kind, C.byref(n), C.byref(ms), C.byref(ev)), ctx)
    return n.value, ms.value, ev.value


def pgm_last_error(ctx) -> str:
    m = lib().pgm_last_error(ctx)
    return m.decode() if m else ""


def pgm_destroy(ctx) -> None:
    lib().pgm_destroy(ctx)


def _as_params(p):
    return p if isinstance(p, pgm_params) else params(p)


# ---- convenience wrapper over torch tensors ----

class Matcher:
    """A libpgm context plus torch-allocated outputs. Images are (h, w, 3) uint8 CUDA (HIP)
    tensors; work is issued on torch's current stream."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        import torch  # device memory and streams only
        self.torch = torch
        self.device = device
        self.ctx = pgm_create(device, workspace_bytes)
        self.last_sizes = None

    def close(self):
        if self.ctx:
            pgm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self, p, w, h, bwd=True, compact=True, count_evals=True):
        torch = self.torch
        s = pgm_query(p, w, h)
        n = s.nx * s.ny
        dev = torch.device("cuda", self.device)
        o = dict(sizes=s, n=n)
        o["fwd"] = torch.empty(n * 6, dtype=torch.int32, device=dev)
        o["bwd"] = torch.empty(n * 6, dtype=torch.int32, device=dev) if bwd else None
        o["n_inliers"] = torch.zeros(1, dtype=torch.int32, device=dev) if compact else None
        o["compact"] = torch.empty(n * 6, dtype=torch.int32, device=dev) if compact else None
        o["n_evals"] = torch.zeros(1, dtype=torch.int64, device=dev) if count_evals else None
        return o

    def match_into(self, p, img1, img2, o, stream=None):
        torch = self.torch
        assert img1.is_cuda and img1.dtype == torch.uint8 and img1.dim() == 3 and img1.shape[2] == 3
        assert img2.shape == img1.shape and img2.dtype == torch.uint8
        assert img1.stride(2) == 1 and img1.stride(1) == 3 and img2.stride(1) == 3 and img2.stride(2) == 1
        assert img1.stride(0) == img2.stride(0)
        h, w = img1.shape[:2]
        ptr = lambda t: None if t is None else t.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        pgm_match(self.ctx, p, img1.data_ptr(), img2.data_ptr(), w, h, img1.stride(0), o["fwd"].data_ptr(),
                  ptr(o["bwd"]), ptr(o["n_inliers"]), ptr(o["compact"]), ptr(o["n_evals"]), stream)
        self.last_sizes = o["sizes"]
        return o

    def match(self, p, img1, img2, bwd=True, compact=True, count_evals=True):
        h, w = img1.shape[:2]
        o = self.outputs(p, w, h, bwd, compact, count_evals)
        return self.match_into(p, img1, img2, o)

    def outputs_batch(self, p, w, h, n_pairs, bwd=True, compact=True, count_evals=True):
        torch = self.torch
        s = pgm_query(p, w, h)
        n = s.nx * s.ny
        dev = torch.device("cuda", self.device)
        o = dict(sizes=s, n=n, n_pairs=n_pairs)
        o["fwd"] = torch.empty(n_pairs * n * 6, dtype=torch.int32, device=dev)
        o["bwd"] = torch.empty(n_pairs * n * 6, dtype=torch.int32, device=dev) if bwd else None
        o["n_inliers"] = torch.zeros(n_pairs, dtype=torch.int32, device=dev) if compact else None
        o["compact"] = torch.empty(n_pairs * n * 6, dtype=torch.int32, device=dev) if compact else None
        o["n_evals"] = torch.zeros(1, dtype=torch.int64, device=dev) if count_evals else None
        return o

    def match_batch_into(self, p, img1, img2, o, stream=None):
        """img1, img2: (B, h, w, 3) uint8 CUDA tensors with the same strides."""
        torch = self.torch
        assert img1.is_cuda and img1.dtype == torch.uint8 and img1.dim() == 4 and img1.shape[3] == 3
        assert img2.shape == img1.shape and img2.dtype == torch.uint8
        assert img1.stride()[1:] == img2.stride()[1:] and img1.stride(0) == img2.stride(0)
        assert img1.stride(3) == 1 and img1.stride(2) == 3
        B, h, w = img1.shape[:3]
        assert B == o["n_pairs"]
        ptr = lambda t: None if t is None else t.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        pgm_match_batch(self.ctx, p, B, img1.data_ptr(), img2.data_ptr(), w, h, img1.stride(1),
                        img1.stride(0), o["fwd"].data_ptr(), ptr(o["bwd"]), ptr(o["n_inliers"]),
                        ptr(o["compact"]), ptr(o["n_evals"]), stream)
        self.last_sizes = o["sizes"]
        return o

    def tune(self, p, img1, img2, o, repeats=3, stream=None):
        """Pick the fastest launch schedule for this workload (pgm_tune) and keep it for later
        calls; img1, img2 and o as for match_batch_into (o holds the matches afterwards; its
        evaluation counter is not written). Returns the chosen SCHED_* flags."""
        torch = self.torch
        assert img1.is_cuda and img1.dtype == torch.uint8 and img1.dim() == 4 and img1.shape[3] == 3
        assert img2.shape == img1.shape and img2.dtype == torch.uint8
        assert img1.stride()[1:] == img2.stride()[1:] and img1.stride(0) == img2.stride(0)
        assert img1.stride(3) == 1 and img1.stride(2) == 3
        B, h, w = img1.shape[:3]
        assert B == o["n_pairs"]
        ptr = lambda t: None if t is None else t.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        self.last_sizes = o["sizes"]
        return pgm_tune(self.ctx, p, B, img1.data_ptr(), img2.data_ptr(), w, h, img1.stride(1), img1.stride(0),
                        o["fwd"].data_ptr(), ptr(o["bwd"]), ptr(o["n_inliers"]), ptr(o["compact"]), repeats, stream)

    def match_batch(self, p, img1, img2, bwd=True, compact=True, count_evals=True):
        B, h, w = img1.shape[:3]
        o = self.outputs_batch(p, w, h, B, bwd, compact, count_evals)
        return self.match_batch_into(p, img1, img2, o)

    def match_groups_into(self, items, n_evals=None, use_graph=False, stream=None):
        """items: a list of (params, img1, img2, outputs) with (B, h, w, 3) uint8 CUDA image
        tensors and outputs from outputs_batch; all groups run in one pgm_match_groups call."""
        torch = self.torch
        ptr = lambda t: None if t is None else t.data_ptr()
        keep, groups = [], []
        for p, img1, img2, o in items:
            assert img1.is_cuda and img1.dtype == torch.uint8 and img1.dim() == 4 and img1.shape[3] == 3
            assert img2.shape == img1.shape and img1.stride() == img2.stride()
            assert img1.stride(3) == 1 and img1.stride(2) == 3
            B, h, w = img1.shape[:3]
            assert B == o["n_pairs"]
            pp = _as_params(p)
            keep.append(pp)
            groups.append(pgm_group(C.pointer(pp), B, w, h, img1.stride(1), img1.stride(0), img1.data_ptr(),
                                    img2.data_ptr(), o["fwd"].data_ptr(), ptr(o["bwd"]), ptr(o["n_inliers"]),
                                    ptr(o["compact"])))
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        pgm_match_groups(self.ctx, groups, ptr(n_evals), use_graph, stream)
        return items

    @staticmethod
    def to_numpy(t, count=None):
        a = t.cpu().numpy().view(MATCH_DTYPE) if t is not None else None
        return a if count is None else a[:count]

    def dump_level(self, level, dir):
        s = self.last_sizes
        return pgm_dump_level(self.ctx, level, dir, s.level_nx[level] * s.level_ny[level])

    def dump_gradient(self, level, image, C2=6, f32=False):
        s = self.last_sizes
        return pgm_dump_gradient(self.ctx, level, image, (s.level_h[level], s.level_w[level], C2), f32)

    def dump_pyramid(self, level, image):
        s = self.last_sizes
        return pgm_dump_pyramid(self.ctx, level, image, s.level_w[level], s.level_h[level])


class Server:
    """A libpgm request server with torch-allocated outputs. submit() takes (h, w, 3) uint8
    CUDA image tensors and returns the tag; poll() returns the tags of finished requests.
    The server keeps references to each request's tensors until its tag has been reported."""

    def __init__(self, device: int = 0, pool_bytes: int = 1 << 30, n_streams: int = 4, max_queued: int = 0,
                 max_batch: int = 0):
        import torch  # device memory and streams only
        self.torch = torch
        self.device = device
        self.h = pgm_server_create(device, pool_bytes, n_streams, max_queued, max_batch)
        self.live = {}
        self.next_tag = 0

    def close(self):
        if self.h:
            pgm_server_destroy(self.h)
            self.h = None
            self.live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, p, img1, img2, bwd=True, compact=True, count_evals=False, tag=None):
        torch = self.torch
        assert img1.is_cuda and img1.dtype == torch.uint8 and img1.dim() == 3 and img1.shape[2] == 3
        assert img2.shape == img1.shape and img1.stride() == img2.stride() and img1.stride(1) == 3
        h, w = img1.shape[:2]
        s = pgm_query(p, w, h)
        n = s.nx * s.ny
        dev = torch.device("cuda", self.device)
        o = dict(sizes=s, n=n, img1=img1, img2=img2)
        o["fwd"] = torch.empty(n * 6, dtype=torch.int32, device=dev)
        o["bwd"] = torch.empty(n * 6, dtype=torch.int32, device=dev) if bwd else None
        o["n_inliers"] = torch.zeros(1, dtype=torch.int32, device=dev) if compact else None
        o["compact"] = torch.empty(n * 6, dtype=torch.int32, device=dev) if compact else None
        o["n_evals"] = torch.zeros(1, dtype=torch.int64, device=dev) if count_evals else None
        if tag is None:
            tag = self.next_tag
            self.next_tag += 1
        ptr = lambda t: None if t is None else t.data_ptr()
        self.live[tag] = o
        # the request runs after the work torch has queued so far (inputs, zero-filled counters)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        try:
            pgm_server_submit(self.h, p, img1.data_ptr(), img2.data_ptr(), w, h, img1.stride(0),
                              o["fwd"].data_ptr(), ptr(o["bwd"]), ptr(o["n_inliers"]), ptr(o["compact"]),
                              ptr(o["n_evals"]), tag, stream)
        except Exception:
            del self.live[tag]
            raise
        return tag

    def poll(self, max_tags: int = 256):
        """[(tag, outputs)] of the requests finished since the last poll; a request whose
        launches failed raises PGMError with its status (its tag is then dropped)."""
        out = []
        for t, st in pgm_server_poll(self.h, max_tags):
            o = self.live.pop(t)
            if st != PGM_OK:
                raise PGMError(st, f"request {t} failed: " + pgm_server_last_error_text(self.h))
            out.append((t, o))
        return out

    def pending(self):
        return pgm_server_pending(self.h)

    def stats(self):
        return pgm_server_stats(self.h)

    def drain(self):
        pgm_server_drain(self.h)
