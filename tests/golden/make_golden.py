"""Writes the frozen oracle runs under tests/golden/ (tiny_*.txt).

Only the CPU oracle (oracle/) computes the stored results; the input images come from the
seeded generators in synth/ and are stored in the file too, so a fixture stays valid if the
generators change. Run from the repository root:

    python tests/golden/make_golden.py

A change to a stored result is a change to the oracle's arithmetic: its commit names the
passage of the paper, or the reading of it, that justifies it.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def _params(**kw):
    p = dict(levels=2, seed_stride=3, patch_fwd=8, patch_bwd=8, iters=[4, 4], radius=2, max_disp=12,
             sobel_ksize=5, feature=0, color=0, fwd_bwd=1, consistency_px=1, init_mode=0, refine_rounds=0,
             min_region_px=0, region_link_px=12, space_fwd=[0, 0], space_bwd=[0, 0], metric=0, rng_seed=7)
    p.update(kw)
    return p


# name -> (description with the passages it exercises, parameters, generator seed, h, w)
CASES = {
    "tiny_grid_40x32": (
        "stride-3 grid, 8x8 patches, absolute differences (Sec. III-B Eq. 3-5), two levels with the "
        "forward-backward check and outlier record (Sec. III-D Eq. 6-8), grid output (Sec. III-G)",
        _params(), 11, 32, 40),
    "tiny_paper_32x24": (
        "the paper's settings (Sec. IV: W=2, S=5, L=3, N=2, 6/4 iterations; Sec. III-E: r=7/5 patches, "
        "Table II colour spaces, 9 px regions) on a dense field",
        _params(levels=3, seed_stride=1, patch_fwd=15, patch_bwd=11, iters=[6, 4, 4], max_disp=0,
                refine_rounds=2, min_region_px=9, space_fwd=[0, 2, 1], space_bwd=[2, 1, 0], rng_seed=3),
        12, 24, 32),
    "tiny_ssd_sign_40x32": (
        "squared differences over literal gradient signs (Sec. III-B Eq. 3, Sec. III-F), exhaustive "
        "start window at the coarsest level (Sec. III-D)",
        _params(metric=1, feature=2, init_mode=1, max_disp=6, rng_seed=5), 13, 32, 40),
}


def write(name):
    desc, p, seed, h, w = CASES[name]
    pair = synth.rect_pair(seed, h=h, w=w, n_rect=3, dmax=p["max_disp"] or 6)
    r = oracle.match(p, pair.img1, pair.img2, trace=False)
    lines = [f"# {desc}",
             "# written by tests/golden/make_golden.py from the CPU oracle; do not edit by hand",
             "params " + json.dumps(p, sort_keys=True),
             f"size {w} {h}"]
    for tag, img in (("img1", pair.img1), ("img2", pair.img2)):
        lines.append(tag)
        lines += [bytes(img[y].reshape(-1)).hex() for y in range(h)]
    lines.append(f"n_inliers {r['n_inliers']}")
    lines.append(f"n_evals {r['n_evals']}")
    for d in ("fwd", "bwd"):
        m = r[d]
        lines.append(f"{d} {len(m)}")
        lines += [" ".join(str(int(m[k][i])) for k in m.dtype.names) for i in range(len(m))]
    with open(os.path.join(HERE, name + ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def read(path):
    """Parse a fixture: (params, img1, img2, fwd, bwd, n_inliers, n_evals); matches as (n, 6) int64."""
    with open(path) as f:
        rows = [ln.rstrip("\n") for ln in f if not ln.startswith("#")]
    it = iter(rows)
    p = json.loads(next(it).split(" ", 1)[1])
    w, h = map(int, next(it).split()[1:])
    imgs = []
    for tag in ("img1", "img2"):
        assert next(it) == tag
        imgs.append(np.stack([np.frombuffer(bytes.fromhex(next(it)), np.uint8) for _ in range(h)]).reshape(h, w, 3))
    nin = int(next(it).split()[1])
    nev = int(next(it).split()[1])
    out = {}
    for d in ("fwd", "bwd"):
        tag, n = next(it).split()
        assert tag == d
        out[d] = np.array([[int(v) for v in next(it).split()] for _ in range(int(n))], np.int64).reshape(-1, 6)
    return p, imgs[0], imgs[1], out["fwd"], out["bwd"], nin, nev


if __name__ == "__main__":
    for name in CASES:
        write(name)
        print("wrote", name)
