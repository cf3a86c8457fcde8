import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def base_params(**kw):
    """Matching parameters as a plain dict (field names of the C structs)."""
    p = dict(levels=3, seed_stride=3, patch_fwd=8, patch_bwd=8, iters=[4, 4, 4], radius=2,
             max_disp=20, sobel_ksize=5, feature=0, color=0, fwd_bwd=1, consistency_px=1,
             init_mode=0, refine_rounds=0, min_region_px=0, region_link_px=12, metric=0, rs_mode=0, rng_seed=1)
    p.update(kw)
    if len(p["iters"]) < p["levels"]:
        p["iters"] = list(p["iters"]) + [p["iters"][-1]] * (p["levels"] - len(p["iters"]))
    for k in ("space_fwd", "space_bwd"):
        p[k] = (list(p.get(k, [])) + [0] * p["levels"])[: p["levels"]]
    return p


# the matching parameters of the five workloads
CONFIG_PARAMS = {
    1: base_params(levels=3, iters=[4, 4, 4], max_disp=20, rng_seed=1000),
    2: base_params(levels=5, iters=[6] * 5, max_disp=200, rng_seed=2000),
    3: base_params(levels=5, iters=[6] * 5, max_disp=250, feature=1, rng_seed=3000),
}


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle
