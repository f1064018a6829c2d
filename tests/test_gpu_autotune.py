"""The autotuner of the single and batched chi^2 through the C ABI: a tuned
choice is a valid configuration, it is recorded per bucket, survives a JSON
round trip (and the LENS_AUTOTUNE_CACHE start-up load), and the results of
the tuned call are identical to those of the default configuration (the hit
sets and the fixed-order chi^2 sums do not depend on the tile shape or the
nodes per thread)."""
import json
import os

import numpy as np
import pytest

import synthlens as S
from conftest import load_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIDES = (65, 130, 257, 190)


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1902_03252_amd as lens
    lens.context()
    return lens


def dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float64, device="cuda")


def chi2_np(res):
    torch.cuda.synchronize()
    return {k: getattr(res, k).cpu().numpy() for k in ("chi2", "chi2_sys", "n_pred", "hits", "img_xy", "stats")}


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_autotune_single_records_and_matches_default(lens, prec, tmp_path):
    prm, grid, obs_np = load_inputs(1)
    ctx = lens.Context()
    p, obs = dev(prm), lens.Obs.from_numpy(obs_np)
    assert lens.autotune_lookup(prec, False, max(grid.nx, grid.ny), prm.shape[1], ctx=ctx) == (0, 0)
    tile, npl, out = lens.autotune_chi2(p, grid, obs, prec=prec, ctx=ctx, reps=2)
    print(f"  {prec}: tile {tile}, field_npl {npl}", flush=True)
    assert tile in (1, 2, 3, 4)
    assert npl in ((1, 2, 4, 8, 0x21, 0x22, 0x24, 0x41, 0x42) if prec == "mixed" else (0,))
    assert lens.autotune_lookup(prec, False, max(grid.nx, grid.ny), prm.shape[1], ctx=ctx) == (tile, npl)
    # the same bucket: any side in (64, 128], any P in (0, 1]
    assert lens.autotune_lookup(prec, False, 100, 1, ctx=ctx) == (tile, npl)
    assert lens.autotune_lookup(prec, False, 129, 1, ctx=ctx) == (0, 0)
    assert lens.autotune_lookup(prec, True, 128, 1, ctx=ctx) == (0, 0)
    tuned = chi2_np(out)
    auto = chi2_np(lens.lens_image_chi2(p, grid, obs, prec=prec, ctx=ctx))
    default = chi2_np(lens.lens_image_chi2(p, grid, obs, prec=prec, ctx=lens.Context(), tile=1))
    n = int(tuned["stats"][0])
    assert n > 0
    for r in (auto, default):
        assert int(r["stats"][0]) == n
        np.testing.assert_array_equal(r["hits"][:n], tuned["hits"][:n])
        np.testing.assert_array_equal(r["img_xy"][:n], tuned["img_xy"][:n])
        np.testing.assert_array_equal(r["n_pred"], tuned["n_pred"])
        np.testing.assert_array_equal(r["chi2_sys"], tuned["chi2_sys"])
        np.testing.assert_array_equal(r["chi2"], tuned["chi2"])

    # JSON round trip into a fresh context, and the start-up load
    path = str(tmp_path / "tune.json")
    lens.autotune_save(path, ctx=ctx)
    doc = json.load(open(path))
    assert doc["arch"].startswith("gfx") and len(doc["entries"]) == 1
    fresh = lens.Context()
    assert lens.autotune_lookup(prec, False, grid.nx, prm.shape[1], ctx=fresh) == (0, 0)
    lens.autotune_load(path, ctx=fresh)
    assert lens.autotune_lookup(prec, False, grid.nx, prm.shape[1], ctx=fresh) == (tile, npl)
    old = os.environ.get("LENS_AUTOTUNE_CACHE")
    os.environ["LENS_AUTOTUNE_CACHE"] = path
    try:
        started = lens.Context()
    finally:
        if old is None:
            del os.environ["LENS_AUTOTUNE_CACHE"]
        else:
            os.environ["LENS_AUTOTUNE_CACHE"] = old
    assert lens.autotune_lookup(prec, False, grid.nx, prm.shape[1], ctx=started) == (tile, npl)


def test_autotune_table_files(lens, tmp_path):
    """Malformed or missing files are rejected and leave the table as it was;
    a file of another GPU architecture adds nothing; a later entry of the same
    bucket replaces the earlier one."""
    ctx = lens.Context()
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"arch": "gfx950", "entries": [
        {"prec": 2, "batched": 1, "n_log2": 11, "p_log2": 7, "tile": 3, "field_npl": 4, "ms": 1.5},
        {"prec": 0, "batched": 0, "n_log2": 10, "p_log2": 6, "tile": 2, "field_npl": 0, "ms": 0.2}]}))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    if arch != "gfx950":
        pytest.skip(f"table files of this test are written for gfx950, device is {arch}")
    lens.autotune_load(str(good), ctx=ctx)
    assert lens.autotune_lookup("mixed", True, 2048, 105, ctx=ctx) == (3, 4)
    assert lens.autotune_lookup("fp64", False, 1024, 50, ctx=ctx) == (2, 0)
    bad = [
        "",
        "{",
        '{"arch": "gfx950", "entries": [{"prec": 2, "batched": 0, "n_log2": 7, "p_log2": 0, "tile": 9, '
        '"field_npl": 1, "ms": 1}]}',
        '{"arch": "gfx950", "entries": [{"prec": 2, "batched": 1, "n_log2": 7, "p_log2": 0, "tile": 1, '
        '"field_npl": 8, "ms": 1}]}',
        '{"arch": "gfx950", "entries": [{"prec": 2, "batched": 0, "n_log2": 7.5, "p_log2": 0, "tile": 1, '
        '"field_npl": 1, "ms": 1}]}',
        '{"entries": []}',
        '{"arch": "gfx950", "entries": []} trailing',
        # nesting far beyond a table file's two levels is refused without recursing through it
        '{"arch": "gfx950", "entries": [], "x": ' + "[" * 200000 + "]" * 200000 + "}",
    ]
    for k, text in enumerate(bad):
        f = tmp_path / f"bad{k}.json"
        f.write_text(text)
        with pytest.raises(RuntimeError, match="invalid"):
            lens.autotune_load(str(f), ctx=ctx)
    with pytest.raises(RuntimeError, match="invalid"):
        lens.autotune_load(str(tmp_path / "missing.json"), ctx=ctx)
    assert lens.autotune_lookup("mixed", True, 2048, 105, ctx=ctx) == (3, 4)
    other = tmp_path / "other.json"
    other.write_text(json.dumps({"arch": "gfx942", "entries": [
        {"prec": 2, "batched": 1, "n_log2": 11, "p_log2": 7, "tile": 1, "field_npl": 1, "ms": 1.0}]}))
    lens.autotune_load(str(other), ctx=ctx)
    assert lens.autotune_lookup("mixed", True, 2048, 105, ctx=ctx) == (3, 4)
    newer = tmp_path / "newer.json"
    newer.write_text(json.dumps({"arch": "gfx950:sramecc+:xnack-", "entries": [
        {"prec": 2, "batched": 1, "n_log2": 11, "p_log2": 7, "tile": 2, "field_npl": 1, "ms": 1.0}]}))
    lens.autotune_load(str(newer), ctx=ctx)
    assert lens.autotune_lookup("mixed", True, 2048, 105, ctx=ctx) == (2, 1)


def test_autotune_batched_matches_default(lens):
    _, _, obs_np = load_inputs(2)
    params, pot_off, grids = S.batch_samples(8, seed_stream=41, p_min=1, p_max=60, grid_sizes=SIDES)
    ctx = lens.Context()
    p, obs = dev(params), lens.Obs.from_numpy(obs_np)
    layout = lens.BatchLayout(pot_off, grids)
    tile, npl, out = lens.autotune_chi2_batched(p, layout, obs, prec="mixed", ctx=ctx, reps=2)
    print(f"  batched: tile {tile}, field_npl {npl}", flush=True)
    assert tile in (1, 2, 3, 4) and npl in (1, 2, 4, 0x21, 0x22, 0x41)
    side = max(max(g.nx, g.ny) for g in grids)
    mean_p = -(-params.shape[1] // len(grids))
    assert lens.autotune_lookup("mixed", True, side, mean_p, ctx=ctx) == (tile, npl)
    torch.cuda.synchronize()
    tuned = {k: getattr(out, k).cpu().numpy() for k in ("chi2", "chi2_sys", "n_pred", "status")}
    ref = lens.lens_image_chi2_batched(p, layout, obs, prec="mixed", ctx=lens.Context())
    torch.cuda.synchronize()
    for k in tuned:
        np.testing.assert_array_equal(getattr(ref, k).cpu().numpy(), tuned[k])
    assert (tuned["status"] == 0).all()
