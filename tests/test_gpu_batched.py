"""GPU parity of the batched chi^2 (many lens models per call, uneven potential
counts and grids) against the FP64 CPU oracle and the single-evaluation path.

Bars: per-sample predicted-image counts identical to the oracle's (integer
work, bit-exact); chi^2 within 1e-9 relative (FP64 path) or 1e-6 (mixed path)
of the oracle; every sample identical, up to 1e-13 relative, to the
single-evaluation entry point on the same inputs."""
import math
import os

import numpy as np
import pytest

import oracle
import synthlens as S
from conftest import load_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = {"fp64": 1e-9, "mixed": 1e-6}
SIDES = (65, 130, 257, 190)  # ragged against the 32 x 8 triangle tiles and the 256-node field rows


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1902_03252_amd as lens
    lens.context()
    return lens


def dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float64, device="cuda")


def split(params, pot_off):
    return [params[:, pot_off[s]:pot_off[s + 1]] for s in range(len(pot_off) - 1)]


_ORACLE = {}


def oracle_of(key, prm, grid, obs):
    if key not in _ORACLE:
        _ORACLE[key] = oracle.image_chi2(prm, grid, obs)
    return _ORACLE[key]


def batch(n=12, seed_stream=40):
    params, pot_off, grids = S.batch_samples(n, seed_stream=seed_stream, p_min=1, p_max=200, grid_sizes=SIDES)
    return params, pot_off, grids


def run_batched(lens, params, pot_off, grids, obs, prec, ctx=None, hits=False, **kw):
    layout = lens.BatchLayout(pot_off, grids)
    o = lens.Obs.from_numpy(obs)
    out = lens.batch_buffers(layout.n, o, "cuda", hits=hits, hit_capacity=kw.get("hit_capacity", 1024))
    res = lens.lens_image_chi2_batched(dev(params), layout, o, prec=prec, ctx=ctx, out=out, **kw)
    torch.cuda.synchronize()
    got = {k: getattr(res, k).cpu().numpy() for k in ("chi2", "chi2_sys", "n_pred", "status", "stats")}
    if hits:
        got["hits"] = [res.sample_hits(s) for s in range(layout.n)]
    return got


POS_TOL = {"fp64": 1e-9, "mixed": 1e-5}


def check_sample(got, s, want, rtol, prec=None):
    """Per-sample counts and chi^2; with the hit lists, also the sorted hit set
    (bit-exact) and the predicted positions (1e-9" FP64, 1e-5" mixed)."""
    if "hits" in got:
        h = got["hits"][s]
        np.testing.assert_array_equal(h["hit_sys"], want["hit_sys"])
        np.testing.assert_array_equal(h["hit_tid"], want["hit_tid"])
        np.testing.assert_allclose(h["hit_x"], want["hit_x"], rtol=0, atol=POS_TOL[prec])
        np.testing.assert_allclose(h["hit_y"], want["hit_y"], rtol=0, atol=POS_TOL[prec])
    np.testing.assert_array_equal(got["n_pred"][s], want["n_pred"])
    fin = np.isfinite(want["chi2_sys"])
    np.testing.assert_array_equal(np.isfinite(got["chi2_sys"][s]), fin)
    np.testing.assert_allclose(got["chi2_sys"][s][fin], want["chi2_sys"][fin], rtol=rtol, atol=1e-12)
    if math.isfinite(want["chi2"]):
        assert got["chi2"][s] == pytest.approx(want["chi2"], rel=rtol)
    else:
        assert got["chi2"][s] == want["chi2"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_matches_oracle_and_single(lens, prec):
    _, _, obs = load_inputs(2)
    params, pot_off, grids = batch()
    print(f"batched {prec}: P={np.diff(pot_off).tolist()} sides={[g.nx for g in grids]}", flush=True)
    got = run_batched(lens, params, pot_off, grids, obs, prec, hits=True)
    assert (got["status"] == 0).all()
    o = lens.Obs.from_numpy(obs)
    hits = 0
    for s, prm in enumerate(split(params, pot_off)):
        want = oracle_of(("b", s), prm, grids[s], obs)
        hits += len(want["hit_sys"])
        check_sample(got, s, want, RTOL[prec], prec)
        single = lens.lens_image_chi2(dev(prm), grids[s], o, prec=prec)
        torch.cuda.synchronize()
        one = single.host()
        np.testing.assert_array_equal(got["n_pred"][s], one["n_pred"])
        np.testing.assert_allclose(got["chi2_sys"][s], one["chi2_sys"], rtol=1e-13, atol=0)
    st = got["stats"]
    print(f"  hits {st[0]} flagged {st[1]} fb-hits {st[5]} tests {st[6]}", flush=True)
    assert st[0] == hits and st[4] == 0 and st[7] == 0
    assert st[6] == sum(g.n_triangles for g in grids) * (len(obs["sys_off"]) - 1)


def test_batched_invalid_empty_and_capacity(lens):
    """A sample with no potentials (identity lens), a sample with an invalid
    ellipticity, and a per-sample hit capacity that some samples exceed: each
    sample gets its own status, the others are unaffected."""
    _, _, obs = load_inputs(2)
    params, pot_off, grids = batch(6, seed_stream=41)
    blocks = split(params, pot_off)
    bad = blocks[2].copy()
    bad[2, 0] = 1.5
    blocks = [blocks[0], np.zeros((7, 0)), bad] + blocks[3:]
    grids = [grids[0], S.square_grid(64, 80.0), grids[2]] + list(grids[3:])
    counts = [b.shape[1] for b in blocks]
    off = np.zeros(len(blocks) + 1, np.int32)
    off[1:] = np.cumsum(counts)
    cat = np.concatenate(blocks, axis=1)
    for prec in ("fp64", "mixed"):
        got = run_batched(lens, cat, off, grids, obs, prec)
        assert got["status"][2] == 1 and math.isnan(got["chi2"][2]) and (got["n_pred"][2] == 0).all()
        assert got["stats"][7] == 1 and got["stats"][4] == 1
        for s in (0, 1, 3, 4, 5):
            assert got["status"][s] == 0
            check_sample(got, s, oracle_of(("c", s, grids[s].nx), blocks[s], grids[s], obs), RTOL[prec])
        # identity lens: at most one predicted image per system (its barycentre, if on the grid)
        assert (got["n_pred"][1] <= 1).all() and got["n_pred"][1].sum() > 0
        # capacity: 3 hits per sample
        cap = run_batched(lens, cat, off, grids, obs, prec, hit_capacity=3)
        for s in (0, 1, 3, 4, 5):
            n = len(oracle_of(("c", s, grids[s].nx), blocks[s], grids[s], obs)["hit_sys"])
            assert cap["status"][s] == (3 if n > 3 else 0), (s, n)
            if n <= 3:
                check_sample(cap, s, oracle_of(("c", s, grids[s].nx), blocks[s], grids[s], obs), RTOL[prec])
            else:
                assert math.isnan(cap["chi2"][s])


def test_batched_chunking_is_bitwise_neutral(lens):
    """A field-memory budget of one sample per chunk gives bit-identical results
    to the single-chunk plan."""
    _, _, obs = load_inputs(2)
    params, pot_off, grids = batch(9, seed_stream=42)
    for prec in ("mixed", "fp64"):
        whole = run_batched(lens, params, pot_off, grids, obs, prec)
        os.environ["LENS_BATCH_FIELD_BYTES"] = "1"
        try:
            ctx = lens.Context()  # fresh plan cache
            parts = run_batched(lens, params, pot_off, grids, obs, prec, ctx=ctx)
            del ctx
        finally:
            del os.environ["LENS_BATCH_FIELD_BYTES"]
        for k in ("chi2", "chi2_sys", "n_pred", "status", "stats"):
            np.testing.assert_array_equal(parts[k], whole[k])


def test_batched_plan_reuse_with_new_parameters(lens):
    """Same layout (cached plan), different parameter values."""
    _, _, obs = load_inputs(2)
    params, pot_off, grids = batch(5, seed_stream=43)
    run_batched(lens, params, pot_off, grids, obs, "mixed")
    g = np.random.default_rng(7)
    moved = params.copy()
    moved[0] += g.normal(0, 0.5, moved.shape[1])
    moved[6] *= 1.0 + 0.02 * g.normal(0, 1, moved.shape[1])
    got = run_batched(lens, moved, pot_off, grids, obs, "mixed")
    for s, prm in enumerate(split(moved, pot_off)):
        check_sample(got, s, oracle_of(("m", s), prm, grids[s], obs), RTOL["mixed"])


def test_batched_graph_replay_matches_eager(lens):
    _, _, obs = load_inputs(2)
    params, pot_off, grids = batch(8, seed_stream=44)
    p = dev(params)
    o = lens.Obs.from_numpy(obs)
    layout = lens.BatchLayout(pot_off, grids)
    small = dev(params[:, :pot_off[1]])
    for prec in ("mixed", "fp64"):
        out = lens.batch_buffers(layout.n, o, "cuda")
        lens.lens_image_chi2_batched(p, layout, o, prec=prec, out=out)
        torch.cuda.synchronize()
        eager = {k: getattr(out, k).cpu().numpy() for k in ("chi2", "chi2_sys", "n_pred", "status", "stats")}
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            lens.lens_image_chi2_batched(p, layout, o, prec=prec, out=out)
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            lens.lens_image_chi2_batched(p, layout, o, prec=prec, out=out)
        for rep in range(3):
            out.chi2.fill_(-1.0)
            out.n_pred.fill_(-1)
            lens.lens_deflect(small, grids[0], "fp32")  # unrelated eager work on the same context
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            for k in ("chi2", "chi2_sys", "n_pred", "status", "stats"):
                np.testing.assert_array_equal(getattr(out, k).cpu().numpy(), eager[k], err_msg=f"{prec} {rep} {k}")
        del graph


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batched_full_workload_sampled_against_oracle(lens, prec):
    """The benchmark's 1024-sample batch (P 10..200, sides 256..2048, 1.49e9 nodes:
    one chunk in mixed precision, two in FP64) with the hit lists; compared with the
    oracle on sampled members: the largest grids with the most potentials, the last
    samples of the batch (the highest node offsets of the chunk's field planes) and
    a 256^2 sample -- hit sets bit-exact, positions and chi^2 within the bars."""
    _, _, obs = load_inputs(2)
    params, pot_off, grids = S.batch_samples(1024)
    got = run_batched(lens, params, pot_off, grids, obs, prec, hits=True)
    assert (got["status"] == 0).all()
    counts = np.diff(pot_off)
    sides = np.array([g.nx for g in grids])
    by_cost = [int(s) for s in np.argsort(-(sides.astype(np.int64) ** 2 * counts), kind="stable")]
    big = [s for s in by_cost if sides[s] == 2048 and counts[s] >= 190]
    last = [1023, 1022, 1021, 1020, 1019]
    small = [int(np.flatnonzero(sides == 256)[-1])]
    pick = set(big[:6] + last + small)
    for s in by_cost:  # the next costliest members when the groups overlap
        if len(pick) >= 12:
            break
        pick.add(s)
    pick = sorted(pick)
    assert len(pick) >= 12
    blocks = split(params, pot_off)
    for s in pick:
        key = ("full", s)
        if key not in _ORACLE:
            _ORACLE[key] = oracle.image_chi2(blocks[s], grids[s], obs, nthreads=min(16, os.cpu_count() or 1))
        want = _ORACLE[key]
        print(f"  {prec} sample {s}: side {sides[s]} P {counts[s]} hits {len(want['hit_sys'])}", flush=True)
        check_sample(got, s, want, RTOL[prec], prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_thin_grids(lens, prec):
    """One batch of thin grids (a few cell rows or columns, narrower than a tile)
    through the cluster workload's lens plane, next to a square one: every
    sample against the oracle, hit sets included."""
    prm, grid0, obs = load_inputs(2)
    h = grid0.h
    j = int(np.argmax(np.abs(obs["x"]) + np.abs(obs["y"]) < 40.0))
    cx, cy = float(obs["x"][j]), float(obs["y"][j])
    shapes = [(4099, 3), (3, 4099), (1537, 10), (10, 1537), (2, 2), (65, 2), (257, 257)]
    grids = [S.Grid(cx - h * (nx - 1) / 2 - 0.37 * h, cy - h * (ny - 1) / 2 + 0.21 * h, h, nx, ny)
             for nx, ny in shapes]
    params = np.concatenate([prm] * len(grids), axis=1)
    pot_off = np.arange(len(grids) + 1, dtype=np.int32) * prm.shape[1]
    got = run_batched(lens, params, pot_off, grids, obs, prec, hits=True)
    assert (got["status"] == 0).all()
    for s, g in enumerate(grids):
        want = oracle_of(("thin", s), prm, g, obs)
        print(f"  {g.nx}x{g.ny} {prec}: oracle hits {len(want['hit_tid'])}", flush=True)
        check_sample(got, s, want, RTOL[prec], prec)
