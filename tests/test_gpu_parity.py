"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Bars (stated per test): triangle-hit sets and predicted-image counts identical
(integer work, bit-exact); FP64 deflections within 1e-10 arcsec; mixed-path
image positions within 1e-5 arcsec and chi^2 within 1e-6 relative; FP32
deflections within the library's stated FP32 error bound."""
import math
import os

import numpy as np
import pytest

import oracle
import synthlens as S
from conftest import load_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1902_03252_amd as lens
    lens.context()
    return lens


def dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float64, device="cuda")


def fp32_alpha_bound(prm, grid):
    """The library's stated FP32 deflection bound (per component):
    u (64 + P) sum_p w_p + sum_p j_p + 1e-9, with w_p = K (1+eps)/sqrt(1-eps) and
    j_p = J_p derr + 2u K (1+eps)/(1-eps)^1.5 (+ 2 w_p for a nearly singular
    profile within 1e-10" of a node without being on it), J_p the Jacobian bound
    at half a node or at the nearest node's distance, whichever is larger."""
    eps, a, s, sig = prm[2], prm[4], prm[5], prm[6]
    b0 = 4 * math.pi * (sig / 299792.458) ** 2 * 206264.80624709636
    K = np.where(np.isinf(s), b0, b0 * s / np.where(np.isinf(s), 1.0, s - a))
    w = K * (1 + eps) / np.sqrt(1 - eps)
    cx = np.rint((prm[0] - grid.x0) / grid.h)
    cy = np.rint((prm[1] - grid.y0) / grid.h)
    fx = -((grid.x0 + cx * grid.h) - prm[0]) / grid.h
    fy = -((grid.y0 + cy * grid.h) - prm[1]) / grid.h
    rn = np.hypot(fx, fy)
    rho = np.sqrt(1 - eps) * grid.h * np.maximum(rn, 0.5)
    J = 2 * K * (1 + eps) / ((1 - eps) * (np.sqrt(a * a + rho * rho) + a))
    span = abs(grid.x0) + abs(grid.y0) + (grid.nx + grid.ny) * grid.h + abs(prm[0]) + abs(prm[1])
    near = (rn > 0) & (grid.h * rn < 1e-10) & (a < 1e-10)
    j = J * (grid.h * 2.0 ** -25 + 1e-15 * span) + 2 * U32 * K * (1 + eps) / (1 - eps) ** 1.5 + np.where(near, 2 * w, 0.0)
    return U32 * (64 + prm.shape[1]) * w.sum() + j.sum() + 1e-9


def obs_of(d):
    import paper_1902_03252_amd as lens
    return lens.Obs.from_numpy(d)


# ----------------------------------------------------------------- deflection

@pytest.mark.parametrize("config,n", [(1, None), (2, 256), (2, None), (1, 77)])
def test_deflect_fp64_and_fp32(lens, config, n):
    prm, grid, _ = load_inputs(config)
    if n is not None:  # ragged smaller grid over the same field of view
        grid = S.Grid(grid.x0, grid.y0, grid.h * (grid.nx - 1) / (n - 1), n, n - 3)
    print(f"deflect config={config} grid={grid.nx}x{grid.ny} P={prm.shape[1]}", flush=True)
    ax_o, ay_o = oracle.alpha_grid(prm, grid)
    p = dev(prm)
    ax, ay = lens.lens_deflect(p, grid, "fp64")
    np.testing.assert_allclose(ax.cpu().numpy(), ax_o, rtol=0, atol=1e-10)
    np.testing.assert_allclose(ay.cpu().numpy(), ay_o, rtol=0, atol=1e-10)
    ax, ay = lens.lens_deflect(p, grid, "fp32")
    err = np.maximum(np.abs(ax.cpu().numpy() - ax_o), np.abs(ay.cpu().numpy() - ay_o))
    bound = fp32_alpha_bound(prm, grid)
    print(f"  fp32 |err| max {err.max():.3e} p99 {np.percentile(err, 99):.3e} bound {bound:.3e}", flush=True)
    assert err.max() <= bound


def test_deflect_singular_and_uncut_kinds(lens):
    """All four radial-profile kinds (cored/singular x cut/uncut), incl. the SIE of Algorithm 1."""
    prm = S.sie_potentials(6, seed=3)
    prm[4, :3] = [0.2, 0.0, 0.4]
    prm[5, 3:] = [30.0, 50.0, np.inf]
    prm[4, 5] = 0.1
    grid = S.Grid(-60.3, -59.1, 0.37, 301, 290)
    ax_o, ay_o = oracle.alpha_grid(prm, grid)
    ax, ay = lens.lens_deflect(dev(prm), grid, "fp64")
    np.testing.assert_allclose(ax.cpu().numpy(), ax_o, rtol=0, atol=1e-10)
    np.testing.assert_allclose(ay.cpu().numpy(), ay_o, rtol=0, atol=1e-10)
    ax, ay = lens.lens_deflect(dev(prm), grid, "fp32")
    err = np.maximum(np.abs(ax.cpu().numpy() - ax_o), np.abs(ay.cpu().numpy() - ay_o))
    assert err.max() <= fp32_alpha_bound(prm, grid)


def test_deflect_zero_and_small_dispersion(lens):
    """Potentials with sigma_v = 0, 1e-9 and 1e-4 km/s (cut and uncut, cored and
    singular) beside ordinary ones: the FP32 table stores the first two with
    K = 0 and divides by K for the others; both precisions against the oracle,
    and the chi^2 with them against the oracle's."""
    prm = S.sie_potentials(10, seed=5)
    prm[4, :4] = [0.3, 0.0, 0.2, 0.0]
    prm[5, :4] = [40.0, 25.0, np.inf, np.inf]
    prm[6, :6] = [0.0, 0.0, 1e-9, 1e-9, 1e-4, 1e-4]
    prm[5, 4] = np.inf
    grid = S.Grid(-50.3, -49.1, 0.35, 289, 283)
    ax_o, ay_o = oracle.alpha_grid(prm, grid)
    ax, ay = lens.lens_deflect(dev(prm), grid, "fp64")
    np.testing.assert_allclose(ax.cpu().numpy(), ax_o, rtol=0, atol=1e-10)
    np.testing.assert_allclose(ay.cpu().numpy(), ay_o, rtol=0, atol=1e-10)
    ax, ay = lens.lens_deflect(dev(prm), grid, "fp32")
    err = np.maximum(np.abs(ax.cpu().numpy() - ax_o), np.abs(ay.cpu().numpy() - ay_o))
    assert np.isfinite(err).all() and err.max() <= fp32_alpha_bound(prm, grid)
    _, _, obs = load_inputs(2)
    want = oracle.image_chi2(prm, grid, obs)
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec)
        compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)


def test_deflect_invalid_parameters_reported(lens):
    prm = S.config1_potentials()
    for k, v in [(2, 1.0), (2, -0.1), (4, -1.0), (5, 0.1), (6, -5.0), (0, np.nan)]:
        bad = prm.copy()
        bad[k, 0] = v
        with pytest.raises(RuntimeError, match="invalid"):
            lens.lens_deflect(dev(bad), S.square_grid(16, 10.0), "fp32")
        ax, _ = lens.lens_deflect(dev(bad), S.square_grid(16, 10.0), "fp64", check=False)
        assert torch.isnan(ax).all()


def test_no_potentials(lens):
    ax, ay = lens.lens_deflect(dev(np.zeros((7, 0))), S.square_grid(33, 5.0), "fp32")
    assert float(ax.abs().max()) == 0.0 and float(ay.abs().max()) == 0.0


# ----------------------------------------------------------------- cosmology and sources

def test_dls_dos(lens):
    zs = np.array([0.2, 0.3, 1.0, 2.0, 3.0, 6.0])
    got = lens.lens_dls_dos(0.3, dev(zs)).cpu().numpy()
    want = np.array([oracle.dls_dos(0.3, z) for z in zs])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("config", [1, 2, 3])
def test_source_positions(lens, config):
    prm, grid, obs = load_inputs(config)
    beta, bar = lens.lens_source_positions(dev(prm), obs_of(obs))
    bx, by, cx, cy = oracle.source_positions(prm, obs["sys_off"], obs["x"], obs["y"], obs["dls"])
    np.testing.assert_allclose(beta.cpu().numpy(), np.stack([bx, by], 1), rtol=0, atol=1e-10)
    np.testing.assert_allclose(bar.cpu().numpy(), np.stack([cx, cy], 1), rtol=0, atol=1e-10)


# ----------------------------------------------------------------- chi^2

def compare_chi2(got, want, pos_tol, chi2_rtol):
    assert got["status"] == 0
    np.testing.assert_array_equal(got["n_pred"], want["n_pred"])
    np.testing.assert_array_equal(got["hit_sys"], want["hit_sys"])
    np.testing.assert_array_equal(got["hit_tid"], want["hit_tid"])
    np.testing.assert_allclose(got["hit_x"], want["hit_x"], rtol=0, atol=pos_tol)
    np.testing.assert_allclose(got["hit_y"], want["hit_y"], rtol=0, atol=pos_tol)
    np.testing.assert_array_equal(got["match"][:len(want["match"])], want["match"])
    fin = np.isfinite(want["chi2_sys"])
    np.testing.assert_array_equal(np.isfinite(got["chi2_sys"]), fin)
    np.testing.assert_allclose(got["chi2_sys"][fin], want["chi2_sys"][fin], rtol=chi2_rtol, atol=1e-12)
    if math.isfinite(want["chi2"]):
        assert got["chi2"] == pytest.approx(want["chi2"], rel=chi2_rtol)
    else:
        assert got["chi2"] == want["chi2"]


def run_chi2(lens, prm, grid, obs, prec, **kw):
    res = lens.lens_image_chi2(dev(prm), grid, obs_of(obs), prec=prec, **kw)
    torch.cuda.synchronize()
    return res.host()


@pytest.mark.parametrize("config,n", [(1, None), (1, 200), (2, None), (2, 333)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chi2_parity(lens, config, n, prec):
    prm, grid, obs = load_inputs(config)
    if n is not None:
        grid = S.Grid(grid.x0, grid.y0, grid.h * (grid.nx - 1) / (n - 1), n, n + 5)
    print(f"chi2 {prec} config={config} grid={grid.nx}x{grid.ny}", flush=True)
    want = oracle.image_chi2(prm, grid, obs)
    got = run_chi2(lens, prm, grid, obs, prec)
    st = got["stats"]
    print(f"  hits {st[0]} flagged {st[1]} tile-pass {st[2]} bbox-pass {st[3]} fb-hits {st[5]}", flush=True)
    compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)


_RAGGED = {}


@pytest.mark.parametrize("tile,npl", [(1, 1), (2, 2), (3, 4), (4, 8), (2, 8), (3, 1)])
def test_chi2_tile_shapes_and_nodes_per_thread(lens, tile, npl):
    """Every triangle-tile shape (32x8, 64x16, 64x8, 32x16) and field width (1..8 nodes per
    thread) on a ragged grid: 333 x 338 nodes, so neither axis is a multiple of a tile."""
    prm, grid, obs = load_inputs(2)
    grid = S.Grid(grid.x0, grid.y0, grid.h * (grid.nx - 1) / 332, 333, 338)
    if "r" not in _RAGGED:
        _RAGGED["r"] = oracle.image_chi2(prm, grid, obs)
    want = _RAGGED["r"]
    for prec in ("mixed", "fp64"):
        got = run_chi2(lens, prm, grid, obs, prec, tile=tile, field_npl=npl)
        compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)


def _many_images_obs(n_sys, n_img, seed):
    """n_img observed images in n_sys systems (at least one each), positions
    uniform over the cluster field, distance ratios in [0.4, 1]."""
    g = np.random.default_rng(seed)
    sizes = 1 + g.multinomial(n_img - n_sys, np.full(n_sys, 1.0 / n_sys))
    sys_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return dict(sys_off=sys_off, x=g.uniform(-60, 60, n_img), y=g.uniform(-60, 60, n_img),
                sigma=np.full(n_img, 0.3), dls=g.uniform(0.4, 1.0, n_sys))


@pytest.mark.parametrize("n_sys,n_img", [(120, 512), (512, 512), (150, 700)])
def test_many_images_both_head_forms(lens, n_sys, n_img):
    """Source positions and chi^2 with many observed images: up to 512 images
    (and fewer than 512 systems) the head spreads the images over its threads,
    beyond it walks each system's images; both against the oracle."""
    prm, grid, _ = load_inputs(2)
    grid = S.Grid(grid.x0, grid.y0, grid.h * (grid.nx - 1) / 200, 201, 201)
    obs = _many_images_obs(n_sys, n_img, seed=n_sys + n_img)
    beta, bar = lens.lens_source_positions(dev(prm), obs_of(obs))
    bx, by, cx, cy = oracle.source_positions(prm, obs["sys_off"], obs["x"], obs["y"], obs["dls"])
    np.testing.assert_allclose(beta.cpu().numpy(), np.stack([bx, by], 1), rtol=0, atol=1e-10)
    np.testing.assert_allclose(bar.cpu().numpy(), np.stack([cx, cy], 1), rtol=0, atol=1e-10)
    want = oracle.image_chi2(prm, grid, obs)
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec, hit_capacity=8192)
        print(f"  {n_sys} systems, {n_img} images, {prec}: hits {got['stats'][0]}", flush=True)
        compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)


def test_chi2_identity_lens_exact_images(lens):
    """No potentials: each system has one predicted image at its barycentre."""
    g = np.random.default_rng(11)
    grid = S.Grid(-5.0, -4.0, 0.1, 101, 91)
    xs = g.uniform(-4, 4, (9, 2))
    obs = dict(sys_off=np.array([0, 2, 3, 6, 9], np.int32), x=xs[:, 0], y=xs[:, 1], sigma=np.full(9, 0.2),
               dls=np.array([0.5, 0.7, 0.9, 1.0]))
    prm = np.zeros((7, 0))
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec)
        want = oracle.image_chi2(prm, grid, obs)
        compare_chi2(got, want, 1e-9, 1e-9)
        assert list(got["n_pred"]) == [1, 1, 1, 1]


def test_chi2_system_without_images_is_infinite(lens):
    prm, grid, obs = load_inputs(1)
    obs = dict(obs)
    obs["x"] = obs["x"].copy()
    obs["y"] = obs["y"].copy()
    j0, j1 = obs["sys_off"][1], obs["sys_off"][2]
    obs["x"][j0:j1] = 500.0  # far outside the grid: its source lies outside every triangle
    obs["y"][j0:j1] = 500.0
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec)
        want = oracle.image_chi2(prm, grid, obs)
        assert got["n_pred"][1] == 0 and math.isinf(got["chi2_sys"][1]) and math.isinf(got["chi2"])
        compare_chi2(got, want, 1e-9, 1e-6)


def test_chi2_capacity_and_invalid_status(lens):
    prm, grid, obs = load_inputs(2)
    got = run_chi2(lens, prm, grid, obs, "mixed", hit_capacity=3)
    assert got["status"] == 3 and got["stats"][0] > 3 and math.isnan(got["chi2"])
    bad = prm.copy()
    bad[2, 4] = 1.5
    got = run_chi2(lens, bad, grid, obs, "fp64")
    assert got["status"] == 1 and math.isnan(got["chi2"])
    # the next call on the same context is unaffected
    got = run_chi2(lens, prm, grid, obs, "fp64")
    assert got["status"] == 0


def sys_vertex_bound(prm, grid, bar_x, bar_y, dls):
    """The library's stated FP32 bound E_B on each component of a source-plane
    vertex offset B - barycentre, per system:
    r E_alpha + 4u Theta + 2u r (W + E_alpha) + 2^-25 h + 1e-9 (times 1 + 1e-6)."""
    e_alpha = fp32_alpha_bound(prm, grid)
    eps, a, s, sig = prm[2], prm[4], prm[5], prm[6]
    b0 = 4 * math.pi * (sig / 299792.458) ** 2 * 206264.80624709636
    K = np.where(np.isinf(s), b0, b0 * s / np.where(np.isinf(s), 1.0, s - a))
    W = float((K * (1 + eps) / np.sqrt(1 - eps)).sum())
    xlo, xhi = grid.x0, grid.x0 + (grid.nx - 1) * grid.h
    ylo, yhi = grid.y0, grid.y0 + (grid.ny - 1) * grid.h
    theta = np.maximum(np.maximum(abs(xlo - bar_x), abs(xhi - bar_x)), np.maximum(abs(ylo - bar_y), abs(yhi - bar_y)))
    eb = dls * e_alpha + 4 * U32 * theta + 2 * U32 * dls * (W + e_alpha) + grid.h * 2.0 ** -25 + 1e-9
    return eb * (1 + 1e-6)


def triangle_margin(prm, grid, sys, tid, bar_x, bar_y, dls, eb):
    """min_k (|c_k| - T_k) of one (system, triangle) test: c_k = d_k x d_k+1 from the
    oracle's FP64 vertices (d = B - barycentre), T_k the bound on how far FP32
    vertices within eb of these (and FP32 products) can move c_k.  A test can be
    decided differently from the exact one by FP32 arithmetic only if this is <= 0."""
    nx = grid.nx
    cell, k = divmod(int(tid), 2)
    j, i = divmod(cell, nx - 1)
    nodes = [(i, j), (i + 1, j), (i, j + 1)] if k == 0 else [(i + 1, j + 1), (i, j + 1), (i + 1, j)]
    th = np.array([(grid.x0 + a * grid.h, grid.y0 + b * grid.h) for a, b in nodes])
    al = oracle.alpha_points(prm, th)
    r = dls[sys]
    d = th - r * al - np.array([bar_x[sys], bar_y[sys]])
    E = eb[sys]
    m = np.inf
    for q in range(3):
        u, v = d[q], d[(q + 1) % 3]
        c = u[0] * v[1] - u[1] * v[0]
        T = E * (abs(u).sum() + abs(v).sum()) + 2 * E * E + 2 * U32 * (abs(u[0] * v[1]) + abs(u[1] * v[0]))
        m = min(m, abs(c) - 1.01 * T)
    return m


def _literal_check(lens, prm, grid, obs, want):
    """Literal fallback rule |c| < tau h^2 (tau = 1e-6): the FP32 sign is taken
    whenever |c| >= tau h^2, which does not guarantee the exact decision.  Every
    hit-set difference from the oracle must be a test that FP32 arithmetic within
    the stated vertex bound can legitimately get wrong (triangle_margin <= 0)."""
    got = run_chi2(lens, prm, grid, obs, "mixed", fb_mode=1, fb_tau=1e-6, hit_capacity=8192)
    assert got["status"] == 0
    a = set(zip(got["hit_sys"].tolist(), got["hit_tid"].tolist()))
    b = set(zip(want["hit_sys"].tolist(), want["hit_tid"].tolist()))
    diff = sorted(a ^ b)
    st = got["stats"]
    print(f"literal mode {grid.nx}x{grid.ny}: flagged {st[1]} of {st[6]} tests ({st[1] / max(st[6], 1):.2e}), "
          f"fallback hits {st[5]}, hits {st[0]} (oracle {len(b)}), hit-set mismatches {len(diff)}", flush=True)
    if diff:
        eb = sys_vertex_bound(prm, grid, want["bar_x"], want["bar_y"], obs["dls"])
        for sys, tid in diff:
            m = triangle_margin(prm, grid, sys, tid, want["bar_x"], want["bar_y"], obs["dls"], eb)
            print(f"  mismatch system {sys} triangle {tid}: margin {m:.3e}", flush=True)
            assert m <= 0.0, (sys, tid, m)
    return got, diff


def test_chi2_literal_threshold_mode(lens):
    prm, grid, obs = load_inputs(2)
    _literal_check(lens, prm, grid, obs, oracle.image_chi2(prm, grid, obs))


@pytest.mark.slow
def test_chi2_literal_threshold_mode_large(lens):
    """The literal rule on the 4096^2 / 200-potential / 100-system workload, against
    the complete oracle run."""
    prm, grid, obs = load_inputs(3)
    _literal_check(lens, prm, grid, obs, _oracle_large())


# ----------------------------------------------------------------- exact ties and edge cases

def _tie_obs():
    """Single-image systems on a grid whose nodes are exact binary fractions
    (x0 = -8, h = 1/8): the barycentre (= the observed image, identity lens) lies
    exactly on a node, on a horizontal / vertical edge, on a cell's anti-diagonal
    (its midpoint and a quarter point), or 1e-12 arcsec off an edge or the
    anti-diagonal, on either side."""
    h, x0 = 0.125, -8.0
    pts = []
    for (i, j) in [(40, 70), (64, 64), (100, 3)]:
        X, Y = x0 + i * h, x0 + j * h
        pts += [(X, Y),                                  # node
                (X + 0.5 * h, Y), (X, Y + 0.5 * h),      # horizontal / vertical edge
                (X + 0.5 * h, Y + 0.5 * h),              # anti-diagonal midpoint
                (X + 0.25 * h, Y + 0.75 * h),            # anti-diagonal, quarter point
                (X + 0.5 * h, Y + 1e-12), (X + 0.5 * h, Y - 1e-12),
                (X + 1e-12, Y + 0.5 * h), (X - 1e-12, Y + 0.5 * h),
                (X + 0.5 * h + 1e-12, Y + 0.5 * h), (X + 0.5 * h - 1e-12, Y + 0.5 * h)]
    pts = np.array(pts)
    n = len(pts)
    return S.Grid(x0, x0, h, 129, 129), dict(sys_off=np.arange(n + 1, dtype=np.int32), x=pts[:, 0],
                                             y=pts[:, 1], sigma=np.full(n, 0.1), dls=np.full(n, 0.8))


def test_chi2_exact_ties_identity_lens(lens):
    """Barycentres exactly on nodes, edges and anti-diagonals are in no triangle
    (strict inequalities decided exactly), and 1e-12 arcsec off an edge they are
    in exactly one; both precisions equal the oracle, and in the mixed path those
    tests are the ones sent to the FP64 fallback."""
    grid, obs = _tie_obs()
    prm = np.zeros((7, 0))
    want = oracle.image_chi2(prm, grid, obs)
    n_off = len(obs["x"]) // 11 * 6
    assert int((want["n_pred"] == 1).sum()) == n_off and int((want["n_pred"] == 0).sum()) == len(obs["x"]) - n_off
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec)
        st = got["stats"]
        print(f"ties {prec}: hits {st[0]} flagged {st[1]} fallback hits {st[5]}", flush=True)
        compare_chi2(got, want, 1e-9, 1e-9)
        if prec == "mixed":
            assert st[1] > 0 and st[5] == n_off  # every hit was decided in FP64


@pytest.mark.parametrize("n_sys", [1023, 1024, 1025])
def test_chi2_systems_at_the_tail_staging_limit(lens, n_sys):
    """1024 systems is the largest count the tail stages in LDS: the last system's
    offsets, n_pred and chi^2 against the oracle at, below and above it."""
    g = np.random.default_rng(n_sys)
    grid = S.Grid(-40.0, -40.0, 0.5, 161, 161)
    n_img = 1024 if n_sys <= 1024 else 1030
    sizes = np.ones(n_sys, np.int64)
    sizes[g.choice(n_sys, n_img - n_sys, replace=False)] += 1
    sys_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    obs = dict(sys_off=sys_off, x=g.uniform(-35, 35, n_img), y=g.uniform(-35, 35, n_img),
               sigma=np.full(n_img, 0.3), dls=g.uniform(0.5, 1.0, n_sys))
    for prm in (np.zeros((7, 0)), S.sie_potentials(2, seed=n_sys, half_width=30.0)):
        want = oracle.image_chi2(prm, grid, obs)
        for prec in ("fp64", "mixed"):
            got = run_chi2(lens, prm, grid, obs, prec, hit_capacity=8192)
            print(f"  {n_sys} systems P={prm.shape[1]} {prec}: hits {got['stats'][0]}", flush=True)
            compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)


def _singular_case(where):
    """A singular isothermal lens (the SIE of Algorithm 1: r_core = 0, r_cut = inf)
    on a 257^2 grid over +-40" whose nodes are exact binary fractions, with its
    centre on the node at the origin, a hair off it, or at an ordinary position;
    a second, singular and cut galaxy-scale potential on another node."""
    off = {"on": (0.0, 0.0), "1e-9 node": (1e-9 * 0.3125, -0.7e-9 * 0.3125), "ordinary": (0.1, -0.07)}[where]
    prm = np.array([[off[0], 2.5], [off[1], -1.25], [0.2, 0.1], [0.5, 1.0], [0.0, 0.0], [np.inf, 20.0],
                    [800.0, 150.0]])
    grid = S.Grid(-40.0, -40.0, 0.3125, 257, 257)
    g = np.random.default_rng(7)
    xs = g.uniform(-20, 20, (7, 2))
    obs = dict(sys_off=np.array([0, 2, 3, 5, 7], np.int32), x=xs[:, 0], y=xs[:, 1], sigma=np.full(7, 0.1),
               dls=np.array([0.6, 0.7, 0.8, 0.9]))
    return prm, grid, obs


@pytest.mark.parametrize("where", ["on", "1e-9 node", "ordinary"])
def test_chi2_singular_centre_on_a_node(lens, where):
    """The FP32 bound stays finite for a singular centre on (or next to) a lattice
    node; both paths against the oracle, the mixed path without a capacity status."""
    prm, grid, obs = _singular_case(where)
    want = oracle.image_chi2(prm, grid, obs)
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec)
        st = got["stats"]
        print(f"singular centre {where} {prec}: status {got['status']} hits {st[0]} flagged {st[1]}", flush=True)
        compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)
        if prec == "mixed":
            assert st[1] < 1000  # the bound admits few undecided tests


def test_deflect_singular_centre_on_a_node_within_bound(lens):
    """FP32 deflections of the same lenses within the stated bound, at every node
    including the one at (or next to) the centre."""
    for where in ("on", "1e-9 node", "ordinary"):
        prm, grid, _ = _singular_case(where)
        ax_o, ay_o = oracle.alpha_grid(prm, grid)
        ax, ay = lens.lens_deflect(dev(prm), grid, "fp64")
        np.testing.assert_allclose(ax.cpu().numpy(), ax_o, rtol=0, atol=1e-10)
        np.testing.assert_allclose(ay.cpu().numpy(), ay_o, rtol=0, atol=1e-10)
        ax, ay = lens.lens_deflect(dev(prm), grid, "fp32")
        err = np.maximum(np.abs(ax.cpu().numpy() - ax_o), np.abs(ay.cpu().numpy() - ay_o))
        bound = fp32_alpha_bound(prm, grid)
        print(f"  {where}: fp32 |err| max {err.max():.3e} bound {bound:.3e}", flush=True)
        assert err.max() <= bound


def test_chi2_deterministic(lens):
    prm, grid, obs = load_inputs(2)
    a = run_chi2(lens, prm, grid, obs, "mixed")
    b = run_chi2(lens, prm, grid, obs, "mixed")
    for k in ("hit_sys", "hit_tid", "hit_x", "hit_y", "n_pred", "chi2_sys"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["chi2"] == b["chi2"]


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_chi2_parity_large(lens, prec):
    """4096^2 grid, 200 potentials, 100 systems: full hit-set parity at the benchmark size."""
    prm, grid, obs = load_inputs(3)
    want = _oracle_large()
    got = run_chi2(lens, prm, grid, obs, prec)
    st = got["stats"]
    print(f"large {prec}: hits {st[0]} flagged {st[1]} ({st[1] / st[6]:.2e} of tests) fb-hits {st[5]}", flush=True)
    compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)


_LARGE = {}


def _oracle_large():
    if "r" not in _LARGE:
        prm, grid, obs = load_inputs(3)
        _LARGE["r"] = oracle.image_chi2(prm, grid, obs, nthreads=min(16, os.cpu_count() or 1))
    return _LARGE["r"]


def test_graph_replay_matches_eager(lens):
    """One chi^2 evaluation captured into a HIP graph: every replay, with eager work and
    synchronisations in between, reproduces the eager result exactly."""
    prm, grid, obs = load_inputs(2)
    p = dev(prm)
    o = obs_of(obs)
    for prec in ("mixed", "fp64"):
        out = lens.chi2_buffers(o, 4096, "cuda")
        lens.lens_image_chi2(p, grid, o, prec=prec, out=out)
        torch.cuda.synchronize()
        eager = out.host()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            lens.lens_image_chi2(p, grid, o, prec=prec, out=out)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lens.lens_image_chi2(p, grid, o, prec=prec, out=out)
        for rep in range(4):
            out.chi2.fill_(-1.0)
            out.hits.fill_(-1)
            lens.lens_deflect(p, grid, "fp32")  # unrelated eager work on the same context
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = out.host()
            assert got["chi2"] == eager["chi2"], (prec, rep)
            for k in ("hit_sys", "hit_tid", "hit_x", "hit_y", "n_pred", "chi2_sys", "match"):
                np.testing.assert_array_equal(got[k], eager[k])
        del g


@pytest.mark.parametrize("nx,ny", [(4099, 3), (3, 4099), (1537, 10), (10, 1537), (2, 2), (65, 2)])
@pytest.mark.parametrize("tile", [1, 2])
def test_chi2_thin_grids(lens, nx, ny, tile):
    """Grids of one or a few cell rows (or columns), narrower than a tile in one
    direction, through the cluster workload's lens plane along an observed
    image of each kind of placement: the tile ranges, halo columns, culling and
    pair tests at the grid's edges, in both precisions, against the oracle."""
    prm, grid0, obs = load_inputs(2)
    h = grid0.h
    j = int(np.argmax(np.abs(obs["x"]) + np.abs(obs["y"]) < 40.0))  # an image near the centre
    cx, cy = float(obs["x"][j]), float(obs["y"][j])
    grid = S.Grid(cx - h * (nx - 1) / 2 - 0.37 * h, cy - h * (ny - 1) / 2 + 0.21 * h, h, nx, ny)
    want = oracle.image_chi2(prm, grid, obs)
    for prec in ("fp64", "mixed"):
        got = run_chi2(lens, prm, grid, obs, prec, tile=tile)
        print(f"  {nx}x{ny} tile {tile} {prec}: hits {got['stats'][0]} (oracle {len(want['hit_tid'])})", flush=True)
        compare_chi2(got, want, 1e-9 if prec == "fp64" else 1e-5, 1e-9 if prec == "fp64" else 1e-6)
