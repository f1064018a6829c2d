"""GPU parity of the paper's mixed-precision SIE gradient (Sec. 3.2, 3.3,
Appendix A.3) against the FP64 CPU oracle, through the C ABI.

Bars: the FP64-block pixels are the oracle's blocks exactly (integer
geometry decided in FP64 on both sides); every FP64 pixel (block or
criteria) within 1e-10 arcsec of the oracle; every FP32 pixel within the
paper's single-precision bound of 2.3e-3 arcsec (Appendix A.3).  The criteria
are decided on the FP32 field, so where the GPU's set of criteria pixels and
the oracle's (decided on its FP64 field) differ, the pixel must lie within
twice the largest observed FP32 error of a threshold, and such pixels must be
rare."""
import numpy as np
import pytest

import oracle
import synthlens as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DP_TOL = 1e-10   # arcsec
SP_BOUND = 2.3e-3  # arcsec, the paper's single-precision bound (Appendix A.3)


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1902_03252_amd as lens
    lens.context()
    return lens


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def criterion_margin(ax, ay, h):
    """Per pixel, the smallest distance of the criteria quantities to their
    thresholds (FP64 reference field), +inf where nothing is evaluated."""
    m = np.full(ax.shape, np.inf)
    d1 = ax[:, 1:] - ax[:, :-1]
    d4 = ay[:, 1:] - ay[:, :-1]
    m[:, 1:] = np.minimum(np.abs(np.abs(h - d1) - oracle.T12), np.abs(np.abs(d4) - oracle.T34))
    d2 = ay[1:, :] - ay[:-1, :]
    d3 = ax[1:, :] - ax[:-1, :]
    m[1:, :] = np.minimum(m[1:, :], np.minimum(np.abs(np.abs(h - d2) - oracle.T12), np.abs(np.abs(d3) - oracle.T34)))
    return m


def check_rows(got_ax, got_ay, mask, ref_ax, ref_ay, ref_patch, ref_crit, margin, what):
    """got/ref arrays of the same rows; ref_crit/margin valid where evaluated."""
    np.testing.assert_array_equal(mask == 1, ref_patch.astype(bool), err_msg=f"{what}: FP64 blocks")
    dp = mask >= 1
    err = np.maximum(np.abs(got_ax - ref_ax), np.abs(got_ay - ref_ay))
    dp_err = err[dp].max() if dp.any() else 0.0
    sp_err = err[~dp].max() if (~dp).any() else 0.0
    gpu_crit = mask == 2
    want = ref_crit.astype(bool) & ~ref_patch.astype(bool)
    diff = gpu_crit != want
    print(f"  {what}: FP64 px {int(dp.sum())} (blocks {int((mask == 1).sum())}, criteria {int(gpu_crit.sum())}, "
          f"oracle criteria {int(want.sum())}, differ {int(diff.sum())}); max err FP64 {dp_err:.2e}, "
          f"FP32 {sp_err:.2e}", flush=True)
    assert dp_err <= DP_TOL
    assert sp_err <= SP_BOUND
    assert (margin[diff] <= 2.0 * sp_err + 1e-12).all(), margin[diff].max()
    assert diff.sum() <= 0.01 * max(int(want.sum()), 1) + 10
    return int(dp.sum())


def test_mixed_gradient_ragged_grid_full_parity(lens):
    """700 x 650 nodes of 0.03 arcsec (ragged against the 256-node rows), the
    paper's two cluster-scale halos and 60 galaxies, the paper's 400/20 blocks."""
    grid = S.paper_grid(700, ny=650)
    prm = S.paper_sie_cluster(grid, n_galaxies=60, seed=3)
    res = lens.lens_deflect_mixed(dev(prm), grid, n_cluster=2)
    torch.cuda.synchronize()
    ax, ay = oracle.alpha_grid(prm, grid)
    patch = oracle.dp_patches(prm, grid, 2)
    crit = oracle.criteria(ax, ay, grid.h)
    mask = res.mask.cpu().numpy()
    n_dp = check_rows(res.ax.cpu().numpy(), res.ay.cpu().numpy(), mask, ax, ay, patch, crit,
                      criterion_margin(ax, ay, grid.h), "700x650")
    st = res.stats.cpu().numpy()
    assert st[3] == 0 and st[0] == (mask == 1).sum() and st[1] == (mask == 2).sum() and st[2] == n_dp
    assert st[1] > 0


@pytest.mark.parametrize("pc,pg", [(0, 0), (64, 7)])
def test_mixed_gradient_block_sizes(lens, pc, pg):
    """No blocks at all, and odd block sizes; the same bars."""
    grid = S.paper_grid(300, ny=257)
    prm = S.paper_sie_cluster(grid, n_galaxies=25, seed=4)
    res = lens.lens_deflect_mixed(dev(prm), grid, n_cluster=2, patch_cluster=pc, patch_galaxy=pg)
    torch.cuda.synchronize()
    ax, ay = oracle.alpha_grid(prm, grid)
    patch = oracle.dp_patches(prm, grid, 2, pc, pg)
    crit = oracle.criteria(ax, ay, grid.h)
    check_rows(res.ax.cpu().numpy(), res.ay.cpu().numpy(), res.mask.cpu().numpy(), ax, ay, patch, crit,
               criterion_margin(ax, ay, grid.h), f"blocks {pc}/{pg}")


def test_mixed_gradient_invalid_and_empty(lens):
    grid = S.paper_grid(130, ny=70)
    prm = S.paper_sie_cluster(grid, n_galaxies=5, seed=5)
    bad = prm.copy()
    bad[4, 3] = 0.2  # a core radius: outside the SIE model of the precision study
    res = lens.lens_deflect_mixed(dev(bad), grid, n_cluster=2)
    st = res.stats.cpu().numpy()
    assert st[3] == 1 and (st[:3] == 0).all()
    assert np.isnan(res.ax.cpu().numpy()).all() and np.isnan(res.ay.cpu().numpy()).all()
    # the next call on the same context is unaffected
    res = lens.lens_deflect_mixed(dev(prm), grid, n_cluster=2)
    assert res.stats.cpu().numpy()[3] == 0 and np.isfinite(res.ax.cpu().numpy()).all()
    # no potentials: zero field, nothing in FP64 (every source pixel is dx long)
    res = lens.lens_deflect_mixed(dev(np.zeros((7, 0))), grid, n_cluster=0)
    torch.cuda.synchronize()
    assert (res.ax.cpu().numpy() == 0).all() and (res.mask.cpu().numpy() == 0).all()
    assert (res.stats.cpu().numpy() == 0).all()
    with pytest.raises(RuntimeError, match="invalid"):
        lens.lens_deflect_mixed(dev(prm), grid, n_cluster=len(prm[0]) + 1)


def test_mixed_gradient_paper_benchmark_sampled_rows(lens):
    """The benchmark of Sec. 4 at full size: 6730^2 pixels, 2 + 700 SIE halos;
    rows sampled through both cluster halos, their blocks' edges, the image
    edges and elsewhere, each checked with the row below it."""
    grid = S.paper_grid()
    prm = S.paper_sie_cluster(grid)
    res = lens.lens_deflect_mixed(dev(prm), grid, n_cluster=2)
    st = res.stats.cpu().numpy()
    print(f"  6730^2: FP64 blocks {st[0]}, criteria {st[1]}, FP64 fraction {st[2] / grid.nx / grid.ny:.4f}",
          flush=True)
    assert st[3] == 0
    kj = [int(round((y - grid.y0) / grid.h)) for y in prm[1, :2]]
    rows = sorted({1, 2, 100, 3000, 6729} | {k + d for k in kj for d in (-200, -199, 0, 199, 200, 300)})
    total = 0
    for j in rows:
        sub = S.Grid(grid.x0, grid.y0 + (j - 1) * grid.h, grid.h, grid.nx, 2)
        ax, ay = oracle.alpha_grid(prm, sub)
        patch = oracle.dp_patches(prm, sub, 2)
        crit = oracle.criteria(ax, ay, grid.h)
        margin = criterion_margin(ax, ay, grid.h)
        ga = res.ax[j].cpu().numpy()[None]
        gb = res.ay[j].cpu().numpy()[None]
        gm = res.mask[j].cpu().numpy()[None]
        # row 1 of the sub-grid is row j (its row 0 is the neighbour below)
        total += check_rows(ga, gb, gm, ax[1:], ay[1:], patch[1:], crit[1:], margin[1:], f"row {j}")
    assert total > 0
