"""GPU parity of the backward form against the FP64 CPU oracle (complex-step
derivatives), through the C ABI.

Bars (per gradient entry, M = the oracle's magnitude sum over nodes of
|g . d alpha/dq|, the scale of the rounding error of any evaluation order):
FP64 products |err| <= 1e-11 M; FP32 products with FP64 accumulation
|err| <= 256 u32 M (u32 = 2^-24: about 40 roundings per product, pieces that
cancel by up to a factor 4, and the FP32 partial sums of 16 nodes).  Source-
plane chi^2 within 1e-12 relative, its gradient within 1e-10 of each
parameter row's largest entry."""
import numpy as np
import pytest

import oracle
import synthlens as S
from conftest import load_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
BAR = {"fp64": 1e-11, "fp32": 256 * U32}


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1902_03252_amd as lens
    lens.context()
    return lens


def dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float64, device="cuda")


_ORACLE = {}


def oracle_vjp(key, prm, grid, gx, gy):
    if key not in _ORACLE:
        _ORACLE[key] = (oracle.alpha_vjp(prm, grid, gx, gy), oracle.alpha_vjp(prm, grid, gx, gy, absolute=True))
    return _ORACLE[key]


def check_vjp(got, want, mag, prec, what):
    err = np.abs(got - want)
    ratio = (err / np.maximum(mag, 1e-300)).max(axis=1)
    print(f"  {what} {prec}: max |err|/M per parameter {np.array2string(ratio, precision=2)}", flush=True)
    assert (err <= BAR[prec] * mag + 1e-300).all(), (what, prec, ratio)


def config5():
    w = S.WORKLOADS[5]
    grid = w.grid
    cot = S.cotangent(grid.nx * grid.ny)
    return S.potentials(5), grid, cot[0].reshape(grid.ny, grid.nx), cot[1].reshape(grid.ny, grid.nx)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deflect_vjp_differentiation_workload(lens, prec):
    """512^2 grid over +-80", the 50 cluster potentials, N(0,1) cotangent."""
    prm, grid, gx, gy = config5()
    want, mag = oracle_vjp("c5", prm, grid, gx, gy)
    got = lens.lens_deflect_backward(dev(prm), grid, dev(gx), dev(gy), prec).cpu().numpy()
    check_vjp(got, want, mag, prec, "config 5")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deflect_vjp_all_profile_kinds_ragged_grid(lens, prec):
    """Cored/singular x cut/uncut profiles (incl. the SIE of Algorithm 1) on a grid
    whose node count is not a multiple of the 4096-node chunk."""
    prm = S.sie_potentials(6, seed=3)
    prm[4, :3] = [0.2, 0.0, 0.4]
    prm[5, 3:] = [30.0, 50.0, np.inf]
    prm[4, 5] = 0.1
    grid = S.Grid(-60.3, -59.1, 0.37, 301, 290)
    g = np.random.default_rng(21)
    gx, gy = g.normal(size=(grid.ny, grid.nx)), g.normal(size=(grid.ny, grid.nx))
    want, mag = oracle_vjp("kinds", prm, grid, gx, gy)
    got = lens.lens_deflect_backward(dev(prm), grid, dev(gx), dev(gy), prec).cpu().numpy()
    check_vjp(got, want, mag, prec, "kinds")
    np.testing.assert_array_equal(got[5][np.isinf(prm[5])], 0.0)


def test_deflect_vjp_invalid_and_empty(lens):
    prm, grid, gx, gy = config5()
    grid = S.square_grid(64, 40.0)
    gx, gy = gx[:64, :64].copy(), gy[:64, :64].copy()
    bad = prm[:, :5].copy()
    bad[2, 3] = 1.2
    with pytest.raises(RuntimeError, match="invalid"):
        lens.lens_deflect_backward(dev(bad), grid, dev(gx), dev(gy), "fp64")
    got = lens.lens_deflect_backward(dev(bad), grid, dev(gx), dev(gy), "fp64", check=False).cpu().numpy()
    assert np.isnan(got[:, 3]).all() and np.isfinite(np.delete(got, 3, axis=1)).all()
    empty = lens.lens_deflect_backward(dev(np.zeros((7, 0))), grid, dev(gx), dev(gy), "fp64")
    assert empty.shape == (7, 0)


def test_deflect_vjp_deterministic(lens):
    prm, grid, gx, gy = config5()
    p, a, b = dev(prm), dev(gx), dev(gy)
    for prec in ("fp64", "fp32"):
        x = lens.lens_deflect_backward(p, grid, a, b, prec).cpu().numpy()
        y = lens.lens_deflect_backward(p, grid, a, b, prec).cpu().numpy()
        np.testing.assert_array_equal(x, y)


def test_src_chi2_and_gradient(lens):
    prm, _, obs = load_inputs(2)
    o = lens.Obs.from_numpy(obs)
    want = oracle.src_chi2(prm, obs)
    gwant = oracle.src_chi2_grad(prm, obs)
    got = float(lens.lens_src_chi2(dev(prm), o).cpu()[0])
    assert got == pytest.approx(want, rel=1e-12)
    g3 = torch.full((1,), 3.0, dtype=torch.float64, device="cuda")
    grad = lens.lens_src_chi2_backward(dev(prm), o, g3).cpu().numpy()
    scale = np.abs(gwant).max(axis=1, keepdims=True)
    err = np.abs(grad - 3.0 * gwant) / (3.0 * scale)
    print(f"  src chi2 {got:.6e} (oracle {want:.6e}); grad max err / row max {err.max():.2e}", flush=True)
    assert err.max() <= 1e-10


def test_src_chi2_invalid_status(lens):
    prm, _, obs = load_inputs(2)
    bad = prm.copy()
    bad[6, 2] = -1.0
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    o = lens.Obs.from_numpy(obs)
    chi2 = lens.lens_src_chi2(dev(bad), o, status=status)
    assert int(status.cpu()[0]) == 1 and np.isnan(float(chi2.cpu()[0]))
    grad = lens.lens_src_chi2_backward(dev(bad), o, status=status).cpu().numpy()
    assert int(status.cpu()[0]) == 1 and np.isnan(grad).all()
    # the next call is unaffected
    chi2 = lens.lens_src_chi2(dev(prm), o, status=status)
    assert int(status.cpu()[0]) == 0 and np.isfinite(float(chi2.cpu()[0]))


def test_autograd_functions(lens):
    """DeflectFn and SrcChi2Fn route torch.autograd through the backward entry points."""
    prm, grid, gx, gy = config5()
    grid = S.square_grid(96, 60.0)
    g = np.random.default_rng(5)
    wx, wy = dev(g.normal(size=(grid.ny, grid.nx))), dev(g.normal(size=(grid.ny, grid.nx)))
    p = dev(prm).requires_grad_(True)
    ax, ay = lens.DeflectFn.apply(p, grid, "fp64")
    ((ax * wx).sum() + (ay * wy).sum()).backward()
    direct = lens.lens_deflect_backward(dev(prm), grid, wx, wy, "fp64")
    assert torch.equal(p.grad, direct)
    _, _, obs = load_inputs(2)
    o = lens.Obs.from_numpy(obs)
    q = dev(prm).requires_grad_(True)
    (gq,) = torch.autograd.grad(2.5 * lens.SrcChi2Fn.apply(q, o), q)
    want = 2.5 * oracle.src_chi2_grad(prm, obs)
    scale = np.abs(want).max(axis=1, keepdims=True)
    assert (np.abs(gq.cpu().numpy() - want) <= 1e-10 * scale).all()


def test_deflect_gradcheck_small(lens):
    """torch.autograd.gradcheck (finite differences of the GPU forward) on a tiny
    FP64 instance: forward and backward kernels agree with each other."""
    prm = S.potentials(2)[:, :2].copy()
    prm[0] = [3.0, -7.0]
    prm[1] = [-2.0, 5.0]
    grid = S.Grid(-20.0, -18.0, 4.3, 9, 8)
    p = dev(prm).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: lens.DeflectFn.apply(x, grid, "fp64"), (p,), eps=1e-6, atol=1e-6,
                                    rtol=1e-5, fast_mode=True)
