"""Plain FP64 CPU oracle (test infrastructure only).

Thin numpy/ctypes wrapper around ``lens_oracle.c``.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import this package;
the GPU library never does, and this package never imports the GPU library.

Functions mirror the steps of Rexroth et al. (2019): Algorithm 1 (deflection
gradient, generalised to the cored/cut isothermal profile), the reformulated
lens equation of Sec. 2.2.2, and the chi^2 re-lensing procedure of
Sec. 2.2.1-2.2.2 (Fig. 1).  See the C source for the readings taken where the
paper is silent.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lens_oracle.c")
_LIB = os.path.join(_HERE, "liblens_oracle.so")
_lib = None

OMEGA_M, OMEGA_L = 0.3, 0.7  # Sec. 4 cosmology


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-adds)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        d, i = C.c_double, C.c_int
        lib.orc_b0.restype = d
        lib.orc_b0.argtypes = [d]
        lib.orc_comoving.restype = d
        lib.orc_comoving.argtypes = [d, d, d]
        lib.orc_dls_dos.restype = d
        lib.orc_dls_dos.argtypes = [d, d, d, d]
        lib.orc_alpha.argtypes = [dp, i, d, d, dp, dp]
        lib.orc_alpha_cplx.argtypes = [dp, i, d, d, d, d, i, i, d, dp]
        lib.orc_alpha_grid.argtypes = [dp, i, d, d, d, i, i, dp, dp, i]
        lib.orc_source_positions.argtypes = [dp, i, i, ip, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_orient.restype = i
        lib.orc_orient.argtypes = [d] * 6
        lib.orc_image_chi2.restype = i
        lib.orc_image_chi2.argtypes = [dp, i, d, d, d, i, i, i, ip, dp, dp, dp, dp, i, i,
                                       ip, ip, dp, dp, ip, dp, dp, ip, lp, dp, dp]
        lib.orc_hits_from_field.restype = i
        lib.orc_hits_from_field.argtypes = [dp, dp, d, d, d, i, i, i, dp, dp, dp, i, i, ip, ip, lp]
        lib.orc_positions_from_field.argtypes = [dp, dp, d, d, d, i, i, ip, ip, dp, dp, dp, dp, dp]
        lib.orc_match_chi2.restype = d
        lib.orc_match_chi2.argtypes = [i, ip, dp, dp, dp, i, ip, dp, dp, ip, dp, ip]
        lib.orc_newton.restype = i
        lib.orc_newton.argtypes = [dp, i, d, d, d, d, d, i, d, dp, dp]
        lib.orc_find_images.restype = i
        lib.orc_find_images.argtypes = [dp, i, d, d, d, d, d, d, i, i, d, d, d, d, d, d, i, dp, dp]
        lib.orc_src_chi2.restype = d
        lib.orc_src_chi2.argtypes = [dp, i, i, ip, dp, dp, dp, dp]
        lib.orc_src_chi2_grad.argtypes = [dp, i, i, ip, dp, dp, dp, dp, dp]
        lib.orc_alpha_vjp.argtypes = [dp, i, d, d, d, i, i, dp, dp, dp, i, i]
        u8p = C.POINTER(C.c_uint8)
        lib.orc_dp_patches.argtypes = [dp, i, i, i, i, d, d, d, i, i, u8p]
        lib.orc_criteria.argtypes = [dp, dp, i, i, d, d, d, u8p]
        lib.orc_nfw_alpha.argtypes = [dp, i, d, d, dp, dp]
        lib.orc_nfw_alpha_grid.argtypes = [dp, i, d, d, d, i, i, dp, dp, i]
        _lib = lib
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _prm(prm):
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    assert prm.ndim == 2 and prm.shape[0] == 7, "potentials are a [7, P] structure of arrays"
    return prm, prm.ctypes.data_as(C.POINTER(C.c_double)), prm.shape[1]


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ---------------------------------------------------------------- scalars

def b0(sigma_v: float) -> float:
    """b0 = 4 pi (sigma_v/c)^2 in arcsec (Sec. 2.2.2)."""
    return _load().orc_b0(float(sigma_v))


def comoving(z: float, om: float = OMEGA_M, ol: float = OMEGA_L) -> float:
    return _load().orc_comoving(float(z), om, ol)


def dls_dos(zl: float, zs: float, om: float = OMEGA_M, ol: float = OMEGA_L) -> float:
    """D_LS / D_OS, flat LambdaCDM (Sec. 2.2.2: computed once per source)."""
    return _load().orc_dls_dos(float(zl), float(zs), om, ol)


def orient(a, b, c) -> int:
    """Exact sign of (a - c) x (b - c) for double inputs."""
    return _load().orc_orient(float(a[0]), float(a[1]), float(b[0]), float(b[1]), float(c[0]), float(c[1]))


# ---------------------------------------------------------------- deflection

def alpha(prm, t1: float, t2: float):
    """grad Psi at one point (Algorithm 1, summed over potentials)."""
    prm, pp, n = _prm(prm)
    a1, a2 = C.c_double(), C.c_double()
    _load().orc_alpha(pp, n, float(t1), float(t2), C.byref(a1), C.byref(a2))
    return a1.value, a2.value


def alpha_points(prm, pts):
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(pts)
    for k, (x, y) in enumerate(pts):
        out[k] = alpha(prm, x, y)
    return out


def alpha_complex(prm, t1: complex, t2: complex, kq: int = -1, pq: int = -1, ih: float = 0.0):
    """Complex evaluation of the same steps: position (t1, t2) may be complex and
    parameter kq of potential pq may carry an imaginary part ih."""
    prm, pp, n = _prm(prm)
    out = np.zeros(4)
    _, op = _d(out)
    t1, t2 = complex(t1), complex(t2)
    _load().orc_alpha_cplx(pp, n, t1.real, t1.imag, t2.real, t2.imag, kq, pq, ih, op)
    return complex(out[0], out[1]), complex(out[2], out[3])


def alpha_grid(prm, grid, nthreads: int | None = None):
    """Deflection at all nodes, arrays [ny, nx] (row-major, node (i,j) at index [j, i])."""
    prm, pp, n = _prm(prm)
    ax = np.empty((grid.ny, grid.nx))
    ay = np.empty((grid.ny, grid.nx))
    _, axp = _d(ax)
    _, ayp = _d(ay)
    _load().orc_alpha_grid(pp, n, grid.x0, grid.y0, grid.h, grid.nx, grid.ny, axp, ayp,
                           nthreads or default_threads())
    return ax, ay


# ---------------------------------------------------------------- sources

def source_positions(prm, sys_off, ox, oy, dls):
    prm, pp, n = _prm(prm)
    sys_off, sp = _i32(sys_off)
    ox, oxp = _d(ox)
    oy, oyp = _d(oy)
    dls, dp_ = _d(dls)
    nimg, nsys = int(sys_off[-1]), len(sys_off) - 1
    bx, by = np.empty(nimg), np.empty(nimg)
    barx, bary = np.empty(nsys), np.empty(nsys)
    _load().orc_source_positions(pp, n, nsys, sp, oxp, oyp, dp_, _d(bx)[1], _d(by)[1],
                                 _d(barx)[1], _d(bary)[1])
    return bx, by, barx, bary


# ---------------------------------------------------------------- chi^2

def image_chi2(prm, grid, obs, nthreads: int | None = None, cap: int = 1 << 16):
    """Full image-plane chi^2 evaluation.  ``obs`` has keys sys_off, x, y, sigma, dls.

    Returns a dict with hits (sys, tid) sorted, positions, n_pred, chi2_sys, chi2,
    match and stats."""
    prm, pp, n = _prm(prm)
    sys_off, sp = _i32(obs["sys_off"])
    ox, oxp = _d(obs["x"])
    oy, oyp = _d(obs["y"])
    os_, osp = _d(obs["sigma"])
    dls, dlp = _d(obs["dls"])
    nsys, nimg = len(sys_off) - 1, int(sys_off[-1])
    hs, ht = np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    hx, hy = np.zeros(cap), np.zeros(cap)
    npred, csys = np.zeros(nsys, np.int32), np.zeros(nsys)
    chi2 = np.zeros(1)
    match = np.zeros(max(nimg, 1), np.int32)
    stats = np.zeros(4, np.int64)
    barx, bary = np.zeros(nsys), np.zeros(nsys)
    nh = _load().orc_image_chi2(
        pp, n, grid.x0, grid.y0, grid.h, grid.nx, grid.ny, nsys, sp, oxp, oyp, osp, dlp,
        nthreads or default_threads(), cap, _i32(hs)[1], _i32(ht)[1], _d(hx)[1], _d(hy)[1],
        _i32(npred)[1], _d(csys)[1], _d(chi2)[1], _i32(match)[1],
        stats.ctypes.data_as(C.POINTER(C.c_int64)), _d(barx)[1], _d(bary)[1])
    if nh > cap:
        raise RuntimeError(f"oracle hit capacity {cap} exceeded ({nh} hits)")
    return dict(hit_sys=hs[:nh].copy(), hit_tid=ht[:nh].copy(), hit_x=hx[:nh].copy(),
                hit_y=hy[:nh].copy(), n_pred=npred, chi2_sys=csys, chi2=float(chi2[0]),
                match=match[:nimg].copy(), stats=stats, bar_x=barx, bar_y=bary)


def hits_from_field(ax, ay, grid, barx, bary, dls, nthreads: int | None = None, cap: int = 1 << 16):
    """Triangle stage on a given field: sorted (sys, tid) of every triangle whose
    source-plane image contains its system's barycentre."""
    ax, axp = _d(ax)
    ay, ayp = _d(ay)
    barx, bxp = _d(np.atleast_1d(barx))
    bary, byp = _d(np.atleast_1d(bary))
    dls, dlp = _d(np.atleast_1d(dls))
    hs, ht = np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    nb = C.c_int64()
    nh = _load().orc_hits_from_field(axp, ayp, grid.x0, grid.y0, grid.h, grid.nx, grid.ny, len(barx),
                                     bxp, byp, dlp, nthreads or default_threads(), cap, _i32(hs)[1],
                                     _i32(ht)[1], C.byref(nb))
    if nh > cap:
        raise RuntimeError(f"oracle hit capacity {cap} exceeded ({nh} hits)")
    return hs[:nh].copy(), ht[:nh].copy()


def positions_from_field(ax, ay, grid, hit_sys, hit_tid, barx, bary, dls):
    ax, axp = _d(ax)
    ay, ayp = _d(ay)
    hit_sys, hsp = _i32(hit_sys)
    hit_tid, htp = _i32(hit_tid)
    barx, bxp = _d(np.atleast_1d(barx))
    bary, byp = _d(np.atleast_1d(bary))
    dls, dlp = _d(np.atleast_1d(dls))
    nh = len(hit_sys)
    hx, hy = np.zeros(max(nh, 1)), np.zeros(max(nh, 1))
    _load().orc_positions_from_field(axp, ayp, grid.x0, grid.y0, grid.h, grid.nx, nh, hsp, htp, bxp, byp,
                                     dlp, _d(hx)[1], _d(hy)[1])
    return hx[:nh], hy[:nh]


def match_chi2(obs, hit_sys, hit_x, hit_y):
    """Matching and chi^2 of Sec. 2.2.1 for hits sorted by system."""
    sys_off, sp = _i32(obs["sys_off"])
    ox, oxp = _d(obs["x"])
    oy, oyp = _d(obs["y"])
    os_, osp = _d(obs["sigma"])
    hit_sys, hsp = _i32(hit_sys)
    hx, hxp = _d(hit_x)
    hy, hyp = _d(hit_y)
    nsys, nimg = len(sys_off) - 1, int(sys_off[-1])
    npred, csys, match = np.zeros(nsys, np.int32), np.zeros(nsys), np.zeros(max(nimg, 1), np.int32)
    chi2 = _load().orc_match_chi2(nsys, sp, oxp, oyp, osp, len(hit_sys), hsp, hxp, hyp, _i32(npred)[1],
                                  _d(csys)[1], _i32(match)[1])
    return dict(n_pred=npred, chi2_sys=csys, chi2=chi2, match=match[:nimg])


# ---------------------------------------------------------------- image finding

def newton(prm, r, beta, seed, maxit: int = 60, tol: float = 1e-11):
    prm, pp, n = _prm(prm)
    rx, ry = C.c_double(), C.c_double()
    ok = _load().orc_newton(pp, n, float(r), float(beta[0]), float(beta[1]), float(seed[0]),
                            float(seed[1]), maxit, tol, C.byref(rx), C.byref(ry))
    return (rx.value, ry.value) if ok else None


def find_images(prm, r, beta, seed_grid, bounds, tol: float = 1e-11, dedup: float = 1e-7, cap: int = 64):
    """Brute-force image finder: Newton from every node of seed_grid; roots inside
    bounds = (xlo, xhi, ylo, yhi), de-duplicated."""
    prm, pp, n = _prm(prm)
    ox, oy = np.zeros(cap), np.zeros(cap)
    k = _load().orc_find_images(pp, n, float(r), float(beta[0]), float(beta[1]), seed_grid.x0,
                                seed_grid.y0, seed_grid.h, seed_grid.nx, seed_grid.ny, *map(float, bounds),
                                tol, dedup, cap, _d(ox)[1], _d(oy)[1])
    k = min(k, cap)
    return np.stack([ox[:k], oy[:k]], axis=1)


# ---------------------------------------------------------------- source-plane chi^2

def src_chi2(prm, obs) -> float:
    prm, pp, n = _prm(prm)
    sys_off, sp = _i32(obs["sys_off"])
    return _load().orc_src_chi2(pp, n, len(sys_off) - 1, sp, _d(obs["x"])[1], _d(obs["y"])[1],
                                _d(obs["sigma"])[1], _d(obs["dls"])[1])


def src_chi2_grad(prm, obs):
    """Complex-step gradient of the source-plane chi^2, shape [7, P]."""
    prm, pp, n = _prm(prm)
    sys_off, sp = _i32(obs["sys_off"])
    x, xp = _d(obs["x"])
    y, yp = _d(obs["y"])
    s, spp = _d(obs["sigma"])
    r, rp = _d(obs["dls"])
    g = np.zeros((7, n))
    _load().orc_src_chi2_grad(pp, n, len(sys_off) - 1, sp, xp, yp, spp, rp, _d(g)[1])
    return g


def alpha_vjp(prm, grid, gx, gy, nthreads: int | None = None, absolute: bool = False):
    """sum over nodes of g . d(alpha)/d(q) for every parameter, shape [7, P];
    absolute=True sums |gx d alpha_1/dq| + |gy d alpha_2/dq| instead."""
    prm, pp, n = _prm(prm)
    gx, gxp = _d(np.asarray(gx).reshape(grid.ny, grid.nx))
    gy, gyp = _d(np.asarray(gy).reshape(grid.ny, grid.nx))
    g = np.zeros((7, n))
    _load().orc_alpha_vjp(pp, n, grid.x0, grid.y0, grid.h, grid.nx, grid.ny, gxp, gyp, _d(g)[1],
                          nthreads or default_threads(), int(bool(absolute)))
    return g


# ---------------------------------------------------------------- the paper's mixed-precision gradient

PATCH_CLUSTER, PATCH_GALAXY = 400, 20   # Sec. 3.2 / Appendix A.3, pixels
T12, T34 = 0.0092, 0.0104               # Sec. 3.3 thresholds for 0.03 arcsec pixels, arcsec


def _u8(shape):
    a = np.zeros(shape, dtype=np.uint8)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint8))


def dp_patches(prm, grid, n_cluster: int, pc: int = PATCH_CLUSTER, pg: int = PATCH_GALAXY):
    """uint8 [ny, nx]: 1 inside the double-precision block of some halo."""
    prm, pp, n = _prm(prm)
    m, mp = _u8((grid.ny, grid.nx))
    _load().orc_dp_patches(pp, n, int(n_cluster), int(pc), int(pg), grid.x0, grid.y0, grid.h, grid.nx, grid.ny, mp)
    return m


def criteria(ax, ay, dx: float, t12: float = T12, t34: float = T34):
    """uint8 [ny, nx]: 1 where the criteria of Sec. 3.3 ask for double precision."""
    ax, axp = _d(ax)
    ay, ayp = _d(ay)
    ny, nx = ax.shape
    f, fp = _u8((ny, nx))
    _load().orc_criteria(axp, ayp, nx, ny, float(dx), float(t12), float(t34), fp)
    return f


# ---------------------------------------------------------------- sampler steps
#
# The paper evaluates chi^2 inside a sampler over the lens parameters
# (Sec. 2.2.1).  These are the textbook steps of two samplers, written out
# plainly: Hamiltonian Monte Carlo (Duane, Kennedy, Pendleton & Roweth 1987;
# the leapfrog form of Neal 2011, "MCMC using Hamiltonian dynamics", Sec. 5.3)
# and random-walk Metropolis (Metropolis et al. 1953).  Random draws are
# arguments.

def hmc_step_generic(q0, step, n_leapfrog: int, momentum, u: float, energy):
    """One HMC step in the coordinates z = q/step with unit masses.
    energy(q) -> (U, dU/dq).  Returns (q, U, accepted)."""
    q0 = np.asarray(q0, dtype=np.float64)
    free = np.asarray(step) != 0
    q = q0.copy()
    p = np.where(free, momentum, 0.0)
    u0, g = energy(q)
    p = p - np.where(free, 0.5 * step * g, 0.0)                      # half kick
    u1 = u0
    for ell in range(1, n_leapfrog + 1):
        q = np.where(free, q + step * p, q)                           # drift
        u1, g = energy(q)
        c = 1.0 if ell < n_leapfrog else 0.5
        p = p - np.where(free, c * step * g, 0.0)                     # kick (half at the end)
    h0 = u0 + 0.5 * float(np.sum(np.where(free, momentum, 0.0) ** 2))
    h1 = u1 + 0.5 * float(np.sum(p ** 2))
    accept = bool(np.isfinite(u0) and np.isfinite(h1) and math.log(u) < h0 - h1)
    return (q, u1, True) if accept else (q0.copy(), u0, False)


def _src_energy(obs):
    def energy(q):
        c = src_chi2(q, obs)
        if not np.isfinite(c):
            return float("nan"), np.full(q.shape, np.nan)
        return 0.5 * c, 0.5 * src_chi2_grad(q, obs)
    return energy


def hmc_step(state, obs, step, n_leapfrog: int, momentum, u: float):
    """HMC on the source-plane chi^2 (U = chi^2/2): returns (state, chi2, accepted)."""
    q, u1, acc = hmc_step_generic(state, step, n_leapfrog, momentum, u, _src_energy(obs))
    return q, 2.0 * u1, acc


def mh_accept(chi2_new: float, chi2_cur: float, u: float, valid: bool) -> bool:
    """Metropolis acceptance for the log-likelihood -chi^2/2; any valid proposal
    replaces a state whose chi^2 is not finite."""
    if not valid or not np.isfinite(chi2_new):
        return False
    return (not np.isfinite(chi2_cur)) or math.log(u) < -0.5 * (chi2_new - chi2_cur)


# ---------------------------------------------------------------- pseudo-elliptical NFW

def _nfw(prm):
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    if prm.ndim != 2 or prm.shape[0] != 6:
        raise ValueError("NFW parameters must be [6, P]: x, y, eps, phi, r_s, kappa_s")
    return prm, prm.ctypes.data_as(C.POINTER(C.c_double)), prm.shape[1]


def nfw_alpha(prm, t1: float, t2: float):
    prm, pp, n = _nfw(prm)
    a1, a2 = C.c_double(), C.c_double()
    _load().orc_nfw_alpha(pp, n, t1, t2, C.byref(a1), C.byref(a2))
    return a1.value, a2.value


def nfw_alpha_grid(prm, grid, nthreads: int | None = None):
    prm, pp, n = _nfw(prm)
    ax, ay = np.empty((grid.ny, grid.nx)), np.empty((grid.ny, grid.nx))
    _load().orc_nfw_alpha_grid(pp, n, grid.x0, grid.y0, grid.h, grid.nx, grid.ny, _d(ax)[1], _d(ay)[1],
                               nthreads or default_threads())
    return ax, ay
