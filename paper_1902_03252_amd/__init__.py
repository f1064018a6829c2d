"""MI355X (gfx950) image-plane chi^2 for strong-lens models.

Python face of the C ABI in include/lens.h (Rexroth et al. 2019: Algorithm 1
deflection generalised to cored/cut isothermal potentials, the lens equation of
Sec. 2.2.2, and the triangle re-lensing chi^2 of Sec. 2.2.1-2.2.2).  The
functions below only marshal torch tensors into the library calls; all
arithmetic runs in the HIP kernels of liblens.so.

Potentials are a float64 CUDA tensor of shape [7, P] (rows x, y, eps, phi,
r_core, r_cut, sigma_v; structure of arrays).  Observations are an ``Obs``
(CSR over systems).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import torch

from . import _lib as L
from ._lib import LENS_FP32, LENS_FP64, LENS_MIXED, STAT_N  # noqa: F401

_PREC = {"fp64": LENS_FP64, "fp32": LENS_FP32, "mixed": LENS_MIXED}


@dataclasses.dataclass
class Obs:
    """Observed multiple-image systems: sys_off [S+1] int32, x, y, sigma [n_img]
    float64, dls [S] float64 (D_LS/D_OS), all on the same CUDA device."""
    sys_off: torch.Tensor
    x: torch.Tensor
    y: torch.Tensor
    sigma: torch.Tensor
    dls: torch.Tensor

    @property
    def n_sys(self) -> int:
        return self.sys_off.numel() - 1

    @property
    def n_img(self) -> int:
        return self.x.numel()

    @staticmethod
    def from_numpy(d, device="cuda"):
        f = lambda a, dt: torch.as_tensor(a, dtype=dt, device=device).contiguous()
        return Obs(f(d["sys_off"], torch.int32), f(d["x"], torch.float64), f(d["y"], torch.float64),
                   f(d["sigma"], torch.float64), f(d["dls"], torch.float64))


def _require_cuda(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _pots(params: torch.Tensor) -> L.LensPotentials:
    _require_cuda(params, torch.float64, "params")
    if params.dim() != 2 or params.shape[0] != 7:
        raise ValueError("params must have shape [7, P]")
    n = params.shape[1]
    rows = [params[k].data_ptr() if n > 0 else None for k in range(7)]
    return L.LensPotentials(n, *rows)


def _grid(grid) -> L.LensGrid:
    return L.LensGrid(float(grid.x0), float(grid.y0), float(grid.h), int(grid.nx), int(grid.ny))


def _obs(obs: Obs) -> L.LensObs:
    _require_cuda(obs.sys_off, torch.int32, "sys_off")
    for name in ("x", "y", "sigma", "dls"):
        _require_cuda(getattr(obs, name), torch.float64, name)
    return L.LensObs(obs.n_sys, obs.n_img, obs.sys_off.data_ptr(), obs.x.data_ptr(), obs.y.data_ptr(),
                     obs.sigma.data_ptr(), obs.dls.data_ptr())


class Context:
    """Owns a lens_ctx (device scratch) on one device."""

    def __init__(self, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available: the lens library has no CPU path")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        torch.cuda.init()
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.lens_create(C.byref(h), self.device.index), "lens_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lens_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def stream(self):
        return L.stream_handle(self.device)

    def set_timing(self, enable: bool):
        """Bracket every deflection-field kernel launch with HIP events."""
        L.check(self._lib.lens_set_timing(self._h, int(bool(enable))), "lens_set_timing")

    def field_timing(self, reset: bool = True):
        """(total kernel milliseconds, number of launches) since the last reset."""
        ms, n = C.c_double(), C.c_int64()
        L.check(self._lib.lens_field_timing(self._h, C.byref(ms), C.byref(n), int(bool(reset))),
                "lens_field_timing")
        return ms.value, n.value


_contexts: dict[int, Context] = {}


def context(device=None) -> Context:
    idx = torch.cuda.current_device() if device is None else torch.device("cuda", device).index
    if idx not in _contexts:
        _contexts[idx] = Context(idx)
    return _contexts[idx]


def lens_dls_dos(z_lens: float, z_src: torch.Tensor, omega_m: float = 0.3, omega_l: float = 0.7,
                 ctx: Context | None = None) -> torch.Tensor:
    """D_LS/D_OS for every source redshift (flat universe, GPU quadrature)."""
    ctx = ctx or context(z_src.device.index)
    _require_cuda(z_src, torch.float64, "z_src")
    out = torch.empty_like(z_src)
    L.check(ctx._lib.lens_dls_dos(ctx.handle, float(z_lens), L.ptr(z_src), z_src.numel(), omega_m, omega_l,
                                  L.ptr(out), ctx.stream()), "lens_dls_dos")
    return out


def lens_deflect(params: torch.Tensor, grid, prec: str = "fp64", ctx: Context | None = None,
                 check: bool = True):
    """grad Psi at every grid node; returns (ax, ay) of shape [ny, nx] (float64 for
    'fp64', float32 for 'fp32'/'mixed')."""
    ctx = ctx or context(params.device.index)
    p = _pots(params)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ax = torch.empty((grid.ny, grid.nx), dtype=dt, device=params.device)
    ay = torch.empty_like(ax)
    status = torch.zeros(1, dtype=torch.int32, device=params.device)
    L.check(ctx._lib.lens_deflect(ctx.handle, C.byref(p), C.byref(_grid(grid)), _PREC[prec], L.ptr(ax), L.ptr(ay),
                                  L.ptr(status), ctx.stream()), "lens_deflect")
    if check and int(status.item()) != L.LENS_OK:
        raise RuntimeError(f"lens_deflect: invalid potential parameters (status {int(status.item())})")
    return ax, ay


def lens_deflect_nfw(halos: torch.Tensor, grid, prec: str = "fp64", ctx: Context | None = None,
                     check: bool = True):
    """Deflection of pseudo-elliptical NFW halos ([6, n] float64 table: x, y,
    eps, phi, r_s, kappa_s) at every node: (ax, ay) [ny, nx], float64 for
    'fp64', float32 for 'fp32'."""
    ctx = ctx or context(halos.device.index)
    if prec not in ("fp64", "fp32"):
        raise ValueError("prec must be 'fp64' or 'fp32'")
    _require_cuda(halos, torch.float64, "halos")
    if halos.dim() != 2 or halos.shape[0] != 6:
        raise ValueError("halos must be a [6, n] table")
    n = halos.shape[1]
    rows = [halos[k].data_ptr() if n else None for k in range(6)]
    h = L.LensNfw(n, *rows)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ax = torch.empty((grid.ny, grid.nx), dtype=dt, device=halos.device)
    ay = torch.empty_like(ax)
    status = torch.zeros(1, dtype=torch.int32, device=halos.device)
    L.check(ctx._lib.lens_deflect_nfw(ctx.handle, C.byref(h), C.byref(_grid(grid)), _PREC[prec], L.ptr(ax),
                                      L.ptr(ay), L.ptr(status), ctx.stream()), "lens_deflect_nfw")
    if check and int(status.item()) != L.LENS_OK:
        raise RuntimeError(f"lens_deflect_nfw: invalid halo parameters (status {int(status.item())})")
    return ax, ay


@dataclasses.dataclass
class MixedResult:
    ax: torch.Tensor     # [ny, nx] float64
    ay: torch.Tensor     # [ny, nx] float64
    mask: torch.Tensor   # [ny, nx] uint8: 0 FP32, 1 FP64 block, 2 FP64 by the criteria
    stats: torch.Tensor  # [4] int64: block nodes, criteria nodes, FP64 nodes, status


def mixed_buffers(grid, device) -> MixedResult:
    z = lambda dt: torch.empty((grid.ny, grid.nx), dtype=dt, device=device)
    return MixedResult(z(torch.float64), z(torch.float64), z(torch.uint8),
                       torch.zeros(4, dtype=torch.int64, device=device))


def lens_deflect_mixed(params: torch.Tensor, grid, n_cluster: int, patch_cluster: int = 400,
                       patch_galaxy: int = 20, t12: float = 0.0092, t34: float = 0.0104,
                       out: MixedResult | None = None, ctx: Context | None = None) -> MixedResult:
    """The paper's mixed-precision gradient of an SIE lens (asynchronous):
    FP32 everywhere, FP64 in blocks around the halos and where the criteria
    of its Sec. 3.3 hold.  The first n_cluster potentials are the cluster-scale halos."""
    ctx = ctx or context(params.device.index)
    p = _pots(params)
    out = out or mixed_buffers(grid, params.device)
    opts = L.LensMixedOpts(int(n_cluster), int(patch_cluster), int(patch_galaxy), float(t12), float(t34))
    L.check(ctx._lib.lens_deflect_mixed(ctx.handle, C.byref(p), C.byref(_grid(grid)), C.byref(opts),
                                        L.ptr(out.ax), L.ptr(out.ay), L.ptr(out.mask), L.ptr(out.stats),
                                        ctx.stream()), "lens_deflect_mixed")
    return out


def lens_source_positions(params: torch.Tensor, obs: Obs, ctx: Context | None = None, check: bool = True):
    """Source positions of the observed images [n_img, 2] and barycentres [n_sys, 2]."""
    ctx = ctx or context(params.device.index)
    p, o = _pots(params), _obs(obs)
    dev = params.device
    bx = torch.empty(obs.n_img, dtype=torch.float64, device=dev)
    by = torch.empty_like(bx)
    cx = torch.empty(obs.n_sys, dtype=torch.float64, device=dev)
    cy = torch.empty_like(cx)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    L.check(ctx._lib.lens_source_positions(ctx.handle, C.byref(p), C.byref(o), L.ptr(bx), L.ptr(by), L.ptr(cx),
                                           L.ptr(cy), L.ptr(status), ctx.stream()), "lens_source_positions")
    if check and int(status.item()) != L.LENS_OK:
        raise RuntimeError(f"lens_source_positions: invalid input (status {int(status.item())})")
    return torch.stack([bx, by], 1), torch.stack([cx, cy], 1)


@dataclasses.dataclass
class Chi2Result:
    chi2: torch.Tensor      # [1] float64
    chi2_sys: torch.Tensor  # [S] float64
    n_pred: torch.Tensor    # [S] int32
    hits: torch.Tensor      # [cap, 2] int32 (system, triangle id); first stats[0] rows valid
    img_xy: torch.Tensor    # [cap, 2] float64
    match: torch.Tensor     # [n_img] int32
    stats: torch.Tensor     # [8] int64

    def host(self) -> dict:
        """Copy to host and trim the hit list (synchronises)."""
        st = self.stats.cpu().numpy()
        n = int(st[L.STAT_HITS]) if st[L.STAT_STATUS] == L.LENS_OK else 0
        return dict(chi2=float(self.chi2.cpu()[0]), chi2_sys=self.chi2_sys.cpu().numpy(),
                    n_pred=self.n_pred.cpu().numpy(), hit_sys=self.hits[:n, 0].cpu().numpy(),
                    hit_tid=self.hits[:n, 1].cpu().numpy(), hit_x=self.img_xy[:n, 0].cpu().numpy(),
                    hit_y=self.img_xy[:n, 1].cpu().numpy(), match=self.match.cpu().numpy(), stats=st,
                    status=int(st[L.STAT_STATUS]))


def chi2_buffers(obs: Obs, hit_capacity: int, device) -> Chi2Result:
    z = lambda *s, dt=torch.float64: torch.zeros(*s, dtype=dt, device=device)
    return Chi2Result(z(1), z(obs.n_sys), z(obs.n_sys, dt=torch.int32), z(hit_capacity, 2, dt=torch.int32),
                      z(hit_capacity, 2), z(max(obs.n_img, 1), dt=torch.int32), z(STAT_N, dt=torch.int64))


def lens_image_chi2(params: torch.Tensor, grid, obs: Obs, prec: str = "mixed", fb_mode: int = 0,
                    fb_tau: float = 1e-6, hit_capacity: int = 4096, out: Chi2Result | None = None,
                    ctx: Context | None = None, field_npl: int = 0, tile: int = 0) -> Chi2Result:
    """Image-plane chi^2 (asynchronous; outputs valid after stream sync)."""
    ctx = ctx or context(params.device.index)
    if prec not in ("fp64", "mixed"):
        raise ValueError("prec must be 'fp64' or 'mixed'")
    p, o = _pots(params), _obs(obs)
    out = out or chi2_buffers(obs, hit_capacity, params.device)
    opts = L.LensChi2Opts(_PREC[prec], int(fb_mode), float(fb_tau), int(out.hits.shape[0]), int(field_npl),
                          int(tile))
    L.check(ctx._lib.lens_image_chi2(ctx.handle, C.byref(p), C.byref(_grid(grid)), C.byref(o), C.byref(opts),
                                     C.byref(_chi2_out(out)), ctx.stream()), "lens_image_chi2")
    return out


def lens_image_chi2_noalloc(params: torch.Tensor, grid, obs: Obs, prec: str = "mixed", fb_mode: int = 0,
                            fb_tau: float = 1e-6, hit_capacity: int = 4096, out: Chi2Result | None = None,
                            field_npl: int = 0, tile: int = 0) -> Chi2Result:
    """lens_image_chi2 through the entry point that allocates no device memory
    (no context; the library's fixed scratch on params' device).  Callers that
    cannot allocate pass `out`; without it the buffers are made here, outside
    the library call."""
    if prec not in ("fp64", "mixed"):
        raise ValueError("prec must be 'fp64' or 'mixed'")
    lib = L.load()
    p, o = _pots(params), _obs(obs)
    out = out or chi2_buffers(obs, hit_capacity, params.device)
    opts = L.LensChi2Opts(_PREC[prec], int(fb_mode), float(fb_tau), int(out.hits.shape[0]), int(field_npl),
                          int(tile))
    with torch.cuda.device(params.device):
        L.check(lib.lens_image_chi2_noalloc(C.byref(p), C.byref(_grid(grid)), C.byref(o), C.byref(opts),
                                            C.byref(_chi2_out(out)), L.stream_handle(params.device)),
                "lens_image_chi2_noalloc")
    return out


def _chi2_out(out: Chi2Result):
    return L.LensChi2Out(out.chi2.data_ptr(), out.chi2_sys.data_ptr(), out.n_pred.data_ptr(), out.hits.data_ptr(),
                         out.img_xy.data_ptr(), out.match.data_ptr(), out.stats.data_ptr())


def _batch_out(out: "BatchResult"):
    hits = out.hits is not None
    return L.LensBatchOut(out.chi2.data_ptr(), out.chi2_sys.data_ptr(), out.n_pred.data_ptr(),
                          out.status.data_ptr(), out.stats.data_ptr(), out.n_hits.data_ptr() if hits else None,
                          out.hits.data_ptr() if hits else None, out.img_xy.data_ptr() if hits else None)


class BatchLayout:
    """Host description of a batch: sample s owns parameter columns
    [pot_off[s], pot_off[s+1]) and is evaluated on grids[s].  Built once and
    reused, it keeps the marshalled host arrays of repeated calls."""

    def __init__(self, pot_off, grids):
        off = [int(v) for v in pot_off]
        if len(off) != len(grids) + 1:
            raise ValueError("pot_off needs one entry more than grids")
        self.n = len(grids)
        self.pot_off = (C.c_int32 * len(off))(*off)
        self.grids = (L.LensGrid * self.n)(*[_grid(g) for g in grids])


@dataclasses.dataclass
class BatchResult:
    chi2: torch.Tensor      # [n] float64
    chi2_sys: torch.Tensor  # [n, S] float64
    n_pred: torch.Tensor    # [n, S] int32
    status: torch.Tensor    # [n] int32
    stats: torch.Tensor     # [8] int64, totals over the batch
    n_hits: torch.Tensor | None = None  # [n] int32 (with hits)
    hits: torch.Tensor | None = None    # [n, hit_capacity, 2] int32 (system, triangle id), sorted
    img_xy: torch.Tensor | None = None  # [n, hit_capacity, 2] float64 predicted image positions

    def sample_hits(self, s: int) -> dict:
        """Host copy of sample s's hits (requires buffers made with hits=True)."""
        k = int(self.n_hits[s])
        h = self.hits[s, :k].cpu().numpy()
        xy = self.img_xy[s, :k].cpu().numpy()
        return dict(hit_sys=h[:, 0].copy(), hit_tid=h[:, 1].copy(), hit_x=xy[:, 0].copy(), hit_y=xy[:, 1].copy())


def batch_buffers(n: int, obs: Obs, device, hits: bool = False, hit_capacity: int = 1024) -> BatchResult:
    """Output buffers of a batched call; with hits=True also the per-sample hit
    lists (the call must then use the same hit_capacity)."""
    z = lambda *s, dt=torch.float64: torch.zeros(*s, dtype=dt, device=device)
    r = BatchResult(z(n), z(n, obs.n_sys), z(n, obs.n_sys, dt=torch.int32), z(n, dt=torch.int32),
                    z(STAT_N, dt=torch.int64))
    if hits:
        r.n_hits = z(n, dt=torch.int32)
        r.hits = z(n, hit_capacity, 2, dt=torch.int32)
        r.img_xy = z(n, hit_capacity, 2)
    return r


def lens_image_chi2_batched(params: torch.Tensor, layout: BatchLayout, obs: Obs, prec: str = "mixed",
                            fb_mode: int = 0, fb_tau: float = 1e-6, hit_capacity: int = 1024,
                            out: BatchResult | None = None, ctx: Context | None = None, field_npl: int = 0,
                            tile: int = 0) -> BatchResult:
    """Image-plane chi^2 of every sample of a batch (asynchronous).  params is
    the [7, sum P_s] concatenation of the samples' potentials."""
    ctx = ctx or context(params.device.index)
    if prec not in ("fp64", "mixed"):
        raise ValueError("prec must be 'fp64' or 'mixed'")
    p, o = _pots(params), _obs(obs)
    out = out or batch_buffers(layout.n, obs, params.device)
    if out.hits is not None and tuple(out.hits.shape) != (layout.n, int(hit_capacity), 2):
        raise ValueError("the hit buffers must be [n_samples, hit_capacity, 2]")
    opts = L.LensChi2Opts(_PREC[prec], int(fb_mode), float(fb_tau), int(hit_capacity), int(field_npl), int(tile))
    L.check(ctx._lib.lens_image_chi2_batched(ctx.handle, C.byref(p), layout.n, layout.pot_off, layout.grids,
                                             C.byref(o), C.byref(opts), C.byref(_batch_out(out)), ctx.stream()),
            "lens_image_chi2_batched")
    return out


# ---------------------------------------------------------------- sampler steps

def _table(t: torch.Tensor, name: str) -> torch.Tensor:
    _require_cuda(t, torch.float64, name)
    if t.dim() != 2 or t.shape[0] != 7 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous [7, n] float64 tensor")
    return t


def hmc_step(state: torch.Tensor, obs: Obs, step: torch.Tensor, n_leapfrog: int, momentum: torch.Tensor,
             u: torch.Tensor, ctx: Context | None = None):
    """One HMC step on the source-plane chi^2 (asynchronous).  state [7, n] is
    updated in place on acceptance; momentum [7, n] N(0,1) and u [1] U(0,1) are
    the step's random draws.  Returns (chi2 [1], accepted [1] int32) tensors."""
    ctx = ctx or context(state.device.index)
    _table(state, "state")
    for name, t in (("step", step), ("momentum", momentum)):
        _require_cuda(t, torch.float64, name)
        if t.shape != state.shape or not t.is_contiguous():
            raise ValueError(f"{name} must match state")
    _require_cuda(u, torch.float64, "u")
    chi2 = torch.empty(1, dtype=torch.float64, device=state.device)
    acc = torch.empty(1, dtype=torch.int32, device=state.device)
    L.check(ctx._lib.lens_hmc_step(ctx.handle, L.ptr(state), state.shape[1], C.byref(_obs(obs)), L.ptr(step),
                                   int(n_leapfrog), L.ptr(momentum), L.ptr(u), L.ptr(chi2), L.ptr(acc),
                                   ctx.stream()), "lens_hmc_step")
    return chi2, acc


def mh_step_batched(states: torch.Tensor, n_chains: int, grid, obs: Obs, step: torch.Tensor, noise: torch.Tensor,
                    u: torch.Tensor, chi2: torch.Tensor, prec: str = "mixed", fb_mode: int = 0,
                    fb_tau: float = 1e-6, hit_capacity: int = 1024, ctx: Context | None = None) -> torch.Tensor:
    """One Metropolis step of n_chains chains on the image-plane chi^2
    (asynchronous).  states [7, n_chains*n] and chi2 [n_chains] are updated in
    place; noise [7, n_chains*n] N(0,1), u [n_chains] U(0,1).  Returns the
    accepted flags [n_chains] int32."""
    ctx = ctx or context(states.device.index)
    _table(states, "states")
    if states.shape[1] % n_chains:
        raise ValueError("states must hold n_chains equal blocks of columns")
    n = states.shape[1] // n_chains
    _require_cuda(step, torch.float64, "step")
    _require_cuda(noise, torch.float64, "noise")
    _require_cuda(u, torch.float64, "u")
    _require_cuda(chi2, torch.float64, "chi2")
    if step.shape != (7, n) or noise.shape != states.shape or u.numel() != n_chains or chi2.numel() != n_chains:
        raise ValueError("step [7, n], noise like states, u and chi2 [n_chains]")
    acc = torch.empty(n_chains, dtype=torch.int32, device=states.device)
    opts = L.LensChi2Opts(_PREC[prec], int(fb_mode), float(fb_tau), int(hit_capacity), 0, 0)
    L.check(ctx._lib.lens_mh_step_batched(ctx.handle, L.ptr(states), int(n_chains), int(n), C.byref(_grid(grid)),
                                          C.byref(_obs(obs)), C.byref(opts), L.ptr(step.contiguous()),
                                          L.ptr(noise.contiguous()), L.ptr(u), L.ptr(chi2), L.ptr(acc),
                                          ctx.stream()), "lens_mh_step_batched")
    return acc


# ---------------------------------------------------------------- autotuning

def autotune_chi2(params: torch.Tensor, grid, obs: Obs, prec: str = "mixed", fb_mode: int = 0,
                  fb_tau: float = 1e-6, hit_capacity: int = 4096, out: Chi2Result | None = None,
                  ctx: Context | None = None, reps: int = 5):
    """Times the tile shapes / FP32 field nodes per thread on this problem and
    records the fastest in the context's table (synchronises the stream).
    Returns (tile, field_npl, out); out holds the result of the chosen configuration."""
    ctx = ctx or context(params.device.index)
    if prec not in ("fp64", "mixed"):
        raise ValueError("prec must be 'fp64' or 'mixed'")
    p, o = _pots(params), _obs(obs)
    out = out or chi2_buffers(obs, hit_capacity, params.device)
    opts = L.LensChi2Opts(_PREC[prec], int(fb_mode), float(fb_tau), int(out.hits.shape[0]), 0, 0)
    t, n = C.c_int32(), C.c_int32()
    L.check(ctx._lib.lens_autotune_chi2(ctx.handle, C.byref(p), C.byref(_grid(grid)), C.byref(o), C.byref(opts),
                                        C.byref(_chi2_out(out)), int(reps), C.byref(t), C.byref(n), ctx.stream()),
            "lens_autotune_chi2")
    return t.value, n.value, out


def autotune_chi2_batched(params: torch.Tensor, layout: BatchLayout, obs: Obs, prec: str = "mixed",
                          fb_mode: int = 0, fb_tau: float = 1e-6, hit_capacity: int = 1024,
                          out: BatchResult | None = None, ctx: Context | None = None, reps: int = 3):
    """autotune_chi2 for the batched form; returns (tile, field_npl, out)."""
    ctx = ctx or context(params.device.index)
    if prec not in ("fp64", "mixed"):
        raise ValueError("prec must be 'fp64' or 'mixed'")
    p, o = _pots(params), _obs(obs)
    out = out or batch_buffers(layout.n, obs, params.device)
    opts = L.LensChi2Opts(_PREC[prec], int(fb_mode), float(fb_tau), int(hit_capacity), 0, 0)
    t, n = C.c_int32(), C.c_int32()
    L.check(ctx._lib.lens_autotune_chi2_batched(ctx.handle, C.byref(p), layout.n, layout.pot_off, layout.grids,
                                                C.byref(o), C.byref(opts), C.byref(_batch_out(out)), int(reps),
                                                C.byref(t), C.byref(n), ctx.stream()),
            "lens_autotune_chi2_batched")
    return t.value, n.value, out


def autotune_lookup(prec: str, batched: bool, n_side: int, n_pot: int, ctx: Context | None = None):
    """The context table's (tile, field_npl) for a bucket; (0, 0) if none."""
    ctx = ctx or context()
    t, n = C.c_int32(), C.c_int32()
    L.check(ctx._lib.lens_autotune_lookup(ctx.handle, _PREC[prec], int(bool(batched)), int(n_side), int(n_pot),
                                          C.byref(t), C.byref(n)), "lens_autotune_lookup")
    return t.value, n.value


def autotune_save(path: str, ctx: Context | None = None):
    ctx = ctx or context()
    L.check(ctx._lib.lens_autotune_save(ctx.handle, os.fsencode(path)), "lens_autotune_save")


def autotune_load(path: str, ctx: Context | None = None):
    ctx = ctx or context()
    L.check(ctx._lib.lens_autotune_load(ctx.handle, os.fsencode(path)), "lens_autotune_load")


# ---------------------------------------------------------------- backward form

def lens_deflect_backward(params: torch.Tensor, grid, g_ax: torch.Tensor, g_ay: torch.Tensor, prec: str = "fp64",
                          ctx: Context | None = None, check: bool = True) -> torch.Tensor:
    """sum over nodes of g . d(alpha)/d(params): gradient [7, P] float64.  prec 'fp64',
    or 'fp32' (FP32 per-node products, FP64 accumulation)."""
    ctx = ctx or context(params.device.index)
    if prec not in ("fp64", "fp32"):
        raise ValueError("prec must be 'fp64' or 'fp32'")
    p = _pots(params)
    for name, t in (("g_ax", g_ax), ("g_ay", g_ay)):
        _require_cuda(t, torch.float64, name)
        if t.numel() != grid.nx * grid.ny:
            raise ValueError(f"{name} must have ny*nx elements")
    grad = torch.empty_like(params)
    status = torch.zeros(1, dtype=torch.int32, device=params.device)
    L.check(ctx._lib.lens_deflect_backward(ctx.handle, C.byref(p), C.byref(_grid(grid)), _PREC[prec], L.ptr(g_ax),
                                           L.ptr(g_ay), L.ptr(grad), L.ptr(status), ctx.stream()),
            "lens_deflect_backward")
    if check and int(status.item()) != L.LENS_OK:
        raise RuntimeError(f"lens_deflect_backward: invalid potential parameters (status {int(status.item())})")
    return grad


def lens_src_chi2(params: torch.Tensor, obs: Obs, ctx: Context | None = None, status: torch.Tensor | None = None):
    """Source-plane chi^2 (FP64), a [1] float64 tensor (asynchronous)."""
    ctx = ctx or context(params.device.index)
    p, o = _pots(params), _obs(obs)
    out = torch.empty(1, dtype=torch.float64, device=params.device)
    L.check(ctx._lib.lens_src_chi2(ctx.handle, C.byref(p), C.byref(o), L.ptr(out), L.ptr(status), ctx.stream()),
            "lens_src_chi2")
    return out


def lens_src_chi2_backward(params: torch.Tensor, obs: Obs, g_chi2: torch.Tensor | None = None,
                           ctx: Context | None = None, status: torch.Tensor | None = None) -> torch.Tensor:
    """g_chi2 * d(chi2_src)/d(params), [7, P] float64 (g_chi2: [1] float64 device tensor or None)."""
    ctx = ctx or context(params.device.index)
    p, o = _pots(params), _obs(obs)
    if g_chi2 is not None:
        _require_cuda(g_chi2, torch.float64, "g_chi2")
    grad = torch.empty_like(params)
    L.check(ctx._lib.lens_src_chi2_backward(ctx.handle, C.byref(p), C.byref(o), L.ptr(g_chi2), L.ptr(grad),
                                            L.ptr(status), ctx.stream()), "lens_src_chi2_backward")
    return grad


class DeflectFn(torch.autograd.Function):
    """(ax, ay) = deflection field of params [7, P] on `grid`; differentiable in params.
    prec 'fp64' (FP64 forward and backward) or 'mixed' (FP32 field, FP32 products with
    FP64 accumulation in the backward pass)."""

    @staticmethod
    def forward(fctx, params, grid, prec="fp64"):
        ax, ay = lens_deflect(params, grid, "fp64" if prec == "fp64" else "fp32")
        fctx.save_for_backward(params)
        fctx.grid, fctx.prec = grid, prec
        return ax, ay

    @staticmethod
    def backward(fctx, g_ax, g_ay):
        (params,) = fctx.saved_tensors
        z = lambda g: (torch.zeros((fctx.grid.ny, fctx.grid.nx), dtype=torch.float64, device=params.device)
                       if g is None else g.to(torch.float64).contiguous())
        grad = lens_deflect_backward(params, fctx.grid, z(g_ax), z(g_ay),
                                     "fp64" if fctx.prec == "fp64" else "fp32", check=False)
        return grad, None, None


class SrcChi2Fn(torch.autograd.Function):
    """Source-plane chi^2 of params [7, P] against `obs` (a 0-d float64 tensor)."""

    @staticmethod
    def forward(fctx, params, obs):
        fctx.save_for_backward(params)
        fctx.obs = obs
        return lens_src_chi2(params, obs).reshape(())

    @staticmethod
    def backward(fctx, g):
        (params,) = fctx.saved_tensors
        g1 = g.reshape(1).to(torch.float64).contiguous()
        return lens_src_chi2_backward(params, fctx.obs, g1), None


__all__ = ["Obs", "Context", "context", "lens_dls_dos", "lens_deflect", "lens_source_positions",
           "lens_image_chi2", "Chi2Result", "chi2_buffers", "BatchLayout", "BatchResult", "batch_buffers",
           "lens_image_chi2_batched", "lens_deflect_backward", "lens_src_chi2", "lens_src_chi2_backward",
           "DeflectFn", "SrcChi2Fn"]
