"""Write the stored inputs of the chi^2 workloads (tests/golden/config{k}_inputs.npz).

Calls only the seeded draws of ``synthlens`` and the CPU oracle: the observed
multiple images of each system are images the oracle solves for (triangle hits
on a search grid, refined by Newton's method on the lens equation), plus
Gaussian noise of 0.1 arcsec per coordinate; D_LS/D_OS comes from the oracle's
flat LambdaCDM quadrature.  Nothing here comes from the GPU library.

    python tests/golden/make_inputs.py [config ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthlens as S  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def solve_images(prm, r, beta, field, search, half_width):
    """Every image the oracle's triangle test finds on the search grid, refined by Newton."""
    ax, ay = field
    hs, ht = oracle.hits_from_field(ax, ay, search, [beta[0]], [beta[1]], [r])
    hx, hy = oracle.positions_from_field(ax, ay, search, hs, ht, [beta[0]], [beta[1]], [r])
    roots = []
    for x, y in zip(hx, hy):
        root = oracle.newton(prm, r, beta, (x, y), maxit=100, tol=1e-11)
        if root is None:
            continue
        if abs(root[0]) > half_width or abs(root[1]) > half_width:
            continue
        if any(np.hypot(root[0] - q[0], root[1] - q[1]) < 1e-6 for q in roots):
            continue
        roots.append(root)
    return np.asarray(roots).reshape(-1, 2)


def make(config: int):
    wl = S.WORKLOADS[config]
    prm = S.potentials(config)
    grid = wl.grid
    search = grid if grid.nx <= 2048 else S.square_grid(2048, wl.half_width)
    t0 = time.time()
    field = oracle.alpha_grid(prm, search)
    g_src, g_noise = S.rng(config, 2), S.rng(config, 3)
    zs, betas, images = [], [], []
    for s in range(wl.n_sources):
        for attempt in range(10000):
            z = wl.z_sources[s] if wl.z_sources else float(S.source_redshifts(g_src, 1)[0])
            r = oracle.dls_dos(S.Z_LENS, z)
            beta = S.disk_points(g_src, 1, wl.source_radius)[0]
            imgs = solve_images(prm, r, beta, field, search, wl.half_width)
            if wl.min_images <= len(imgs) <= wl.max_images:
                break
        else:
            raise RuntimeError(f"config {config}: no source with {wl.min_images}-{wl.max_images} images")
        zs.append(z)
        betas.append(beta)
        images.append(imgs)
    sys_off = np.zeros(len(images) + 1, np.int32)
    sys_off[1:] = np.cumsum([len(i) for i in images])
    true_xy = np.concatenate(images, axis=0)
    obs_xy = true_xy + S.position_noise(g_noise, len(true_xy))
    zs = np.asarray(zs)
    dls = np.array([oracle.dls_dos(S.Z_LENS, z) for z in zs])
    path = os.path.join(OUT, f"config{config}_inputs.npz")
    np.savez(path, params=prm, grid=np.array([grid.x0, grid.y0, grid.h, grid.nx, grid.ny]),
             z_lens=S.Z_LENS, z_src=zs, dls=dls, beta_true=np.asarray(betas), sys_off=sys_off,
             x=obs_xy[:, 0].copy(), y=obs_xy[:, 1].copy(), sigma=np.full(len(obs_xy), S.OBS_SIGMA),
             img_true=true_xy)
    print(f"config {config}: {len(images)} systems, {len(true_xy)} images, "
          f"{time.time() - t0:.1f}s -> {os.path.relpath(path, ROOT)}")


if __name__ == "__main__":
    cfgs = [int(a) for a in sys.argv[1:]] or [1, 2, 3]
    for c in cfgs:
        make(c)
