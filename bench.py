"""Throughput of the image-plane chi^2 on one MI355X.

One step = one complete chi^2 evaluation (source positions, deflection field,
triangle containment, FP64 fallback, image positions, matching, chi^2) of the
largest single-GPU workload: 1 cluster halo + 199 galaxy potentials on a
4096^2 grid over +-100", 100 multiple-image systems, inputs resident in HBM,
mixed precision (FP32 bulk, FP64 fallback / positions / chi^2), captured once
into a HIP graph and replayed.  Beside it: the FP64 path on the same workload,
the literal fallback rule |c| < 1e-6 h^2 on it, the cluster workload (50
potentials, 1024^2, 20 systems), a batch of 1024 sampler proposals (uneven
potential counts and grids, one batched call), the backward form, the
paper's own benchmark and the sampler steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.  The CPU baseline is the plain FP64 oracle on the same
workload: full evaluations on the threads of the job's CPU share, and one
thread on a band of grid rows (extrapolated to the whole grid).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "image-plane χ² evals/sec and grid triangles/s, mixed vs FP64, 1 MI355X"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector peak
FLOPS_PER_SIE = 26         # flops of one SIE pixel-potential evaluation (Algorithm 1, cos/sin hoisted)
# The paper's runtimes for its benchmark (Table 2): seconds, (double precision, mixed precision)
PAPER_TABLE2_S = {"Xeon E5-2680 v3, 12 cores": (8.1, 7.40), "GTX 1080 Ti (+Xeon)": (6.8, 1.58),
                  "P100 (+Xeon)": (0.71, 0.58), "V100 (+Xeon)": (0.46, 0.39)}
FLOPS_PER_EVAL = 34        # flops of one cored/cut pixel-potential evaluation, counted on the formula
                           # (+,-,x = 1, fma = 2, sqrt = 1, div = 1): translate 2, rotate 6, R^2 5,
                           # two square roots 4, f 5, lens-frame gradient 4, rotate back + sum 8
FLOPS_PER_VJP = 78         # flops of one cored/cut (node, potential) term of the deflection VJP in its factored
                           # form (seven node sums, per-potential constants applied once), counted as above:
                           # m and R^2 9, square roots 4, reciprocals 1/(A_ B_ S), 1/qa, 1/qs and f 13,
                           # F' 11, df/da, df/ds 4, g.m and F'(g.m) 5, the seven sums 32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_field32_large.txt")
# FP32 field layout (lens_chi2_opts.field_npl) and triangle tile shape of the timed calls: the
# library's defaults for each grid size, passed explicitly so that the profiled variant is the timed one
HEADLINE_FIELD = 0x41     # 1 column x 4 rows of nodes per thread
HEADLINE_TILE = 1         # 32 x 8 cells
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1902_03252_amd", "csrc", f)
                  for f in ("lens_kernels.hip", "lens_path.hpp", "lens_device.hpp")]


def load_workload(config: int):
    import synthlens as S
    d = np.load(os.path.join(ROOT, "tests", "golden", f"config{config}_inputs.npz"))
    x0, y0, h, nx, ny = d["grid"]
    grid = S.Grid(float(x0), float(y0), float(h), int(nx), int(ny))
    obs = dict(sys_off=d["sys_off"].astype(np.int32), x=d["x"], y=d["y"], sigma=d["sigma"], dls=d["dls"])
    return d["params"], grid, obs


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch(npl: int):
    """HBM bytes per launch of the field kernel from the committed rocprofv3 PMC
    summary, or None when it was taken on a different kernel source or nodes
    per thread."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash() or kv.get("field_npl") != hex(npl):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_kernels(torch, ctx, fn, steps, warmup):
    """Wall time per call of `steps` calls after `warmup` untimed ones, and the
    library's event-timed kernel milliseconds and launch count of the timed
    calls only."""
    ctx.set_timing(True)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.field_timing(reset=True)
    dt = time_steps(torch, fn, steps, 0)
    kms, nl = ctx.field_timing(reset=True)
    ctx.set_timing(False)
    return dt, kms, nl


def time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def autotune(args, lens, ctx, prec, batched, grid, n_pot, tune):
    """Tunes a bucket the context's table does not hold yet (with --autotune);
    returns the (tile, field_npl) the timed calls use, (0, 0) for the defaults."""
    side = max(grid.nx, grid.ny)
    if args.autotune and lens.autotune_lookup(prec, batched, side, n_pot, ctx=ctx) == (0, 0):
        tune()
    return lens.autotune_lookup(prec, batched, side, n_pot, ctx=ctx)


def chi2_leg(torch, lens, ctx, p, grid, obs, prec, steps, warmup, **kw):
    """W untimed and K timed eager calls with the field kernel bracketed by HIP
    events on the call's stream (the kernel average covers the K timed calls),
    then the same call captured once into a HIP graph and K replays."""
    out = lens.chi2_buffers(obs, 4096, "cuda")
    step = lambda: lens.lens_image_chi2(p, grid, obs, prec=prec, out=out, ctx=ctx, **kw)
    eager_s, kern_ms, launches = timed_kernels(torch, ctx, step, steps, warmup)
    eager = out.host()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    graph_s = time_steps(torch, g.replay, steps, warmup)
    replay = out.host()
    same = (replay["chi2"] == eager["chi2"] and np.array_equal(replay["hit_tid"], eager["hit_tid"])
            and np.array_equal(replay["hit_x"], eager["hit_x"]))
    del g
    return dict(eager_s=eager_s, graph_s=graph_s, kern_ms=kern_ms / max(launches, 1), launches=launches,
                result=eager, graph_matches_eager=bool(same))


def gpu_bench(args):
    import torch
    import paper_1902_03252_amd as lens

    ctx = lens.context(0)
    if args.tune_cache and os.path.exists(args.tune_cache):
        lens.autotune_load(args.tune_cache, ctx=ctx)
    tuned = {}
    # headline: the 4096^2 / 200-potential / 100-system workload
    prm, grid, obs_np = load_workload(3)
    p = torch.as_tensor(prm, dtype=torch.float64, device="cuda")
    obs = lens.Obs.from_numpy(obs_np)
    res = {}
    for prec in ("mixed", "fp64"):
        kw = dict(tile=HEADLINE_TILE, field_npl=HEADLINE_FIELD if prec == "mixed" else 0)
        res[prec] = chi2_leg(torch, lens, ctx, p, grid, obs, prec, args.steps, args.warmup, **kw)
    # the literal fallback rule on the same workload (reported; compared with the oracle below)
    out = lens.chi2_buffers(obs, 4096, "cuda")
    lens.lens_image_chi2(p, grid, obs, prec="mixed", fb_mode=1, fb_tau=1e-6, out=out, ctx=ctx,
                         tile=HEADLINE_TILE, field_npl=HEADLINE_FIELD)
    torch.cuda.synchronize()
    res["literal"] = out.host()
    # the cluster workload
    cluster = {}
    prm2, grid2, obs2_np = load_workload(2)
    p2 = torch.as_tensor(prm2, dtype=torch.float64, device="cuda")
    obs2 = lens.Obs.from_numpy(obs2_np)
    for prec in ("mixed", "fp64"):
        if args.autotune:
            tuned[f"cluster_{prec}"] = autotune(
                args, lens, ctx, prec, False, grid2, prm2.shape[1],
                lambda: lens.autotune_chi2(p2, grid2, obs2, prec=prec, out=lens.chi2_buffers(obs2, 4096, "cuda"),
                                           ctx=ctx, reps=5))
        cluster[prec] = chi2_leg(torch, lens, ctx, p2, grid2, obs2, prec, 10 * args.steps, args.warmup)
    batched = batched_bench(torch, lens, ctx, obs2, obs2_np, args, tuned) if args.batch > 0 else None
    paper = paper_bench(torch, lens, ctx, args) if args.paper else None
    sampler = sampler_bench(torch, lens, ctx, args) if args.sampler else None
    precision = precision_bench(torch, lens, ctx, args) if args.paper else None
    backward = backward_bench(torch, lens, ctx, obs2, args) if args.backward else None
    if args.tune_cache:
        lens.autotune_save(args.tune_cache, ctx=ctx)
    return (prm, grid, obs_np, res, (prm2, grid2, obs2_np, cluster), batched, backward, tuned, paper, sampler,
            precision)


def paper_bench(torch, lens, ctx, args):
    """The paper's own benchmark (Sec. 4, Table 2): grad Psi at every pixel of a
    6730^2 HST ACS image (0.03 arcsec pixels) for 2 cluster-scale + 700
    galaxy-scale SIE halos: the paper's mixed-precision gradient (FP32, FP64
    blocks of 400^2 / 20^2 pixels, FP64 where the criteria of Sec. 3.3 hold),
    and the pure FP64 and FP32 gradients, beside the paper's runtimes."""
    import synthlens as S
    grid = S.paper_grid()
    prm = S.paper_sie_cluster(grid)
    p = torch.as_tensor(prm, dtype=torch.float64, device="cuda")
    evals = float(grid.nx * grid.ny * prm.shape[1])
    out = lens.mixed_buffers(grid, "cuda")
    legs = {"mixed": lambda: lens.lens_deflect_mixed(p, grid, 2, out=out, ctx=ctx),
            "fp64": lambda: lens.lens_deflect(p, grid, "fp64", ctx=ctx, check=False),
            "fp32": lambda: lens.lens_deflect(p, grid, "fp32", ctx=ctx, check=False)}
    res = {}
    for name, step in legs.items():
        dt, kms, nl = timed_kernels(torch, ctx, step, 5, 2)
        res[name] = dict(ms=dt * 1e3, pixel_potential_evals_per_s=evals / dt,
                         field_kernel_ms=kms / max(nl, 1))
    st = out.stats.cpu().numpy()
    assert st[3] == 0
    n = grid.nx * grid.ny
    res["mixed"].update(fp64_block_px=int(st[0]), fp64_criteria_px=int(st[1]), fp64_fraction=float(st[2]) / n)
    res["fp32"]["field_tflops"] = FLOPS_PER_SIE * evals / (res["fp32"]["field_kernel_ms"] / 1e3) / 1e12
    res["fp64"]["field_tflops"] = FLOPS_PER_SIE * evals / (res["fp64"]["field_kernel_ms"] / 1e3) / 1e12
    res["paper_table2_s"] = {k: {"dp": v[0], "mixed": v[1]} for k, v in PAPER_TABLE2_S.items()}
    v100_dp, v100_mixed = PAPER_TABLE2_S["V100 (+Xeon)"]
    res["speedup_vs_v100"] = {"mixed": v100_mixed / (res["mixed"]["ms"] / 1e3),
                              "fp64": v100_dp / (res["fp64"]["ms"] / 1e3)}
    res["workload"] = (f"{grid.nx}^2 pixels of {grid.h} arcsec, 2 + {prm.shape[1] - 2} SIE halos, "
                       f"{evals:.3e} pixel-potential evaluations (Sec. 4); other hardware's times are context")
    return res


def sp_safe(torch, a32, a64, h):
    """FP32 error against FP64 and the share of pixels where single precision
    is accurate enough: |error_i| <= 7.5e-3" / M_i (a quarter pixel of 0.03"
    over the magnification along axis i, Sec. 3.2), with M_i = dx / |dx - d_i|
    from the FP64 field (d_1, d_2 the differences of Sec. 3.3)."""
    ex = (a32[0].double() - a64[0]).abs()
    ey = (a32[1].double() - a64[1]).abs()
    d1 = torch.zeros_like(a64[0])
    d2 = torch.zeros_like(a64[1])
    d1[:, 1:] = a64[0][:, 1:] - a64[0][:, :-1]
    d2[1:, :] = a64[1][1:, :] - a64[1][:-1, :]
    ok = (ex <= 7.5e-3 * (h - d1).abs() / h) & (ey <= 7.5e-3 * (h - d2).abs() / h)
    e = torch.maximum(ex, ey)
    return dict(fp32_max_err_arcsec=float(e.max()), frac_within_2p3e_3=float((e <= 2.3e-3).double().mean()),
                frac_sp_safe_with_magnification=float(ok.double().mean()))


def precision_bench(torch, lens, ctx, args):
    """The precision study the paper asks for beyond the SIE (Sec. 5): on the
    benchmark image (6730^2 pixels of 0.03"), the FP32 field against the FP64
    field for the SIE cluster (2 + 700 halos) and for the same cluster of
    pseudo-elliptical NFW halos, with the FP32 / FP64 field times."""
    import synthlens as S
    grid = S.paper_grid()
    out = {}
    for name, prm, fn in (("sie", S.paper_sie_cluster(grid), lens.lens_deflect),
                          ("nfw", S.nfw_cluster(grid), lens.lens_deflect_nfw)):
        p = torch.as_tensor(prm, dtype=torch.float64, device="cuda")
        res = {}
        fields = {}
        for prec in ("fp32", "fp64"):
            dt, kms, nl = timed_kernels(torch, ctx, lambda: fn(p, grid, prec, ctx=ctx, check=False), 3, 1)
            fields[prec] = fn(p, grid, prec, ctx=ctx)
            res[f"{prec}_ms"] = dt * 1e3
            res[f"{prec}_field_kernel_ms"] = kms / max(nl, 1)
        res.update(sp_safe(torch, fields["fp32"], fields["fp64"], grid.h))
        res["halos"] = int(prm.shape[1])
        out[name] = res
        del fields
    out["workload"] = f"{grid.nx}^2 pixels of {grid.h} arcsec; SIE and NFW clusters of 2 + 700 halos"
    return out


def sampler_bench(torch, lens, ctx, args):
    """Sampler steps on the cluster model (50 potentials, 20 systems): HMC with
    10 leapfrog steps on the source-plane chi^2 (free: the halo's centre,
    eps, phi, core and sigma_v, every galaxy's sigma_v), graph-replayed; and one
    random-walk Metropolis step of 256 chains on the 512^2 grid (one batched
    mixed chi^2 of all proposals per step)."""
    import synthlens as S
    prm, _, obs_np = load_workload(2)
    obs = lens.Obs.from_numpy(obs_np)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    st = np.zeros_like(prm)
    st[0, 0] = st[1, 0] = 2e-3
    st[2, 0], st[3, 0], st[4, 0], st[6, 0] = 2e-4, 2e-3, 2e-3, 0.5
    st[6, 1:] = 0.2
    state, step = dev(prm), dev(st)
    mom = torch.randn(prm.shape, dtype=torch.float64, device="cuda")
    u = torch.rand(1, dtype=torch.float64, device="cuda")
    L = 10
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lens.hmc_step(state.clone(), obs, step, L, mom, u, ctx=ctx)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        _, acc = lens.hmc_step(state, obs, step, L, mom, u, ctx=ctx)
    n_acc = torch.zeros(1, dtype=torch.int64, device="cuda")

    def hmc():
        mom.normal_()
        u.uniform_()
        graph.replay()
        n_acc.add_(acc)

    dt = time_steps(torch, hmc, 50, 5)
    hmc_res = dict(ms_per_step=dt * 1e3, leapfrog_steps_per_s=L / dt, acceptance=float(n_acc.item()) / 55,
                   free_parameters=int((st != 0).sum()), n_leapfrog=L)
    del graph
    B, n = 256, prm.shape[1]
    grid = S.WORKLOADS[5].grid
    states = dev(np.tile(prm, (1, B)))
    layout = lens.BatchLayout([b * n for b in range(B + 1)], [grid] * B)
    chi2 = lens.lens_image_chi2_batched(states, layout, obs, ctx=ctx).chi2.clone()
    mh_st = dev(st * 0.5)
    noise = torch.empty_like(states)
    uu = torch.empty(B, dtype=torch.float64, device="cuda")
    accs = []

    def mh():
        noise.normal_()
        uu.uniform_()
        accs.append(lens.mh_step_batched(states, B, grid, obs, mh_st, noise, uu, chi2, ctx=ctx))

    dt = time_steps(torch, mh, 5, 1)
    rate = float(torch.stack(accs).double().mean().item())
    mh_res = dict(chains=B, ms_per_step=dt * 1e3, chain_steps_per_s=B / dt, acceptance=rate,
                  grid=f"{grid.nx}x{grid.ny}", precision="mixed")
    return {"hmc_source_plane": hmc_res, "metropolis_image_plane": mh_res}


def backward_bench(torch, lens, ctx, obs, args):
    """Differentiation workload: the 50 cluster potentials on a 512^2 grid over
    +-80", N(0,1) cotangent; deflection VJP (FP64 and FP32 products) and the
    source-plane chi^2 gradient of the 20 systems."""
    import synthlens as S
    w = S.WORKLOADS[5]
    grid = w.grid
    prm = S.potentials(5)
    cot = S.cotangent(grid.nx * grid.ny)
    p = torch.as_tensor(prm, dtype=torch.float64, device="cuda")
    gx = torch.as_tensor(cot[0], dtype=torch.float64, device="cuda")
    gy = torch.as_tensor(cot[1], dtype=torch.float64, device="cuda")
    flops = FLOPS_PER_VJP * float(grid.nx * grid.ny * prm.shape[1])
    out = {"workload": f"{prm.shape[1]} potentials, {grid.nx}^2 grid, 7 parameters each, N(0,1) cotangent"}
    for prec in ("fp64", "fp32"):
        step = lambda: lens.lens_deflect_backward(p, grid, gx, gy, prec, ctx=ctx, check=False)
        dt, kms, nl = timed_kernels(torch, ctx, step, 20, 3)
        kern_s = kms / 1e3 / max(nl, 1)
        peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
        out[prec] = dict(ms_per_vjp=dt * 1e3, vjp_kernel_ms=kern_s * 1e3, tflops=flops / kern_s / 1e12,
                         frac_of_peak=flops / kern_s / 1e12 / peak)
    dt = time_steps(torch, lambda: lens.lens_src_chi2_backward(p, obs, ctx=ctx), 20, 3)
    out["src_chi2_grad_ms"] = dt * 1e3
    return out


def batched_bench(torch, lens, ctx, obs, obs_np, args, tuned):
    """A sampler's batch: n lens models with P ~ U{10..200} potentials and grid
    sides drawn from {256, 512, 1024, 2048} over +-80", evaluated by one batched
    call, captured into a HIP graph and replayed."""
    import synthlens as S
    params, pot_off, grids = S.batch_samples(args.batch)
    p = torch.as_tensor(params, dtype=torch.float64, device="cuda")
    layout = lens.BatchLayout(pot_off, grids)
    nodes = np.array([g.nx * g.ny for g in grids], dtype=np.float64)
    n_pot = np.diff(pot_off).astype(np.float64)
    tri = float(sum(g.n_triangles for g in grids))
    flops = FLOPS_PER_EVAL * float((nodes * n_pot).sum())
    out_res = {}
    for prec in ("mixed", "fp64"):
        out = lens.batch_buffers(layout.n, obs, "cuda")
        side = max(max(g.nx, g.ny) for g in grids)
        tuned[f"batched_{prec}"] = autotune(args, lens, ctx, prec, True, S.Grid(0.0, 0.0, 1.0, side, side),
                                            -(-params.shape[1] // len(grids)),
                                            lambda: lens.autotune_chi2_batched(p, layout, obs, prec=prec, out=out,
                                                                               ctx=ctx, reps=2))
        step = lambda: lens.lens_image_chi2_batched(p, layout, obs, prec=prec, out=out, ctx=ctx)
        step()  # builds and caches the plan
        torch.cuda.synchronize()
        eager_s, kms, nl = timed_kernels(torch, ctx, step, 3, 1)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        dt = time_steps(torch, g.replay, args.batch_steps, 1)
        st = out.stats.cpu().numpy()
        status = out.status.cpu().numpy()
        field_s = kms / 1e3 / 3.0  # field kernels of one batch (3 timed calls)
        peak = PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
        out_res[prec] = dict(chi2_evals_per_s=args.batch / dt, ms_per_batch=dt * 1e3,
                             eager_ms_per_batch=eager_s * 1e3, grid_triangles_per_s=tri / dt,
                             field_ms_per_batch=field_s * 1e3, field_tflops=flops / field_s / 1e12,
                             field_frac_of_peak=flops / field_s / 1e12 / peak,
                             samples_ok=int((status == 0).sum()), hits=int(st[0]), flagged_tests=int(st[1]),
                             fallback_rate=float(st[1]) / float(st[6]))
        del g
    out_res["speedup_mixed_vs_fp64"] = out_res["fp64"]["ms_per_batch"] / out_res["mixed"]["ms_per_batch"]
    out_res["workload"] = (f"{args.batch} samples, P ~ U{{10..200}} (mean {n_pot.mean():.1f}), grid sides "
                           f"{{256, 512, 1024, 2048}}, {nodes.sum() / 1e9:.2f} G nodes, 20 systems")
    return out_res


def cpu_threads() -> int:
    """Threads of the CPU baseline: the CPUs this process may run on, at most 16
    (the host's CPU share of a one-GPU job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(prm, grid, obs_np, budget_s: float, band_rows: int):
    """The FP64 oracle on the headline workload: complete chi^2 evaluations on
    cpu_threads() threads until budget_s has passed (at least one), and one
    thread on a band of band_rows grid rows -- its deflection field and triangle
    stage, the two parts whose work scales with the grid -- extrapolated
    linearly to the grid's triangles."""
    import oracle
    import synthlens as S
    threads = cpu_threads()
    t0 = time.perf_counter()
    n = 0
    want = None
    while True:
        want = oracle.image_chi2(prm, grid, obs_np, nthreads=threads)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    j0 = (grid.ny - band_rows) // 2
    band = S.Grid(grid.x0, grid.y0 + j0 * grid.h, grid.h, grid.nx, band_rows)
    t1 = time.perf_counter()
    ax, ay = oracle.alpha_grid(prm, band, nthreads=1)
    oracle.hits_from_field(ax, ay, band, want["bar_x"], want["bar_y"], obs_np["dls"], nthreads=1)
    t_band = time.perf_counter() - t1
    t_one = t_band * (grid.ny - 1) / (band_rows - 1)
    base = dict(value=n / dt, unit="chi2 evals/s", cores=threads, kind="oracle",
                sample=(f"{n} full chi^2 evaluations of the 4096^2 / 200-potential / 100-system workload "
                        f"(FP64, {threads} threads, {dt:.1f} s)"),
                one_core=dict(value=1.0 / t_one, unit="chi2 evals/s", cores=1,
                              sample=(f"deflection field and triangle stage of a band of {band_rows} of the "
                                      f"{grid.ny} grid rows on one thread ({t_band:.1f} s), extrapolated to the "
                                      f"grid's {grid.ny - 1} cell rows")),
                host_cpus=os.cpu_count())
    return base, want


def cpu_extras(obs2_np, batch: int, batch_samples: int):
    """The FP64 oracle on the batched and backward legs' workloads, as context
    beside the GPU figures: chi^2 of batch_samples evenly spaced samples of the
    batch on cpu_threads() threads, extrapolated to the whole batch in
    proportion to sum N^2 P, and one deflection VJP of the differentiation
    workload (512^2 grid, 50 potentials) on the same threads."""
    import oracle
    import synthlens as S
    threads = cpu_threads()
    out = {}
    if batch > 0 and batch_samples > 0:
        params, pot_off, grids = S.batch_samples(batch)
        cost = np.array([g.nx * g.ny for g in grids], dtype=np.float64) * np.diff(pot_off)
        step = max(1, batch // batch_samples)
        idx = list(range(0, batch, step))[:batch_samples]
        t0 = time.perf_counter()
        for s in idx:
            oracle.image_chi2(params[:, pot_off[s]:pot_off[s + 1]], grids[s], obs2_np, nthreads=threads)
        dt = time.perf_counter() - t0
        t_batch = dt * cost.sum() / cost[idx].sum()
        out["batched"] = dict(value=batch / t_batch, unit="chi2 evals/s", cores=threads, kind="oracle",
                              sample=(f"{len(idx)} of the {batch} samples (every {step}th, {dt:.1f} s), "
                                      f"extrapolated to the batch in proportion to sum N^2 P"))
    w = S.WORKLOADS[5]
    cot = S.cotangent(w.grid.nx * w.grid.ny)
    prm5 = S.potentials(5)
    t0 = time.perf_counter()
    oracle.alpha_vjp(prm5, w.grid, cot[0].reshape(w.grid.ny, w.grid.nx), cot[1].reshape(w.grid.ny, w.grid.nx),
                     nthreads=threads)
    dt = time.perf_counter() - t0
    out["backward"] = dict(value=1.0 / dt, unit="deflection VJPs/s", cores=threads, kind="oracle",
                           sample=f"one VJP of the 512^2 / 50-potential workload ({dt:.2f} s)")
    return out


def hit_set(r):
    return set(zip(np.asarray(r["hit_sys"]).tolist(), np.asarray(r["hit_tid"]).tolist()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed calls before each timed loop (the first ~10 launches of the 4096^2 step run "
                         "slower while the device clock rises)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="seconds of full oracle evaluations for the baseline (at least one)")
    ap.add_argument("--cpu-band", type=int, default=48, help="grid rows of the one-thread oracle sample")
    ap.add_argument("--cpu-batch-samples", type=int, default=8,
                    help="batch samples the oracle evaluates for its batched figure (0 skips it)")
    ap.add_argument("--batch", type=int, default=1024, help="samples of the batched leg (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=5, help="timed replays of the batched leg")
    ap.add_argument("--no-backward", dest="backward", action="store_false", help="skip the backward leg")
    ap.add_argument("--no-sampler", dest="sampler", action="store_false", help="skip the sampler-step leg")
    ap.add_argument("--no-paper", dest="paper", action="store_false",
                    help="skip the paper's own benchmark (6730^2 SIE gradient, mixed / FP64 / FP32)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the cluster and batched legs' tile shape / field layout (the headline always "
                         "runs the library's default for its size, passed explicitly)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune table (JSON) merged before tuning and written at the end; buckets it holds "
                         "are not tuned again")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device-to-device 3 times (a known-size kernel that calibrates the "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this path has no multi-GPU form); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    (prm, grid, obs_np, res, (prm2, grid2, obs2_np, cluster), batched, backward, tuned, paper, sampler,
     precision) = gpu_bench(args)
    mixed, fp64 = res["mixed"], res["fp64"]
    step_s = mixed["graph_s"]
    n_tri = grid.n_triangles
    evals = grid.nx * grid.ny * prm.shape[1]
    flops = FLOPS_PER_EVAL * evals
    kern_s = mixed["kern_ms"] / 1e3
    achieved = flops / kern_s / 1e12
    traffic = traffic_per_launch(HEADLINE_FIELD)

    cpu, want = (None, None) if args.no_cpu else cpu_baseline(prm, grid, obs_np, args.cpu_budget, args.cpu_band)
    if cpu is not None:
        cpu.update(cpu_extras(obs2_np, args.batch, args.cpu_batch_samples))
    parity = None
    lit = res["literal"]
    literal = {"rule": "FP64 fallback when |c_k| < 1e-6 h^2 (FP32 sign taken otherwise)",
               "flagged_tests": int(lit["stats"][1]), "tests": int(lit["stats"][6]),
               "rate": float(lit["stats"][1]) / float(lit["stats"][6]), "fallback_hits": int(lit["stats"][5]),
               "hits": int(lit["stats"][0]), "status": int(lit["status"])}
    if want is not None:
        got = mixed["result"]
        parity = dict(hit_set_equal_to_oracle=hit_set(got) == hit_set(want),
                      chi2_rel_err=abs(got["chi2"] - want["chi2"]) / abs(want["chi2"]),
                      max_position_err_arcsec=float(max(np.abs(got["hit_x"] - want["hit_x"]).max(),
                                                        np.abs(got["hit_y"] - want["hit_y"]).max()))
                      if hit_set(got) == hit_set(want) else None,
                      fp64_hit_set_equal_to_oracle=hit_set(fp64["result"]) == hit_set(want),
                      fp64_chi2_rel_err=abs(fp64["result"]["chi2"] - want["chi2"]) / abs(want["chi2"]))
        literal["hit_set_mismatches_vs_oracle"] = len(hit_set(lit) ^ hit_set(want))

    st = mixed["result"]["stats"]
    n_tri2 = grid2.n_triangles
    flops2 = FLOPS_PER_EVAL * grid2.nx * grid2.ny * prm2.shape[1]
    cm, cf = cluster["mixed"], cluster["fp64"]
    line = {
        "metric": METRIC,
        "value": 1.0 / step_s,
        "unit": "chi2 evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "large cluster: 1 halo + 199 galaxy potentials, 4096^2 grid over +-100 arcsec, "
                               "100 multiple-image systems",
                   "grid": f"{grid.nx}x{grid.ny}", "potentials": int(prm.shape[1]), "systems": len(obs_np["dls"]),
                   "precision": "mixed (FP32 bulk, FP64 fallback/positions/chi2)",
                   "mode": "HIP graph replay of one evaluation",
                   "field_layout": f"{HEADLINE_FIELD:#x} (1 column x 4 rows of nodes per thread)",
                   "tile": "32x8 cells"},
        "grid_triangles_per_s": n_tri / step_s,
        "triangle_source_tests_per_s": float(st[6]) / step_s,
        "pixel_potential_evals_per_s": evals / step_s,
        "eager_chi2_evals_per_s": 1.0 / mixed["eager_s"],
        "whole_step_tflops": (flops + 4 * grid.nx * grid.ny * len(obs_np["dls"])) / step_s / 1e12,
        "fp64": {"chi2_evals_per_s": 1.0 / fp64["graph_s"], "ms_per_eval": fp64["graph_s"] * 1e3,
                 "eager_chi2_evals_per_s": 1.0 / fp64["eager_s"],
                 "grid_triangles_per_s": n_tri / fp64["graph_s"], "field_kernel_ms": fp64["kern_ms"],
                 "field_frac_of_fp64_peak": flops / (fp64["kern_ms"] / 1e3) / 1e12 / PEAK_FP64_TFLOPS},
        "speedup_mixed_vs_fp64": fp64["graph_s"] / step_s,
        "graph_replay_matches_eager": mixed["graph_matches_eager"] and fp64["graph_matches_eager"],
        "fallback": {"flagged_tests": int(st[1]), "tests": int(st[6]), "rate": float(st[1]) / float(st[6]),
                     "fallback_hits": int(st[5]), "hits": int(st[0])},
        "literal": literal,
        "roofline": {"bound": "alu", "kernel": f"k_field32h<1,4> (FP32 deflection field, 1 x 4 nodes per thread; "
                                                  f"its first workgroups run the head's source-plane part)",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "flops_per_launch": flops, "avg_launch_ms": mixed["kern_ms"], "launches_timed": mixed["launches"]},
        "cluster": {"workload": "1 halo + 49 galaxy potentials, 1024^2 grid over +-80 arcsec, 20 systems",
                    "mixed": {"chi2_evals_per_s": 1.0 / cm["graph_s"], "ms_per_eval": cm["graph_s"] * 1e3,
                              "eager_chi2_evals_per_s": 1.0 / cm["eager_s"],
                              "grid_triangles_per_s": n_tri2 / cm["graph_s"], "field_kernel_ms": cm["kern_ms"],
                              "field_frac_of_peak": flops2 / (cm["kern_ms"] / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
                              "flagged_tests": int(cm["result"]["stats"][1]), "hits": int(cm["result"]["stats"][0])},
                    "fp64": {"chi2_evals_per_s": 1.0 / cf["graph_s"], "ms_per_eval": cf["graph_s"] * 1e3,
                             "grid_triangles_per_s": n_tri2 / cf["graph_s"], "field_kernel_ms": cf["kern_ms"],
                             "field_frac_of_fp64_peak": flops2 / (cf["kern_ms"] / 1e3) / 1e12 / PEAK_FP64_TFLOPS},
                    "speedup_mixed_vs_fp64": cf["graph_s"] / cm["graph_s"],
                    "graph_replay_matches_eager": cm["graph_matches_eager"] and cf["graph_matches_eager"]},
        "batched": batched,
        "backward": backward,
        "paper_benchmark": paper,
        "sampler": sampler,
        "precision_study": precision,
        "autotuned": {k: {"tile": t, "field_npl": n} for k, (t, n) in tuned.items() if t} or None,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
