"""The entry point that allocates nothing (lens_image_chi2_noalloc, fixed
device scratch) against lens_image_chi2 on the same inputs: identical outputs,
on consecutive calls whose second input is smaller than the first, in both
precisions, under graph replay, and a clear error for an input beyond the
fixed scratch."""
import ctypes as C

import numpy as np
import pytest

from conftest import load_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("chi2", "chi2_sys", "n_pred", "hits", "img_xy", "match", "stats")


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1902_03252_amd as lens
    return lens


def _inputs(lens, config):
    prm, grid, obs_np = load_inputs(config)
    return torch.as_tensor(prm, dtype=torch.float64, device="cuda"), grid, lens.Obs.from_numpy(obs_np), obs_np


def _host(out):
    """Every output, the hit list and positions trimmed to the hits found (the
    rows beyond are not written)."""
    torch.cuda.synchronize()
    h = {k: getattr(out, k).cpu().numpy().copy() for k in KEYS}
    n = int(h["stats"][0]) if h["stats"][4] == 0 else 0
    h["hits"], h["img_xy"] = h["hits"][:n], h["img_xy"][:n]
    return h


def _same(a, b, what):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{what}: {k}")


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_matches_context_entry_point_on_consecutive_calls(lens, prec):
    """Large input first, then a smaller one: the second call's buffers sit at
    other offsets of the fixed array over the first call's leftovers."""
    for config in (2, 1):
        p, grid, obs, obs_np = _inputs(lens, config)
        want = _host(lens.lens_image_chi2(p, grid, obs, prec=prec))
        got = _host(lens.lens_image_chi2_noalloc(p, grid, obs, prec=prec))
        print(f"noalloc {prec} config {config}: chi2 {got['chi2'][0]:.9g} hits {got['stats'][0]}", flush=True)
        assert got["stats"][4] == 0
        _same(got, want, f"{prec} config {config}")


def test_noalloc_full_size_workload_both_precisions(lens):
    """The 4096^2 / 200-potential / 100-system workload fits the fixed scratch
    in either precision; mixed, then FP64, then mixed again."""
    p, grid, obs, _ = _inputs(lens, 3)
    for prec in ("mixed", "fp64", "mixed"):
        want = _host(lens.lens_image_chi2(p, grid, obs, prec=prec))
        got = _host(lens.lens_image_chi2_noalloc(p, grid, obs, prec=prec))
        print(f"noalloc {prec} 4096^2: chi2 {got['chi2'][0]:.9g} hits {got['stats'][0]}", flush=True)
        _same(got, want, f"{prec} 4096^2")


def test_noalloc_graph_replay(lens):
    """Captured into a graph and replayed with unrelated eager calls (other
    inputs, the same fixed scratch) between the replays."""
    p, grid, obs, _ = _inputs(lens, 2)
    p1, grid1, obs1, _ = _inputs(lens, 1)
    out = lens.chi2_buffers(obs, 4096, "cuda")
    want = _host(lens.lens_image_chi2(p, grid, obs, prec="mixed"))
    lens.lens_image_chi2_noalloc(p, grid, obs, prec="mixed", out=out)  # first call outside capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lens.lens_image_chi2_noalloc(p, grid, obs, prec="mixed", out=out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lens.lens_image_chi2_noalloc(p, grid, obs, prec="mixed", out=out)
    for rep in range(3):
        for k in KEYS:
            getattr(out, k).fill_(-1)
        lens.lens_image_chi2_noalloc(p1, grid1, obs1, prec="fp64")  # eager, other input
        torch.cuda.synchronize()
        g.replay()
        _same(_host(out), want, f"replay {rep}")
    del g


def test_noalloc_rejects_input_beyond_the_fixed_scratch(lens):
    """An 8192^2 FP64 evaluation needs more than the fixed scratch: the call
    returns LENS_ERR_SCRATCH before anything is enqueued, and a following call
    still works."""
    import synthlens as S
    from paper_1902_03252_amd import _lib as L
    p, grid, obs, _ = _inputs(lens, 2)
    big = S.Grid(-80.0, -80.0, 160.0 / 8191, 8192, 8192)
    with pytest.raises(RuntimeError, match="fixed no-allocation buffer"):
        lens.lens_image_chi2_noalloc(p, big, obs, prec="fp64")
    assert L.load().lens_strerror(L.LENS_ERR_SCRATCH) == b"input needs more scratch than the fixed no-allocation buffer holds"
    want = _host(lens.lens_image_chi2(p, grid, obs, prec="fp64"))
    _same(_host(lens.lens_image_chi2_noalloc(p, grid, obs, prec="fp64")), want, "after the rejected call")
