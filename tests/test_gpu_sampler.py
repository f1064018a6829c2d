"""GPU parity of the sampler steps (HMC on the source-plane chi^2, batched
random-walk Metropolis on the image-plane chi^2) against the oracle's plain
FP64 steps on the same random draws, through the C ABI.

Bars: acceptance decisions identical (draws within 1e-6 of the acceptance
threshold are re-drawn); HMC end states within 1e-7 of a step of the oracle's
(the trajectories differ only by the gradients' rounding, <= 1e-10 relative);
chi^2 within 1e-9 relative; Metropolis proposals bit-identical to the
oracle's state + step * noise (multiply and add rounded separately), so
accepted states are bit-identical and rejected states untouched."""
import math

import numpy as np
import pytest

import oracle
import synthlens as S
from conftest import load_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lens():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1902_03252_amd as lens
    lens.context()
    return lens


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def hmc_steps_table(prm, scale=1.0):
    """Step sizes: the halo's centre, ellipticity, angle, core and sigma, and
    the galaxies' sigma; r_cut and the galaxies' positions held fixed."""
    st = np.zeros_like(prm)
    st[0, 0] = st[1, 0] = 2e-3
    st[2, 0], st[3, 0], st[4, 0], st[6, 0] = 2e-4, 2e-3, 2e-3, 0.5
    st[6, 1:] = 0.2
    return st * scale


def hmc_energy_gap(prm, obs, st, L, mom):
    """H0 - H1 of the oracle trajectory (for keeping draws away from ties)."""
    e = oracle._src_energy(obs)
    free = st != 0
    q, p = prm.copy(), np.where(free, mom, 0.0)
    u0, g = e(q)
    p = p - np.where(free, 0.5 * st * g, 0.0)
    u1 = u0
    for ell in range(1, L + 1):
        q = np.where(free, q + st * p, q)
        u1, g = e(q)
        p = p - np.where(free, (1.0 if ell < L else 0.5) * st * g, 0.0)
    return (u0 + 0.5 * np.sum(np.where(free, mom, 0.0) ** 2)) - (u1 + 0.5 * np.sum(p ** 2))


@pytest.mark.parametrize("scale", [1.0, 6.0])
def test_hmc_steps_match_oracle(lens, scale):
    """Three consecutive HMC steps (L = 5) from a perturbed cluster model; in
    the large-step case the trajectories diverge (finite energy errors far
    above 1), which exercises the Metropolis rejection of valid trajectories."""
    prm, _, obs_np = load_inputs(2)
    obs = lens.Obs.from_numpy(obs_np)
    st = hmc_steps_table(prm, scale)
    g = np.random.default_rng(7)
    state_np = prm.copy()
    state_np[6] *= 1.0 + 0.01 * g.normal(size=prm.shape[1])
    state = dev(state_np)
    step = dev(st)
    decisions = []
    for k in range(3):
        mom = g.normal(size=prm.shape)
        gap = hmc_energy_gap(state_np, obs_np, st, 5, mom)
        u = g.uniform()
        while np.isfinite(gap) and abs(math.log(u) - gap) < 1e-6:
            u = g.uniform()
        want_q, want_c, want_acc = oracle.hmc_step(state_np, obs_np, st, 5, mom, u)
        chi2, acc = lens.hmc_step(state, obs, step, 5, dev(mom), dev([u]))
        got_q = state.cpu().numpy()
        got_c, got_acc = float(chi2.cpu()[0]), bool(acc.cpu()[0])
        print(f"  step {k}: accepted {got_acc} (oracle {want_acc}), dH {gap:.3e}, chi2 {got_c:.6e}", flush=True)
        assert got_acc == want_acc
        assert got_c == pytest.approx(want_c, rel=1e-9)
        assert (np.abs(got_q - want_q) <= 1e-7 * st + 1e-13 * np.abs(want_q)).all()
        decisions.append(got_acc)
        state_np = want_q
        if scale > 1.0:
            assert np.isfinite(gap)
    if scale > 1.0:
        assert not all(decisions)


def test_hmc_invalid_trajectory_rejected(lens):
    """A trajectory that leaves the model's domain (eps pushed below 0) is
    rejected: the state is unchanged and chi^2 is the start's."""
    prm, _, obs_np = load_inputs(2)
    obs = lens.Obs.from_numpy(obs_np)
    st = np.zeros_like(prm)
    st[2, 0] = 0.2
    mom = np.zeros_like(prm)
    mom[2, 0] = -5.0
    state = dev(prm)
    chi2, acc = lens.hmc_step(state, obs, dev(st), 3, dev(mom), dev([0.5]))
    want = oracle.src_chi2(prm, obs_np)
    assert not bool(acc.cpu()[0])
    assert float(chi2.cpu()[0]) == pytest.approx(want, rel=1e-12)
    assert torch.equal(state, dev(prm))


def test_hmc_step_graph_replay(lens):
    """One HMC step captured into a HIP graph and replayed with fresh draws
    copied into the captured inputs: every replay equals the eager step."""
    prm, _, obs_np = load_inputs(2)
    obs = lens.Obs.from_numpy(obs_np)
    st = dev(hmc_steps_table(prm))
    g = np.random.default_rng(3)
    state, mom, u = dev(prm), dev(np.zeros_like(prm)), dev([0.5])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lens.hmc_step(state.clone(), obs, st, 4, mom, u)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        chi2_g, acc_g = lens.hmc_step(state, obs, st, 4, mom, u)
    ref_state = dev(prm)
    for k in range(3):
        m, uu = g.normal(size=prm.shape), g.uniform()
        mom.copy_(dev(m))
        u.copy_(dev([uu]))
        graph.replay()
        torch.cuda.synchronize()
        chi2_e, acc_e = lens.hmc_step(ref_state, obs, st, 4, dev(m), dev([uu]))
        torch.cuda.synchronize()
        assert torch.equal(state, ref_state) and torch.equal(chi2_g, chi2_e) and torch.equal(acc_g, acc_e), k


def test_mh_batched_steps_match_oracle(lens):
    """12 chains of the 50-potential cluster model on a 512^2 grid, FP64 chi^2;
    chain 3's proposal leaves the domain (negative core radius) and is rejected."""
    prm, _, obs_np = load_inputs(2)
    obs = lens.Obs.from_numpy(obs_np)
    grid = S.WORKLOADS[5].grid
    B, n = 12, prm.shape[1]
    g = np.random.default_rng(19)
    states_np = np.tile(prm, (1, B))
    for b in range(B):
        states_np[0, b * n] += 0.002 * g.normal()
        states_np[6, b * n] *= 1.0 + 0.0002 * g.normal()
    st = np.zeros_like(prm)
    st[0, 0] = st[1, 0] = 0.002
    st[2, 0], st[3, 0], st[4, 0], st[6, 0] = 2e-4, 2e-3, 5e-3, 0.3
    st[6, 1:] = 0.2
    states = dev(states_np)
    chi2_cur = np.array([oracle.image_chi2(states_np[:, b * n:(b + 1) * n], grid, obs_np)["chi2"]
                         for b in range(B)])
    layout = lens.BatchLayout([b * n for b in range(B + 1)], [grid] * B)
    res = lens.lens_image_chi2_batched(states, layout, obs, prec="fp64")
    chi2 = res.chi2.clone()
    np.testing.assert_allclose(chi2.cpu().numpy(), chi2_cur, rtol=1e-9)
    for k in range(2):
        noise = g.normal(size=states_np.shape)
        if k == 0:
            noise[4, 3 * n] = -1e3  # chain 3: r_core < 0
        prop = states_np + np.tile(st, (1, B)) * noise
        chi2_prop, valid = np.empty(B), np.empty(B, bool)
        for b in range(B):
            q = prop[:, b * n:(b + 1) * n]
            valid[b] = bool(((q[2] >= 0) & (q[2] < 1) & (q[4] >= 0) & (q[5] > q[4]) & (q[6] >= 0)).all())
            chi2_prop[b] = oracle.image_chi2(q, grid, obs_np)["chi2"] if valid[b] else np.nan
        u = g.uniform(size=B)
        for b in range(B):
            if valid[b] and np.isfinite(chi2_prop[b]) and np.isfinite(chi2_cur[b]):
                while abs(math.log(u[b]) + 0.5 * (chi2_prop[b] - chi2_cur[b])) < 1e-6 * (1 + abs(chi2_cur[b])):
                    u[b] = g.uniform()
        acc = lens.mh_step_batched(states, B, grid, obs, dev(st), dev(noise), dev(u), chi2, prec="fp64")
        got_acc = acc.cpu().numpy().astype(bool)
        want_acc = np.array([oracle.mh_accept(chi2_prop[b], chi2_cur[b], u[b], valid[b]) for b in range(B)])
        print(f"  MH step {k}: accepted {int(got_acc.sum())}/{B}", flush=True)
        np.testing.assert_array_equal(got_acc, want_acc)
        for b in range(B):
            sl = slice(b * n, (b + 1) * n)
            if want_acc[b]:
                states_np[:, sl] = prop[:, sl]
                chi2_cur[b] = chi2_prop[b]
        np.testing.assert_array_equal(states.cpu().numpy(), states_np)
        np.testing.assert_allclose(chi2.cpu().numpy(), chi2_cur, rtol=1e-9)
        if k == 0:
            assert not got_acc[3]
        assert 0 < got_acc.sum() < B
