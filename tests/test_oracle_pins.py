"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms printed in the paper, textbook values, invariants of a gradient
field, exact rational arithmetic, library quadrature and brute force.

Each test names the mistake it is meant to catch."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

import oracle
import synthlens as S

C_KMS = 299792.458


def pot(x=0.0, y=0.0, eps=0.0, phi=0.0, rc=0.0, rcut=np.inf, sig=300.0):
    p = np.zeros((7, 1))
    p[:, 0] = (x, y, eps, phi, rc, rcut, sig)
    return p


def rand_dpie(g, n):
    p = np.zeros((7, n))
    p[0] = g.uniform(-20, 20, n)
    p[1] = g.uniform(-20, 20, n)
    p[2] = g.uniform(0, 0.5, n)
    p[3] = g.uniform(0, math.pi, n)
    p[4] = g.uniform(0.05, 3.0, n)
    p[5] = p[4] + g.uniform(5, 200, n)
    p[6] = g.uniform(100, 1000, n)
    return p


# --------------------------------------------------------------- normalisation

def test_b0_textbook_einstein_radius():
    """A singular isothermal sphere with sigma_v = 200 km/s has an Einstein radius of
    1.15 arcsec for D_LS/D_OS = 1 (Narayan & Bartelmann 1996, eq. for theta_E of the
    SIS).  Catches a wrong unit conversion, a wrong c or a missing 4 pi."""
    assert oracle.b0(200.0) == pytest.approx(1.15, abs=0.006)
    # quadratic in sigma_v (Sec. 2.2.2: b0 = 4 pi (sigma_v/c)^2)
    assert oracle.b0(400.0) == pytest.approx(4.0 * oracle.b0(200.0), rel=1e-15)


def test_sis_deflection_magnitude_is_constant():
    """Sec. 2.1: for the SIS |alpha| = theta_E everywhere, directed away from the centre
    (the lens equation is beta = theta - alpha).  Catches translation/rotation sign
    errors and a wrong radial profile."""
    g = np.random.default_rng(1)
    p = pot(x=3.0, y=-2.0, phi=0.7, sig=700.0)
    b0 = oracle.b0(700.0)
    for _ in range(50):
        t = g.uniform(-50, 50, 2)
        a = np.array(oracle.alpha(p, *t))
        d = t - np.array([3.0, -2.0])
        assert np.linalg.norm(a) == pytest.approx(b0, rel=1e-13)
        np.testing.assert_allclose(a / b0, d / np.linalg.norm(d), rtol=0, atol=1e-13)


def test_sie_orientation_convention():
    """Sec. 2.2.2: the pseudo-elliptical potential is stretched along its semi-major axis,
    which makes the angle Phi counter-clockwise from theta_1.  Along the major axis the
    SIE deflection is sqrt(1-eps) b0, along the minor axis sqrt(1+eps) b0 (from
    alpha_i = (1 -/+ eps) b0 theta_i / R).  Catches a rotation by +Phi instead of -Phi
    and swapped (1-eps)/(1+eps) factors."""
    eps, phi, sig = 0.3, 0.4, 500.0
    b0 = oracle.b0(sig)
    p = pot(x=1.0, y=2.0, eps=eps, phi=phi, sig=sig)
    for rho in (0.5, 7.0, 40.0):
        major = np.array([1.0, 2.0]) + rho * np.array([math.cos(phi), math.sin(phi)])
        minor = np.array([1.0, 2.0]) + rho * np.array([-math.sin(phi), math.cos(phi)])
        a_major = np.array(oracle.alpha(p, *major))
        a_minor = np.array(oracle.alpha(p, *minor))
        assert np.linalg.norm(a_major) == pytest.approx(math.sqrt(1 - eps) * b0, rel=1e-13)
        assert np.linalg.norm(a_minor) == pytest.approx(math.sqrt(1 + eps) * b0, rel=1e-13)
        # both point radially along the axes
        np.testing.assert_allclose(a_major / np.linalg.norm(a_major), [math.cos(phi), math.sin(phi)], atol=1e-13)
        np.testing.assert_allclose(a_minor / np.linalg.norm(a_minor), [-math.sin(phi), math.cos(phi)], atol=1e-13)


def test_sie_gradient_formula_in_complex_rotation():
    """The SIE gradient of Sec. 2.2.2, (1 -/+ eps) b0 theta_i / R in the lens frame, with the
    frame rotation written as multiplication by exp(-i Phi) / exp(+i Phi) (a formulation
    independent of the oracle's real-arithmetic rotations)."""
    g = np.random.default_rng(2)
    for _ in range(40):
        xc, yc = g.uniform(-30, 30, 2)
        eps, phi, sig = g.uniform(0, 0.6), g.uniform(-4, 4), g.uniform(50, 1200)
        p = pot(xc, yc, eps, phi, 0.0, np.inf, sig)
        t = g.uniform(-60, 60, 2)
        z = complex(t[0] - xc, t[1] - yc) * complex(math.cos(phi), -math.sin(phi))
        R = math.sqrt((1 - eps) * z.real ** 2 + (1 + eps) * z.imag ** 2)
        b0 = 4 * math.pi * (sig / C_KMS) ** 2 * 180 * 3600 / math.pi
        w = complex((1 - eps) * b0 * z.real / R, (1 + eps) * b0 * z.imag / R) * complex(math.cos(phi), math.sin(phi))
        a = oracle.alpha(p, *t)
        assert a[0] == pytest.approx(w.real, rel=1e-12, abs=1e-12)
        assert a[1] == pytest.approx(w.imag, rel=1e-12, abs=1e-12)


# --------------------------------------------------------------- dPIE profile

def test_dpie_limits():
    """r_core -> 0 and r_cut -> inf recover the SIS (|alpha| = b0); far outside the cut
    radius the profile is a point mass, |alpha| R -> b0 * r_cut (the enclosed mass of
    the cored/cut isothermal profile).  Catches a wrong K = b0 s/(s-a) or a wrong f."""
    b0 = oracle.b0(600.0)
    p = pot(rc=1e-9, rcut=1e12, sig=600.0)
    for r in (0.1, 3.0, 80.0):
        assert np.linalg.norm(oracle.alpha(p, r, 0.0)) == pytest.approx(b0, rel=1e-6)
    p = pot(rc=0.7, rcut=30.0, sig=600.0)
    R = 3.0e6
    assert np.linalg.norm(oracle.alpha(p, 0.0, R)) * R == pytest.approx(b0 * 30.0, rel=1e-5)


def test_dpie_divergence_equals_twice_convergence():
    """grad . alpha = 2 kappa (Sec. 2.1: alpha = grad psi and psi solves the 2-D Poisson
    equation with source 2 kappa).  For eps = 0 the cored/cut isothermal convergence is
    kappa(R) = (K/2) (1/sqrt(a^2+R^2) - 1/sqrt(s^2+R^2)) (Eliasdottir et al. 2007), with
    K = b0 s/(s-a).  Checked by central differences."""
    a, s, sig = 0.8, 40.0, 800.0
    K = oracle.b0(sig) * s / (s - a)
    p = pot(x=1.5, y=-0.5, rc=a, rcut=s, sig=sig)
    h = 1e-4
    for t in [(2.0, 0.3), (-5.0, 7.0), (30.0, -20.0), (1.7, -0.4)]:
        ax_p = oracle.alpha(p, t[0] + h, t[1])[0]
        ax_m = oracle.alpha(p, t[0] - h, t[1])[0]
        ay_p = oracle.alpha(p, t[0], t[1] + h)[1]
        ay_m = oracle.alpha(p, t[0], t[1] - h)[1]
        div = (ax_p - ax_m) / (2 * h) + (ay_p - ay_m) / (2 * h)
        R = math.hypot(t[0] - 1.5, t[1] + 0.5)
        kappa = 0.5 * K * (1 / math.sqrt(a * a + R * R) - 1 / math.sqrt(s * s + R * R))
        assert div == pytest.approx(2 * kappa, rel=1e-6, abs=1e-8)


def test_deflection_is_curl_free():
    """alpha is a gradient (Sec. 2.1), so d alpha_2/d theta_1 = d alpha_1/d theta_2.
    Catches a back-rotation with the wrong sign or a mis-placed (1 +/- eps)."""
    g = np.random.default_rng(3)
    p = rand_dpie(g, 6)
    h = 1e-5
    for _ in range(30):
        t = g.uniform(-40, 40, 2)
        d21 = (oracle.alpha(p, t[0] + h, t[1])[1] - oracle.alpha(p, t[0] - h, t[1])[1]) / (2 * h)
        d12 = (oracle.alpha(p, t[0], t[1] + h)[0] - oracle.alpha(p, t[0], t[1] - h)[0]) / (2 * h)
        scale = abs(d21) + abs(d12) + 1e-3
        assert abs(d21 - d12) < 1e-5 * scale


def test_symmetries_and_superposition():
    """Point reflection about the centre, invariance under Phi -> Phi + pi, covariance
    under a rigid rotation of the whole configuration, and linearity in the list of
    potentials (the superposition of Sec. 2.2.2)."""
    g = np.random.default_rng(4)
    p = rand_dpie(g, 1)
    c = p[:2, 0]
    for _ in range(10):
        d = g.uniform(-15, 15, 2)
        np.testing.assert_allclose(oracle.alpha(p, *(c + d)), -np.array(oracle.alpha(p, *(c - d))), atol=1e-12)
    q = p.copy()
    q[3] += math.pi
    for _ in range(10):
        t = g.uniform(-40, 40, 2)
        np.testing.assert_allclose(oracle.alpha(p, *t), oracle.alpha(q, *t), rtol=1e-12, atol=1e-12)
    # rigid rotation by omega about the origin
    w = 0.9
    Rw = np.array([[math.cos(w), -math.sin(w)], [math.sin(w), math.cos(w)]])
    pr = p.copy()
    pr[:2, 0] = Rw @ p[:2, 0]
    pr[3] += w
    for _ in range(10):
        t = g.uniform(-40, 40, 2)
        np.testing.assert_allclose(oracle.alpha(pr, *(Rw @ t)), Rw @ np.array(oracle.alpha(p, *t)),
                                   rtol=1e-11, atol=1e-11)
    # superposition
    pp = rand_dpie(g, 5)
    for _ in range(10):
        t = g.uniform(-40, 40, 2)
        parts = sum(np.array(oracle.alpha(pp[:, k:k + 1], *t)) for k in range(5))
        np.testing.assert_allclose(oracle.alpha(pp, *t), parts, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------- cosmology

def test_einstein_de_sitter_closed_form():
    """Omega_m = 1: chi(z) = 2 (1 - 1/sqrt(1+z)) c/H0, so D_LS/D_OS =
    (1/sqrt(1+z_l) - 1/sqrt(1+z_s)) / (1 - 1/sqrt(1+z_s))."""
    for zl, zs in [(0.3, 2.0), (0.1, 0.5), (0.5, 6.0)]:
        want = (1 / math.sqrt(1 + zl) - 1 / math.sqrt(1 + zs)) / (1 - 1 / math.sqrt(1 + zs))
        assert oracle.dls_dos(zl, zs, 1.0, 0.0) == pytest.approx(want, rel=1e-12)
    assert oracle.dls_dos(0.5, 0.4) == 0.0


def test_lcdm_against_library_quadrature():
    """Flat LambdaCDM (0.3, 0.7) of Sec. 4 against scipy's adaptive quadrature."""
    f = lambda z: 1 / math.sqrt(0.3 * (1 + z) ** 3 + 0.7)
    for zl, zs in [(0.3, 1.0), (0.3, 2.0), (0.3, 3.0), (0.3, 6.0)]:
        cl = integrate.quad(f, 0, zl, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
        cs = integrate.quad(f, 0, zs, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
        assert oracle.dls_dos(zl, zs) == pytest.approx((cs - cl) / cs, rel=1e-12)


# --------------------------------------------------------------- exact predicate

def _fr_orient(a, b, c):
    A = [Fraction(v) for v in (*a, *b, *c)]
    det = (A[0] - A[4]) * (A[3] - A[5]) - (A[1] - A[5]) * (A[2] - A[4])
    return (det > 0) - (det < 0)


def test_orient_matches_exact_rationals():
    """Exact sign against Python's rational arithmetic, on random, nearly collinear,
    exactly collinear, tiny, huge and subnormal inputs."""
    g = np.random.default_rng(5)
    cases = []
    for _ in range(300):
        cases.append(tuple(g.uniform(-100, 100, 6)))
    for _ in range(300):  # c on (or next to) the segment a-b
        a, b = g.uniform(-100, 100, 2), g.uniform(-100, 100, 2)
        t = g.uniform(0, 1)
        c = a + t * (b - a)
        c = c + g.choice([0.0, 1e-14, -1e-14, 1e-300]) * g.uniform(-1, 1, 2)
        cases.append((*a, *b, *c))
    for _ in range(100):  # exactly collinear with representable coordinates
        k = g.integers(-50, 50, 3)
        cases.append((0.5, 0.25, 0.5 + k[0], 0.25 + 2.0 * k[0], 0.5 + k[1], 0.25 + 2.0 * k[1]))
    cases += [(1e-300, 0, 0, 1e-300, 0, 0), (5e-324, 0, 0, 5e-324, 0, 0), (1e300, 1, -1e300, 1, 0, 1),
              (1e200, 1e-200, 3.0, 7.0, 1e-180, 5e150), (0, 0, 0, 0, 0, 0)]
    for cs in cases:
        a, b, c = cs[0:2], cs[2:4], cs[4:6]
        assert oracle.orient(a, b, c) == _fr_orient(a, b, c), cs


# --------------------------------------------------------------- triangles and images

def test_identity_lens_single_exact_image():
    """With no potentials the lens equation is beta = theta: every source inside the grid
    has exactly one image, at beta itself (barycentric interpolation is exact for a linear
    map), in the cell that contains it, on the side of the anti-diagonal it lies on.
    Catches wrong triangle vertices, ids, orientation handling and transposed weights."""
    grid = S.Grid(-3.0, -2.0, 0.5, 13, 11)
    empty = np.zeros((7, 0))
    ax, ay = oracle.alpha_grid(empty, grid)
    g = np.random.default_rng(6)
    for _ in range(60):
        b = np.array([g.uniform(-2.9, 2.9), g.uniform(-1.9, 2.9)])
        hs, ht = oracle.hits_from_field(ax, ay, grid, [b[0]], [b[1]], [0.7])
        assert len(ht) == 1
        fx, fy = (b[0] - grid.x0) / grid.h, (b[1] - grid.y0) / grid.h
        i, j = int(fx), int(fy)
        k = 0 if (fx - i) + (fy - j) < 1 else 1
        assert ht[0] == 2 * (j * (grid.nx - 1) + i) + k
        hx, hy = oracle.positions_from_field(ax, ay, grid, hs, ht, [b[0]], [b[1]], [0.7])
        assert hx[0] == pytest.approx(b[0], abs=1e-13) and hy[0] == pytest.approx(b[1], abs=1e-13)


def test_points_on_edges_are_misses():
    """READING of the containment test: strict inequalities, so a barycentre exactly on a
    grid node or on a triangle edge is inside no triangle."""
    grid = S.Grid(0.0, 0.0, 1.0, 5, 5)
    ax, ay = oracle.alpha_grid(np.zeros((7, 0)), grid)
    for b in [(2.0, 2.0), (1.5, 1.0), (2.0, 1.25), (1.5, 1.5)]:  # node, edges, diagonal
        hs, ht = oracle.hits_from_field(ax, ay, grid, [b[0]], [b[1]], [1.0])
        assert len(ht) == 0, b


def test_sis_two_images_closed_form():
    """SIS (Sec. 2.1): a source at beta has images at theta = beta_hat (|beta| +/- theta_E)
    with theta_E = b0 D_LS/D_OS.  Both the brute-force Newton finder and the triangle
    method (to O(h^2)) find them."""
    sig, r = 600.0, 0.77
    p = pot(sig=sig, x=0.013, y=-0.021)
    tE = r * oracle.b0(sig)
    beta = np.array([1.1, 0.7])
    bn = np.linalg.norm(beta)
    want = np.array([(bn + tE) * beta / bn, (bn - tE) * beta / bn]) + np.array([0.013, -0.021])
    # the source plane is centred on the lens: shift beta by the lens centre
    found = oracle.find_images(p, r, beta + np.array([0.013, -0.021]), S.square_grid(41, 30.0), (-30, 30, -30, 30))
    assert len(found) == 2
    for w in want:
        assert np.min(np.linalg.norm(found - w, axis=1)) < 1e-9
    grid = S.square_grid(401, 30.0)
    ax, ay = oracle.alpha_grid(p, grid)
    bb = beta + np.array([0.013, -0.021])
    hs, ht = oracle.hits_from_field(ax, ay, grid, [bb[0]], [bb[1]], [r])
    hx, hy = oracle.positions_from_field(ax, ay, grid, hs, ht, [bb[0]], [bb[1]], [r])
    pts = np.stack([hx, hy], axis=1)
    for w in want:
        assert np.min(np.linalg.norm(pts - w, axis=1)) < grid.h ** 2 / 4  # O(h^2) interpolation
    # any other hit sits in a cell touching the singular centre
    centre = np.array([0.013, -0.021])
    for q in pts:
        if min(np.linalg.norm(q - w) for w in want) > grid.h ** 2 / 4:
            assert np.linalg.norm(q - centre) < 2 * grid.h


def test_einstein_ring():
    """Sec. 2.1: a source exactly behind a SIS is imaged onto the ring |theta| = theta_E."""
    sig, r = 500.0, 0.8
    p = pot(sig=sig, x=0.0317, y=0.0129)
    tE = r * oracle.b0(sig)
    grid = S.square_grid(201, 20.0)
    ax, ay = oracle.alpha_grid(p, grid)
    hs, ht = oracle.hits_from_field(ax, ay, grid, [0.0317], [0.0129], [r])
    hx, hy = oracle.positions_from_field(ax, ay, grid, hs, ht, [0.0317], [0.0129], [r])
    rad = np.hypot(hx - 0.0317, hy - 0.0129)
    ring = rad > 2 * grid.h
    assert ring.sum() > 2 * math.pi * tE / grid.h * 0.5
    np.testing.assert_allclose(rad[ring], tE, atol=grid.h)


def test_exact_images_map_to_one_source():
    """Newton-exact images of one source all lens back onto that source, so their
    barycentre is the source (Sec. 2.2.2), and the triangle method recovers each image
    to O(h^2)."""
    prm = S.config1_potentials()
    r = oracle.dls_dos(0.3, 2.0)
    beta = np.array([0.4, -0.3])
    imgs = oracle.find_images(prm, r, beta, S.square_grid(161, 40.0), (-40, 40, -40, 40))
    assert len(imgs) >= 3
    obs = dict(sys_off=np.array([0, len(imgs)]), x=imgs[:, 0], y=imgs[:, 1], sigma=np.full(len(imgs), 0.1),
               dls=np.array([r]))
    bx, by, barx, bary = oracle.source_positions(prm, obs["sys_off"], obs["x"], obs["y"], obs["dls"])
    np.testing.assert_allclose(bx, beta[0], atol=1e-10)
    np.testing.assert_allclose(by, beta[1], atol=1e-10)
    res = oracle.image_chi2(prm, S.square_grid(513, 40.0), obs)
    assert res["n_pred"][0] == len(imgs)
    pts = np.stack([res["hit_x"], res["hit_y"]], axis=1)
    for im in imgs:
        assert np.min(np.linalg.norm(pts - im, axis=1)) < 5e-3


def test_match_and_chi2_rules():
    """chi^2 of Sec. 2.2.1 with the nearest-image pairing (READING): zero when each observed
    image sits on a predicted one, sum |d|^2/sigma^2 for known offsets, ties to the earlier
    hit, +inf for a system with no predicted image."""
    obs = dict(sys_off=np.array([0, 2, 3, 4]), x=np.array([0.0, 5.0, 1.0, 9.0]),
               y=np.array([0.0, 0.0, 1.0, 9.0]), sigma=np.array([0.1, 0.2, 0.5, 1.0]))
    hit_sys = np.array([0, 0, 1, 1])
    hx = np.array([0.0, 5.0, 1.0 + 0.3, 1.0 - 0.3])
    hy = np.array([0.0, 0.0, 1.0, 1.0])
    res = oracle.match_chi2(obs, hit_sys, hx, hy)
    assert list(res["n_pred"]) == [2, 2, 0]
    assert res["chi2_sys"][0] == 0.0
    assert res["chi2_sys"][1] == pytest.approx(0.3 ** 2 / 0.25)
    assert list(res["match"][:3]) == [0, 1, 2]  # tie between hits 2 and 3 -> earlier hit
    assert math.isinf(res["chi2_sys"][2]) and math.isinf(res["chi2"])
    hx2 = hx + np.array([0.01, -0.02, 0.0, 0.0])
    res = oracle.match_chi2(dict(obs, sys_off=np.array([0, 2, 3])), hit_sys, hx2, hy)
    assert res["chi2"] == pytest.approx(0.01 ** 2 / 0.01 + 0.02 ** 2 / 0.04 + 0.3 ** 2 / 0.25, rel=1e-12)


# --------------------------------------------------------------- derivatives

def test_complex_evaluation_matches_real():
    g = np.random.default_rng(7)
    p = rand_dpie(g, 4)
    for _ in range(10):
        t = g.uniform(-30, 30, 2)
        a1, a2 = oracle.alpha_complex(p, t[0], t[1])
        np.testing.assert_allclose([a1.real, a2.real], oracle.alpha(p, *t), rtol=1e-14, atol=1e-14)


def test_complex_step_identities():
    """d alpha / d sigma_v = 2 alpha / sigma_v (alpha is proportional to b0, quadratic in
    sigma_v); d alpha / d x_c = - d alpha / d theta_1 (translation invariance);
    d alpha / d Phi = Omega alpha - J Omega (theta - theta_c) (rotation covariance, with
    Omega the 90-degree rotation and J the Jacobian of alpha); complex step against
    central differences."""
    g = np.random.default_rng(8)
    p = rand_dpie(g, 1)
    ih = 1e-30
    Om = np.array([[0.0, -1.0], [1.0, 0.0]])
    for _ in range(10):
        t = g.uniform(-30, 30, 2)
        a = np.array(oracle.alpha(p, *t))
        ds = np.array([v.imag for v in oracle.alpha_complex(p, t[0], t[1], 6, 0, ih)]) / ih
        np.testing.assert_allclose(ds, 2 * a / p[6, 0], rtol=1e-12, atol=1e-15)
        dxc = np.array([v.imag for v in oracle.alpha_complex(p, t[0], t[1], 0, 0, ih)]) / ih
        dt1 = np.array([v.imag for v in oracle.alpha_complex(p, t[0] + ih * 1j, t[1])]) / ih
        dt2 = np.array([v.imag for v in oracle.alpha_complex(p, t[0], t[1] + ih * 1j)]) / ih
        np.testing.assert_allclose(dxc, -dt1, rtol=1e-12, atol=1e-14)
        J = np.stack([dt1, dt2], axis=1)
        dphi = np.array([v.imag for v in oracle.alpha_complex(p, t[0], t[1], 3, 0, ih)]) / ih
        np.testing.assert_allclose(dphi, Om @ a - J @ (Om @ (t - p[:2, 0])), rtol=1e-10, atol=1e-12)
        for k in range(7):
            h = 1e-6 * max(abs(p[k, 0]), 1.0)
            pp, pm = p.copy(), p.copy()
            pp[k, 0] += h
            pm[k, 0] -= h
            fd = (np.array(oracle.alpha(pp, *t)) - np.array(oracle.alpha(pm, *t))) / (2 * h)
            cs = np.array([v.imag for v in oracle.alpha_complex(p, t[0], t[1], k, 0, ih)]) / ih
            np.testing.assert_allclose(cs, fd, rtol=1e-6, atol=1e-8)


def _exact_src_chi2(sys_off, bx, by, sig):
    """sum_i sum_j |beta_ij - mean_j beta_ij|^2 / sigma_ij^2 in exact rational
    arithmetic (every float converted exactly)."""
    tot = Fraction(0)
    for i in range(len(sys_off) - 1):
        j0, j1 = int(sys_off[i]), int(sys_off[i + 1])
        if j1 == j0:
            continue
        X = [Fraction(float(v)) for v in bx[j0:j1]]
        Y = [Fraction(float(v)) for v in by[j0:j1]]
        mx, my = sum(X) / len(X), sum(Y) / len(Y)
        for k in range(j1 - j0):
            s2 = Fraction(float(sig[j0 + k])) ** 2
            tot += ((X[k] - mx) ** 2 + (Y[k] - my) ** 2) / s2
    return tot


def test_src_chi2_identity_lens_is_the_exact_scatter():
    """With no potential the lens equation gives beta = theta, so the source-plane
    chi^2 (reading of the smooth companion of the image-plane chi^2) is the
    sigma-weighted scatter of each system's observed images about their unweighted
    mean, computed here in exact rational arithmetic.  Catches sigma instead of
    sigma^2, a weighted or wrongly delimited mean, a dropped component, a
    missing system or a wrong normalisation."""
    g = np.random.default_rng(31)
    sizes = [1, 2, 3, 5, 4]
    sys_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(sys_off[-1])
    obs = dict(sys_off=sys_off, x=g.uniform(-30, 30, n), y=g.uniform(-30, 30, n),
               sigma=g.choice([0.05, 0.1, 0.25, 0.7], n), dls=g.uniform(0.4, 0.9, len(sizes)))
    want = _exact_src_chi2(sys_off, obs["x"], obs["y"], obs["sigma"])
    got = oracle.src_chi2(np.zeros((7, 0)), obs)
    assert abs(Fraction(got) - want) <= Fraction(1, 10 ** 12) * want
    # a single-image system contributes nothing; moving one image moves only its system's term
    obs2 = dict(obs, x=obs["x"].copy())
    obs2["x"][0] += 3.0
    assert oracle.src_chi2(np.zeros((7, 0)), obs2) == pytest.approx(got, rel=1e-14)


def test_src_chi2_vanishes_on_exact_images_of_a_singular_isothermal_sphere():
    """A singular isothermal sphere at theta_c maps its two images theta_c + u(|b| +/- r b0)
    (u the unit vector of the source offset b; the closed form of Sec. 2.1 with the
    distance ratio r) onto one source, so their source-plane chi^2 is zero up to
    rounding; a wrong sign or a misplaced distance ratio in the lens equation
    separates them by ~2 r b0."""
    xc, yc, sig = 1.5, -0.75, 600.0
    b0 = 4 * math.pi * (sig / C_KMS) ** 2 * 180 * 3600 / math.pi
    prm = pot(x=xc, y=yc, sig=sig)
    xs, ys, sys_off, dls = [], [], [0], []
    for (bx, by, r) in [(0.8, 0.3, 0.7), (-1.2, 2.0, 0.9), (0.05, -0.4, 0.55)]:
        bl = math.hypot(bx, by)
        ux, uy = bx / bl, by / bl
        for t in (bl + r * b0, bl - r * b0):
            xs.append(xc + ux * t)
            ys.append(yc + uy * t)
        sys_off.append(len(xs))
        dls.append(r)
    obs = dict(sys_off=np.array(sys_off, np.int32), x=np.array(xs), y=np.array(ys), sigma=np.full(len(xs), 0.1),
               dls=np.array(dls))
    assert oracle.src_chi2(prm, obs) <= 1e-18
    bad = dict(obs, dls=obs["dls"] * 1.01)
    assert oracle.src_chi2(prm, bad) > 1.0


def test_nfw_grid_indexing_matches_pointwise_deflection():
    """The NFW field at node (i, j) of a grid with nx != ny, x0 != y0, is the
    pointwise deflection at (x0 + i h, y0 + j h), stored at row j, column i
    (catches a transposed or mis-strided layout, or swapped axes)."""
    prm = np.stack([nfw(x=1.3, y=-2.1, eps=0.2, phi=0.7, rs=6.0, ks=0.3)[:, 0],
                    nfw(x=-4.0, y=3.5, eps=0.1, phi=2.0, rs=3.0, ks=0.1)[:, 0]], axis=1)
    grid = S.Grid(-7.3, -5.1, 0.61, 23, 17)
    ax, ay = oracle.nfw_alpha_grid(prm, grid)
    assert ax.shape == (17, 23)
    for j in range(grid.ny):
        for i in range(grid.nx):
            a = oracle.nfw_alpha(prm, grid.x0 + i * grid.h, grid.y0 + j * grid.h)
            assert ax[j, i] == a[0] and ay[j, i] == a[1], (i, j)


def test_src_chi2_gradient_against_finite_differences():
    """Complex-step gradient of the source-plane chi^2 vs central differences with
    h = 1e-6 relative (1e-6 absolute for parameters equal to zero)."""
    prm, grid, obs = _small_cluster()
    val = oracle.src_chi2(prm, obs)
    assert val > 0
    grad = oracle.src_chi2_grad(prm, obs)
    for k in range(7):
        for pi in range(prm.shape[1]):
            h = 1e-6 * max(abs(prm[k, pi]), 1.0)
            pp, pm = prm.copy(), prm.copy()
            pp[k, pi] += h
            pm[k, pi] -= h
            fd = (oracle.src_chi2(pp, obs) - oracle.src_chi2(pm, obs)) / (2 * h)
            assert grad[k, pi] == pytest.approx(fd, rel=2e-5, abs=1e-6 * (abs(val) + 1))


def test_alpha_vjp_against_finite_differences():
    prm, grid, obs = _small_cluster()
    g = np.random.default_rng(9)
    grid = S.square_grid(9, 20.0)
    gx, gy = g.normal(size=(grid.ny, grid.nx)), g.normal(size=(grid.ny, grid.nx))
    vjp = oracle.alpha_vjp(prm, grid, gx, gy)
    for k in range(7):
        for pi in range(prm.shape[1]):
            h = 1e-6 * max(abs(prm[k, pi]), 1.0)
            pp, pm = prm.copy(), prm.copy()
            pp[k, pi] += h
            pm[k, pi] -= h
            axp, ayp = oracle.alpha_grid(pp, grid)
            axm, aym = oracle.alpha_grid(pm, grid)
            fd = (np.sum(gx * (axp - axm)) + np.sum(gy * (ayp - aym))) / (2 * h)
            assert vjp[k, pi] == pytest.approx(fd, rel=1e-5, abs=1e-6)


def test_alpha_vjp_magnitude_mode_is_the_sum_of_node_magnitudes():
    """absolute=True equals the sum over nodes of |gx d alpha_1/dq| + |gy d alpha_2/dq|,
    each node's term taken from the signed VJP on a one-node grid with one cotangent
    component at a time; it bounds the signed VJP."""
    prm, _, _ = _small_cluster()
    grid = S.Grid(-13.0, -7.5, 2.25, 5, 4)
    g = np.random.default_rng(12)
    gx, gy = g.normal(size=(grid.ny, grid.nx)), g.normal(size=(grid.ny, grid.nx))
    mag = oracle.alpha_vjp(prm, grid, gx, gy, absolute=True)
    want = np.zeros_like(mag)
    one, zero = np.ones((1, 1)), np.zeros((1, 1))
    for j in range(grid.ny):
        for i in range(grid.nx):
            node = S.Grid(grid.x0 + i * grid.h, grid.y0 + j * grid.h, 1.0, 1, 1)
            want += np.abs(gx[j, i] * oracle.alpha_vjp(prm, node, one, zero))
            want += np.abs(gy[j, i] * oracle.alpha_vjp(prm, node, zero, one))
    np.testing.assert_allclose(mag, want, rtol=1e-12, atol=0)
    assert (np.abs(oracle.alpha_vjp(prm, grid, gx, gy)) <= mag * (1 + 1e-12)).all()


def _small_cluster():
    prm = S.cluster_potentials(3, 2)
    grid = S.square_grid(65, 40.0)
    r = np.array([oracle.dls_dos(0.3, 2.5), oracle.dls_dos(0.3, 4.0)])
    g = np.random.default_rng(10)
    xs = g.uniform(-20, 20, (6, 2))
    obs = dict(sys_off=np.array([0, 3, 6], np.int32), x=xs[:, 0], y=xs[:, 1], sigma=np.full(6, 0.1), dls=r)
    return prm, grid, obs


# --------------------------------------------------------------- the paper's mixed-precision gradient

def test_dp_patches_block_geometry():
    """Blocks of Sec. 3.2 / Appendix A.3 by hand-counted integer geometry: an
    interior block has p^2 pixels spanning [k - p/2, k - p/2 + p); halves round
    away from zero; blocks clip at the grid edge; overlapping blocks count once;
    only the first n_cluster halos get the large block.  Catches an off-by-one
    in the span, a round-half-even centre, a missing clip or a swapped axis."""
    g = S.Grid(0.0, 0.0, 0.5, 120, 90)
    # (5.25 - 0)/0.5 = 10.5 -> 11; (7.0)/0.5 = 14
    m = oracle.dp_patches(pot(x=5.25, y=7.0), g, 0, 400, 20)
    rows, cols = np.nonzero(m)
    assert m.sum() == 400
    assert (cols.min(), cols.max(), rows.min(), rows.max()) == (1, 20, 4, 23)
    # -1.25/0.5 = -2.5 -> -3: columns [-13, 7) clipped to [0, 7)
    m = oracle.dp_patches(pot(x=-1.25, y=20.0), g, 0, 400, 20)
    rows, cols = np.nonzero(m)
    assert (cols.min(), cols.max(), rows.min(), rows.max()) == (0, 6, 30, 49) and m.sum() == 7 * 20
    # two galaxy blocks at nodes (50, 40) and (60, 45): 400 + 400 - 10 * 15
    two = np.concatenate([pot(x=25.0, y=20.0), pot(x=30.0, y=22.5)], axis=1)
    assert oracle.dp_patches(two, g, 0, 400, 20).sum() == 650
    # the first potential is cluster-scale: a 30 x 30 block (clipped at y = 89) plus a 20 x 20 one
    m = oracle.dp_patches(two, g, 1, 30, 20)
    big = (np.arange(35, 65), np.arange(25, 55))
    assert m[np.ix_(big[1], big[0])].all()
    assert m.sum() == 30 * 30 + 20 * 20 - len(range(50, 65)) * len(range(35, 55))


def test_criteria_sis_axis_closed_form():
    """Criteria of Sec. 3.3 on the oracle's own SIS field, along the row through
    the centre, against their closed forms: with R = (i - ic) h and the
    neighbour row one pixel below, d1 = d4 = 0, d2 = b0 h / sqrt(R^2 + h^2)
    (the tangential stretch that vanishes on the Einstein ring) and
    d3 = b0 (1 - R / sqrt(R^2 + h^2)).  Catches a swapped difference direction
    (i+1 for i-1), d2 and d3 exchanged, a wrong threshold comparison (<= vs >,
    |d| vs d) or an axis mix-up."""
    h, b0 = 0.03, oracle.b0(1000.0)
    ic, nx = 20, 1500
    g = S.Grid(-ic * h, -h, h, nx, 3)  # centre at node (20, 1)
    ax, ay = oracle.alpha_grid(pot(sig=1000.0), g, nthreads=2)
    f = oracle.criteria(ax, ay, h)
    R = (np.arange(ic + 2, nx) - ic) * h
    q = np.sqrt(R * R + h * h)
    d2 = b0 * h / q
    d3 = b0 * (1.0 - R / q)
    a = np.abs(h - d2) - oracle.T12
    b = d3 - oracle.T34
    want = (a < 0) | (b > 0)
    clear = (np.abs(a) > 1e-9) & (np.abs(b) > 1e-9)
    got = f[1, ic + 2:].astype(bool)
    assert clear.sum() > 1000
    np.testing.assert_array_equal(got[clear], want[clear])
    # both bands are present: the core (d3) and the Einstein ring (d2, b0 = 28.8")
    assert want[R < 1.0].all() and not want[(R > 2.0) & (R < 20.0)].any() and want[np.abs(R - b0) < 1.0].all()


def test_criteria_edges_and_linear_fields():
    """Fields whose differences are constant: a flag appears exactly where the
    difference is evaluated, never on the first column (d1, d4) or first row
    (d2, d3) of the image.  Catches a wrap-around neighbour or an evaluated edge."""
    h = 0.03
    i = np.arange(40)[None, :] * np.ones((30, 1))
    j = np.arange(30)[:, None] * np.ones((1, 40))
    zero = np.zeros((30, 40))
    f = oracle.criteria((h - 0.001) * i, zero, h)          # |h - d1| = 0.001
    np.testing.assert_array_equal(f, (i >= 1).astype(np.uint8))
    f = oracle.criteria(zero, (h - 0.001) * j, h)          # |h - d2| = 0.001
    np.testing.assert_array_equal(f, (j >= 1).astype(np.uint8))
    f = oracle.criteria(0.02 * j, zero, h)                 # d3 = 0.02 > 0.0104
    np.testing.assert_array_equal(f, (j >= 1).astype(np.uint8))
    f = oracle.criteria(zero, -0.02 * i, h)                # |d4| = 0.02
    np.testing.assert_array_equal(f, (i >= 1).astype(np.uint8))
    f = oracle.criteria(0.005 * j, 0.005 * j, h)           # source pixels h long, |d3| < t34: nothing
    assert f.sum() == 0
    f = oracle.criteria(h * i, zero, h)                    # d1 = h: source pixel of length 0
    np.testing.assert_array_equal(f, (i >= 1).astype(np.uint8))


# --------------------------------------------------------------- sampler steps

def test_hmc_leapfrog_matches_harmonic_map():
    """For U = q^2 / (2 sigma^2) the leapfrog map in z = q/step with omega =
    step/sigma is the linear map M = [[1 - w/2, 1], [-w (1 - w/4), 1 - w/2]],
    w = omega^2 (kick-drift-kick with unit step); L steps are M^L (numpy matrix
    power).  Catches a missing half kick, the kick/drift order, the step
    scaling or the sign of the gradient."""
    sigma, s, L = 1.7, 0.4, 7
    w = (s / sigma) ** 2
    M = np.array([[1 - w / 2, 1.0], [-w * (1 - w / 4), 1 - w / 2]])
    energy = lambda q: (0.5 * float(np.sum(q * q)) / sigma ** 2, q / sigma ** 2)
    q0, p0 = np.array([0.9, -2.1]), np.array([0.3, 1.2])
    q, _, acc = oracle.hmc_step_generic(q0, np.full(2, s), L, p0, 1e-300, energy)
    assert acc
    ML = np.linalg.matrix_power(M, L)
    for k in range(2):
        z, _ = ML @ np.array([q0[k] / s, p0[k]])
        assert q[k] == pytest.approx(z * s, rel=1e-12)
    # a frozen coordinate (step 0) does not move
    q, _, _ = oracle.hmc_step_generic(q0, np.array([s, 0.0]), L, p0, 1e-300, energy)
    assert q[1] == q0[1]


def test_hmc_reversible_and_samples_a_gaussian():
    """Leapfrog is reversible (negated end momentum returns to the start), and
    the chain's moments match N(0, sigma^2) (seeded; 5-sigma sampling bounds).
    Catches a non-symmetric integrator or a wrong acceptance sign."""
    sigma = 2.5
    energy = lambda q: (0.5 * float(np.sum(q * q)) / sigma ** 2, q / sigma ** 2)
    q0, p0, s, L = np.array([1.3]), np.array([0.7]), np.array([0.9]), 6
    w = (s[0] / sigma) ** 2
    M = np.linalg.matrix_power(np.array([[1 - w / 2, 1.0], [-w * (1 - w / 4), 1 - w / 2]]), L)
    z1, p1 = M @ np.array([q0[0] / s[0], p0[0]])
    back, _, _ = oracle.hmc_step_generic(np.array([z1 * s[0]]), s, L, np.array([-p1]), 1e-300, energy)
    assert back[0] == pytest.approx(q0[0], rel=1e-12)
    g = np.random.default_rng(11)
    q, xs = np.zeros(1), []
    for _ in range(20000):
        q, _, _ = oracle.hmc_step_generic(q, np.array([1.1]), 5, g.normal(size=1), g.uniform(), energy)
        xs.append(q[0])
    xs = np.array(xs[1000:])
    n_eff = len(xs) / 4  # conservative
    assert abs(xs.mean()) < 5 * sigma / math.sqrt(n_eff)
    assert abs(xs.var() / sigma ** 2 - 1) < 5 * math.sqrt(2 / n_eff)


def test_metropolis_acceptance_rule():
    """log-likelihood -chi^2/2: a chi^2 larger by 2 is accepted exactly when
    u < 1/e; invalid proposals never; any valid proposal from an infinite chi^2."""
    e = math.exp(-1.0)
    assert oracle.mh_accept(12.0, 10.0, e * 0.999, True) and not oracle.mh_accept(12.0, 10.0, e * 1.001, True)
    assert oracle.mh_accept(5.0, 10.0, 0.999999, True)
    assert not oracle.mh_accept(5.0, 10.0, 0.5, False) and not oracle.mh_accept(math.inf, 10.0, 0.5, True)
    assert oracle.mh_accept(1e9, math.inf, 0.999, True)


# --------------------------------------------------------------- pseudo-elliptical NFW

def nfw(x=0.0, y=0.0, eps=0.0, phi=0.0, rs=10.0, ks=0.2):
    p = np.zeros((6, 1))
    p[:, 0] = (x, y, eps, phi, rs, ks)
    return p


def test_nfw_deflection_is_the_enclosed_projected_density():
    """The circular NFW deflection alpha(R) = R * (mean convergence inside R),
    with the convergence obtained by integrating the 3D density
    rho ~ 1 / (r (1 + r)^2) along the line of sight (scipy quadrature, no
    closed form involved): alpha = (2 r_s / x) int_0^x x' k(x') dx',
    k(x') = 2 kappa_s int_0^inf dz / (s (1 + s)^2), s = sqrt(x'^2 + z^2).
    Catches a wrong F(x) branch, a missing log term or a wrong normalisation."""
    rs, ks = 10.0, 0.2

    def kappa(xp):
        f = lambda z: 1.0 / (math.hypot(xp, z) * (1.0 + math.hypot(xp, z)) ** 2)
        a = integrate.quad(f, 0.0, xp, limit=200, epsabs=0, epsrel=1e-12)[0]
        b = integrate.quad(f, xp, np.inf, limit=200, epsabs=0, epsrel=1e-12)[0]
        return 2.0 * ks * (a + b)

    for x in (0.05, 0.5, 0.999, 1.0, 1.001, 2.0, 7.0):
        inner = integrate.quad(lambda xp: xp * kappa(xp), 0.0, x, limit=200, epsabs=0, epsrel=1e-10)[0]
        want = 2.0 * rs * inner / x
        got, zero = oracle.nfw_alpha(nfw(rs=rs, ks=ks), x * rs, 0.0)
        assert zero == 0.0
        assert got == pytest.approx(want, rel=1e-7), x


def test_nfw_limits_and_continuity():
    """Series limits of g(x) = ln(x/2) + F(x): x -> 0, g ~ (x^2/2)(ln(2/x) - 1/2);
    x -> inf, g ~ ln(x/2) + pi/(2x) - 1/x^2; and the three branches of F join
    continuously at x = 1 (g(1) = 1 - ln 2)."""
    rs, ks = 10.0, 0.2
    a = lambda x: oracle.nfw_alpha(nfw(rs=rs, ks=ks), x * rs, 0.0)[0]
    for x in (1e-3, 1e-4):
        g = 0.5 * x * x * (math.log(2 / x) - 0.5)
        assert a(x) == pytest.approx(4 * ks * rs * g / x, rel=3 * x * x * math.log(1 / x))
    for x in (1e3, 1e4):
        g = math.log(x / 2) + math.pi / (2 * x) - 1 / x ** 2
        assert a(x) == pytest.approx(4 * ks * rs * g / x, rel=2 / x ** 3)
    assert a(1.0) == pytest.approx(4 * ks * rs * (1 - math.log(2)), rel=1e-15)
    assert abs(a(1 - 1e-9) - a(1.0)) < 1e-8 and abs(a(1 + 1e-9) - a(1.0)) < 1e-8


def test_nfw_pseudo_elliptical_field_is_a_rotated_gradient():
    """Rotating the point about the centre together with Phi rotates the
    deflection (Algorithm 1's frame change), and the field is curl-free (a
    gradient of the pseudo-elliptical potential): d a1/d t2 = d a2/d t1 by
    central differences.  Catches a wrong rotation sign or eps on the wrong axis."""
    p0 = nfw(x=1.5, y=-2.0, eps=0.3, phi=0.0, rs=8.0, ks=0.3)
    phi = 0.7
    p1 = p0.copy()
    p1[3, 0] = phi
    c, s = math.cos(phi), math.sin(phi)
    for d in ((3.0, 1.0), (-0.4, 5.0), (12.0, -9.0)):
        a0 = np.array(oracle.nfw_alpha(p0, 1.5 + d[0], -2.0 + d[1]))
        r = (c * d[0] - s * d[1], s * d[0] + c * d[1])
        a1 = np.array(oracle.nfw_alpha(p1, 1.5 + r[0], -2.0 + r[1]))
        np.testing.assert_allclose(a1, [c * a0[0] - s * a0[1], s * a0[0] + c * a0[1]], rtol=1e-12, atol=1e-14)
    p = nfw(x=0.0, y=0.0, eps=0.25, phi=0.4, rs=6.0, ks=0.25)
    h = 1e-5
    for t in ((2.0, 1.0), (-7.0, 3.0), (0.5, -0.3)):
        d12 = (oracle.nfw_alpha(p, t[0], t[1] + h)[0] - oracle.nfw_alpha(p, t[0], t[1] - h)[0]) / (2 * h)
        d21 = (oracle.nfw_alpha(p, t[0] + h, t[1])[1] - oracle.nfw_alpha(p, t[0] - h, t[1])[1]) / (2 * h)
        assert d12 == pytest.approx(d21, rel=1e-6, abs=1e-9)
