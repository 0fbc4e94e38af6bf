"""Pins for the dense FP64 oracle: exact physics it must satisfy whatever its
implementation (moment identities, the propagation direction of eq. (1), the
bounce-back rule, conservation, forcing, and the Poiseuille closed form)."""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres, init_fields
from oracle import dense
from oracle.d3q19 import C, W, OPP, Q


def test_equilibrium_moments():
    rng = np.random.default_rng(1)
    rho = 1 + 0.1 * rng.standard_normal(50)
    u = 0.05 * rng.standard_normal((3, 50))
    feq = dense.equilibrium(rho, u)
    c = C.astype(float)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-14)
    for a in range(3):
        np.testing.assert_allclose((c[:, a, None] * feq).sum(0), rho * u[a], rtol=1e-12, atol=1e-16)
        for b in range(3):
            want = rho * (u[a] * u[b] + (1.0 / 3.0 if a == b else 0.0))
            np.testing.assert_allclose((c[:, a, None] * c[:, b, None] * feq).sum(0), want,
                                       rtol=1e-12, atol=1e-16)


def test_moments_of_equilibrium_roundtrip():
    rng = np.random.default_rng(2)
    rho = 1 + 0.01 * rng.standard_normal((4, 5, 6))
    u = 0.01 * rng.standard_normal((3, 4, 5, 6))
    r2, u2 = dense.macroscopic(dense.equilibrium(rho, u))
    np.testing.assert_allclose(r2, rho, rtol=1e-14)
    for a in range(3):
        np.testing.assert_allclose(u2[a], u[a], rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("q", range(1, 19))
def test_stream_moves_along_c(q):
    # eq. (1): the post-collision value f*_q(x) arrives at x + c_q
    shape = (5, 6, 7)
    solid = np.zeros(shape, bool)
    fs = np.zeros((Q,) + shape)
    x0 = np.array([2, 3, 4])
    fs[q][tuple(x0)] = 1.0
    out = dense.stream(fs, solid, (True, True, True))
    hit = np.argwhere(out[q] == 1.0)
    assert hit.shape == (1, 3)
    assert tuple(hit[0]) == tuple((x0 + C[q]) % np.array(shape))
    assert np.count_nonzero(out) == 1


@pytest.mark.parametrize("q", range(1, 19))
def test_bounce_back_at_wall(q):
    # a value heading into a solid site returns to its own site, reversed
    shape = (5, 5, 5)
    solid = np.zeros(shape, bool)
    x0 = np.array([2, 2, 2])
    solid[tuple(x0 + C[q])] = True
    fs = np.zeros((Q,) + shape)
    fs[q][tuple(x0)] = 1.0
    out = dense.stream(fs, solid, (True, True, True))
    out[:, solid] = 0
    assert out[OPP[q]][tuple(x0)] == 1.0
    assert np.count_nonzero(out) == 1


@pytest.mark.parametrize("axis", range(3))
def test_outside_is_solid_on_closed_axes(axis):
    shape = (4, 4, 4)
    solid = np.zeros(shape, bool)
    periodic = [True, True, True]
    periodic[axis] = False
    q = 1 + 2 * axis  # +axis direction
    x0 = [1, 1, 1]
    x0[axis] = shape[axis] - 1
    fs = np.zeros((Q,) + shape)
    fs[q][tuple(x0)] = 1.0
    out = dense.stream(fs, solid, tuple(periodic))
    assert out[OPP[q]][tuple(x0)] == 1.0 and np.count_nonzero(out) == 1


def test_rest_state_is_a_fixed_point():
    mask = rsa_spheres((16, 16, 16), 2.5, 0.2, (True, False, False), seed=3).astype(bool)
    f = dense.run(mask, (True, False, False), 0.8, (0.0, 0.0, 0.0), 20)
    # the rest weights do not sum to exactly 1.0 in floating point, so the
    # state may move by an ulp, but it must not drift
    for q in range(Q):
        assert np.max(np.abs(f[q][~mask] - W[q])) < 1e-15


def test_mass_conservation():
    mask = rsa_spheres((16, 16, 16), 2.5, 0.2, (True, False, False), seed=4).astype(bool)
    rho0, u0 = init_fields(mask.shape, seed=5)
    f0 = dense.initial_state(mask, rho0, u0)
    m0 = dense.macroscopic(f0)[0][~mask].sum()
    f = dense.run(mask, (True, False, False), 0.7, (1e-5, 0, 0), 200, f0=f0)
    m1 = dense.macroscopic(f)[0][~mask].sum()
    assert abs(m1 - m0) / m0 < 1e-13


def test_uniform_periodic_box_gains_force():
    # sum_q S_q = 0 and sum_q c_q S_q = F: j grows by F every step everywhere
    shape = (3, 4, 5)
    solid = np.zeros(shape, bool)
    F = (2e-5, -1e-5, 3e-6)
    f = dense.initial_state(solid)
    for t in range(1, 31):
        f = dense.step(f, solid, (True, True, True), 0.9, F)
        rho, j = dense.density_and_momentum(f)
        np.testing.assert_allclose(rho, 1.0, rtol=0, atol=1e-14)
        for a in range(3):
            np.testing.assert_allclose(j[a], t * F[a], rtol=1e-11, atol=1e-18)


def poiseuille(H, tau, F):
    """Steady BGK plane Poiseuille flow with halfway bounce-back and simple
    forcing. Fluid rows y = 1..H, walls at 1/2 and H + 1/2:
    u(y) = F/(2 nu) (y - 1/2)(H + 1/2 - y) + F (16 tau^2 - 20 tau + 3) / (4 (2 tau - 1)),
    nu = (tau - 1/2)/3. The second term is the BGK bounce-back slip, from the
    x-antisymmetric populations (derivation in the design notes)."""
    y = np.arange(1, H + 1, dtype=float)
    nu = (tau - 0.5) / 3.0
    return F / (2 * nu) * (y - 0.5) * (H + 0.5 - y) + F * (16 * tau ** 2 - 20 * tau + 3) / (4 * (2 * tau - 1))


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_poiseuille_closed_form(tau):
    H, F = 8, 1e-5
    shape = (2, H, 2)
    solid = np.zeros(shape, bool)
    nu = (tau - 0.5) / 3
    steps = int(30 * H * H / (nu * np.pi ** 2)) + 1
    f = dense.run(solid, (True, False, True), tau, (F, 0, 0), steps)
    rho, u = dense.macroscopic(f)
    want = poiseuille(H, tau, F)
    got = u[0][0, :, 0]
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-10
    np.testing.assert_allclose(rho, 1.0, atol=1e-13)
    assert np.max(np.abs(u[1])) < 1e-15 * F * 1e6 and np.max(np.abs(u[2])) < 1e-15 * F * 1e6


def test_cone_sites_match_full_run():
    mask = rsa_spheres((12, 10, 9), 2.0, 0.2, (True, False, False), seed=6).astype(bool)
    periodic = (True, False, False)
    rho0, u0 = init_fields(mask.shape, seed=7)
    f = dense.run(mask, periodic, 0.7, (1e-5, 0, 0), 3, rho0, u0)
    fl = np.argwhere(~mask)
    sites = fl[np.random.default_rng(8).choice(len(fl), 12, replace=False)]
    got = dense.cone_sites(mask, periodic, 0.7, (1e-5, 0, 0), 3, rho0, u0, sites)
    want = np.stack([f[:, s[0], s[1], s[2]] for s in sites])
    assert np.array_equal(got, want)


# ------------------------------------------------------------------ TRT ----

def poiseuille_trt(H, tau, F, magic):
    """Steady TRT plane Poiseuille flow with halfway bounce-back and simple
    forcing: the wall-location error depends on Lambda only, and u = j/rho
    without the half-force shift lags the parabola by F/2:
    u(y) = F/(2 nu) ((y - 1/2)(H + 1/2 - y) + (16 Lambda - 3)/12) - F/2.
    For BGK (Lambda = (tau - 1/2)^2) this is the closed form above."""
    y = np.arange(1, H + 1, dtype=float)
    nu = (tau - 0.5) / 3.0
    return F / (2 * nu) * ((y - 0.5) * (H + 0.5 - y) + (16 * magic - 3) / 12) - F / 2


def test_trt_closed_form_reduces_to_bgk():
    for tau in (0.6, 0.8, 1.3):
        np.testing.assert_allclose(poiseuille_trt(8, tau, 1e-5, (tau - 0.5) ** 2),
                                   poiseuille(8, tau, 1e-5), rtol=1e-12)


@pytest.mark.parametrize("tau,magic", [(0.8, 3 / 16), (1.3, 3 / 16), (0.7, 1 / 12), (1.0, 0.25)])
def test_trt_poiseuille_closed_form(tau, magic):
    H, F = 8, 1e-5
    solid = np.zeros((2, H, 2), bool)
    nu = (tau - 0.5) / 3
    om = dense.trt_omega_minus(tau, magic)
    steps = int(40 * H * H / (nu * np.pi ** 2)) + int(200 / min(1 / tau, om))
    f = dense.run(solid, (True, False, True), tau, (F, 0, 0), steps, magic=magic)
    rho, u = dense.macroscopic(f)
    want = poiseuille_trt(H, tau, F, magic)
    assert np.max(np.abs(u[0][0, :, 0] - want)) / np.max(np.abs(want)) < 1e-10


def test_trt_with_bgk_magic_is_bgk():
    mask = rsa_spheres((10, 10, 10), 2.0, 0.2, (True, False, False), seed=12).astype(bool)
    rho0, u0 = init_fields(mask.shape, seed=13)
    tau = 0.8
    a = dense.run(mask, (True, False, False), tau, (1e-5, 0, 0), 10, rho0, u0)
    b = dense.run(mask, (True, False, False), tau, (1e-5, 0, 0), 10, rho0, u0, magic=(tau - 0.5) ** 2)
    np.testing.assert_allclose(b[:, ~mask], a[:, ~mask], rtol=0, atol=1e-15)


def test_trt_conservation_and_force():
    mask = rsa_spheres((14, 12, 10), 2.5, 0.2, (True, False, False), seed=14).astype(bool)
    rho0, u0 = init_fields(mask.shape, seed=15)
    f0 = dense.initial_state(mask, rho0, u0)
    m0 = dense.macroscopic(f0)[0][~mask].sum()
    f = dense.run(mask, (True, False, False), 0.7, (1e-5, 0, 0), 100, f0=f0, magic=0.1)
    assert abs(dense.macroscopic(f)[0][~mask].sum() - m0) / m0 < 1e-13
    shape = (3, 4, 5)
    solid = np.zeros(shape, bool)
    g = dense.initial_state(solid)
    for t in range(1, 11):
        g = dense.step(g, solid, (True, True, True), 0.9, (2e-5, -1e-5, 3e-6), magic=0.2)
        _, j = dense.density_and_momentum(g)
        np.testing.assert_allclose(j[0], t * 2e-5, rtol=1e-11)
