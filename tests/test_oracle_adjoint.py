"""Pins for the partial-bounce-back forward and the autograd gradient oracle:
ns = 0 is plain BGK bitwise, the torch forward equals the numpy oracle, and
autograd agrees with central finite differences of the numpy oracle."""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres, pbb_fraction
from oracle import dense, adjoint

PER = (True, False, False)


@pytest.fixture(scope="module")
def small():
    mask = rsa_spheres((10, 9, 8), 2.0, 0.2, PER, seed=31)
    ns = pbb_fraction(mask, seed=32)
    w = np.zeros(mask.shape)
    w[-1] = 1.0
    w[mask != 0] = 0.0
    return mask.astype(bool), ns, w


def test_zero_fraction_is_bgk(small):
    solid, ns, _ = small
    a = dense.run(solid, PER, 0.8, (1e-5, 0, 0), 6)
    b = dense.run(solid, PER, 0.8, (1e-5, 0, 0), 6, ns=np.zeros(solid.shape))
    assert np.array_equal(a, b)


def test_torch_forward_matches_numpy(small):
    solid, ns, w = small
    f = dense.run(solid, PER, 0.8, (1e-5, 0, 0), 8, ns=ns)
    _, j = dense.density_and_momentum(f)
    want = float((w * j[0]).sum())
    import torch
    got = adjoint.objective(torch.from_numpy(ns), solid, PER, 0.8, (1e-5, 0, 0), 8, w)
    assert float(got) == want


def test_full_bounce_back_site_reverses(small):
    # ns = 1 returns every PDF of a site to the opposite direction unchanged
    solid, _, _ = small
    rng = np.random.default_rng(3)
    f = dense.initial_state(solid) + 1e-3 * rng.random((19,) + solid.shape)
    ns = np.ones(solid.shape)
    post = dense.collide(f, 0.8, (0, 0, 0), ns=ns)
    from oracle.d3q19 import OPP
    for q in range(19):
        assert np.array_equal(post[q], f[OPP[q]])


def test_autograd_matches_finite_differences(small):
    solid, ns, w = small
    steps, tau, F = 12, 0.8, (1e-5, 0, 0)
    J, g = adjoint.gradient(ns, solid, PER, tau, F, steps, w)
    fluid = np.argwhere(~solid)
    big = fluid[np.argsort(-np.abs(g[~solid]))[:6]]

    def Jn(x):
        f = dense.run(solid, PER, tau, F, steps, ns=x)
        return float((w * dense.density_and_momentum(f)[1][0]).sum())

    for s in big:
        s = tuple(s)
        def D(h):
            p, m = ns.copy(), ns.copy()
            p[s] += h
            m[s] -= h
            return (Jn(p) - Jn(m)) / (2 * h)
        fd = (4 * D(5e-4) - D(1e-3)) / 3  # Richardson
        assert abs(fd - g[s]) <= 1e-6 * abs(g[s]), (s, fd, g[s])
