"""Hand-written adjoint of the AA step (partial bounce-back, FP64) through the
C ABI: forward parity with the oracle, gradients against autograd through the
dense torch oracle, and central finite differences at the 128^3 sphere pack
(porosity 0.5, 200 steps, checkpoints every 20)."""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres, pbb_fraction, workload
from oracle import dense, adjoint as adj_oracle
from tests.gpu_util import solver_for, oracle_at_nodes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PER = (True, False, False)


def outlet_weight(mask):
    w = np.zeros(mask.shape)
    w[-1] = 1.0
    w[mask != 0] = 0.0
    return w


@pytest.fixture(scope="module")
def small():
    mask = rsa_spheres((10, 9, 8), 2.0, 0.2, PER, seed=31)
    ns = pbb_fraction(mask, seed=32)
    return mask, ns, outlet_weight(mask)


def nodes_of(lat, field):
    return field.reshape(-1)[lat.node_voxel().astype(np.int64)]


@pytest.mark.parametrize("ria", [False, True, "direction"])
def test_pbb_forward_every_step(small, ria):
    mask, ns, _ = small
    tau, F = 0.8, (1e-5, 0, 0)
    lat, s = solver_for(mask, PER, tau, F, "aa", ria, pbb=True)
    s.set_solid_fraction(torch.from_numpy(nodes_of(lat, ns)).cuda())
    s.init()
    f = dense.initial_state(mask.astype(bool))
    for t in range(1, 7):
        s.step(1)
        f = dense.step(f, mask.astype(bool), PER, tau, F, ns=ns)
        assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f)), t


def test_pbb_zero_fraction_is_plain_step(small):
    mask, _, _ = small
    lat, a = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", True, pbb=True)
    _, b = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", True)
    a.init(); b.init()
    a.step(9); b.step(9)
    assert np.array_equal(a.export_pdfs().cpu().numpy(), b.export_pdfs().cpu().numpy())


def fluid_slots(n_fluid):
    """Element offsets of every (q, n) slot of the fluid nodes in the
    tile-major grid: direction q of node n = 64t + l at (19t + q)*64 + l."""
    n = np.arange(n_fluid)
    return (((19 * (n // 64))[None, :] + np.arange(19)[:, None]) * 64 + (n % 64)[None, :]).reshape(-1)


@pytest.mark.parametrize("ria", [False, True, "direction"])
@pytest.mark.parametrize("pbb", [True, False])
def test_step_save(small, ria, pbb):
    # step_save keeps the state each step reads and steps exactly like step
    mask, ns, _ = small
    lat, a = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", ria, pbb=pbb)
    _, b = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", ria, pbb=pbb)
    if pbb:
        x = torch.from_numpy(nodes_of(lat, ns)).cuda()
        a.set_solid_fraction(x)
        b.set_solid_fraction(x)
    a.init()
    b.init()
    idx = torch.from_numpy(fluid_slots(lat.n_fluid)).cuda()
    save = torch.full_like(a.pdf[0], float("nan"))
    for t in range(5):  # both parities
        before = a.pdf[0].clone()
        a.step_save(save)
        b.step(1)
        assert torch.equal(save[idx], before[idx]), t
        assert torch.equal(a.pdf[0][idx], b.pdf[0][idx]), t
    assert a.t == b.t == 5


def test_step_save_needs_aa_fp64_bgk(small):
    from paper_1410_0412_amd import LbmError
    mask, _, _ = small
    _, s = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", True, pbb=True)
    s.init()
    with pytest.raises(LbmError):
        s.step_save(s.pdf[0])  # the solver's own grid
    for kw in (dict(pattern="osnt"), dict(pattern="aa", precision="f32"), dict(pattern="aa", trt_magic=0.25)):
        pattern = kw.pop("pattern")
        _, s = solver_for(mask, PER, 0.8, (1e-5, 0, 0), pattern, True, **kw)
        s.init()
        with pytest.raises(LbmError):
            s.step_save(torch.empty(19 * s.ldf, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("ria", [False, True, "direction"])
@pytest.mark.parametrize("every", [1, 5, 12])
def test_gradient_matches_autograd(small, ria, every):
    from paper_1410_0412_amd import outlet_flux
    mask, ns, w = small
    tau, F, T = 0.8, (1e-5, 0, 0), 12
    J_ref, g_ref = adj_oracle.gradient(ns, mask.astype(bool), PER, tau, F, T, w)
    lat, s = solver_for(mask, PER, tau, F, "aa", ria, pbb=True)
    x = torch.from_numpy(nodes_of(lat, ns)).cuda().requires_grad_(True)
    J = outlet_flux(x, s, T, every, torch.from_numpy(nodes_of(lat, w)).cuda())
    assert abs(J.item() - J_ref) <= 1e-13 * abs(J_ref)
    J.backward()
    g = x.grad.cpu().numpy()
    gr = nodes_of(lat, g_ref)
    err = np.max(np.abs(g - gr)) / np.max(np.abs(gr))
    print("gradient vs autograd (ria=%s, every=%d): %.3e" % (ria, every, err), flush=True)
    assert err <= 2e-12, err


def test_checkpoint_interval_does_not_change_gradient(small):
    from paper_1410_0412_amd import outlet_flux
    mask, ns, w = small
    grads = []
    for every in (1, 3, 7, 13):
        lat, s = solver_for(mask, PER, 0.7, (1e-5, 0, 0), "aa", True, pbb=True)
        x = torch.from_numpy(nodes_of(lat, ns)).cuda().requires_grad_(True)
        outlet_flux(x, s, 13, every, torch.from_numpy(nodes_of(lat, w)).cuda()).backward()
        grads.append(x.grad.cpu().numpy())
    for g in grads[1:]:
        assert np.array_equal(g, grads[0])


def test_finite_differences_spherepack128():
    from paper_1410_0412_amd import outlet_flux
    mask, p = workload("spherepack-128", seed=0)
    ns_vox = pbb_fraction(mask, seed=1)
    w_vox = outlet_weight(mask)
    T, every = p["steps"], 20
    lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], "aa", True, p["order"], p["block"], pbb=True)
    ns = torch.from_numpy(nodes_of(lat, ns_vox)).cuda()
    w = torch.from_numpy(nodes_of(lat, w_vox)).cuda()
    x = ns.clone().requires_grad_(True)
    J = outlet_flux(x, s, T, every, w)
    J.backward()
    g = x.grad.cpu().numpy()
    print("spherepack-128: N=%d J=%.6e max|g|=%.3e" % (lat.n_fluid, J.item(), np.abs(g).max()), flush=True)
    top = np.argsort(-np.abs(g))[:32]
    assert np.abs(g[top]).min() >= 1e-3 * np.abs(g).max()

    def Jat(i, h):
        y = ns.clone()
        y[i] += h
        return outlet_flux(y, s, T, every, w).item()

    # J is a polynomial of degree ~T in each ns, so the step must be small:
    # Richardson's O(h^4) remainder is ~1e-2 at h = 1e-2 but negligible at
    # h = 5e-4, where FP64 cancellation stays below 1e-8 relative
    worst = 0.0
    for i in top:
        D = lambda h: (Jat(int(i), h) - Jat(int(i), -h)) / (2 * h)
        fd = (4 * D(2.5e-4) - D(5e-4)) / 3  # Richardson
        worst = max(worst, abs(fd - g[i]) / abs(g[i]))
    print("finite differences: worst relative deviation %.3e over 32 nodes" % worst, flush=True)
    assert worst <= 1e-6
