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


@pytest.mark.parametrize("ria", [False, True, "direction"])
def test_wide_slots_gradient_bitwise(small, ria):
    # the partial-bounce-back, state-saving and adjoint step kernels with
    # 64-bit slot offsets (the form grids of more than 2^31 - 1 elements
    # take) give the same J and gradient as the 32-bit form, bit for bit
    from paper_1410_0412_amd import outlet_flux
    mask, ns, w = small
    out = []
    for wide in (False, True):
        lat, s = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", ria, pbb=True, wide_slots=wide)
        x = torch.from_numpy(nodes_of(lat, ns)).cuda().requires_grad_(True)
        J = outlet_flux(x, s, 12, 5, torch.from_numpy(nodes_of(lat, w)).cuda())
        J.backward()
        out.append((J.item(), x.grad.cpu().numpy()))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


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


def test_backward_uses_its_own_forward_and_restores_the_solver(small):
    # forward(ns1), forward(ns2), then the backward of the first: the
    # gradient equals that of forward(ns1) alone, bitwise, and the solver
    # keeps the grid, time and solid fraction the second forward left
    from paper_1410_0412_amd import outlet_flux
    mask, ns, w = small
    T, every = 12, 5
    lat, s = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", "direction", pbb=True)
    wt = torch.from_numpy(nodes_of(lat, w)).cuda()
    ns1 = torch.from_numpy(nodes_of(lat, ns)).cuda()
    ns2 = (ns1 * 0.5).flip(0)
    x_ref = ns1.clone().requires_grad_(True)
    outlet_flux(x_ref, s, T, every, wt).backward()
    x1 = ns1.clone().requires_grad_(True)
    x2 = ns2.clone().requires_grad_(True)
    J1 = outlet_flux(x1, s, T, every, wt)
    J2 = outlet_flux(x2, s, T + 1, every, wt)
    after_pdf, after_t, after_ns = s.pdf[0].clone(), s.t, s.solid_frac[: s.n_fluid].clone()
    assert after_t == T + 1 and torch.equal(after_ns, ns2)
    J1.backward()
    assert torch.equal(x1.grad, x_ref.grad)
    assert torch.equal(s.pdf[0], after_pdf) and s.t == after_t
    assert torch.equal(s.solid_frac[: s.n_fluid], after_ns)
    # the solver steps on from the restored state exactly as before
    J2.backward()
    x2_ref = ns2.clone().requires_grad_(True)
    _, s2 = solver_for(mask, PER, 0.8, (1e-5, 0, 0), "aa", "direction", pbb=True)
    outlet_flux(x2_ref, s2, T + 1, every, wt).backward()
    assert torch.equal(x2.grad, x2_ref.grad)


def ridders(D, h0, levels=7, c=2.0):
    """Derivative from central differences D(h) by Ridders' method (C. J. F.
    Ridders, Adv. Eng. Software 4(2), 1982): a Neville tableau extrapolates
    D(h0), D(h0/c), D(h0/c^2), ... to h = 0 in powers of h^2; the entry whose
    neighbours in the tableau agree best is kept, and the sweep stops once
    the diagonal drifts away by more than twice that agreement. Returns
    (estimate, error estimate). The estimate uses only values of J."""
    prev = [D(h0)]
    best, err = prev[0], float("inf")
    h = h0
    for i in range(1, levels):
        h /= c
        row = [D(h)]
        f = c * c
        for j in range(1, i + 1):
            row.append((row[j - 1] * f - prev[j - 1]) / (f - 1))
            f *= c * c
            e = max(abs(row[j] - row[j - 1]), abs(row[j] - prev[j - 1]))
            if e <= err:
                err, best = e, row[j]
        if abs(row[i] - prev[i - 1]) >= 2 * err:
            break
        prev = row
    return best, err


def spherepack128_gradient(force, ria):
    from paper_1410_0412_amd import outlet_flux
    mask, p = workload("spherepack-128", seed=0)
    ns_vox = pbb_fraction(mask, seed=1)
    T, every = p["steps"], 20
    lat, s = solver_for(mask, p["periodic"], p["tau"], force, "aa", ria, p["order"], p["block"], pbb=True)
    ns = torch.from_numpy(nodes_of(lat, ns_vox)).cuda()
    w = torch.from_numpy(nodes_of(lat, outlet_weight(mask))).cuda()
    x = ns.clone().requires_grad_(True)
    J = outlet_flux(x, s, T, every, w)
    J.backward()
    g = x.grad.cpu().numpy()
    print("spherepack-128, F = %g, index %s: N=%d J=%.6e max|g|=%.3e" % (force[0], s.index, lat.n_fluid, J.item(),
                                                                         np.abs(g).max()), flush=True)

    def fd(i):
        def Jat(h):
            y = ns.clone()
            y[i] += h
            return outlet_flux(y, s, T, every, w).item()

        def D(h):
            return (Jat(h) - Jat(-h)) / (2 * h)
        # J is a polynomial of degree ~T in each ns: steps from 8e-3 down
        est, _ = ridders(D, 8e-3)
        return abs(est - g[i]) / abs(g[i])

    return mask, lat, ns_vox, g, fd


@pytest.mark.parametrize("ria", [True, "direction"])
def test_finite_differences_spherepack128(ria):
    # the benchmark's adjoint case (F = 1e-6): the 32 largest gradients, with
    # the paper's runs and with per-direction runs (the automatic choice on
    # this lattice)
    _, _, _, g, fd = spherepack128_gradient((1e-6, 0.0, 0.0), ria)
    top = np.argsort(-np.abs(g))[:32]
    assert np.abs(g[top]).min() >= 1e-3 * np.abs(g).max()
    worst = max(fd(int(i)) for i in top)
    print("finite differences, F = 1e-6: worst relative deviation %.3e over the 32 largest |g|" % worst, flush=True)
    assert worst <= 1e-6


def test_finite_differences_spherepack128_sampled_nodes():
    # A seeded sample of the nodes with |g| >= 1e-3 max|g| beyond the 32
    # largest: 8 on the outlet plane (where J is taken), 8 next to the y/z
    # walls of the box, 8 partial-bounce-back nodes (0 < ns < 1, next to a
    # sphere) and 8 anywhere; and the 32 largest again. At F = 1e-6 the FP64
    # rounding of J (about 1e-15 absolute against J = 1.6e-2) puts a floor of
    # about 1e-5 on the relative accuracy of any finite difference for
    # gradients near 1e-3 max|g| (Ridders' own error estimate reaches 1e-5
    # there). At F = 1e-4, J and max|g| are 100.00 times larger (the flow is
    # nearly linear in F at these speeds) against the same rounding, and the
    # finite differences resolve about 1e-7 relative.
    mask, lat, ns_vox, g, fd = spherepack128_gradient((1e-4, 0.0, 0.0), "direction")
    top = np.argsort(-np.abs(g))[:32]
    nv = lat.node_voxel().astype(np.int64)
    x, y, z = np.unravel_index(nv, mask.shape)
    ok = np.abs(g) >= 1e-3 * np.abs(g).max()
    ok[top] = False
    nsn = nodes_of(lat, ns_vox)
    groups = {"outlet plane": ok & (x == mask.shape[0] - 1),
              "box walls": ok & ((y == 0) | (y == mask.shape[1] - 1) | (z == 0) | (z == mask.shape[2] - 1)),
              "partial bounce-back": ok & (nsn > 0),
              "anywhere": ok}
    rng = np.random.default_rng(7)
    picked = []
    for name, sel in groups.items():
        cand = np.setdiff1d(np.flatnonzero(sel), np.array(picked, dtype=np.int64))
        assert len(cand) >= 8, name
        pick = rng.choice(cand, 8, replace=False)
        picked.extend(int(i) for i in pick)
        errs = [fd(int(i)) for i in pick]
        print("finite differences, F = 1e-4, %s: worst relative deviation %.3e over 8 nodes (|g| / max|g| from "
              "%.1e to %.1e)" % (name, max(errs), np.abs(g[pick]).min() / np.abs(g).max(),
                                 np.abs(g[pick]).max() / np.abs(g).max()), flush=True)
        assert max(errs) <= 1e-6, name
    worst = max(fd(int(i)) for i in top)
    print("finite differences, F = 1e-4: worst relative deviation %.3e over the 32 largest |g|" % worst, flush=True)
    assert worst <= 1e-6
