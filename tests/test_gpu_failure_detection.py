"""Failure detection: lbm_solver_moments reports non-finite mass or momentum
totals (a NaN or an infinity in the PDFs) as LBM_ERANGE. The NaN is put in
from the host through the import call; no kernel faults."""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PER = (True, False, False)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("pattern,t", [("aa", 0), ("aa", 1), ("osnt", 0)])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_moments_flags_nonfinite_totals(prec, pattern, t, bad):
    from paper_1410_0412_amd import LbmError, Lattice, Solver
    from paper_1410_0412_amd._capi import LBM_ERANGE
    mask = rsa_spheres((16, 16, 16), 2.5, 0.2, PER, seed=0)
    lat = Lattice(mask, PER, "lex", 0)
    s = Solver(lat, 0.8, (1e-5, 0.0, 0.0), pattern=pattern, precision=prec)
    s.init()
    s.step(3)
    rho, _, tot = s.moments()  # finite state: no error
    assert torch.isfinite(tot).all()
    f = s.export_pdfs()
    node = lat.n_fluid // 2
    f[7, node] = bad
    s.import_pdfs(f, t=t)
    print("case", prec, pattern, t, bad, flush=True)
    with pytest.raises(LbmError) as e:
        s.moments()
    assert e.value.code == LBM_ERANGE and "non-finite" in str(e.value)
    # a step spreads it; the next moments call still reports it
    s.step(1)
    with pytest.raises(LbmError) as e:
        s.moments()
    assert e.value.code == LBM_ERANGE
    # a fresh initial state clears the condition
    s.init()
    _, _, tot = s.moments()
    assert torch.isfinite(tot).all()
