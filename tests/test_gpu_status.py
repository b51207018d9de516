"""Numerical status reporting (mnf_status) through the C ABI: non-finite
input intensities are reported as MNF_ENONFINITE by the next status call,
which clears the record; a finite run reports MNF_OK."""
import numpy as np
import pytest
import torch

from paper_2608_01746_amd import lib as L
from paper_2608_01746_amd import synth

from _cases import tiny_scan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


def _run(api, I, err=True):
    O, P, pos, _ = tiny_scan(96, 32, 32, 4, 16, 4, seed=5)
    Og = torch.ones((96, 96), dtype=torch.complex64, device=DEV)
    Pg = torch.from_numpy(P.astype(np.complex64)).to(DEV)
    e = api.ptycho_iterate(Og, Pg, torch.from_numpy(I.astype(np.float32)).to(DEV), pos, 3, alg="rpie",
                           alpha=0.2, beta=0.2, batch=4, update_probe=True, order=synth.random_orders(len(pos), 3, 1))
    return e


def test_finite_run_reports_ok(api):
    _, _, _, I = tiny_scan(96, 32, 32, 4, 16, 4, seed=5)
    api.status()  # clear anything earlier tests left
    e = _run(api, I)
    assert api.status() == 0
    assert torch.isfinite(e).all()


def test_nan_intensity_reports_nonfinite_once(api):
    _, _, _, I = tiny_scan(96, 32, 32, 4, 16, 4, seed=5)
    api.status()
    I = I.copy()
    I[3, 10, 11] = np.nan
    _run(api, I)
    assert api.status() == L.MNF_ENONFINITE
    assert api.status() == 0  # the record was cleared
    with pytest.raises(api.MnfError):
        _run(api, I)
        api.check_status()


def test_nan_in_gradient_loss_reports_nonfinite(api):
    O, P, pos, I = tiny_scan(96, 32, 32, 4, 16, 4, seed=5)
    api.status()
    I = I.copy()
    I[0, 0, 0] = np.inf
    api.ptycho_grad(torch.from_numpy(O.astype(np.complex64)).to(DEV), torch.from_numpy(P.astype(np.complex64)).to(DEV),
                    torch.from_numpy(I.astype(np.float32)).to(DEV), pos, "poisson", 1e-6, 4)
    assert api.status() == L.MNF_ENONFINITE


def test_device_upstream_scales_the_gradient(api):
    O, P, pos, I = tiny_scan(96, 32, 32, 4, 16, 4, seed=6)
    Ot = torch.from_numpy((O * 0.9).astype(np.complex64)).to(DEV)
    Pt = torch.from_numpy(P.astype(np.complex64)).to(DEV)
    It = torch.from_numpy(I.astype(np.float32)).to(DEV)
    _, g1, p1 = api.ptycho_grad(Ot, Pt, It, pos, "poisson", 1e-6, 4)
    up = torch.tensor(-2.5, dtype=torch.float64, device=DEV)
    _, g2, p2 = api.ptycho_grad(Ot, Pt, It, pos, "poisson", 1e-6, 4, up)
    torch.testing.assert_close(g2, -2.5 * g1, rtol=1e-6, atol=1e-6 * float(g1.abs().max()))
    torch.testing.assert_close(p2, -2.5 * p1, rtol=1e-6, atol=1e-6 * float(p1.abs().max()))
