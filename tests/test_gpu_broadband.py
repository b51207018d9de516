"""Discrete-spectrum measurement (Eq. 4) on the GPU against the float64
oracle: the resampling of one pattern and the two-line forward model."""
import numpy as np
import pytest
import torch

from oracle import broadband, ptycho
from paper_2608_01746_amd import synth

from _cases import c64, f32

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("Nd,s", [(32, 0.818), (64, 0.9), (64, 1.0), (65, 0.75), (128, 1.2)])
def test_resample_matches_oracle(api, Nd, s):
    rng = np.random.default_rng(Nd)
    I = f32(rng.gamma(0.5, 10.0, size=(3, Nd, Nd)))
    got = api.detector_resample(torch.from_numpy(I.astype(np.float32)).to(DEV), np.float32(s), 0.5)
    want = 0.5 * broadband.resample(I, float(np.float32(s)))
    assert rel(got.cpu().numpy(), want) < 1e-5


def test_two_line_forward_model_matches_oracle(api):
    # the XUV source's 9th and 11th harmonics of 515 nm, reference the 11th
    O = c64(synth.make_object(96, 5))
    P = c64(synth.make_probe(32, 8.0, np.pi))
    pos = synth.raster_positions(3, 12, 10)
    scales = [1.0, float(np.float32(9.0 / 11.0))]
    weights = [0.6, 0.4]
    got = api.broadband_forward(torch.from_numpy(O.astype(np.complex64)).to(DEV),
                                torch.from_numpy(P.astype(np.complex64)).to(DEV), pos, 64, scales, weights)
    ref = ptycho.forward_intensity(O, P, pos, 64)
    want = broadband.broadband(ref, scales, weights)
    assert rel(got.cpu().numpy(), want) < 1e-5


def test_resample_accumulates_and_rejects_aliasing(api):
    I = torch.rand((2, 16, 16), device=DEV)
    a = api.detector_resample(I, 1.0, 1.0)
    api.detector_resample(I, 1.0, 2.0, out=a, accumulate=True)
    assert torch.allclose(a, 3.0 * I)
    with pytest.raises(api.MnfError, match="alias"):
        api.detector_resample(I, 0.9, out=I)
    with pytest.raises(api.MnfError, match="MNF_EINVAL"):
        api.detector_resample(I, 0.0)
