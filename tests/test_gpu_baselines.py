"""The linear fusion baselines on the GPU against the float64 oracle, on the
small workload's exposure stack (CPU-simulated, saturated and noisy)."""
import numpy as np
import pytest
import torch

from oracle import baselines

from _cases import small_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


@pytest.mark.parametrize("dark", [0.0, 3.0])
def test_linear_integration_matches_oracle(api, dark):
    c = small_case()
    w = c["w"]
    raw = c["raw"]
    assert (raw == w.sat).any()  # saturated pixels are present
    got = api.fuse_linear(torch.from_numpy(raw).to(DEV), w.t, w.sat, dark)
    want = baselines.linear_integration(raw, w.t, w.sat, dark)
    g = got.cpu().numpy()
    # integer count sums are exact in float32; one float32 division and product remain
    assert np.all(np.abs(g - want) <= 2e-7 * np.abs(want) + 1e-6)


def test_shortest_frame_matches_oracle(api):
    c = small_case()
    w = c["w"]
    got = api.fuse_linear(torch.from_numpy(c["raw"]).to(DEV), w.t, w.sat, 1.0,
                          mode="shortest")
    assert np.array_equal(got.cpu().numpy(), baselines.single_exposure(c["raw"], 1.0).astype(np.float32))


def test_linear_rejects_bad_arguments(api):
    raw = torch.zeros((1, 2, 8, 8), dtype=torch.uint16, device=DEV)
    with pytest.raises(api.MnfError, match="MNF_EINVAL"):
        api.fuse_linear(raw, [1.0, 0.0], 4095.0)
    with pytest.raises(api.MnfError, match="MNF_EINVAL"):
        api.fuse_linear(raw, [1.0, 2.0], 0.0, 1.0)
