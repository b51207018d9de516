"""Launch timing: every launch of a class, or a sample of every k-th launch
(the first included), counted per class from the last reset."""
import math

import numpy as np
import pytest
import torch

from _cases import tiny_scan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


def test_sampled_launch_timing(api):
    O, P, pos, I = tiny_scan(200, 128, 128, 3, 30, 5, seed=11)
    Ig = torch.from_numpy(np.asarray(I, np.float32)).to(DEV)

    def run(n_iter):
        Og = torch.ones((200, 200), dtype=torch.complex64, device=DEV)
        Pg = torch.from_numpy(P.astype(np.complex64)).to(DEV)
        api.ptycho_iterate(Og, Pg, Ig, pos, n_iter, alg="rpie", batch=4, update_probe=False)
        torch.cuda.synchronize()

    J, B, n_iter = len(pos), 4, 5
    per_pass = n_iter * math.ceil(J / B)  # launches of each pass: 5 iterations x 3 mini-batches
    try:
        api.profile(["rows_fwd", "object_update"])
        api.profile_reset()
        run(n_iter)
        every_launch = api.profile_read()
        assert every_launch["rows_fwd"][0] == per_pass and every_launch["object_update"][0] == per_pass
        for k in (2, 4, 7):
            api.profile(["rows_fwd"], every=k)
            api.profile_reset()
            run(n_iter)
            got = api.profile_read()
            assert set(got) == {"rows_fwd"}
            n, ms = got["rows_fwd"]
            assert n == math.ceil(per_pass / k)  # launches 0, k, 2k, ...
            assert ms > 0.0
        # a reset restarts the count: the next launch is timed again
        api.profile(["rows_fwd"], every=per_pass + 1)
        api.profile_reset()
        run(1)
        assert api.profile_read()["rows_fwd"][0] == 1
        with pytest.raises(api.MnfError):
            api.profile(["rows_fwd"], every=0)
    finally:
        api.profile([])
