"""The screener's forward pass without allocation (nep_mlp_forward_noalloc) against
nep_mlp_forward with a caller-allocated workspace: identical probabilities (the same
kernels and arithmetic), on two calls in a row with the second one smaller, so that a
stale or misaddressed activation array would show; and the batch limit."""
import numpy as np
import pytest

import gen
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def test_forward_without_allocation_matches_the_workspace_forward():
    import torch
    assert torch.cuda.is_available()
    from paper_2312_13117_amd import nep as N
    N.lib()
    say("case forward without allocation: B = 3000 then 37")
    rng = np.random.default_rng(71)
    params = torch.from_numpy(gen.mlp_init(7)).to("cuda")
    rows = 5000
    X = torch.from_numpy(rng.standard_normal((rows, 32)).astype(np.float32)).to("cuda")
    for B in (3000, 37):
        idx = torch.from_numpy(rng.choice(rows, size=B, replace=False).astype(np.int32)).to("cuda")
        ref = torch.empty((B, 4), dtype=torch.float32, device="cuda")
        work = torch.empty(N.nep_mlp_workspace_floats(B), dtype=torch.float32, device="cuda")
        N.nep_mlp_forward(params, X, idx, B, ref, work)
        got = torch.full((B, 4), -1.0, dtype=torch.float32, device="cuda")
        N.nep_mlp_forward_noalloc(params, X, idx, B, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"B = {B}"
        assert float(got.min()) > 0.0 and float(got.max()) < 1.0
    # beyond the array: rejected before any launch
    too_many = N.NEP_MLP_NOALLOC_MAX_B + 1
    idx = torch.zeros(too_many, dtype=torch.int32, device="cuda")
    out = torch.empty((too_many, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(N.NepError) as e:
        N.nep_mlp_forward_noalloc(params, X, idx, too_many, out)
    assert e.value.status == -5                                  # NEP_ERR_CAPACITY
