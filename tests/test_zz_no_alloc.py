"""The allocation-free projection blp_sine_project_noalloc, through the C
ABI, against blp_sine_project (same kernels and order of summation, so the
two agree bit for bit): two calls in a row on one GPU, the second with a
smaller input (the fixed scratch array keeps the first call's contents),
then a request larger than the scratch array, which must be refused with
BLP_E_SCRATCH, and a normal call after it."""
import sys

import numpy as np
import pytest

from paper_2108_13468_amd import inputs

pytestmark = pytest.mark.gpu

BLP_E_SCRATCH = -6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_projection_matches_allocating_one():
    import torch
    assert torch.cuda.is_available()
    from paper_2108_13468_amd import blp
    rng = np.random.default_rng(77)
    cases = [(1024, 64, 48), (256, 8, 5)]  # (N, K, L): the second call is smaller
    probs = []
    for N, K, L in cases:
        p = blp.from_instance(inputs.plain(N, 1e-5, seed=78))
        probs.append(p)
        w = torch.as_tensor(rng.standard_normal((N - 1) ** 2), device="cuda")
        say("noalloc projection N=%d K=%d L=%d" % (N, K, L))
        g0 = p.sine_project(w, K, L)
        g1 = p.sine_project_noalloc(w, K, L)
        assert g1.shape == (L, K)
        assert np.array_equal(g0, g1), np.abs(g0 - g1).max()
    # a request beyond the 4 MiB array is refused, and the array stays usable
    p = probs[0]
    w = torch.zeros((1024 - 1) ** 2, dtype=torch.float64, device="cuda")
    with pytest.raises(blp.BlpError) as e:
        p.sine_project_noalloc(w, 300, 300)
    assert e.value.code == BLP_E_SCRATCH
    w = torch.as_tensor(rng.standard_normal((1024 - 1) ** 2), device="cuda")
    assert np.array_equal(p.sine_project(w, 16, 16), p.sine_project_noalloc(w, 16, 16))
