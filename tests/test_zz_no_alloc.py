"""mtp_grade_from_b_noalloc (the grade of section 2.3 with its product
c = b A^{-1} in the library's fixed device scratch instead of allocated
memory) against mtp_grade_from_b on the same rows, through the C ABI: two
calls in a row, the second with fewer rows, then a size beyond the scratch
rejected before any launch."""
import numpy as np
import pytest
import torch

from gpu_common import log, pot_path

pytestmark = pytest.mark.gpu


def test_grade_noalloc_matches_grade_from_b():
    from paper_2007_08555_amd import Potential
    from paper_2007_08555_amd._lib import MTPError
    import os
    A = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "active_lev16_s3.npz"))["A"]
    P = Potential(pot_path("lev16_s3"))
    P.set_active_set(A)
    rng = np.random.default_rng(11)
    scale = np.abs(A).max(axis=0)
    for n in (3000, 700):
        # rows like descriptor rows: active rows mixed and perturbed, column scales of A
        mix = rng.normal(size=(n, A.shape[0])) @ A / np.sqrt(A.shape[0])
        b = torch.as_tensor(mix + 0.01 * rng.normal(size=mix.shape) * scale, device="cuda:0").contiguous()
        g_ref, a_ref = P.grade_from_b(b)
        gamma = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
        arg = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
        P.grade_from_b_noalloc(b, gamma, arg)
        torch.cuda.synchronize()
        log(f"[no-alloc grade] n={n}: gamma {gamma.min().item():.3g}..{gamma.max().item():.3g}")
        # same kernels on the same inputs: identical results
        assert torch.equal(gamma, g_ref) and torch.equal(arg, a_ref)
    too_many = (1 << 21) // P.m + 1
    big = torch.zeros((too_many, P.m), dtype=torch.float64, device="cuda:0")
    g = torch.empty(too_many, dtype=torch.float64, device="cuda:0")
    a = torch.empty(too_many, dtype=torch.int32, device="cuda:0")
    with pytest.raises(MTPError, match="fixed scratch"):
        P.grade_from_b_noalloc(big, g, a)
