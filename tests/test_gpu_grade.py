"""GPU parity of the extrapolation grade (paper, section 2.3) against the
FP64 oracle: c = b A^{-1}, gamma = max |c_j|, argmax, and A^{-1} itself."""
import os

import numpy as np
import pytest

import synth
from gpu_common import log, pot_path
from oracle import grade as og
from oracle import mtp as omtp
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu

ACTIVE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "active_lev16_s3.npz")


@pytest.fixture(scope="module")
def setup():
    from paper_2007_08555_amd import Potential
    P = Potential(pot_path("lev16_s3"))
    A = np.load(ACTIVE)["A"]
    P.set_active_set(A)
    return P, read_potential(pot_path("lev16_s3")), A


def oracle_rows(pot, batch):
    return np.array([omtp.evaluate(pot, *synth.config_of(batch, k))["b"] for k in range(len(batch["n_atoms"]))])


def _compare(gam, arg, c, gam_o, arg_o, c_o, rtol):
    scale = np.abs(c_o).max(axis=1, keepdims=True)
    err = np.abs(c - c_o) / scale
    log(f"[grade] max rel error of c: {err.max():.3e}, gamma range {gam_o.min():.3g}..{gam_o.max():.3g}")
    assert err.max() <= rtol
    assert np.allclose(gam, gam_o, rtol=rtol)
    for r in range(len(gam)):
        if arg[r] != arg_o[r]:   # a near-tie: both indices must attain the maximum within tolerance
            assert abs(abs(c_o[r, arg[r]]) - gam_o[r]) <= rtol * scale[r, 0]


def test_grade_from_b_matches_oracle(setup):
    P, pot, A = setup
    batch = synth.mixed_batch(seed=11, n_configs=24, n_min=8, n_max=64, n_species_model=3)
    b = oracle_rows(pot, batch)
    gam, arg, c = P.grade_from_b(b, want_c=True)
    gam_o, arg_o, c_o = og.grade(b, A)
    _compare(gam.cpu().numpy(), arg.cpu().numpy(), c.cpu().numpy(), gam_o, arg_o, c_o, 1e-8)


def test_active_rows_have_grade_one(setup):
    P, _pot, A = setup
    gam, arg, c = P.grade_from_b(A, want_c=True)
    assert np.allclose(gam.cpu().numpy(), 1.0, atol=1e-8)
    assert np.array_equal(arg.cpu().numpy(), np.arange(len(A)))
    assert np.allclose(c.cpu().numpy(), np.eye(len(A)), atol=1e-8)


def test_grade_end_to_end(setup):
    P, pot, A = setup
    batch = synth.mixed_batch(seed=12, n_configs=16, n_min=8, n_max=96, n_species_model=3)
    from paper_2007_08555_amd import Batch
    gam, arg = P.grade(Batch.from_arrays(batch), precision="fp64")
    gam_o, arg_o, c_o = og.grade(oracle_rows(pot, batch), A)
    g = gam.cpu().numpy()
    log(f"[grade e2e] gamma gpu {g[:4]} oracle {gam_o[:4]}")
    assert np.allclose(g, gam_o, rtol=1e-7)


def test_singular_active_set_is_rejected(setup):
    from paper_2007_08555_amd import Potential
    from paper_2007_08555_amd._lib import MTPError
    P2 = Potential(pot_path("lev16_s3"))
    _P, _pot, A = setup
    bad = A.copy()
    bad[3] = bad[7]
    with pytest.raises(MTPError, match="singular"):
        P2.set_active_set(bad)
    with pytest.raises(MTPError, match="active set"):
        P2.grade_from_b(A[:2])
