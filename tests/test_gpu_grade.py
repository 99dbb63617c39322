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


@pytest.mark.parametrize("name,n_species,step", [("lev12_s2", 2, 6), ("lev16_s3", 3, 17)])
def test_theta_rows_match_the_oracle(name, n_species, step):
    """Rows dE_k/dtheta of the nonlinear grade (mtp_theta_rows) against the
    oracle's complex-step rows: every xi column and a sample of c columns
    (every species pair at level 16 with three species)."""
    from paper_2007_08555_amd import Batch, Potential
    P = Potential(pot_path(name))
    pot = read_potential(pot_path(name))
    batch = synth.mixed_batch(seed=21, n_configs=4, n_min=8, n_max=20, n_species_model=n_species)
    m, nc = len(pot["xi"]), pot["c"].size
    # every xi column at level 12; at level 16 a few (the xi part is b, checked
    # against the oracle by the grade tests above)
    idx = (list(range(m)) if m <= 40 else [0, m // 2, m - 1]) + list(range(m, m + nc, step)) + [m + nc - 1]
    log(f"[theta rows] configs 4 atoms {int(batch['n_atoms'].sum())} columns {len(idx)} of {m + nc}")
    R = P.theta_rows(Batch.from_arrays(batch), precision="fp64").cpu().numpy()
    assert R.shape == (4, m + nc)
    Ro = og.theta_rows(pot, batch, indices=idx)
    scale = np.maximum(np.abs(Ro).max(axis=0), 1e-300)
    err = np.abs(R[:, idx] - Ro) / scale
    log(f"[theta rows] max error relative to each column's scale {err.max():.3e}")
    assert err.max() <= 1e-10
    c_cols = [t for t, q in enumerate(idx) if q >= m]
    assert np.abs(Ro[:, c_cols]).max() > 0
    R32 = P.theta_rows(Batch.from_arrays(batch), precision="fp32").cpu().numpy()
    err32 = np.abs(R32[:, idx] - Ro) / scale
    log(f"[theta rows] FP32 kernels: {err32.max():.3e}")
    assert err32.max() <= 1e-4


def test_theta_rows_are_bitwise_repeatable():
    """The c part of the rows is summed per configuration in a fixed order
    (no floating-point atomics), also for configurations larger than a
    workgroup: two calls agree bit for bit."""
    from paper_2007_08555_amd import Batch, Potential
    P = Potential(pot_path("lev16_s3"))
    batch = synth.mixed_batch(seed=22, n_configs=16, n_min=200, n_max=400, n_species_model=3)
    assert batch["n_atoms"].max() > 256
    B = Batch.from_arrays(batch)
    R = [P.theta_rows(B, precision="fp64").cpu().numpy() for _ in range(3)]
    assert np.abs(R[0]).max() > 0
    assert all(np.array_equal(R[0], r) for r in R[1:])


def test_nonlinear_grade_matches_the_oracle():
    """gamma over theta rows (oracle rows, restricted to independent columns
    chosen by pivoted QR: the full rows are rank-deficient by one relation per
    radial function) against an active set chosen by pivoted elimination: the
    oracle's grade on the same rows, and grade one with argmax = own index on
    the active rows themselves."""
    import scipy.linalg
    from paper_2007_08555_amd import Potential
    P = Potential(pot_path("lev8_s1"))
    pot = read_potential(pot_path("lev8_s1"))
    batch = synth.mixed_batch(seed=22, n_configs=48, n_min=8, n_max=24, n_species_model=1)
    R = og.theta_rows(pot, batch)
    Rs = R / np.abs(R).max(axis=0).clip(1e-300)
    _q, rr, piv = scipy.linalg.qr(Rs, pivoting=True)
    rank = int((np.abs(np.diag(rr)) > 1e-10 * abs(rr[0, 0])).sum())
    cols = np.sort(piv[:rank])
    Rc = R[:, cols]
    rows = og.initial_rows(Rc)
    A = Rc[rows]
    P.set_active_set_theta(A)
    gam, arg = P.grade_theta(Rc)
    gam_o, arg_o, c_o = og.grade(Rc, A)
    g = gam.cpu().numpy()
    log(f"[nonlinear grade] {R.shape[1]} theta columns, rank {rank}, gamma {g.min():.3g}..{g.max():.3g}")
    assert rank < R.shape[1]
    assert np.allclose(g, gam_o, rtol=1e-8)
    ga, aa = P.grade_theta(A)
    assert np.allclose(ga.cpu().numpy(), 1.0, atol=1e-8)
    assert np.array_equal(aa.cpu().numpy(), np.arange(rank))
    # MaxVol over the theta pool: the same swaps and final rows as the oracle's
    sel, swaps = P.maxvol_theta(Rc)
    sel_o, swaps_o = og.maxvol(Rc)
    log(f"[nonlinear maxvol] swaps gpu {swaps} oracle {swaps_o}")
    assert swaps == swaps_o
    assert np.array_equal(sel.cpu().numpy(), np.asarray(sel_o))
    P.set_active_set_theta(Rc[sel.cpu().numpy()])
    g3, _ = P.grade_theta(Rc)
    assert g3.max().item() <= 1.0 + 1e-3 + 1e-9
