"""GPU MaxVol selection (mtp_maxvol; paper, section 2.3) against the
oracle's MaxVol (oracle.grade.maxvol): the same starting rows (pivot rows of
Gaussian elimination with partial pivoting), the same swaps, the same final
rows in position order, on seeded pools; the final selection is dominant
(max |pool A^{-1}| <= 1 + delta, checked in numpy); error cases."""
import numpy as np
import pytest

import synth
from gpu_common import log, pot_path
from oracle import grade as og
from oracle import mtp as omtp
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu


def random_pool(seed, K, m):
    rng = np.random.default_rng(seed)
    # columns spanning six decades, like descriptor rows of different degree
    return rng.normal(size=(K, m)) * 10.0 ** rng.uniform(-3, 3, size=m)


def dominance(B, rows):
    _, _, C = og.grade(B, B[rows])
    return float(np.abs(C).max())


@pytest.mark.parametrize("name,K,seed", [("lev12_s2", 128, 1), ("lev16_s3", 464, 2), ("lev16_s3", 1000, 3)])
def test_maxvol_matches_oracle_on_random_pools(name, K, seed):
    from paper_2007_08555_amd import Potential
    P = Potential(pot_path(name))
    B = random_pool(seed, K, P.m)
    rows_o, swaps_o = og.maxvol(B)
    rows_g, swaps_g = P.maxvol(B)
    rows_g = rows_g.cpu().numpy()
    log(f"[maxvol {name} K={K}] swaps gpu {swaps_g} oracle {swaps_o}; rows equal {np.array_equal(rows_g, rows_o)}; "
        f"max |C| {dominance(B, rows_g):.6f}")
    assert np.array_equal(np.sort(og.initial_rows(B)), np.sort(P.maxvol(B, max_swaps=0)[0].cpu().numpy()))
    assert swaps_g == swaps_o and np.array_equal(rows_g, rows_o)
    assert dominance(B, rows_g) <= 1.0 + 1e-3 + 1e-9


def test_maxvol_on_descriptor_rows():
    # b rows of seeded configurations from the oracle, level 12 (m = 32)
    from paper_2007_08555_amd import Potential
    pot = read_potential(pot_path("lev12_s2"))
    batch = synth.mixed_batch(seed=41, n_configs=96, n_min=6, n_max=24, n_species_model=2)
    B = np.array([omtp.evaluate(pot, *synth.config_of(batch, k))["b"] for k in range(96)])
    rows_o, swaps_o = og.maxvol(B)
    rows_g, swaps_g = Potential(pot_path("lev12_s2")).maxvol(B)
    rows_g = rows_g.cpu().numpy()
    log(f"[maxvol descriptors] swaps gpu {swaps_g} oracle {swaps_o}; max |C| {dominance(B, rows_g):.6f}")
    assert swaps_g == swaps_o and np.array_equal(rows_g, rows_o)


def test_maxvol_from_given_rows_and_errors():
    from paper_2007_08555_amd import Potential
    from paper_2007_08555_amd._lib import MTPError
    P = Potential(pot_path("lev12_s2"))
    m = P.m
    B = random_pool(5, 200, m)
    start = np.arange(50, 50 + m)
    rows_o, swaps_o = og.maxvol(B, start=start)
    rows_g, swaps_g = P.maxvol(B, rows=start)
    log(f"[maxvol given start] swaps gpu {swaps_g} oracle {swaps_o}")
    assert swaps_g == swaps_o and np.array_equal(rows_g.cpu().numpy(), rows_o)
    # a cap on the swaps: the oracle's loop stops at the same point
    rows_o, swaps_o = og.maxvol(B, start=start, max_swaps=3)
    rows_g, swaps_g = P.maxvol(B, rows=start, max_swaps=3)
    assert swaps_g == swaps_o == 3 and np.array_equal(rows_g.cpu().numpy(), rows_o)
    with pytest.raises(MTPError):
        P.maxvol(B[: m - 1])                      # fewer rows than the basis size
    with pytest.raises(MTPError):
        P.maxvol(B, rows=np.r_[0, np.arange(m - 1)])   # repeated starting row
    low = B.copy()
    low[:, 1] = low[:, 0]                         # rank below m
    with pytest.raises(MTPError):
        P.maxvol(low)
