"""Level 24 (the precision study's basis: 2007 functions, 727 connected
contractions, 581 moment components; table-driven contraction): FP64
evaluation against the FP64 oracle on small configurations, then on sampled
atoms of the 256 000-atom disordered fcc alloy (40^3 cells, a = 3.6 A,
sigma = 0.2 A, three species), and FP32 / compensated FP32 against FP64 over
the whole box, held to the stated absolute bounds (an expected failure, with
the numbers, where FP32 misses them); the same for the mixed-precision path
(FP32 moments, everything else in FP64)."""
import numpy as np
import pytest

import synth
from gpu_common import errors, gpu_batch, log, oracle_batch, pot_path
from oracle import mtp as omtp
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu

TOL64 = {"energy_per_atom": 1e-11, "site": 1e-11, "force": 1e-10, "virial": 1e-9, "b_rel": 1e-10}


@pytest.fixture(scope="module")
def lev24():
    from paper_2007_08555_amd import Potential
    return Potential(pot_path("lev24_s3")), read_potential(pot_path("lev24_s3"))


def test_level24_small_configurations(lev24):
    P, pot = lev24
    cfgs = [synth.config_of(synth.mixed_batch(seed=61, n_configs=3, n_min=4, n_max=10, n_species_model=3), k)
            for k in range(3)]
    # a periodic cell narrower than 2 R_cut (atoms see their own images)
    cfgs.append((np.array([[0.0, 0.0, 0.0], [1.7, 1.7, 0.05]]), np.array([2, 0], np.int32), np.eye(3) * 3.4, 1))
    batch = synth._batch(cfgs)
    log(f"[lev24 small] {len(cfgs)} configurations, {int(batch['n_atoms'].sum())} atoms")
    g = gpu_batch(P, batch, "fp64")
    rep = errors(batch, g, oracle_batch(pot, batch))
    log(f"[lev24 fp64] {rep}")
    for k, v in TOL64.items():
        assert rep[k] <= v, (k, rep[k], v)


def _box_results(P, precisions):
    from paper_2007_08555_amd import Batch
    box = synth.fcc_alloy(seed=0)
    B = Batch.from_arrays(box, "cuda:0")
    out = {}
    for p in precisions:
        o = P.eval(B, precision=p, site=True)
        out[p] = {k: v.cpu().numpy() for k, v in o.items()}
    return box, out


def test_level24_alloy_box_sampled_atoms(lev24):
    P, pot = lev24
    box, res = _box_results(P, ["fp64"])
    N = int(box["n_atoms"][0])
    rng = np.random.default_rng(24)
    e_atoms = np.sort(rng.choice(N, size=3, replace=False))
    f_atoms = e_atoms[:1]
    log(f"[lev24 box] sampled site energies of atoms {e_atoms.tolist()}, force on {f_atoms.tolist()}")
    v_o, f_o = omtp.evaluate_sampled(pot, *synth.config_of(box, 0), e_atoms, f_atoms, chunk=8)
    r = res["fp64"]
    e_err = np.abs(r["site"][e_atoms] - v_o).max()
    f_err = np.abs(r["forces"][f_atoms] - f_o).max()
    log(f"[lev24 box fp64] site error {e_err:.3e} eV, force error {f_err:.3e} eV/A "
        f"(site scale {np.abs(v_o).max():.3g}, force scale {np.abs(f_o).max():.3g})")
    assert e_err <= 1e-11 * max(1.0, np.abs(v_o).max())
    assert f_err <= 1e-10 * max(1.0, np.abs(f_o).max())
    # momentum conservation and a symmetric virial over the whole box
    F = r["forces"]
    assert np.abs(F.sum(axis=0)).max() <= 1e-9 * np.abs(F).max() * np.sqrt(N)


@pytest.mark.parametrize("precision", ["fp32", "fp32c", "mixed"])
def test_level24_alloy_box_fp32(lev24, precision):
    P, _ = lev24
    box, res = _box_results(P, ["fp64", precision])
    N = int(box["n_atoms"][0])
    r64, r32 = res["fp64"], res[precision]
    fscale = np.abs(r64["forces"]).max()
    de = abs(float(r32["energy"][0]) - float(r64["energy"][0])) / N
    df = np.abs(r32["forces"] - r64["forces"]).max()
    ds = np.abs(r32["site"] - r64["site"]).max()
    dw = np.abs(r32["virial"] - r64["virial"]).max() / N
    log(f"[lev24 box {precision}] energy per atom {de:.3e} eV, largest site error {ds:.3e} eV, "
        f"largest force error {df:.3e} eV/A (largest force {fscale:.3g}), virial per atom {dw:.3e} eV")
    # guard at FP32's rounding level, then the stated absolute bounds
    assert de <= 1e-5 and df <= 1e-4 * fscale
    miss = {k: v for k, v, b in (("energy_per_atom", de, 1e-6), ("force", df, 1e-5), ("virial_per_atom", dw, 5e-5))
            if v > b}
    if miss:
        pytest.xfail(f"level-24 alloy box, {precision}: misses the absolute bounds: measured {miss}")
