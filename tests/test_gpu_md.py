"""The 16 000-atom bcc box (level 16, two species) evaluated as 100 MD-style
steps: before each step after the first, every coordinate moves by seeded
N(0, 0.002^2) A jitter (the same draws on the host and, added in FP64, on the
device), and the library rebuilds the neighbour lists and evaluates E, F and
the virial.  Site energies of 64 sampled atoms and forces of 8 of them are
compared with the FP64 oracle at the first and the last step.

Bounds: FP64 as in the other parity tests.  FP32 and FP32 compensated: the
energy per atom within 1e-6 eV, estimated by the mean signed site-energy
error over the sample (the box's energy per atom is its mean site energy; the
oracle takes minutes for all 16 000 sites); each site energy within 5e-6 eV
(one FP32 contraction chain per site, measured near 1e-6 eV); each force
component within 1e-5 eV/A."""
import functools

import numpy as np
import pytest

import synth
from gpu_common import log, pot_path
from oracle import mtp as omtp
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu

N_STEPS = 100
CHECK = (0, N_STEPS - 1)
N_SITES, N_FORCES = 64, 8


@functools.lru_cache(maxsize=1)
def trajectory():
    """The box, the per-step jitter, positions at the checked steps and the
    sampled atoms."""
    box = synth.bcc_alloy(seed=0)
    N = int(box["n_atoms"][0])
    jitter = list(synth.md_jitter(seed=1, n_atoms=N, n_steps=N_STEPS - 1))
    pos = box["pos"].copy()
    at = {0: pos.copy()}
    for t, d in enumerate(jitter, start=1):
        pos = pos + d
        if t in CHECK:
            at[t] = pos.copy()
    atoms = np.sort(np.random.default_rng(4).choice(N, size=N_SITES, replace=False))
    return box, jitter, at, atoms


@functools.lru_cache(maxsize=None)
def oracle_at(step):
    box, _, at, atoms = trajectory()
    pot = read_potential(pot_path("lev16_s2"))
    _, sp, cell, pbc = synth.config_of(box, 0)
    return omtp.evaluate_sampled(pot, at[step], sp, cell, pbc, atoms, atoms[:N_FORCES])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32c"])
def test_md_steps_bcc16000(precision):
    import torch
    from paper_2007_08555_amd import Batch, Potential
    box, jitter, at, atoms = trajectory()
    P = Potential(pot_path("lev16_s2"))
    B = Batch.from_arrays(box, "cuda:0")
    got = {}
    for t in range(N_STEPS):
        if t > 0:
            B.pos.add_(torch.as_tensor(jitter[t - 1], device="cuda:0"))
        out = P.eval(B, precision=precision, site=True)
        if t in CHECK:
            got[t] = (out["site"].cpu().numpy()[atoms], out["forces"].cpu().numpy()[atoms[:N_FORCES]])
    assert np.array_equal(B.pos.cpu().numpy(), at[N_STEPS - 1])
    P.status()
    for t in CHECK:
        v_o, f_o = oracle_at(t)
        e_err = np.abs(got[t][0] - v_o).max()
        e_mean = abs(np.mean(got[t][0] - v_o))
        f_err = np.abs(got[t][1] - f_o).max()
        log(f"[md {precision} step {t}] {N_SITES} sites: largest error {e_err:.3e} eV, mean signed "
            f"{e_mean:.3e} eV; forces of atoms {atoms[:N_FORCES].tolist()}: error {f_err:.3e} eV/A "
            f"(largest force {np.abs(f_o).max():.3g})")
        if precision == "fp64":
            assert e_err <= 1e-11 and f_err <= 1e-10
        else:
            assert e_mean <= 1e-6 and e_err <= 5e-6 and f_err <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_md_steps_with_verlet_skin(precision):
    """The same 100 steps with a 0.3 A Verlet skin (mtp_set_skin): the lists
    are built once out to R_cut + 0.3 A and reused while no atom has moved
    more than 0.15 A; every reused step equals a search on every step (a
    second potential without skin on the same positions) up to the rounding
    of the summation order, and the last step matches the oracle."""
    import torch
    from paper_2007_08555_amd import Batch, Potential
    box, jitter, at, atoms = trajectory()
    P = Potential(pot_path("lev16_s2"))
    P.set_skin(0.3)
    Q = Potential(pot_path("lev16_s2"))
    B = Batch.from_arrays(box, "cuda:0")
    reused, worst = 0, {"energy": 0.0, "forces": 0.0, "virial": 0.0}
    for t in range(N_STEPS):
        if t > 0:
            B.pos.add_(torch.as_tensor(jitter[t - 1], device="cuda:0"))
        out = P.eval(B, precision=precision, site=True)
        reused += P.stats()["lists_reused"]
        if t % 11 == 0 or t == N_STEPS - 1:
            ref = Q.eval(B, precision=precision, site=True)
            for k in worst:
                d = (out[k] - ref[k]).abs().max().item() / max(ref[k].abs().max().item(), 1e-300)
                worst[k] = max(worst[k], d)
    st = P.stats()
    log(f"[md skin {precision}] list builds {st['list_builds']}, reused on {reused} of {N_STEPS} steps; "
        f"largest relative difference to a search on every step {worst}")
    assert st["list_builds"] >= 1 and reused >= N_STEPS - st["list_builds"] - 1
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert max(worst.values()) <= tol
    if precision == "fp64":
        v_o, f_o = oracle_at(N_STEPS - 1)
        e_err = np.abs(out["site"].cpu().numpy()[atoms] - v_o).max()
        f_err = np.abs(out["forces"].cpu().numpy()[atoms[:N_FORCES]] - f_o).max()
        log(f"[md skin fp64 step {N_STEPS - 1}] site error {e_err:.3e} eV, force error {f_err:.3e} eV/A")
        assert e_err <= 1e-11 and f_err <= 1e-10
    P.status()
