"""GPU parity of the training loss and its parameter gradient (paper,
section 2.2) against the FP64 oracle (complex-step derivatives)."""
import numpy as np
import pytest

import synth
from gpu_common import log, pot_path
from oracle import loss as ol
from oracle import mtp as omtp
from oracle.potential import read_potential

pytestmark = pytest.mark.gpu


def make_targets(pot, batch, seed=3):
    """Targets from a perturbed copy of the potential plus N(0, 1e-3^2) noise."""
    ref = dict(pot)
    rng = np.random.default_rng(seed)
    ref["xi"] = pot["xi"] * (1.0 + 0.2 * rng.normal(size=pot["xi"].shape))
    ref["c"] = pot["c"] * (1.0 + 0.05 * rng.normal(size=pot["c"].shape))
    E, F, W = [], [], []
    for k in range(len(batch["n_atoms"])):
        r = omtp.evaluate(ref, *synth.config_of(batch, k))
        E.append(r["energy"] + rng.normal(0, 1e-3))
        F.append(r["forces"] + rng.normal(0, 1e-3, r["forces"].shape))
        W.append(r["virial"] + rng.normal(0, 1e-3, (3, 3)))
    return {"energy": np.array(E), "forces": np.concatenate(F), "virial": np.array(W)}


@pytest.mark.parametrize("name,scaling", [("lev12_s2", "vibrations"), ("lev12_s2", "structures"),
                                          ("lev12_s2", "molecules"), ("lev16_s3", "vibrations")])
def test_loss_gradient_matches_oracle(name, scaling):
    from paper_2007_08555_amd import Batch, Potential
    pot = read_potential(pot_path(name))
    S = pot["n_species"]
    batch = synth.mixed_batch(seed=21, n_configs=6, n_min=8, n_max=28, n_species_model=S)
    assert batch["pbc"].any() and not batch["pbc"].all()
    tg = make_targets(pot, batch)
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling=scaling)
    P = Potential(pot_path(name))
    loss, grad = P.loss_grad(Batch.from_arrays(batch), tg["energy"], tg["forces"], tg["virial"], precision="fp64", **w)
    loss, grad = loss.item(), grad.cpu().numpy()
    L_o = ol.loss(pot, batch, tg, **w)
    m, nc = len(pot["xi"]), pot["c"].size
    rng = np.random.default_rng(0)
    idx = sorted(set(rng.choice(m, size=min(m, 24), replace=False).tolist()) |
                 set((m + rng.choice(nc, size=24, replace=False)).tolist()))
    g_o = ol.loss_grad(pot, batch, tg, indices=idx, **w)
    scale = np.abs(g_o).max()
    err = np.abs(grad[idx] - g_o) / scale
    log(f"[loss {name} {scaling}] loss gpu {loss:.10e} oracle {L_o:.10e}; grad max rel err {err.max():.3e} "
        f"(scale {scale:.3e})")
    assert abs(loss - L_o) <= 1e-10 * abs(L_o)
    assert err.max() <= 1e-8
