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


def test_loss_gradient_on_a_training_shaped_batch():
    """The training workload's shape (configurations of 32-128 atoms, three
    species, level 16): about 1500 atoms over many workgroups, so the
    per-workgroup partial sums of dL/dc and their final reduction are
    compared with the oracle too (on a sample of gradient entries)."""
    from paper_2007_08555_amd import Batch, Potential
    pot = read_potential(pot_path("lev16_s3"))
    batch = synth.mixed_batch(seed=29, n_configs=20, n_min=32, n_max=110, n_species_model=3)
    n_atoms = int(batch["n_atoms"].sum())
    log(f"[loss training-shaped] {len(batch['n_atoms'])} configurations, {n_atoms} atoms")
    assert n_atoms > 20 * 64
    tg = make_targets(pot, batch, seed=5)
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations")
    P = Potential(pot_path("lev16_s3"))
    loss, grad = P.loss_grad(Batch.from_arrays(batch), tg["energy"], tg["forces"], tg["virial"], precision="fp64", **w)
    loss, grad = loss.item(), grad.cpu().numpy()
    L_o = ol.loss(pot, batch, tg, **w)
    m, nc = len(pot["xi"]), pot["c"].size
    rng = np.random.default_rng(4)
    idx = sorted(set(rng.choice(m, size=3, replace=False).tolist()) |
                 set((m + rng.choice(nc, size=3, replace=False)).tolist()))
    g_o = ol.loss_grad(pot, batch, tg, indices=idx, **w)
    err = np.abs(grad[idx] - g_o) / np.abs(g_o).max()
    log(f"[loss training-shaped] loss gpu {loss:.10e} oracle {L_o:.10e}; grad entries {idx}: max rel err {err.max():.3e}")
    assert abs(loss - L_o) <= 1e-10 * abs(L_o)
    assert err.max() <= 1e-8


def test_loss_gradient_on_the_training_workload():
    """The training workload itself (1024 configurations of 32-128 atoms,
    82 106 atoms, level 16), where the oracle is too slow: properties that
    hold at any size.  (1) The loss of eq. Fitting is a sum over
    configurations, so the loss and gradient of the batch equal those of its
    two halves added (this checks the multi-workgroup reduction of dL/dc
    over the whole batch); (2) the gradient along a random direction d equals
    the central difference of the loss, (L(theta + h d) - L(theta - h d)) / 2h.
    Targets are seeded random numbers (no evaluation supplies them)."""
    from paper_2007_08555_amd import Batch, Potential
    batch = synth.mixed_batch(seed=4, n_configs=1024, n_min=32, n_max=128, n_species_model=3)
    K, N = len(batch["n_atoms"]), int(batch["n_atoms"].sum())
    offs = batch["atom_offsets"]
    rng = np.random.default_rng(11)
    E_t = rng.normal(-3.0, 0.5, K) * batch["n_atoms"]
    F_t = rng.normal(0.0, 1.0, (N, 3))
    W_t = rng.normal(0.0, 1.0, (K, 3, 3)) * batch["n_atoms"][:, None, None]
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations", precision="fp64")
    P = Potential(pot_path("lev16_s3"))
    log(f"[loss training workload] {K} configurations, {N} atoms")
    L, g = P.loss_grad(Batch.from_arrays(batch), E_t, F_t, W_t, **w)
    L, g = L.item(), g.cpu().numpy()
    # (1) additivity over a split of the configurations
    h = K // 2
    parts = []
    for ks in (range(0, h), range(h, K)):
        sub = synth._batch([synth.config_of(batch, k) for k in ks])
        a0, a1 = offs[ks[0]], offs[ks[-1] + 1]
        Lp, gp = P.loss_grad(Batch.from_arrays(sub), E_t[list(ks)], F_t[a0:a1], W_t[list(ks)], **w)
        parts.append((Lp.item(), gp.cpu().numpy()))
    dL = abs(L - parts[0][0] - parts[1][0]) / abs(L)
    dg = np.abs(g - parts[0][1] - parts[1][1]).max() / np.abs(g).max()
    log(f"[loss training workload] loss {L:.10e}; halves: loss {dL:.2e}, gradient {dg:.2e} (relative)")
    assert dL <= 1e-12 and dg <= 1e-10
    # (2) central difference along a random direction, relative to each entry
    c0, xi0 = P.get_params()
    m = len(xi0)
    d = rng.normal(size=g.shape)
    d[:m] *= np.abs(xi0)
    d[m:] *= np.abs(c0.ravel())
    step = 1e-5
    vals = []
    for sgn in (1.0, -1.0):
        P.set_params(c=(c0.ravel() + sgn * step * d[m:]).reshape(c0.shape), xi=xi0 + sgn * step * d[:m])
        Ls, _ = P.loss_grad(Batch.from_arrays(batch), E_t, F_t, W_t, **w)
        vals.append(Ls.item())
    P.set_params(c=c0, xi=xi0)
    fd = (vals[0] - vals[1]) / (2 * step)
    an = float(g @ d)
    log(f"[loss training workload] directional derivative: gradient {an:.10e}, central difference {fd:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_loss_gradient_is_bitwise_repeatable():
    """Every sum of the loss path runs in a fixed order (no floating-point
    atomics): two calls on the same inputs agree bit for bit."""
    from paper_2007_08555_amd import Batch, Potential
    batch = synth.mixed_batch(seed=30, n_configs=64, n_min=32, n_max=128, n_species_model=3)
    K, N = len(batch["n_atoms"]), int(batch["n_atoms"].sum())
    rng = np.random.default_rng(12)
    E_t = rng.normal(-3.0, 0.5, K) * batch["n_atoms"]
    F_t = rng.normal(0.0, 1.0, (N, 3))
    W_t = rng.normal(0.0, 1.0, (K, 3, 3))
    P = Potential(pot_path("lev16_s3"))
    B = Batch.from_arrays(batch)
    runs = [P.loss_grad(B, E_t, F_t, W_t, precision="fp64") for _ in range(3)]
    for L, g in runs[1:]:
        assert L.item() == runs[0][0].item()
        assert np.array_equal(g.cpu().numpy(), runs[0][1].cpu().numpy())


@pytest.mark.parametrize("name,scaling", [("lev12_s2", "vibrations"), ("lev16_s3", "structures")])
def test_position_gradient_matches_oracle_differences(name, scaling):
    """dL/dx (grad_pos of mtp_loss_grad: -a_k F_i plus the Hessian-vector
    product of E with the force and stress residuals) against central
    differences of the oracle's loss in single coordinates."""
    from paper_2007_08555_amd import Batch, Potential
    pot = read_potential(pot_path(name))
    batch = synth.mixed_batch(seed=23, n_configs=4, n_min=6, n_max=14, n_species_model=pot["n_species"])
    assert batch["pbc"].any() and not batch["pbc"].all()
    tg = make_targets(pot, batch, seed=9)
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling=scaling)
    P = Potential(pot_path(name))
    _, _, gpos = P.loss_grad(Batch.from_arrays(batch), tg["energy"], tg["forces"], tg["virial"], pos=True, **w)
    gpos = gpos.cpu().numpy()
    N = int(batch["n_atoms"].sum())
    rng = np.random.default_rng(10)
    picks = [(int(a), int(d)) for a, d in zip(rng.choice(N, size=8, replace=False), rng.integers(0, 3, 8))]
    h = 1e-5
    fd = []
    for a, d in picks:
        vals = []
        for sgn in (1.0, -1.0):
            b = {k: np.array(v, copy=True) for k, v in batch.items()}
            b["pos"][a, d] += sgn * h
            vals.append(ol.loss(pot, b, tg, **w))
        fd.append((vals[0] - vals[1]) / (2 * h))
    got = np.array([gpos[a, d] for a, d in picks])
    fd = np.array(fd)
    scale = np.abs(gpos).max()
    err = np.abs(got - fd).max() / scale
    log(f"[grad_pos {name} {scaling}] {len(picks)} coordinates: max |GPU - central difference| / max|dL/dx| "
        f"{err:.3e} (scale {scale:.3e})")
    assert err <= 1e-6


def test_position_gradient_on_the_training_workload():
    """At the training workload's size (1024 configurations, 82 106 atoms):
    the position gradient along a random displacement field equals the
    central difference of the loss, in FP64; FP32 kernels agree with FP64 to
    1e-3 of the largest entry."""
    from paper_2007_08555_amd import Batch, Potential
    batch = synth.mixed_batch(seed=4, n_configs=1024, n_min=32, n_max=128, n_species_model=3)
    K, N = len(batch["n_atoms"]), int(batch["n_atoms"].sum())
    rng = np.random.default_rng(13)
    E_t = rng.normal(-3.0, 0.5, K) * batch["n_atoms"]
    F_t = rng.normal(0.0, 1.0, (N, 3))
    W_t = rng.normal(0.0, 1.0, (K, 3, 3)) * batch["n_atoms"][:, None, None]
    w = dict(w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations")
    P = Potential(pot_path("lev16_s3"))
    _, _, gpos = P.loss_grad(Batch.from_arrays(batch), E_t, F_t, W_t, pos=True, **w)
    gpos = gpos.cpu().numpy()
    d = rng.normal(size=(N, 3))
    step = 1e-6
    vals = []
    for sgn in (1.0, -1.0):
        b = dict(batch, pos=batch["pos"] + sgn * step * d)
        L, _ = P.loss_grad(Batch.from_arrays(b), E_t, F_t, W_t, **w)
        vals.append(L.item())
    fd = (vals[0] - vals[1]) / (2 * step)
    an = float(np.sum(gpos * d))
    log(f"[grad_pos training workload] directional derivative {an:.10e}, central difference {fd:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
    _, _, g32 = P.loss_grad(Batch.from_arrays(batch), E_t, F_t, W_t, pos=True, precision="fp32", **w)
    e32 = np.abs(g32.cpu().numpy() - gpos).max() / np.abs(gpos).max()
    log(f"[grad_pos training workload] FP32 against FP64: {e32:.3e} of the largest entry")
    assert e32 <= 1e-3
