"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same seeded inputs and compare."""
import os
import sys

import numpy as np

import synth
from oracle import mtp as omtp
from oracle.potential import read_potential

POT_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "potentials")


def pot_path(name):
    return os.path.join(POT_DIR, name + ".mtp")


def oracle_batch(pot, batch):
    """Per-config oracle results stacked like the GPU outputs."""
    E, F, W, V, b = [], [], [], [], []
    for k in range(len(batch["n_atoms"])):
        r = omtp.evaluate(pot, *synth.config_of(batch, k))
        E.append(r["energy"])
        F.append(r["forces"])
        W.append(r["virial"])
        V.append(r["site"])
        b.append(r["b"])
    cat = lambda x, shape: np.concatenate(x) if x else np.zeros(shape)
    return {"energy": np.array(E), "forces": cat(F, (0, 3)), "virial": np.array(W).reshape(-1, 3, 3),
            "site": cat(V, (0,)), "b": np.array(b).reshape(len(E), -1)}


def gpu_batch(P, batch, precision, **kw):
    import torch
    from paper_2007_08555_amd import Batch
    out = P.eval(Batch.from_arrays(batch), precision=precision, site=True, b=True, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def errors(batch, g, o):
    n = np.maximum(batch["n_atoms"], 1).astype(float)
    rep = {
        "energy_per_atom": float(np.max(np.abs(g["energy"] - o["energy"]) / n)) if len(n) else 0.0,
        "site": float(np.max(np.abs(g["site"] - o["site"]))) if len(o["site"]) else 0.0,
        "force": float(np.max(np.abs(g["forces"] - o["forces"]))) if len(o["forces"]) else 0.0,
        "virial": float(np.max(np.abs(g["virial"] - o["virial"]))) if len(o["virial"]) else 0.0,
    }
    dw = np.abs(g["virial"] - o["virial"]).reshape(len(n), -1).max(axis=1) if len(n) else np.zeros(0)
    rep["virial_per_atom"] = float(np.max(dw / n)) if len(n) else 0.0
    scale_b = np.maximum(np.abs(o["b"]).max(axis=0), 1e-300) if o["b"].size else 1.0
    rep["b_rel"] = float(np.max(np.abs(g["b"] - o["b"]) / scale_b)) if o["b"].size else 0.0
    rep["force_scale"] = float(np.abs(o["forces"]).max()) if len(o["forces"]) else 0.0
    rep["site_scale"] = float(np.abs(o["site"]).max()) if len(o["site"]) else 0.0
    return rep


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()
