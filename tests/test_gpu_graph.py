"""mtp_eval_async captured in a HIP graph (torch.cuda.CUDAGraph): every
replay must reproduce the eager mtp_eval result bit for bit (the path is
deterministic), also after the positions are updated in place."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import log, pot_path

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager(precision):
    from paper_2007_08555_amd import Batch, Potential
    P = Potential(pot_path("lev16_s3"))
    b = synth.mixed_batch(seed=41, n_configs=64, n_min=8, n_max=128, n_species_model=3)
    B = Batch.from_arrays(b)
    ref = P.eval(B, precision=precision, forces=True, virial=True, site=True)   # sizes the workspace
    torch.cuda.synchronize()
    out = P.outputs(B, site=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.eval_async(B, out, precision=precision, stream=side)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.eval_async(B, out, precision=precision)
    for rep in range(3):
        for v in out.values():
            v.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("energy", "forces", "virial", "site"):
            assert torch.equal(out[k], ref[k]), (rep, k)
        P.status()
    # new positions in the same buffer: the replay evaluates them
    B.pos.add_(0.01 * torch.randn_like(B.pos))
    ref2 = P.eval(B, precision=precision, forces=True, virial=True, site=True)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for k in ("energy", "forces", "virial", "site"):
        assert torch.equal(out[k], ref2[k]), k
    assert not torch.equal(ref2["energy"], ref["energy"])
    log(f"[graph {precision}] 4 replays equal to eager evaluation")


def test_async_needs_a_sized_workspace():
    from paper_2007_08555_amd import Batch, Potential
    from paper_2007_08555_amd._lib import MTPError
    P = Potential(pot_path("lev8_s1"))
    B = Batch.from_arrays(synth.fcc108(seed=2))
    with pytest.raises(MTPError, match="workspace"):
        P.eval_async(B, P.outputs(B), precision="fp64")
    torch.cuda.synchronize()
