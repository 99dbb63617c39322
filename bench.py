#!/usr/bin/env python
"""Throughput of batched MTP E + F + stress evaluation on one MI355X.

One step is one pass of the whole evaluation path over one batch resident in
HBM: neighbour lists, radial functions, moments, contractions, adjoint,
force gather, per-configuration energy / virial / basis sums, and the
extrapolation grade gamma of every configuration against a fixed FP64 active
set (c = b A^-1, gamma = max |c|).  The step is captured once in a HIP graph
(mtp_eval_async + mtp_grade_from_b) and replayed; eager calls are timed too.

Workload (default): 4096 configurations of 8..256 atoms (about 530 k atoms),
random fcc/bcc/hcp periodic cells with vacancies and free fragments,
displacements sigma in [0.05, 0.3] A, 1..3 species per configuration drawn
from 3, level-16 MTP with N_Q = 8, R_cut = 5 A (seeded synthetic data; the
calibrated potential tests/golden/potentials/lev16_s3.mtp).

Prints one JSON line.  Besides the contract fields it reports the roofline
of the evaluation kernels, the plain one-configuration-per-launch path on the
same configurations, the 16 000-atom bcc box as 100 MD-style steps, the
256 000-atom alloy in FP64, FP32 and compensated FP32, the training workload
(loss gradient and normal equations), and the FP64 CPU oracle timed on a
bounded sample of the same workload (one thread and one process per core).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-evals/s (E+F+stress) MTP lev16; batched vs plain at force err ≤1e-5 eV/Å"
# TFLOP/s, MI355X vector FP64 / FP32 (the mixed path does all but the moments in FP64)
PEAK = {"fp64": 78.6, "fp32": 157.3, "fp32c": 157.3, "mixed": 78.6}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp32c": "f32", "mixed": "f64 (moments f32)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_MD = os.path.join(ROOT, "profiles", "eval_lev16_batch4096_fp64_s{}_hbm.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2007_08555_amd", "csrc", "generated", "gen_lev16.inc")


def measured_traffic(schedule):
    """HBM bytes per launch of the evaluation kernels of one FP64 schedule
    from the committed FETCH_SIZE / WRITE_SIZE summary, when it was taken on
    the kernels built here (same FP64 evaluation part of the generated
    source); else None."""
    from paper_2007_08555_amd.prof import eval_part_digest
    try:
        fields = dict(line.split(": ", 1) for line in open(TRAFFIC_MD.format(schedule)).read().splitlines()
                      if ": " in line
                      and line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "kernel_part_sha256"))
        digest = eval_part_digest(KERNEL_SRC)
    except OSError:
        return None
    if fields.get("kernel_part_sha256", "").strip() != digest:
        return None
    return float(fields["traffic_bytes_per_launch"])


def training_level20():
    """The training workload at its own basis, level 20 (1024 configurations
    of 32-128 atoms, three species, targets from the reference potential
    plus noise), when the library was built with level 20."""
    from paper_2007_08555_amd import Potential
    from paper_2007_08555_amd._lib import MTPError
    pdir = os.path.join(ROOT, "tests", "golden", "potentials")
    try:
        P = Potential(os.path.join(pdir, "lev20_s3.mtp"))
    except MTPError as e:
        return {"error": str(e)}
    return training_extras(P, os.path.join(pdir, "lev20_s3.mtp"), "fp64",
                           ref_path=os.path.join(pdir, "lev20_s3_ref.mtp"))


def training_extras(P, pot_path, precision, ref_path=None):
    """The training-side rows on a batch shaped like the paper's training
    sets (1024 configurations of 32-128 atoms, three species): loss and
    gradient in all parameters (mtp_loss_grad), and the normal equations in
    xi with their solve (mtp_normal_equations, mtp_solve_normal).  Targets
    are E, F and virial of the reference potential at ref_path (by default
    the same potential with xi scaled by 1.1) plus N(0, 1e-3^2) noise."""
    import numpy as np
    import torch

    import synth
    from paper_2007_08555_amd import Batch
    tb = synth.mixed_batch(seed=4, n_configs=1024, n_min=32, n_max=128, n_species_model=3)
    n_atoms = int(tb["n_atoms"].sum())
    B = Batch.from_arrays(tb, "cuda:0")
    if ref_path is None:
        c, xi = P.get_params()
        P.set_params(xi=xi * 1.1)
        ref = P.eval(B, precision="fp64", forces=True, virial=True)
        P.set_params(xi=xi)
    else:
        from paper_2007_08555_amd import Potential
        ref = Potential(ref_path).eval(B, precision="fp64", forces=True, virial=True)
    g = torch.Generator(device="cuda:0").manual_seed(0)
    noise = lambda t: t + 1e-3 * torch.randn(t.shape, generator=g, device=t.device, dtype=t.dtype)
    Et, Ft, Wt = noise(ref["energy"]), noise(ref["forces"]), noise(ref["virial"])
    res = {"workload": f"1024 configurations, 32-128 atoms ({n_atoms} atoms), 3 species, level {P.level}, FP64",
           "atoms": n_atoms}
    for name, fn in (("loss_grad", lambda: P.loss_grad(B, Et, Ft, Wt, precision="fp64")),
                     ("normal_equations", lambda: P.solve_normal(*P.normal_equations(B, Et, Ft, Wt)[:2]))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"ms_per_call": dt * 1e3, "atom_evals_per_s": n_atoms / dt}
    res["normal_equations"]["note"] = f"m = {P.m} evaluations with xi = e_alpha, Gram product and solve"
    return res


def active_learning_extras(P, batch):
    """The selection and relaxation rows on the benchmark batch: MaxVol over
    its descriptor rows b (mtp_maxvol), the rows dE/dtheta over xi and c
    (mtp_theta_rows), MaxVol and the grade over those rows restricted to
    independent columns (mtp_maxvol_theta, mtp_grade_theta; the columns are
    chosen on the host by pivoted QR, outside the timings), and one FIRE step
    of every configuration (mtp_fire_step).  Each entry reports its error
    instead of a time if the call fails."""
    import numpy as np
    import scipy.linalg
    import torch

    from paper_2007_08555_amd import Batch, md
    B = Batch.from_arrays(batch, "cuda:0")
    K, N = B.n_configs, B.n_atoms
    res = {"workload": f"the benchmark batch: {K} configurations, {N} atoms, level {P.level}, FP64"}

    def timed(fn, reps=3):
        out = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) / reps * 1e3

    out = P.eval(B, precision="fp64", forces=True, virial=False, b=True)
    try:
        (_rows, swaps), ms = timed(lambda: P.maxvol(out["b"]), reps=1)
        res["maxvol_b"] = {"ms_per_call": ms, "swaps": swaps, "pool": [K, P.m]}
    except Exception as e:   # noqa: BLE001 - reported in the JSON line
        res["maxvol_b"] = {"error": str(e)}
    try:
        R, ms = timed(lambda: P.theta_rows(B))
        res["theta_rows"] = {"ms_per_call": ms, "configs_per_s": K / ms * 1e3, "atom_evals_per_s": N / ms * 1e3,
                             "columns": P.m + P.n_c}
        Rh = R.cpu().numpy()
        Rs = Rh / np.maximum(np.abs(Rh).max(axis=0), 1e-300)
        _q, rr, piv = scipy.linalg.qr(Rs, pivoting=True, mode="economic")
        rank = int((np.abs(np.diag(rr)) > 1e-10 * abs(rr[0, 0])).sum())
        cols = torch.as_tensor(np.sort(piv[:rank]), device=R.device)
        Rc = R[:, cols].contiguous()
        (sel, swaps_t), ms = timed(lambda: P.maxvol_theta(Rc), reps=1)
        res["maxvol_theta"] = {"ms_per_call": ms, "swaps": swaps_t, "pool": [K, rank]}
        P.set_active_set_theta(Rc[sel.long()])
        _, ms = timed(lambda: P.grade_theta(Rc))
        res["grade_theta"] = {"ms_per_call": ms, "configs_per_s": K / ms * 1e3}
    except Exception as e:   # noqa: BLE001
        res["theta_error"] = str(e)
    try:
        vel = torch.zeros((N, 3), dtype=torch.float64, device=B.pos.device)
        state = md.fire_state(B)
        pos0 = B.pos.clone()
        masses = np.full(P.n_species, 50.0)
        _, ms = timed(lambda: md.fire_step(P, B, vel, out["forces"], masses, state), reps=10)
        B.pos.copy_(pos0)
        res["fire_step"] = {"ms_per_call": ms, "atoms_per_s": N / ms * 1e3}
    except Exception as e:   # noqa: BLE001
        res["fire_step"] = {"error": str(e)}
    return res


def plain_path(P, batch, precision, stream):
    """One configuration per launch sequence: mtp_eval_async on each of the
    batch's configurations in turn (views into the resident batch arrays and
    output buffers, no host synchronisation between them), timed over the
    whole batch between two synchronisations.  The results are compared with
    the batched call's."""
    import ctypes

    import numpy as np
    import torch

    from paper_2007_08555_amd import Batch, _lib
    B = Batch.from_arrays(batch, "cuda:0")
    K = B.n_configs
    offs = batch["atom_offsets"]
    ref = P.eval(B, precision=precision, b=False, stream=stream)     # sizes the workspace for every configuration
    out = P.outputs(B, forces=True, virial=True)
    one = torch.zeros((K, 2), dtype=torch.int64, device="cuda:0")
    one[:, 1] = torch.as_tensor(batch["n_atoms"], device="cuda:0")
    calls = []
    for k in range(K):
        a, n = int(offs[k]), int(offs[k + 1] - offs[k])
        bs = _lib.mtp_batch(1, n, one[k].data_ptr(), B.pos.data_ptr() + 24 * a, B.species.data_ptr() + 4 * a,
                            B.cell.data_ptr() + 72 * k, B.pbc.data_ptr() + k)
        o = _lib.mtp_out(out["energy"].data_ptr() + 8 * k, out["forces"].data_ptr() + 24 * a,
                         out["virial"].data_ptr() + 72 * k, None, None)
        calls.append((bs, o))
    fn, h, prec, sp = _lib.lib().mtp_eval_async, P._h, _lib.PRECISIONS[precision], ctypes.c_void_p(stream.cuda_stream)

    def run():
        for bs, o in calls:
            rc = fn(h, ctypes.byref(bs), ctypes.byref(o), prec, sp)
            if rc:
                _lib.check(rc, "mtp_eval_async")

    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    P.status(stream)
    tp = float(np.median(times))
    n_atoms = int(batch["n_atoms"].sum())
    dE = float((out["energy"] - ref["energy"]).abs().max())
    dF = float((out["forces"] - ref["forces"]).abs().max())
    return {"value": n_atoms / tp, "unit": "atom-evals/s", "configs": K, "ms_per_batch": tp * 1e3,
            "ms_per_batch_all": [t * 1e3 for t in times],
            "max_abs_diff_vs_batched": {"energy_eV": dE, "forces_eV_per_A": dF},
            "note": "every configuration of the batch on its own: one mtp_eval_async launch sequence per "
                    "configuration (neighbour lists, evaluation kernels, force gather, sums) on one stream, "
                    "one synchronisation at the end; median of 3 passes over the batch"}


def precision_study(stream, level=24):
    """The 256 000-atom disordered fcc alloy (40^3 cells, a = 3.6 A, sigma =
    0.2 A, three species) at the given level (24: the workload's own basis,
    table-driven contraction; 16: the headline's basis): throughput of FP64,
    FP32 and FP32 with compensated moment sums, the FP32 errors against the
    FP64 path (which the tests pin to the oracle) over every atom, and the
    FP64 oracle's own rate on a few site energies of the same box."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import mtp as omtp
    from oracle.potential import read_potential
    from paper_2007_08555_amd import Batch, Potential
    box = synth.fcc_alloy(seed=0)
    N = int(box["n_atoms"][0])
    path = os.path.join(ROOT, "tests", "golden", "potentials", f"lev{level}_s3.mtp")
    P = Potential(path, device=0)
    B = Batch.from_arrays(box, "cuda:0")
    res, outs = {"workload": f"{N}-atom periodic disordered fcc alloy, 3 species, level {level} (E, F, virial)"}, {}
    reps = 5 if level <= 16 else 2
    for p in ("fp64", "fp32", "fp32c", "mixed"):
        for _ in range(2 if level <= 16 else 1):
            P.eval(B, precision=p, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = P.eval(B, precision=p, site=True, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        outs[p] = {k: v.cpu().numpy() for k, v in out.items()}
        res[p] = {"value": N / dt, "unit": "atom-evals/s", "ms_per_step": dt * 1e3}
    r64 = outs["fp64"]
    for p in ("fp32", "fp32c", "mixed"):
        res[p]["vs_fp64"] = {
            "energy_per_atom_eV": abs(float(outs[p]["energy"][0]) - float(r64["energy"][0])) / N,
            "site_max_eV": float(np.abs(outs[p]["site"] - r64["site"]).max()),
            "force_max_eV_per_A": float(np.abs(outs[p]["forces"] - r64["forces"]).max()),
            "virial_per_atom_eV": float(np.abs(outs[p]["virial"] - r64["virial"]).max()) / N,
            "largest_force_eV_per_A": float(np.abs(r64["forces"]).max())}
        res[p]["vs_fp64"]["force_rel"] = res[p]["vs_fp64"]["force_max_eV_per_A"] / \
            res[p]["vs_fp64"]["largest_force_eV_per_A"]
    if level > 16:
        # the oracle on one host thread: site energies of a few seeded atoms
        pot = read_potential(path)
        atoms = np.sort(np.random.default_rng(1).choice(N, size=8, replace=False))
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            site, _ = omtp.evaluate_sampled(pot, *synth.config_of(box, 0), atoms, [], chunk=8)
            dt = time.perf_counter() - t0
        res["oracle"] = {"value": len(atoms) / dt, "unit": "site energies/s", "cores": 1,
                         "sample": f"site energies of {len(atoms)} seeded atoms of the box (no forces), FP64, "
                                   f"{dt:.1f} s on one host thread",
                         "site_max_abs_diff_vs_gpu_fp64_eV": float(np.abs(site - r64["site"][atoms]).max())}
    return res


def fp32_accuracy(P, batch, stream):
    """Errors of the FP32, compensated FP32 and mixed paths against the FP64
    path (which the tests pin to the oracle) over every configuration of a
    batch: energy per atom, absolute force error and the force error relative
    to each configuration's largest force, virial per atom; and each
    precision's time per evaluation (eager calls, each with its host
    synchronisation)."""
    import numpy as np
    import torch

    from paper_2007_08555_amd import Batch
    B = Batch.from_arrays(batch, "cuda:0")
    n = np.maximum(batch["n_atoms"], 1).astype(float)
    precs = ("fp64", "fp32", "fp32c", "mixed")
    outs, ms = {}, {}
    for p in precs:
        P.eval(B, precision=p, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            out = P.eval(B, precision=p, stream=stream)
        torch.cuda.synchronize()
        ms[p] = (time.perf_counter() - t0) / 5 * 1e3
        outs[p] = {k: v.cpu().numpy() for k, v in out.items()}
    r64 = outs["fp64"]
    cfg_of_atom = np.repeat(np.arange(len(n)), batch["n_atoms"])
    fmax_cfg = np.zeros(len(n))
    np.maximum.at(fmax_cfg, cfg_of_atom, np.abs(r64["forces"]).max(axis=1))
    res = {"eager_ms_per_eval": ms}
    for p in ("fp32", "fp32c", "mixed"):
        dF = np.abs(outs[p]["forces"] - r64["forces"]).max(axis=1)
        dF_cfg = np.zeros(len(n))
        np.maximum.at(dF_cfg, cfg_of_atom, dF)
        res[p] = {"energy_per_atom_eV": float(np.max(np.abs(outs[p]["energy"] - r64["energy"]) / n)),
                  "force_max_eV_per_A": float(dF.max()),
                  "force_rel": float(np.max(dF_cfg / np.maximum(fmax_cfg, 1e-300))),
                  "virial_per_atom_eV": float(np.max(np.abs(outs[p]["virial"] - r64["virial"]).reshape(len(n), -1)
                                                     .max(axis=1) / n)),
                  "configs_within_1e-5_eV_per_A": int((dF_cfg <= 1e-5).sum()),
                  "configs": int(len(n))}
    res["largest_force_eV_per_A"] = float(np.abs(r64["forces"]).max())
    return res


_POOL = {}


def _pool_init(sample, pot_path):
    from threadpoolctl import threadpool_limits

    from oracle.potential import read_potential
    _POOL["limits"] = threadpool_limits(limits=1)   # one thread per worker process
    _POOL["sample"], _POOL["pot"] = sample, read_potential(pot_path)


def _pool_eval(k):
    import synth
    from oracle import mtp as omtp
    omtp.evaluate(_POOL["pot"], *synth.config_of(_POOL["sample"], k))
    return int(_POOL["sample"]["n_atoms"][k])


def cpu_baseline_pool(batch, pot_path, rate1, budget_s):
    """The same oracle in one single-threaded worker process per host core
    (at most 16), over whole configurations from the start of the batch,
    sized for about budget_s seconds of wall time."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import synth
    cores = min(16, len(os.sched_getaffinity(0)))
    target = rate1 * cores * budget_s
    n_cfg, atoms = 0, 0
    while n_cfg < len(batch["n_atoms"]) and atoms < target:
        atoms += int(batch["n_atoms"][n_cfg])
        n_cfg += 1
    sample = synth.subset(batch, list(range(n_cfg)))
    # fresh interpreters (spawn): the workers never touch the GPU
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn"),
                                initializer=_pool_init, initargs=(sample, pot_path)) as ex:
        list(ex.map(abs, range(4 * cores)))   # start every worker
        t0 = time.perf_counter()
        done = sum(ex.map(_pool_eval, range(n_cfg), chunksize=2))
        dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_cfg} configurations ({done} atoms) of the benchmark batch, E+F+virial in FP64, "
                      f"{dt:.1f} s on {cores} worker processes of one thread each"}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, pot_path, budget_s):
    """The FP64 oracle on the host, one thread, over whole configurations of
    the same batch until budget_s seconds have passed."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import mtp as omtp
    from oracle.potential import read_potential
    pot = read_potential(pot_path)
    atoms, done = 0, 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for k in range(len(batch["n_atoms"])):
            omtp.evaluate(pot, *synth.config_of(batch, k))
            atoms += int(batch["n_atoms"][k])
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    dt = time.perf_counter() - t0
    return {"value": atoms / dt, "unit": "atom-evals/s", "cores": 1, "kind": "oracle",
            "host": f"{host_cpu()}, os.cpu_count() = {os.cpu_count()}",
            "sample": f"first {done} configurations ({atoms} atoms) of the benchmark batch, "
                      f"E+F+virial in FP64, {dt:.1f} s on one host thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32c", "mixed"])
    ap.add_argument("--configs", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true", help="skip plain path, bcc box and CPU baseline")
    ap.add_argument("--no-graph", action="store_true", help="time eager calls instead of HIP-graph replays")
    ap.add_argument("--schedule", type=int, default=-1,
                    help="FP64 schedule of the evaluation kernels (default: the autotuner's choice)")
    ap.add_argument("--batch-cache", default="",
                    help="npz file holding the generated batch (written if missing, read if present)")
    ap.add_argument("--study", type=int, default=0,
                    help="only the 256 000-atom alloy precision study at this level (16, 20 or 24), "
                         "printed as one JSON line (for profiling that workload alone)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (reference for HBM counters)")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(configurations would be sharded across GPUs by cost with no exchange during evaluation)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2007_08555_amd import Batch, Potential

    if a.study:
        print(json.dumps({"precision_study": precision_study(torch.cuda.current_stream(), level=a.study)}),
              flush=True)
        return

    pot_path = os.path.join(ROOT, "tests", "golden", "potentials", "lev16_s3.mtp")
    t0 = time.time()
    if a.batch_cache and os.path.exists(a.batch_cache):
        with np.load(a.batch_cache) as z:
            batch = {k: z[k] for k in z.files}
        assert len(batch["n_atoms"]) == a.configs, "batch cache holds another batch size"
    else:
        batch = synth.mixed_batch(seed=0, n_configs=a.configs, n_min=8, n_max=256, n_species_model=3)
        if a.batch_cache:
            np.savez(a.batch_cache, **batch)
    n_atoms = int(batch["n_atoms"].sum())
    log(f"generated {a.configs} configurations, {n_atoms} atoms in {time.time() - t0:.1f} s")
    P = Potential(pot_path, device=0)
    B = Batch.from_arrays(batch, "cuda:0")
    P.set_active_set(np.load(os.path.join(ROOT, "tests", "golden", "active_lev16_s3.npz"))["A"])
    stream = torch.cuda.current_stream()
    if a.calib_copy_mib > 0:
        src = torch.ones(a.calib_copy_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {a.calib_copy_mib} MiB read, {a.calib_copy_mib} MiB written")
        del src, dst

    # the library's autotuner picks the FP64 pass split for this batch
    t_at = time.perf_counter()
    # the step writes the basis values of the descriptor sums (for the grade)
    # (the mixed path runs all but its moments with the FP64 schedules)
    tune_precision = "fp64" if a.precision == "mixed" else a.precision
    chosen, sched_ms = P.autotune(B, precision=tune_precision, repeats=3, with_b=True)
    if a.schedule >= 0:
        P.set_schedule(a.schedule, precision=tune_precision)
        chosen = a.schedule
    log(f"autotune: schedule {chosen} of {len(sched_ms)} ({', '.join(f'{t:.3f}' for t in sched_ms)} ms "
        f"evaluation kernels), {time.perf_counter() - t_at:.2f} s")

    def step():
        out = P.eval(B, precision=a.precision, forces=True, virial=True, energy=True, b=True, stream=stream)
        out["gamma"], out["argmax"] = P.grade_from_b(out["b"], stream=stream)
        return out

    for _ in range(max(1, a.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    dt_eager = (time.perf_counter() - t0) / a.steps
    log(f"batched, eager calls: {dt_eager * 1e3:.3f} ms/step")
    dt = dt_eager
    replay_ms = None
    if not a.no_graph:
        # the same step captured once in a HIP graph and replayed
        out = P.outputs(B, b=True)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            P.eval_async(B, out, precision=a.precision, stream=side)
            P.grade_from_b(out["b"], want_c=True, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            P.eval_async(B, out, precision=a.precision)
            gamma, argmax, _ = P.grade_from_b(out["b"], want_c=True)
        for _ in range(a.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            graph.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        # the same replays one by one between HIP events: median and minimum
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * a.steps)]
        for k in range(a.steps):
            ev[2 * k].record()
            graph.replay()
            ev[2 * k + 1].record()
        torch.cuda.synchronize()
        per = np.array([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(a.steps)])
        replay_ms = {"median": float(np.median(per)), "min": float(per.min()), "max": float(per.max())}
        P.status()   # raises if a replay met a capacity or input problem
        ref = step()
        torch.cuda.synchronize()
        if not (torch.equal(ref["energy"], out["energy"]) and torch.equal(ref["gamma"], gamma)):
            raise RuntimeError("graph replay differs from the eager step")
        log(f"batched, graph replay: {dt * 1e3:.3f} ms/step (gamma max {gamma.max().item():.3g}); "
            f"single replays {replay_ms}")
    value = n_atoms / dt
    log(f"batched: {dt * 1e3:.3f} ms/step, {value:.4g} atom-evals/s")

    # per-phase device times of the same call, HIP events on the call's stream
    P.set_timing(True)
    ms = {"ms_neighbours": [], "ms_eval": [], "ms_forces": [], "ms_reduce": []}
    for _ in range(5):
        step()
        st = P.stats()
        for k in ms:
            ms[k].append(st[k])
    P.set_timing(False)
    ms = {k: float(np.mean(v)) for k, v in ms.items()}
    flops = st["n_pairs"] * (st["flops_pair_fwd"] + st["flops_pair_bwd"]) + st["n_atoms"] * st["flops_atom"]
    achieved = flops / (ms["ms_eval"] * 1e-3) / 1e12
    traffic = measured_traffic(chosen) if (a.precision == "fp64" and a.configs == 4096) else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK[a.precision], "unit": "TFLOP/s",
                "frac": achieved / PEAK[a.precision], "traffic": traffic,
                "traffic_hbm_TBps": None if traffic is None else traffic / (ms["ms_eval"] * 1e-3) / 1e12,
                "kernel": "evaluation kernel (moments, contractions, adjoint)",
                "flops_per_launch": flops, "kernel_ms": ms["ms_eval"],
                "n_pairs": st["n_pairs"], "phase_ms": ms}
    log(f"roofline: {roofline}")

    line = {"metric": METRIC, "value": value, "unit": "atom-evals/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": DTYPE[a.precision], "data": "synthetic",
            "config": {"workload": f"batched: {a.configs} mixed fcc/bcc/hcp cells and fragments, 8-256 atoms, "
                                   f"{n_atoms} atoms, 1-3 of 3 species, MTP level 16, N_Q 8, R_cut 5 A; "
                                   f"E, F, stress and the extrapolation grade per configuration",
                       "precision": a.precision, "level": 16, "atoms": n_atoms, "configs": a.configs,
                       "graph_replay": not a.no_graph, "schedule": chosen, "schedule_ms": sched_ms},
            "roofline": roofline, "eager_ms_per_step": dt_eager * 1e3,
            "replay_ms_per_step": replay_ms}

    if not a.no_extras:
        # the plain path: every configuration of the batch on its own, one
        # mtp_eval_async launch sequence per configuration on the same stream,
        # one synchronisation at the end (same precision, same outputs)
        line["plain"] = plain_path(P, batch, a.precision, stream)
        line["batched_over_plain"] = value / line["plain"]["value"]
        log(f"plain: {line['plain']}")
        # the 16 000-atom bcc box (two species) as 100 MD-style steps: before
        # each step after the first every coordinate moves by N(0, 0.002^2) A,
        # then neighbour lists, E, F and virial; FP32 (the workload's precision)
        # and FP64
        box = synth.bcc_alloy(seed=0)
        P2 = Potential(os.path.join(ROOT, "tests", "golden", "potentials", "lev16_s2.mtp"), device=0)
        Bb = Batch.from_arrays(box, "cuda:0")
        nb = int(box["n_atoms"][0])
        jit = torch.as_tensor(np.stack(list(synth.md_jitter(1, nb, 99))), device="cuda:0")
        pos0 = Bb.pos.clone()
        torch.zeros_like(pos0).add_(jit[0])   # the first elementwise add loads its kernel (tens of ms)
        line["bcc16000"] = {"workload": f"{nb}-atom periodic bcc box, 2 species, level 16, 100 MD-style steps "
                                        f"(jitter N(0, 0.002^2) A per step, lists rebuilt every step)"}
        for prec in ("fp32", "mixed", "fp64"):
            for _ in range(2):
                P2.eval(Bb, precision=prec, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for t in range(100):
                if t:
                    Bb.pos.add_(jit[t - 1])
                P2.eval(Bb, precision=prec, stream=stream)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) / 100
            Bb.pos.copy_(pos0)
            P2.set_timing(True)
            P2.eval(Bb, precision=prec, stream=stream)
            st2 = P2.stats()
            P2.set_timing(False)
            line["bcc16000"][prec] = {"value": nb / tb, "unit": "atom-evals/s", "ms_per_step": tb * 1e3,
                                      "phase_ms": {k: st2[k] for k in ("ms_neighbours", "ms_eval", "ms_forces",
                                                                        "ms_reduce")}}
            log(f"bcc16000 {prec}: {nb / tb:.4g} atom-evals/s, {tb * 1e3:.3f} ms/step")
        # the same steps with a 0.3 A Verlet skin: lists built out to
        # R_cut + 0.3 A and reused while no atom moved more than 0.15 A
        for prec in ("fp32", "fp64"):
            P3 = Potential(os.path.join(ROOT, "tests", "golden", "potentials", "lev16_s2.mtp"), device=0)
            P3.set_skin(0.3)
            for _ in range(2):
                P3.eval(Bb, precision=prec, stream=stream)
            torch.cuda.synchronize()
            reused = 0
            t0 = time.perf_counter()
            for t in range(100):
                if t:
                    Bb.pos.add_(jit[t - 1])
                P3.eval(Bb, precision=prec, stream=stream)
                reused += P3.stats()["lists_reused"]
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) / 100
            Bb.pos.copy_(pos0)
            line["bcc16000"][prec + "_skin0.3"] = {"value": nb / tb, "unit": "atom-evals/s", "ms_per_step": tb * 1e3,
                                                   "lists_reused_steps": reused,
                                                   "list_builds": P3.stats()["list_builds"]}
            log(f"bcc16000 {prec}, skin 0.3 A: {nb / tb:.4g} atom-evals/s, {tb * 1e3:.3f} ms/step, "
                f"lists reused on {reused} of 100 steps")
            del P3
        line["fp32_accuracy"] = {"batched": fp32_accuracy(P, batch, stream)}
        P2b = Potential(os.path.join(ROOT, "tests", "golden", "potentials", "lev16_s2.mtp"), device=0)
        line["fp32_accuracy"]["bcc16000"] = fp32_accuracy(P2b, synth.bcc_alloy(seed=0), stream)
        del P2b
        log(f"fp32 accuracy: {line['fp32_accuracy']}")
        line["precision_study"] = precision_study(stream, level=24)
        log(f"precision study: {line['precision_study']}")
        line["precision_study_level16"] = precision_study(stream, level=16)
        log(f"precision study, level 16: {line['precision_study_level16']}")
        line["training"] = training_extras(P, pot_path, a.precision)
        log(f"training: {line['training']}")
        line["active_learning"] = active_learning_extras(P, batch)
        log(f"active learning and relaxation: {line['active_learning']}")
        line["training_level20"] = training_level20()
        log(f"training, level 20: {line['training_level20']}")
        line["cpu_baseline"] = cpu_baseline(batch, pot_path, a.cpu_seconds)
        log(f"cpu baseline: {line['cpu_baseline']}")
        line["cpu_baseline"]["all_cores"] = cpu_baseline_pool(batch, pot_path, line["cpu_baseline"]["value"],
                                                              a.cpu_seconds)
        log(f"cpu baseline, all cores: {line['cpu_baseline']['all_cores']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
