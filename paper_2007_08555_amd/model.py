"""Python front end of libmtp: argument marshalling between torch device
tensors and the C ABI.  No arithmetic of the potential happens here."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Batch:
    """Configurations resident on one GPU (the mtp_batch of the C ABI).

    Arrays: atom_offsets int64 [n_cfg+1], pos float64 [N,3], species int32 [N],
    cell float64 [n_cfg,3,3], pbc uint8 [n_cfg]."""

    def __init__(self, atom_offsets, pos, species, cell, pbc):
        self.atom_offsets = atom_offsets
        self.pos = pos
        self.species = species
        self.cell = cell
        self.pbc = pbc
        self.n_configs = int(atom_offsets.numel()) - 1
        self.n_atoms = int(pos.shape[0])

    @classmethod
    def from_arrays(cls, batch, device="cuda"):
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
        return cls(t(batch["atom_offsets"], torch.int64), t(batch["pos"], torch.float64).reshape(-1, 3),
                   t(batch["species"], torch.int32), t(batch["cell"], torch.float64).reshape(-1, 3, 3),
                   t(batch["pbc"], torch.uint8))

    def c_struct(self):
        return _lib.mtp_batch(self.n_configs, self.n_atoms, self.atom_offsets.data_ptr(), self.pos.data_ptr(),
                              self.species.data_ptr(), self.cell.data_ptr(), self.pbc.data_ptr())


class Potential:
    """A loaded MTP (mtp_load) on one HIP device."""

    def __init__(self, path, device=0):
        h = ctypes.c_void_p()
        check(lib().mtp_load(str(path).encode(), int(device), ctypes.byref(h)), f"mtp_load({path})")
        self._h = h
        self.device = torch.device("cuda", device)
        info = _lib.mtp_info()
        check(lib().mtp_model_info(self._h, ctypes.byref(info)), "mtp_model_info")
        self.level, self.m, self.n_mu = info.level, info.m, info.n_mu
        self.n_species, self.n_q, self.n_c = info.n_species, info.n_q, info.n_c
        self.r_min, self.r_cut = info.r_min, info.r_cut
        self.n_schedules = info.n_schedules

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().mtp_free(h)
            except Exception:   # interpreter shutdown: the process releases everything
                pass
            self._h = None

    # parameters -------------------------------------------------------
    def get_params(self):
        c = np.zeros(self.n_c)
        xi = np.zeros(self.m)
        check(lib().mtp_get_params(self._h, c.ctypes.data_as(ctypes.c_void_p), xi.ctypes.data_as(ctypes.c_void_p)),
              "mtp_get_params")
        return c, xi

    def set_params(self, c=None, xi=None):
        cc = None if c is None else np.ascontiguousarray(np.asarray(c, dtype=np.float64).ravel())
        xx = None if xi is None else np.ascontiguousarray(np.asarray(xi, dtype=np.float64).ravel())
        if cc is not None and cc.size != self.n_c or xx is not None and xx.size != self.m:
            raise ValueError("parameter sizes do not match the potential")
        check(lib().mtp_set_params(self._h, None if cc is None else cc.ctypes.data_as(ctypes.c_void_p),
                                   None if xx is None else xx.ctypes.data_as(ctypes.c_void_p)), "mtp_set_params")

    # evaluation -------------------------------------------------------
    def eval(self, batch: Batch, precision="fp32", forces=True, virial=True, site=False, b=False,
             energy=True, stream=None):
        """Returns a dict of device tensors: energy [K], forces [N,3], virial [K,3,3],
        site [N], b [K,m] (those requested)."""
        dev = self.device
        K, N = batch.n_configs, batch.n_atoms
        res = {}
        if energy:
            res["energy"] = torch.empty(K, dtype=torch.float64, device=dev)
        if forces:
            res["forces"] = torch.empty((N, 3), dtype=torch.float64, device=dev)
        if virial:
            res["virial"] = torch.empty((K, 3, 3), dtype=torch.float64, device=dev)
        if site:
            res["site"] = torch.empty(N, dtype=torch.float64, device=dev)
        if b:
            res["b"] = torch.empty((K, self.m), dtype=torch.float64, device=dev)
        out = _lib.mtp_out(*[res[k].data_ptr() if k in res else None
                             for k in ("energy", "forces", "virial", "site", "b")])
        bs = batch.c_struct()
        check(lib().mtp_eval(self._h, ctypes.byref(bs), ctypes.byref(out), _lib.PRECISIONS[precision],
                             _stream(stream)), "mtp_eval")
        return res

    def loss_grad(self, batch: Batch, E_t, F_t, W_t, w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations",
                  precision="fp64", stream=None, pos=False):
        """Loss of eq. Fitting and dL/d(xi, c) (mtp_loss_grad); targets are
        device or host arrays: E_t [K], F_t [N,3], W_t [K,3,3] (virial, eV).
        With pos=True also dL/dx [N,3] (the gradient in the positions)."""
        dev = self.device
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
        E_t, F_t, W_t = t(E_t), t(F_t), t(W_t)
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        grad = torch.empty(self.m + self.n_c, dtype=torch.float64, device=dev)
        gpos = torch.empty((batch.n_atoms, 3), dtype=torch.float64, device=dev) if pos else None
        bs = batch.c_struct()
        check(lib().mtp_loss_grad(self._h, ctypes.byref(bs), _ptr(E_t), _ptr(F_t), _ptr(W_t), float(w_e), float(w_f),
                                  float(w_s), _lib.SCALINGS[scaling], _lib.PRECISIONS[precision], _ptr(loss),
                                  _ptr(grad), _ptr(gpos) if pos else None, _stream(stream)), "mtp_loss_grad")
        return (loss, grad, gpos) if pos else (loss, grad)

    def normal_equations(self, batch: Batch, E_t, F_t, W_t, w_e=1.0, w_f=0.01, w_s=0.001, scaling="vibrations",
                         precision="fp64", out=None, stream=None):
        """H = J^T W J, g = J^T W y, yy = y^T W y of the loss in xi at the
        current c (mtp_normal_equations).  With out=(H, g, yy) from an earlier
        call the batch's terms are added to them (a training set in several
        batches)."""
        dev = self.device
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
        E_t, F_t, W_t = t(E_t), t(F_t), t(W_t)
        acc = out is not None
        if out is None:
            out = (torch.empty((self.m, self.m), dtype=torch.float64, device=dev),
                   torch.empty(self.m, dtype=torch.float64, device=dev),
                   torch.empty(1, dtype=torch.float64, device=dev))
        H, g, yy = out
        bs = batch.c_struct()
        check(lib().mtp_normal_equations(self._h, ctypes.byref(bs), _ptr(E_t), _ptr(F_t), _ptr(W_t), float(w_e),
                                         float(w_f), float(w_s), _lib.SCALINGS[scaling], _lib.PRECISIONS[precision],
                                         int(acc), _ptr(H), _ptr(g), _ptr(yy), _stream(stream)),
              "mtp_normal_equations")
        return H, g, yy

    def solve_normal(self, H, g, stream=None):
        """xi minimising xi^T H xi - 2 g^T xi (mtp_solve_normal)."""
        xi = torch.empty(self.m, dtype=torch.float64, device=self.device)
        check(lib().mtp_solve_normal(self._h, _ptr(H), _ptr(g), _ptr(xi), _stream(stream)), "mtp_solve_normal")
        return xi

    def fit_xi(self, batch: Batch, E_t, F_t, W_t, precision="fp64", stream=None, **weights):
        """Least-squares xi of eq. Fitting at fixed c, installed in the model;
        returns it (device tensor, file basis order)."""
        H, g, _ = self.normal_equations(batch, E_t, F_t, W_t, precision=precision, stream=stream, **weights)
        xi = self.solve_normal(H, g, stream=stream)
        self.set_params(xi=xi.cpu().numpy())
        return xi

    def set_schedule(self, schedule, precision="fp64"):
        """Selects the pass split of the evaluation kernels (mtp_set_schedule)."""
        check(lib().mtp_set_schedule(self._h, _lib.PRECISIONS[precision], int(schedule)), "mtp_set_schedule")

    def autotune(self, batch: Batch, precision="fp64", repeats=3, stream=None, with_b=False):
        """Times every schedule on `batch` and keeps the fastest, without and
        with the per-atom basis values of the descriptor sums (mtp_autotune).
        Returns (chosen index, [ms per schedule]); with_b=True returns the
        schedule and times of evaluations that write the basis values."""
        ms = (ctypes.c_float * 64)()
        chosen = ctypes.c_int(-1)
        bs = batch.c_struct()
        check(lib().mtp_autotune(self._h, ctypes.byref(bs), _lib.PRECISIONS[precision], int(repeats), ms, 64,
                                 ctypes.byref(chosen), _stream(stream)), "mtp_autotune")
        n = 1 if precision != "fp64" else self.n_schedules
        times = [float(ms[k]) for k in range(2 * n)]
        if with_b:
            t_b = times[n:]
            return int(min(range(n), key=lambda k: t_b[k])), t_b
        return chosen.value, times[:n]

    def outputs(self, batch: Batch, forces=True, virial=True, site=False, b=False, energy=True):
        """Preallocated output tensors for eval_async (dict as returned by eval)."""
        dev = self.device
        K, N = batch.n_configs, batch.n_atoms
        res = {}
        if energy:
            res["energy"] = torch.empty(K, dtype=torch.float64, device=dev)
        if forces:
            res["forces"] = torch.empty((N, 3), dtype=torch.float64, device=dev)
        if virial:
            res["virial"] = torch.empty((K, 3, 3), dtype=torch.float64, device=dev)
        if site:
            res["site"] = torch.empty(N, dtype=torch.float64, device=dev)
        if b:
            res["b"] = torch.empty((K, self.m), dtype=torch.float64, device=dev)
        return res

    def eval_async(self, batch: Batch, out: dict, precision="fp32", stream=None):
        """mtp_eval_async into preallocated outputs: no host synchronisation or
        allocation, so it can be captured in a HIP graph (torch.cuda.graph).
        Check self.status() afterwards."""
        o = _lib.mtp_out(*[out[k].data_ptr() if k in out else None
                           for k in ("energy", "forces", "virial", "site", "b")])
        bs = batch.c_struct()
        check(lib().mtp_eval_async(self._h, ctypes.byref(bs), ctypes.byref(o), _lib.PRECISIONS[precision],
                                   _stream(stream)), "mtp_eval_async")
        return out

    def set_skin(self, skin):
        """Verlet skin in Angstrom (mtp_set_skin); 0 searches on every call."""
        check(lib().mtp_set_skin(self._h, float(skin)), "mtp_set_skin")

    def set_timing(self, enable=True):
        check(lib().mtp_set_timing(self._h, 1 if enable else 0), "mtp_set_timing")

    def stats(self):
        st = _lib.mtp_stats()
        check(lib().mtp_get_stats(self._h, ctypes.byref(st)), "mtp_get_stats")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def status(self, stream=None):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib().mtp_status(self._h, _stream(stream), ctypes.byref(a), ctypes.byref(b)), "mtp_status")
        return {"below_rmin": a.value, "list_errors": b.value}

    # grade ------------------------------------------------------------
    def set_active_set(self, A, stream=None):
        A = torch.as_tensor(A, dtype=torch.float64).to(self.device).contiguous()
        if tuple(A.shape) != (self.m, self.m):
            raise ValueError(f"active set must be [{self.m}, {self.m}]")
        check(lib().mtp_set_active_set(self._h, _ptr(A), _stream(stream)), "mtp_set_active_set")

    def grade_from_b(self, b, want_c=False, stream=None):
        b = torch.as_tensor(b, dtype=torch.float64).to(self.device).contiguous()
        n = int(b.shape[0])
        gamma = torch.empty(n, dtype=torch.float64, device=self.device)
        arg = torch.empty(n, dtype=torch.int32, device=self.device)
        c = torch.empty((n, self.m), dtype=torch.float64, device=self.device) if want_c else None
        check(lib().mtp_grade_from_b(self._h, n, _ptr(b), _ptr(gamma), _ptr(arg), _ptr(c), _stream(stream)),
              "mtp_grade_from_b")
        return (gamma, arg, c) if want_c else (gamma, arg)

    def grade_from_b_noalloc(self, b, gamma, argmax, stream=None):
        """mtp_grade_from_b_noalloc: gamma [n] float64 and argmax [n] int32
        are preallocated device tensors; the library allocates nothing."""
        n = int(b.shape[0])
        if b.dtype != torch.float64 or not b.is_contiguous() or b.dim() != 2 or int(b.shape[1]) != self.m:
            raise ValueError("b must be a contiguous float64 [n, m] device tensor")
        if gamma.dtype != torch.float64 or argmax.dtype != torch.int32 or gamma.numel() < n or argmax.numel() < n:
            raise ValueError("gamma must be float64 [n] and argmax int32 [n]")
        check(lib().mtp_grade_from_b_noalloc(self._h, n, _ptr(b), _ptr(gamma), _ptr(argmax), _stream(stream)),
              "mtp_grade_from_b_noalloc")
        return gamma, argmax

    # nonlinear grade: rows dE/dtheta over theta = (xi, c) ------------------
    def theta_rows(self, batch: Batch, precision="fp64", stream=None):
        """dE_k/dtheta [K, m + n_c] FP64 on the device (mtp_theta_rows)."""
        rows = torch.empty((batch.n_configs, self.m + self.n_c), dtype=torch.float64, device=self.device)
        bs = batch.c_struct()
        check(lib().mtp_theta_rows(self._h, ctypes.byref(bs), _lib.PRECISIONS[precision], _ptr(rows),
                                   _stream(stream)), "mtp_theta_rows")
        return rows

    def set_active_set_theta(self, A, stream=None):
        """A [n, n]: theta rows of the active configurations restricted to n
        chosen columns (mtp_set_active_set_theta)."""
        A = torch.as_tensor(A, dtype=torch.float64).to(self.device).contiguous()
        n = int(A.shape[0])
        if A.dim() != 2 or tuple(A.shape) != (n, n) or not 1 <= n <= self.m + self.n_c:
            raise ValueError(f"active set must be square with at most {self.m + self.n_c} columns")
        check(lib().mtp_set_active_set_theta(self._h, n, _ptr(A), _stream(stream)), "mtp_set_active_set_theta")

    def grade_theta(self, rows, stream=None):
        rows = torch.as_tensor(rows, dtype=torch.float64).to(self.device).contiguous()
        n = int(rows.shape[0])
        gamma = torch.empty(n, dtype=torch.float64, device=self.device)
        arg = torch.empty(n, dtype=torch.int32, device=self.device)
        check(lib().mtp_grade_theta(self._h, n, _ptr(rows), _ptr(gamma), _ptr(arg), _stream(stream)),
              "mtp_grade_theta")
        return gamma, arg

    def maxvol_theta(self, pool, rows=None, delta=1e-3, max_swaps=-1, stream=None):
        """MaxVol selection of n rows of a pool of theta rows restricted to n
        columns ([K, n] FP64) by mtp_maxvol_theta; as maxvol otherwise."""
        pool = torch.as_tensor(pool, dtype=torch.float64).to(self.device).contiguous()
        K, n_cols = int(pool.shape[0]), int(pool.shape[1])
        if rows is None:
            r = torch.zeros(n_cols, dtype=torch.int32, device=self.device)
        else:
            r = torch.as_tensor(rows, dtype=torch.int32).to(self.device).clone().contiguous()
        n = ctypes.c_int32()
        check(lib().mtp_maxvol_theta(self._h, n_cols, K, _ptr(pool), _ptr(r), 0 if rows is None else 1,
                                     float(delta), int(max_swaps), ctypes.byref(n), _stream(stream)),
              "mtp_maxvol_theta")
        return r, n.value

    def maxvol(self, pool, rows=None, delta=1e-3, max_swaps=-1, stream=None):
        """MaxVol selection of m rows of pool [K, m] (FP64, file order) by
        mtp_maxvol; rows = starting rows, or None for the pivot rows of
        Gaussian elimination.  Returns (rows int32 [m] on the device, swaps)."""
        pool = torch.as_tensor(pool, dtype=torch.float64).to(self.device).contiguous()
        K = int(pool.shape[0])
        if rows is None:
            r = torch.zeros(self.m, dtype=torch.int32, device=self.device)
        else:
            r = torch.as_tensor(rows, dtype=torch.int32).to(self.device).clone().contiguous()
        n = ctypes.c_int32()
        check(lib().mtp_maxvol(self._h, K, _ptr(pool), _ptr(r), 0 if rows is None else 1, float(delta),
                               int(max_swaps), ctypes.byref(n), _stream(stream)), "mtp_maxvol")
        return r, n.value

    def grade(self, batch: Batch, precision="fp32", stream=None):
        gamma = torch.empty(batch.n_configs, dtype=torch.float64, device=self.device)
        arg = torch.empty(batch.n_configs, dtype=torch.int32, device=self.device)
        bs = batch.c_struct()
        check(lib().mtp_grade(self._h, ctypes.byref(bs), _ptr(gamma), _ptr(arg), _lib.PRECISIONS[precision],
                              _stream(stream)), "mtp_grade")
        return gamma, arg
