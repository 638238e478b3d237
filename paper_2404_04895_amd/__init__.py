"""Tensorized Ant Colony Optimization for the Euclidean TSP on MI355X (gfx950).

Python binding of libaco.so (C ABI: include/aco.h).  This layer only marshals
arguments: every step of an iteration runs in the library's HIP kernels.
PyTorch provides the device memory (one workspace tensor per colony) and the
stream the library enqueues on.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import (BATCH_SORTED_MAX_N, SCHED_AUTO, SCHED_G16, SCHED_G32, SCHED_G32_LIVE,
                      SCHED_G64, SCHED_G64_LIVE, SCHED_SORTED, SCHEDULES, SORTED_SCHEDULES,
                      AcoError, AcoParams, BatchView, ScheduleEntry, check, lib)

__all__ = ["Colony", "Batch", "MlpTrainer", "edge_ranks", "mlp_eta", "mlp_features",
           "mlp_targets", "mlp_round", "mlp_gradient_noalloc", "MLP_PARAMS", "AcoError", "uniforms", "gamma_schedule", "workspace_bytes",
           "leading_dim", "MAX_CITIES", "SCHEDULES", "SCHED_AUTO", "SCHED_SORTED",
           "SORTED_SCHEDULES", "BATCH_SORTED_MAX_N"]

MAX_CITIES = _native.MAX_CITIES
MLP_PARAMS = _native.MLP_PARAMS


def _torch():
    import torch
    return torch


def leading_dim(n: int) -> int:
    return lib().aco_leading_dim(n)


def workspace_bytes(n: int, m_max: int) -> int:
    return lib().aco_workspace_bytes(n, m_max)


def gamma_schedule(t: int, T: int, gamma_max: float, gamma_min: float) -> float:
    return lib().aco_gamma_schedule(t, T, gamma_max, gamma_min)


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def uniforms(seed: int, iter: int, ant: int, step: int, count: int, device="cuda", stream=None):
    """The deviates r_j (j < count) ant `ant` draws at `step` of `iter`, from the device generator."""
    torch = _torch()
    out = torch.empty(count, dtype=torch.float32, device=device)
    check(lib().aco_uniforms(seed, iter, ant, step, count, ctypes.c_void_p(out.data_ptr()),
                             _stream_handle(stream)), "aco_uniforms")
    return out


class Colony:
    """One TSP instance and its pheromone state on one GPU.

    dist: (n, n) float32 distance matrix, a CUDA tensor or anything numpy accepts.
    """

    def __init__(self, dist, alpha: float, beta: float, rho: float, Q: float = 1.0,
                 m_max: int | None = None, *, tau0: float = 1.0, elite_k: int = 0,
                 gamma_max: float = 1.5, gamma_min: float = 1.0, device="cuda", stream=None):
        torch = _torch()
        if not isinstance(dist, torch.Tensor):
            dist = torch.from_numpy(np.ascontiguousarray(dist, dtype=np.float32))
        if dist.device.type != "cuda":
            dist = dist.to(device)
        dist = dist.to(torch.float32).contiguous()
        if dist.dim() != 2 or dist.shape[0] != dist.shape[1]:
            raise ValueError("dist must be a square matrix")
        n = int(dist.shape[0])
        self.n = n
        self.m_max = int(m_max if m_max is not None else n)
        self.device = dist.device
        self.ld = leading_dim(n)
        self._stream = stream
        self._ctx = None
        nbytes = workspace_bytes(n, self.m_max)
        if nbytes == 0:
            check(_native.ACO_EINVAL if n < 3 or n > MAX_CITIES else _native.ACO_EINVAL,
                  "aco_workspace_bytes(n=%d, m_max=%d)" % (n, self.m_max))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace tensor is not 256-byte aligned")
        ctx = ctypes.c_void_p()
        check(lib().aco_create(ctypes.c_void_p(dist.data_ptr()), n, alpha, beta, rho, Q,
                               self.m_max, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                               _stream_handle(stream), ctypes.byref(ctx)), "aco_create")
        self._ctx = ctx
        self.alpha, self.beta, self.rho, self.Q = alpha, beta, rho, Q
        self.params = AcoParams(tau0, elite_k, gamma_max, gamma_min)
        if (tau0, elite_k, gamma_max, gamma_min) != (1.0, 0, 1.5, 1.0):
            self.set_params(tau0=tau0, elite_k=elite_k, gamma_max=gamma_max,
                            gamma_min=gamma_min)

    # ---- lifetime ---------------------------------------------------------
    def close(self):
        if self._ctx is not None:
            lib().aco_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- configuration ----------------------------------------------------
    def set_params(self, *, tau0=None, elite_k=None, gamma_max=None, gamma_min=None):
        p = AcoParams(self.params.tau0 if tau0 is None else tau0,
                      self.params.elite_k if elite_k is None else elite_k,
                      self.params.gamma_max if gamma_max is None else gamma_max,
                      self.params.gamma_min if gamma_min is None else gamma_min)
        check(lib().aco_set_params(self._ctx, ctypes.byref(p)), "aco_set_params")
        self.params = p

    def set_eta(self, eta):
        """Replace eta = 1/d by a caller heuristic ((n, n) float32), or None for 1/d.
        Returns True if the heuristic is in use (False: it was rejected, 1/d is used)."""
        torch = _torch()
        if eta is None:
            check(lib().aco_set_eta(self._ctx, None), "aco_set_eta")
            return False
        if not isinstance(eta, torch.Tensor):
            eta = torch.from_numpy(np.ascontiguousarray(eta, dtype=np.float32))
        eta = eta.to(self.device, torch.float32).contiguous()
        check(lib().aco_set_eta(self._ctx, ctypes.c_void_p(eta.data_ptr())), "aco_set_eta")
        return bool(lib().aco_eta_active(self._ctx))

    def set_schedule(self, schedule: int):
        check(lib().aco_set_schedule(self._ctx, schedule), "aco_set_schedule")

    def set_selection(self, selection: str):
        """"adair" (argmax of P * r, the default), "adair-sorted" (the same
        selection, bit for bit, by a walk of each row sorted by P) or
        "roulette" (the Roulette Wheel baseline: city j with probability
        P[c,j] over the unvisited sum)."""
        code = {"adair": _native.SELECT_ADAIR, "roulette": _native.SELECT_ROULETTE,
                "adair-sorted": _native.SELECT_ADAIR_SORTED}[selection]
        check(lib().aco_set_selection(self._ctx, code), "aco_set_selection")

    def set_tau_bounds(self, tau_min: float = 0.0, tau_max: float = float("inf")):
        """MAX-MIN bounds on tau after each update (0, inf: none)."""
        check(lib().aco_set_tau_bounds(self._ctx, tau_min, tau_max), "aco_set_tau_bounds")

    def set_sorted_walk(self, batches: int):
        """Batches of 64 sorted entries a step reads before it scans (adair-sorted)."""
        check(lib().aco_set_sorted_walk(self._ctx, batches), "aco_set_sorted_walk")

    def sorted_walk_stats(self):
        """(batches read, steps scanned, blocks scanned) of the last adair-sorted construct."""
        out = np.zeros(3, np.uint64)
        check(lib().aco_sorted_walk_stats(self._ctx, out.ctypes.data_as(ctypes.c_void_p)),
              "aco_sorted_walk_stats")
        return tuple(int(v) for v in out)

    def sorted_rows(self):
        """(values, cities) of the rows of P sorted by the last adair-sorted construct:
        the K entries each row keeps (n x K)."""
        torch = _torch()
        K = int(lib().aco_sorted_prefix(self._ctx))
        Ps = self._view(lib().aco_sorted_rows(self._ctx), torch.float32, (self.n, K))
        Js = self._view(lib().aco_sorted_cities(self._ctx), torch.int16, (self.n, K))
        return Ps, Js

    def set_stream(self, stream):
        self._stream = stream
        check(lib().aco_set_stream(self._ctx, _stream_handle(stream)), "aco_set_stream")

    # ---- the iteration ----------------------------------------------------
    def transition(self, gamma: float):
        check(lib().aco_transition(self._ctx, gamma), "aco_transition")

    def construct(self, m: int, seed: int, iter: int):
        check(lib().aco_construct(self._ctx, m, seed, iter), "aco_construct")

    def update(self, gamma_next: float):
        check(lib().aco_update(self._ctx, gamma_next), "aco_update")

    def run(self, m: int, seed: int, iters: int):
        tour = np.zeros(self.n, np.int32)
        length = ctypes.c_float()
        check(lib().aco_run(self._ctx, m, seed, iters, tour.ctypes.data_as(ctypes.c_void_p),
                            ctypes.byref(length)), "aco_run")
        return tour, float(length.value)

    def best(self):
        tour = np.zeros(self.n, np.int32)
        length = ctypes.c_float()
        it = ctypes.c_int32()
        check(lib().aco_best(self._ctx, tour.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(length), ctypes.byref(it)), "aco_best")
        return tour, float(length.value), int(it.value)

    def sync(self):
        check(lib().aco_sync(self._ctx), "aco_sync")

    @property
    def deposit_scale(self) -> int:
        return lib().aco_deposit_scale(self._ctx)

    # ---- device views -----------------------------------------------------
    def _view(self, ptr, dtype, shape):
        torch = _torch()
        itemsize = torch.empty((), dtype=dtype).element_size()
        count = int(np.prod(shape))
        off = ptr - self.workspace.data_ptr()
        assert 0 <= off and off + count * itemsize <= self.workspace.numel()
        return self.workspace[off:off + count * itemsize].view(dtype).view(*shape)

    def tau_padded(self):
        return self._view(lib().aco_pheromone(self._ctx), _torch().float32, (self.n, self.ld))

    def P_padded(self):
        return self._view(lib().aco_transition_matrix(self._ctx), _torch().float32,
                          (self.n, self.ld))

    def tau(self):
        return self.tau_padded()[:, :self.n]

    def P(self):
        return self.P_padded()[:, :self.n]

    def tours(self, m: int | None = None):
        t = self._view(lib().aco_tours(self._ctx), _torch().int32, (self.m_max, self.n))
        return t if m is None else t[:m]

    def lengths(self, m: int | None = None):
        L = self._view(lib().aco_lengths(self._ctx), _torch().float32, (self.m_max,))
        return L if m is None else L[:m]

    # ---- checkpoint -------------------------------------------------------
    def get_state(self):
        torch = _torch()
        tau = torch.empty((self.n, self.ld), dtype=torch.float32, device=self.device)
        it = ctypes.c_uint32()
        check(lib().aco_get_state(self._ctx, ctypes.c_void_p(tau.data_ptr()), ctypes.byref(it)),
              "aco_get_state")
        return tau, int(it.value)

    def set_state(self, tau_padded, iter: int):
        tau_padded = tau_padded.to(self.device).contiguous()
        assert tuple(tau_padded.shape) == (self.n, self.ld)
        check(lib().aco_set_state(self._ctx, ctypes.c_void_p(tau_padded.data_ptr()), iter),
              "aco_set_state")


class Batch:
    """Many independent instances advanced together on one GPU.

    dists: list of (n_i, n_i) float32 distance matrices; ants: list of m_i
    (default n_i); seeds: list of generator seeds (default 0..count-1).
    Instance i evolves exactly as Colony(dists[i], ..., m_max=m_i).run(m_i, seeds[i], T).
    """

    def __init__(self, dists, alpha, beta, rho, Q=1.0, ants=None, seeds=None, *, tau0=1.0,
                 elite_k=0, gamma_max=1.5, gamma_min=1.0, device="cuda", stream=None):
        torch = _torch()
        mats = [np.ascontiguousarray(d, dtype=np.float32) for d in dists]
        self.count = len(mats)
        self.ns = np.array([d.shape[0] for d in mats], dtype=np.int32)
        self.ms = np.array(self.ns if ants is None else ants, dtype=np.int32)
        self.seeds = np.array(range(self.count) if seeds is None else seeds, dtype=np.uint64)
        offsets = np.zeros(self.count, dtype=np.int64)
        offsets[1:] = np.cumsum((self.ns.astype(np.int64) ** 2))[:-1]
        flat = np.concatenate([d.ravel() for d in mats])
        dev_dists = torch.from_numpy(flat).to(device)
        self.device = dev_dists.device
        self._stream = stream
        nbytes = lib().aco_batch_workspace_bytes(self.ns.ctypes.data_as(ctypes.c_void_p),
                                                 self.ms.ctypes.data_as(ctypes.c_void_p),
                                                 self.count)
        if nbytes == 0:
            raise ValueError("invalid batch sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        params = AcoParams(tau0, elite_k, gamma_max, gamma_min)
        handle = ctypes.c_void_p()
        self._b = None
        check(lib().aco_batch_create(ctypes.c_void_p(dev_dists.data_ptr()),
                                     offsets.ctypes.data_as(ctypes.c_void_p),
                                     self.ns.ctypes.data_as(ctypes.c_void_p),
                                     self.ms.ctypes.data_as(ctypes.c_void_p),
                                     self.seeds.ctypes.data_as(ctypes.c_void_p), self.count,
                                     alpha, beta, rho, Q, ctypes.byref(params),
                                     ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                     _stream_handle(stream), ctypes.byref(handle)),
              "aco_batch_create")
        self._b = handle

    def close(self):
        if self._b is not None:
            lib().aco_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedules(self, table, persistent_waves=0):
        """table: list of (n_max, schedule) pairs."""
        arr = (ScheduleEntry * max(len(table), 1))(*[ScheduleEntry(a, b) for a, b in table])
        check(lib().aco_batch_set_schedules(self._b, arr, len(table), persistent_waves),
              "aco_batch_set_schedules")

    def run(self, iters, use_graph=True, time_construct=False):
        flags = (_native.BATCH_GRAPH if use_graph else 0) | (
            _native.BATCH_TIME_CONSTRUCT if time_construct else 0)
        check(lib().aco_batch_run(self._b, iters, flags), "aco_batch_run")

    def construct_time(self):
        """(total ms, launches) of the construct launches timed by the last run."""
        ms = ctypes.c_double()
        k = ctypes.c_int32()
        check(lib().aco_batch_construct_time(self._b, ctypes.byref(ms), ctypes.byref(k)),
              "aco_batch_construct_time")
        return float(ms.value), int(k.value)

    def sync(self):
        check(lib().aco_batch_sync(self._b), "aco_batch_sync")

    def sorted_walk_stats(self):
        """(entries read, steps scanned, blocks scanned) of the sorted walks of the
        members with SCHED_SORTED since the previous call; resets the counts."""
        out = np.zeros(3, np.uint64)
        check(lib().aco_batch_sorted_walk_stats(self._b, out.ctypes.data_as(ctypes.c_void_p)),
              "aco_batch_sorted_walk_stats")
        return tuple(int(v) for v in out)

    def best(self):
        lens = np.zeros(self.count, np.float32)
        its = np.zeros(self.count, np.int32)
        tours = np.zeros(int(self.ns.sum()), np.int32)
        check(lib().aco_batch_best(self._b, lens.ctypes.data_as(ctypes.c_void_p),
                                   its.ctypes.data_as(ctypes.c_void_p),
                                   tours.ctypes.data_as(ctypes.c_void_p)), "aco_batch_best")
        split = np.split(tours, np.cumsum(self.ns)[:-1])
        return lens, its, split

    def view(self, i):
        v = BatchView()
        check(lib().aco_batch_instance(self._b, i, ctypes.byref(v)), "aco_batch_instance")
        return v

    def _dev(self, ptr, dtype, shape):
        torch = _torch()
        itemsize = torch.empty((), dtype=dtype).element_size()
        count = int(np.prod(shape))
        off = ptr - self.workspace.data_ptr()
        assert 0 <= off and off + count * itemsize <= self.workspace.numel()
        return self.workspace[off:off + count * itemsize].view(dtype).view(*shape)

    def tau(self, i):
        v = self.view(i)
        return self._dev(v.tau, _torch().float32, (v.n, v.ld))[:, :v.n]

    def P(self, i):
        v = self.view(i)
        return self._dev(v.P, _torch().float32, (v.n, v.ld))[:, :v.n]

    def tours(self, i):
        v = self.view(i)
        return self._dev(v.tours, _torch().int32, (v.m, v.n))

    def lengths(self, i):
        v = self.view(i)
        return self._dev(v.lengths, _torch().float32, (v.m,))


# ---------------------------------------------------------------------------
# Learned edge heuristic
# ---------------------------------------------------------------------------
def _dev_f32(x, device="cuda"):
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    return x.to(device=device, dtype=torch.float32).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def edge_ranks(dist, stream=None):
    """(rank (n, n) int32, nearest-neighbour distance (n,), mean (1,) float64), on the device."""
    torch = _torch()
    d = _dev_f32(dist)
    n = d.shape[0]
    rank = torch.empty((n, n), dtype=torch.int32, device=d.device)
    nn = torch.empty(n, dtype=torch.float32, device=d.device)
    mean = torch.empty(1, dtype=torch.float64, device=d.device)
    check(lib().aco_edge_ranks(_ptr(d), n, _ptr(rank), _ptr(nn), _ptr(mean),
                               _stream_handle(stream)), "aco_edge_ranks")
    return rank, nn, mean


def mlp_eta(bf16_params, dist, rank=None, mean=None, stream=None, kappa=1.0, lam=0.0):
    """(eta (n, n) float32, number of non-finite outputs); eta = sigmoid(z)^kappa / f1^lam."""
    torch = _torch()
    d = _dev_f32(dist)
    n = d.shape[0]
    if rank is None or mean is None:
        rank, _, mean = edge_ranks(d, stream)
    params = _dev_f32(bf16_params, d.device)
    eta = torch.empty((n, n), dtype=torch.float32, device=d.device)
    bad = torch.zeros(1, dtype=torch.int32, device=d.device)
    check(lib().aco_mlp_eta(_ptr(params), _ptr(d), _ptr(rank), _ptr(mean), n, kappa, lam,
                            _ptr(eta), _ptr(bad), _stream_handle(stream)), "aco_mlp_eta")
    return eta, bad


def mlp_features(dist, rank=None, mean=None, stream=None):
    torch = _torch()
    d = _dev_f32(dist)
    n = d.shape[0]
    if rank is None or mean is None:
        rank, _, mean = edge_ranks(d, stream)
    feats = torch.empty((n * (n - 1), 3), dtype=torch.float32, device=d.device)
    check(lib().aco_mlp_features(_ptr(d), _ptr(rank), _ptr(mean), n, _ptr(feats),
                                 _stream_handle(stream)), "aco_mlp_features")
    return feats


def mlp_targets(tau_padded, n, stream=None):
    torch = _torch()
    tau = tau_padded.contiguous()
    y = torch.empty(n * (n - 1), dtype=torch.float32, device=tau.device)
    check(lib().aco_mlp_targets(_ptr(tau), n, tau.shape[1], _ptr(y), _stream_handle(stream)),
          "aco_mlp_targets")
    return y


def mlp_round(params, stream=None):
    torch = _torch()
    p = _dev_f32(params)
    out = torch.empty_like(p)
    check(lib().aco_mlp_round(_ptr(p), _ptr(out), _stream_handle(stream)), "aco_mlp_round")
    return out


class MlpTrainer:
    """Minibatch Adam training of the edge MLP on the device."""

    def __init__(self, init_params, batch, device="cuda", stream=None):
        torch = _torch()
        p = _dev_f32(init_params, device)
        assert p.numel() == MLP_PARAMS
        self.batch = int(batch)
        self._stream = stream
        nbytes = lib().aco_mlp_trainer_workspace_bytes(self.batch)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=p.device)
        h = ctypes.c_void_p()
        self._t = None
        check(lib().aco_mlp_trainer_create(_ptr(p), self.batch, _ptr(self.workspace), nbytes,
                                           _stream_handle(stream), ctypes.byref(h)),
              "aco_mlp_trainer_create")
        self._t = h
        self.device = p.device

    def close(self):
        if self._t is not None:
            lib().aco_mlp_trainer_destroy(self._t)
            self._t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gradient(self, feats, y):
        torch = _torch()
        f = _dev_f32(feats, self.device).reshape(-1, 3).contiguous()
        yy = _dev_f32(y, self.device)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        check(lib().aco_mlp_trainer_gradient(self._t, _ptr(f), _ptr(yy), f.shape[0], _ptr(g)),
              "aco_mlp_trainer_gradient")
        return g

    def apply(self, lr):
        check(lib().aco_mlp_trainer_apply(self._t, lr), "aco_mlp_trainer_apply")

    def step(self, feats, y, seed, lr):
        check(lib().aco_mlp_trainer_step(self._t, _ptr(feats), _ptr(y), y.numel(), seed, lr),
              "aco_mlp_trainer_step")

    def loss(self):
        v = ctypes.c_double()
        check(lib().aco_mlp_trainer_loss(self._t, ctypes.byref(v)), "aco_mlp_trainer_loss")
        return float(v.value)

    def params(self):
        torch = _torch()
        master = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        eff = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        check(lib().aco_mlp_trainer_params(self._t, _ptr(master), _ptr(eff)),
              "aco_mlp_trainer_params")
        return master, eff


def mlp_gradient_noalloc(bf16_params, feats, y, grad_out, loss_out=None, stream=None):
    """aco_mlp_gradient_noalloc: the gradient of the mean loss at BF16
    parameters into grad_out (and the mean loss into loss_out), with no device
    allocation in the library or here.  Every argument is a contiguous CUDA
    tensor already: bf16_params, feats (count, 3), y, grad_out float32,
    loss_out one float64 or None."""
    check(lib().aco_mlp_gradient_noalloc(_ptr(bf16_params), _ptr(feats), _ptr(y),
                                         feats.shape[0], _ptr(grad_out),
                                         None if loss_out is None else _ptr(loss_out),
                                         _stream_handle(stream)), "aco_mlp_gradient_noalloc")
