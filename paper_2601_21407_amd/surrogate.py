"""Learned k-step surrogate for the cortical channel set: data generation with
the plain fused kernel, training with the library's MLP forward/backward and
Adam kernels, packing for the MFMA inference, deployment with per-neuron
fallback, and the spike-time comparison against the plain integrator.

Every step of the method runs in libhh kernels: the plain trajectories, the
transition samples and their mean input, the feature normalization, the
network's forward and backward, Adam, the inference and the deployment.
torch holds device buffers, draws the seeded synthetic input currents and
the minibatch permutation, and gathers minibatches.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import hh
from . import workloads as W

K_STEPS = 10          # surrogate step = 10 plain steps of 0.025 ms
V_FALLBACK = -50.0    # mV
CHECK_EVERY = 20      # calls (200 plain steps, 5 ms); the configuration fixes no period
CHECK_TOL = 0.5       # mV


ACT = "hardswish"     # hidden activation of the deployed network (or "silu")


def generate_transitions(n_traj=5000, T=10000, seed=5, seg=400, k=K_STEPS, dev="cuda"):
    """Trajectories of the plain FP32 kernel (cortical set, nominal rates,
    dt = 0.025 ms) under piecewise-constant currents U[0, 20) plus 3 z per
    step; every step t with V <= -50 mV at t and t + k gives one transition
    (x_t, mean I over [t, t+k)) -> x_{t+k} - x_t, formed by the library.
    Returns (X [S,7], dY [S,6]) on the device (FP32, un-normalized)."""
    m = W.custom_channels(dt=0.025)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    M = hh.Model(m, n_traj)
    st = M.new_state()
    v0 = -75.0 + 15.0 * torch.rand(n_traj, generator=gen, device=dev)
    M.init_state(st, v0=v0)
    nseg = (T + seg - 1) // seg
    levels = 20.0 * torch.rand((nseg, n_traj), generator=gen, device=dev)
    I = levels.repeat_interleave(seg, dim=0)[:T] + 3.0 * torch.randn((T, n_traj), generator=gen,
                                                                        device=dev)
    I = I.contiguous()
    traj = torch.empty((T, M.n_state, n_traj), device=dev)
    M.step_n(st, T, 0, i_dense=I, ckpt=traj, ckpt_every=1)
    status, bad = M.check()
    if status != 0:
        raise RuntimeError("plain kernel failed while generating data (%d)" % status)
    return hh.surrogate_transitions(traj, I, k, V_FALLBACK, (T - k) * n_traj)


def norm_stats(X, dY):
    """Per-feature mean and standard deviation (library kernel): norm[0:7]
    input mean, [8:15] input std, [16:22] output mean, [24:30] output std."""
    return hh.mlp_norm(X, dY)


def init_params(seed=0, dev="cuda"):
    rng = np.random.default_rng(seed)
    p = np.zeros(hh.MLP_NPARAM, np.float32)
    off = 0
    for a, b in ((7, 64), (64, 64), (64, 6)):
        p[off: off + a * b] = (rng.standard_normal(a * b) * np.sqrt(2.0 / a)).astype(np.float32)
        off += a * b + b
    return torch.tensor(p, device=dev)


def train(X, dY, norm, *, epochs=8, batch=16384, lr=2e-3, seed=0, act=ACT, log=None):
    """Adam on the normalized MSE with bf16-quantized forward (the deployed
    numerics).  Returns (params, history of mean epoch losses)."""
    dev = X.device
    S = X.shape[0]
    params = init_params(seed, dev)
    grad = torch.zeros_like(params)
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    loss = torch.zeros(1, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed + 1)
    ws = None
    hist = []
    step = 0
    total = epochs * (S // batch)
    for ep in range(epochs):
        perm = torch.randperm(S, generator=gen, device=dev)
        acc = torch.zeros(1, device=dev)
        nb = S // batch
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            xb, yb = X[idx].contiguous(), dY[idx].contiguous()
            ws = hh.mlp_grad(params, norm, xb, yb, grad, loss, quantize=True, act=act, workspace=ws)
            step += 1
            # cosine decay of the learning rate
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * step / total))
            hh.adam_step(params, grad, m1, m2, step, lr_t)
            acc += loss
        hist.append(float(acc.item()) / max(nb, 1))
        if log:
            log("epoch %d loss %.4e" % (ep, hist[-1]))
    return params, hist


def evaluate(params, X, dY, norm, act=ACT):
    """Normalized MSE of the quantized network on a held-out set (the loss
    of the library's gradient kernel)."""
    grad = torch.empty_like(params)
    loss = torch.zeros(1, device=X.device)
    hh.mlp_grad(params, norm, X.contiguous(), dY.contiguous(), grad, loss, quantize=True, act=act)
    return float(loss.item())


def spike_time_error(ref_bits, bits, n, dt_ref, dt_test, window_ms=2.0, max_neurons=None):
    """Match spikes of a test raster to the reference raster (greedy, in time
    order, within +-window_ms).  Returns dict with mean and p95 |dt| (ms) of
    matched spikes, the unmatched fraction (of reference + test spikes) and
    counts.  Rasters are [T][words] uint32 bit rows (numpy)."""
    def times(bits_, dt):
        b = np.unpackbits(np.ascontiguousarray(bits_).view(np.uint8).reshape(bits_.shape[0], -1),
                          axis=1, bitorder="little")[:, :n]
        t, i = np.nonzero(b)
        order = np.lexsort((t, i))
        return i[order], (t[order] + 1) * dt
    ri, rt = times(ref_bits, dt_ref)
    ti, tt = times(bits, dt_test)
    nn = n if max_neurons is None else min(n, max_neurons)
    rs = np.searchsorted(ri, np.arange(nn + 1))
    ts = np.searchsorted(ti, np.arange(nn + 1))
    diffs = []
    unmatched = 0
    for j in range(nn):
        a = rt[rs[j]:rs[j + 1]]
        b = tt[ts[j]:ts[j + 1]]
        used = np.zeros(len(b), bool)
        for x in a:
            if len(b) == 0:
                unmatched += 1
                continue
            c = np.abs(b - x)
            c[used] = np.inf
            q = int(np.argmin(c))
            if c[q] <= window_ms:
                used[q] = True
                diffs.append(c[q])
            else:
                unmatched += 1
        unmatched += int((~used).sum())
    diffs = np.asarray(diffs)
    n_ref = int(rs[nn])
    return {"matched": int(len(diffs)), "ref_spikes": n_ref,
            "mean_abs_ms": float(diffs.mean()) if len(diffs) else 0.0,
            "p95_abs_ms": float(np.percentile(diffs, 95)) if len(diffs) else 0.0,
            "unmatched_frac": unmatched / max(n_ref + int(ts[nn]), 1)}


class SurrogateRun:
    """Model, state, fallback flags, spike words and call counts of a
    deployment on n neurons (cortical set, nominal rates) for T plain-step
    equivalents, allocated once; run() starts the simulation from rest, so
    repeated runs time only the simulation."""

    def __init__(self, n, T, *, spikes=True, dev="cuda"):
        self.T = T
        self.M = hh.Model(W.custom_channels(dt=0.025), n)
        self.st = self.M.new_state()
        self.flags = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.bits = torch.zeros((T, self.M.words), dtype=torch.int32, device=dev) if spikes else None
        self.stats = torch.zeros(3, dtype=torch.int64, device=dev)

    def run(self, packed, *, i_dense=None, noise=None, check_every=CHECK_EVERY,
            v_fallback=V_FALLBACK, check_tol=CHECK_TOL, k=K_STEPS, act=ACT):
        """Returns (model, state, spike bits or None, stats [surrogate calls,
        plain calls, failed checks])."""
        self.M.init_state(self.st, v0_scalar=-65.0)
        self.flags.zero_()
        self.stats.zero_()
        hh.surrogate_step_n(self.M, packed, self.st, self.flags, self.T, k, 0, i_dense=i_dense,
                            noise=noise, v_fallback=v_fallback, check_every=check_every,
                            check_tol=check_tol, spikes=self.bits, stats=self.stats, act=act)
        return self.M, self.st, self.bits, self.stats


class PlainRun:
    """The plain kernel on the same workload, allocated once; table =
    (v_lo, v_hi, n_nodes) switches to tabulated gate kinetics."""

    def __init__(self, n, T, *, dt=0.025, v_method="fe", spikes=True, table=None, dev="cuda"):
        self.T = T
        self.M = hh.Model(W.custom_channels(dt=dt, v_method=v_method), n)
        if table is not None:
            self.M.set_rate_table(*table)
        self.st = self.M.new_state()
        self.bits = torch.zeros((T, self.M.words), dtype=torch.int32, device=dev) if spikes else None

    def run(self, *, i_dense=None, noise=None):
        self.M.init_state(self.st, v0_scalar=-65.0)
        self.M.step_n(self.st, self.T, 0, i_dense=i_dense, noise=noise, spikes=self.bits)
        return self.M, self.st, self.bits


def deploy(packed, n, T, *, i_dense=None, noise=None, spikes=True, check_every=CHECK_EVERY,
           v_fallback=V_FALLBACK, check_tol=CHECK_TOL, k=K_STEPS, act=ACT, dev="cuda"):
    """One deployment run (SurrogateRun allocated and run once)."""
    return SurrogateRun(n, T, spikes=spikes, dev=dev).run(
        packed, i_dense=i_dense, noise=noise, check_every=check_every, v_fallback=v_fallback,
        check_tol=check_tol, k=k, act=act)


def plain_run(n, T, *, dt=0.025, v_method="fe", i_dense=None, noise=None, spikes=True,
              dev="cuda", table=None):
    """One plain run (PlainRun allocated and run once)."""
    return PlainRun(n, T, dt=dt, v_method=v_method, spikes=spikes, table=table,
                    dev=dev).run(i_dense=i_dense, noise=noise)


def coarse_input(I, r):
    """Block means of a dense fine-step input over r consecutive steps (the
    same input integral at a coarser dt)."""
    T, n = I.shape
    return I[: (T // r) * r].view(T // r, r, n).mean(1).contiguous()


def timed(fn, reps=3):
    torch.cuda.synchronize()
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps
