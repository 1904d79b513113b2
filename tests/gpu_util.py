"""Shared helpers of the GPU parity tests (comparison logic only)."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21407_amd import hh  # noqa: F401  (fails loudly if libhh is missing)
    return torch


def spike_trains(raster: np.ndarray):
    return [np.nonzero(raster[:, i])[0] for i in range(raster.shape[1])]


def spike_mismatch(r_gpu: np.ndarray, r_ora: np.ndarray, tol_steps: int = 1):
    """Indices of neurons whose spike trains differ: different counts, or any
    paired spike time more than tol_steps apart."""
    bad = []
    for i in range(r_gpu.shape[1]):
        a = np.nonzero(r_gpu[:, i])[0]
        b = np.nonzero(r_ora[:, i])[0]
        if len(a) != len(b) or (len(a) and np.max(np.abs(a - b)) > tol_steps):
            bad.append(i)
    return np.array(bad, dtype=np.int64)


def print_case(msg: str):
    print("[case] " + msg, flush=True)


# 1e-6 relative probes of the oracle's own sensitivity: input current,
# capacitance, initial V and initial gates, each scaled by (1 +- 1e-6).  The
# GPU computes in FP32, which perturbs every quantity by ~6e-8 relative per
# operation; a neuron whose FP64 trajectory moves by more than the tolerance
# under one of these (16x larger) probes is ill-conditioned: reported, not
# failed.  Typical cases are near-miss excursions that stop just below the
# spike threshold, and spikes triggered close to rheobase.
PROBE = 1e-6


def _subset_kw(kw, idx, n):
    out = {}
    for k, v in kw.items():
        if isinstance(v, np.ndarray) and v.ndim == 1 and v.shape[0] == n:
            out[k] = v[idx]
        elif k in ("coef", "i_dense") and v is not None:
            out[k] = v[:, idx]
        else:
            out[k] = v
    return out


def ill_conditioned(O, model, st0, T, idx, base_kw, *, v_tol=1e-3):
    """Returns (spike_ill, trace_ill): boolean arrays over idx.  spike_ill: a
    probe moves the oracle's spike train by more than one dt (or changes its
    count); trace_ill: a probe moves V by more than v_tol at some step."""
    idx = np.asarray(idx, dtype=np.int64)
    n = st0.shape[1]
    if len(idx) == 0:
        return np.zeros(0, bool), np.zeros(0, bool)
    kw = _subset_kw(base_kw, idx, n)
    cm = kw.get("cm")
    if cm is None:
        cm = np.full(len(idx), float(model["C"]))
    ref = O.run(model, st0[:, idx].copy(), T, record_v=True, **dict(kw, cm=cm))
    probes = []
    for f in (1 + PROBE, 1 - PROBE):
        if kw.get("i_const") is not None:
            probes.append(dict(kw, cm=cm, i_const=kw["i_const"] * f))
        if kw.get("noise_mu") is not None:
            probes.append(dict(kw, cm=cm, noise_mu=kw["noise_mu"] * f))
        if kw.get("i_dense") is not None:
            probes.append(dict(kw, cm=cm, i_dense=kw["i_dense"] * f))
        probes.append(dict(kw, cm=cm * f))
    s0 = st0[:, idx]
    starts = [s0] * len(probes)
    # initial-state probes: V0 and every gate scaled by (1 +- 1e-6)
    G = len(model["gates"])
    for f in (1 + PROBE, 1 - PROBE):
        for rows in ([0], list(range(1, 1 + G))):
            s1 = s0.copy()
            s1[rows] *= f
            probes.append(dict(kw, cm=cm))
            starts.append(s1)
    sp = np.zeros(len(idx), bool)
    tr = np.zeros(len(idx), bool)
    for p, s_init in zip(probes, starts):
        r = O.run(model, s_init.copy(), T, record_v=True, **p)
        bad = spike_mismatch(r["spikes"], ref["spikes"])
        sp[bad] = True
        tr |= np.max(np.abs(r["v"] - ref["v"]), axis=0) > v_tol
    return sp, tr
