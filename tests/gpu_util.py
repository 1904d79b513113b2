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
        if k == "sine" and v is not None:  # (amplitudes [n], frequencies [n])
            out[k] = (np.asarray(v[0])[idx], np.asarray(v[1])[idx])
        elif isinstance(v, np.ndarray) and v.ndim == 1 and v.shape[0] == n:
            out[k] = v[idx]
        elif k in ("coef", "i_dense") and v is not None:
            out[k] = v[:, idx]
        else:
            out[k] = v
    return out


def nominal_coef(model, count):
    """The model's rate coefficients as a per-element table [G*8][count]."""
    G = len(model["gates"])
    nom = np.zeros(G * 8)
    for g, gate in enumerate(model["gates"]):
        for r, rt in enumerate(gate["rates"]):
            nom[g * 8 + r * 4: g * 8 + r * 4 + 4] = rt[1:5]
    return np.repeat(nom[:, None], count, axis=1)


def input_probes(kw, f):
    """Copies of the oracle arguments with the input scaled by f: the
    constant, noise-mean or dense input, or the background amplitudes."""
    out = []
    for key in ("i_const", "noise_mu", "i_dense"):
        if kw.get(key) is not None:
            out.append(dict(kw, **{key: kw[key] * f}))
    if kw.get("background") is not None:
        lam, mu, sigma = kw["background"]
        out.append(dict(kw, background=(lam, mu * f, sigma * f)))
    if kw.get("sine") is not None:
        amp, freq = kw["sine"]
        out.append(dict(kw, sine=(np.asarray(amp) * f, freq)))
    return out


def ill_conditioned(O, model, st0, T, idx, base_kw, *, v_tol=1e-3):
    """Returns (spike_ill, trace_ill): boolean arrays over idx.  spike_ill: a
    probe moves the oracle's spike train by more than one dt (or changes its
    count); trace_ill: a probe moves V by more than v_tol at some step.  The
    probes are those of spike_horizons (input, capacitance, one group of rate
    coefficients) and the initial state."""
    idx = np.asarray(idx, dtype=np.int64)
    n = st0.shape[1]
    if len(idx) == 0:
        return np.zeros(0, bool), np.zeros(0, bool)
    kw = _subset_kw(base_kw, idx, n)
    cm = kw.get("cm")
    if cm is None:
        cm = np.full(len(idx), float(model["C"]))
    ref = O.run(model, st0[:, idx].copy(), T, record_v=True, **dict(kw, cm=cm))
    coef = kw.get("coef")
    if coef is None and len(model["gates"]):
        coef = nominal_coef(model, len(idx))
    probes = []
    for f in (1 + PROBE, 1 - PROBE):
        probes += [dict(p, cm=cm) for p in input_probes(kw, f)]
        probes.append(dict(kw, cm=cm * f))
        if coef is not None:
            for j in range(3):  # A, B, K rows of every rate
                c2 = coef.copy()
                c2[j::4] *= f
                probes.append(dict(kw, cm=cm, coef=c2))
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
    # representation probe: the same FP64 steps with the state stored in
    # FP32 after every step (what any FP32 integrator must at least incur);
    # ill-conditioned when that alone uses half the trace tolerance
    s = s0.copy()
    vr = np.zeros((T, len(idx)))
    spk = np.zeros((T, len(idx)), np.uint8)
    kw1 = dict(kw, cm=cm)
    dense = kw1.pop("i_dense", None)
    t0 = int(kw1.pop("t0", 0))
    for k in range(T):
        extra = {} if dense is None else {"i_dense": dense[k:k + 1]}
        r = O.run(model, s, 1, t0=t0 + k, record_v=True, **kw1, **extra)
        s[:] = s.astype(np.float32).astype(np.float64)
        vr[k] = r["v"][0]
        spk[k] = r["spikes"][0]
    sp[spike_mismatch(spk, ref["spikes"])] = True
    tr |= np.max(np.abs(vr - ref["v"]), axis=0) > 0.5 * v_tol
    return sp, tr


def _interp_times(v, thr):
    """Upward threshold crossings, interpolated within the step (in steps)."""
    out = []
    for j in range(v.shape[1]):
        x = v[:, j]
        ks = np.nonzero((x[:-1] < thr) & (x[1:] >= thr))[0] + 1
        t = [k - 1 + (thr - x[k - 1]) / (x[k] - x[k - 1]) for k in ks]
        if x[0] >= thr:  # crossing in the first step is not interpolable here
            t = [0.0] + t
        out.append(np.array(t))
    return out


def spike_horizons(O, model, st0, T, idx, base_kw, *, shift_tol=0.1):
    """Per neuron in idx: the number of leading oracle spikes whose timing is
    well conditioned.  A spike is ill-conditioned when its interpolated time
    moves by more than shift_tol steps under a 1e-6 relative probe of the
    input, the capacitance or one group (A, B or K) of rate coefficients;
    that spike and all later ones lie beyond the neuron's predictability
    horizon.  Returns (horizon counts, oracle spike-step lists)."""
    idx = np.asarray(idx, dtype=np.int64)
    n = st0.shape[1]
    kw = _subset_kw(base_kw, idx, n)
    cm = kw.get("cm")
    if cm is None:
        cm = np.full(len(idx), float(model["C"]))
    coef = kw.get("coef")
    if coef is None:
        coef = nominal_coef(model, len(idx))
    kw = dict(kw, cm=cm, coef=coef)
    s0 = st0[:, idx]
    thr = float(model["v_th"])
    ref = O.run(model, s0.copy(), T, record_v=True, **kw)
    v0 = np.vstack([s0[0:1], ref["v"]])
    base_t = _interp_times(v0, thr)
    probes = []
    for f in (1 + PROBE, 1 - PROBE):
        probes += input_probes(kw, f)
        probes.append(dict(kw, cm=cm * f))
        for j in range(3):  # A, B, K rows of every rate
            c2 = coef.copy()
            c2[j::4] *= f
            probes.append(dict(kw, coef=c2))
    h = np.array([len(b) for b in base_t])
    for p in probes:
        r = O.run(model, s0.copy(), T, record_v=True, **p)
        tt = _interp_times(np.vstack([s0[0:1], r["v"]]), thr)
        for j, (a, b) in enumerate(zip(tt, base_t)):
            m_ = min(len(a), len(b))
            d = np.abs(a[:m_] - b[:m_]) > shift_tol
            first = int(np.argmax(d)) if d.any() else m_
            if len(a) != len(b):
                first = min(first, m_)
            h[j] = min(h[j], first)
    steps = [np.nonzero(ref["spikes"][:, j])[0] for j in range(len(idx))]
    return h, steps


def match_to_horizon(g_steps, o_steps, h, tol_steps=1):
    """GPU spike steps agree with the first h oracle spikes within tol_steps,
    and the GPU has no other spike before the horizon."""
    if h >= len(o_steps):
        return len(g_steps) == len(o_steps) and (
            len(o_steps) == 0 or np.max(np.abs(np.asarray(g_steps) - o_steps)) <= tol_steps)
    cutoff = o_steps[h] - tol_steps - 1
    g_before = np.asarray([t for t in g_steps if t < cutoff])
    if len(g_before) != h:
        return False
    return h == 0 or np.max(np.abs(g_before - o_steps[:h])) <= tol_steps
