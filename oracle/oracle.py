"""FP64 reference oracle for the Hodgkin-Huxley hot path (ctypes + numpy).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke entry
and the CPU-baseline leg of the benchmark import this module.  It shares no
code with the HIP library: the C part (``hh_oracle.c``) integrates the model of
Methods, Eq. (1)-(2) step by step in double precision; the numpy part holds the
dense pieces (input projection, readout, cross entropy, the MLP surrogate and
Adam), each written from its plain definition.

Models are given as plain dictionaries (see ``model_to_struct``) so that the
oracle and the HIP library each translate the same description into their own
representation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhh_oracle.so")

MAX_GATES = 8
MAX_CH = 8
FORMS = {"exp": 0, "sigmoid": 1, "linoid": 2, "bell": 3}
KINDS = {"ab": 0, "inftau": 1}
VMETH = {"fe": 0, "ee": 1}
IN_NONE, IN_CONST, IN_NOISE, IN_DENSE, IN_BACKGROUND = 0, 1, 2, 3, 4


_OMP_PATH = os.path.join(_HERE, "libhh_oracle_omp.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, no fast-math), and the same
    source with OpenMP (the all-core timing leg: independent neurons split
    over threads, each neuron's arithmetic unchanged)."""
    src = os.path.join(_HERE, "hh_oracle.c")
    newest = max(os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "hh_oracle.h")))
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off"]
                + extra + ["-o", tmp, src, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


class OraModel(ctypes.Structure):
    _fields_ = [
        ("n_gates", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("v_method", ctypes.c_int32),
        ("has_syn", ctypes.c_int32),
        ("gate_kind", ctypes.c_int32 * MAX_GATES),
        ("rate_form", (ctypes.c_int32 * 2) * MAX_GATES),
        ("rate_coef", ((ctypes.c_double * 4) * 2) * MAX_GATES),
        ("ch_n", ctypes.c_int32 * MAX_CH),
        ("ch_gate", (ctypes.c_int32 * 4) * MAX_CH),
        ("ch_expo", (ctypes.c_int32 * 4) * MAX_CH),
        ("ch_gbar", ctypes.c_double * MAX_CH),
        ("ch_E", ctypes.c_double * MAX_CH),
        ("C", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("v_th", ctypes.c_double),
        ("tau_e", ctypes.c_double),
        ("tau_i", ctypes.c_double),
        ("E_e", ctypes.c_double),
        ("E_i", ctypes.c_double),
        ("tab_n", ctypes.c_int32),
        ("tab_vlo", ctypes.c_double),
        ("tab_h", ctypes.c_double),
    ]


def model_to_struct(model: dict) -> OraModel:
    """Translate a model dictionary into the oracle's C struct.

    model = {"gates": [{"kind": "ab"|"inftau", "rates": [(form, A, B, K, c), (form, A, B, K, c)]}],
             "channels": [{"gbar": g, "E": E, "gates": [(gate_index, exponent), ...]}],
             "C": C_m, "dt": dt, "v_th": theta, "v_method": "fe"|"ee",
             "syn": None | {"tau_e", "tau_i", "E_e", "E_i"},
             "table": absent | (v_lo, v_hi, n_nodes)}   # tabulated gate kinetics
    """
    s = OraModel()
    gates, chans = model["gates"], model["channels"]
    s.n_gates, s.n_channels = len(gates), len(chans)
    s.v_method = VMETH[model["v_method"]]
    syn = model.get("syn")
    s.has_syn = 1 if syn else 0
    for g, gate in enumerate(gates):
        s.gate_kind[g] = KINDS[gate["kind"]]
        for r, rate in enumerate(gate["rates"]):
            s.rate_form[g][r] = FORMS[rate[0]]
            for j in range(4):
                s.rate_coef[g][r][j] = float(rate[1 + j])
    for c, ch in enumerate(chans):
        s.ch_n[c] = len(ch["gates"])
        for k, (gi, ex) in enumerate(ch["gates"]):
            s.ch_gate[c][k] = gi
            s.ch_expo[c][k] = ex
        s.ch_gbar[c] = float(ch["gbar"])
        s.ch_E[c] = float(ch["E"])
    s.C, s.dt, s.v_th = float(model["C"]), float(model["dt"]), float(model["v_th"])
    if syn:
        s.tau_e, s.tau_i = float(syn["tau_e"]), float(syn["tau_i"])
        s.E_e, s.E_i = float(syn["E_e"]), float(syn["E_i"])
    tab = model.get("table")
    if tab is not None:
        v_lo, v_hi, n_nodes = float(tab[0]), float(tab[1]), int(tab[2])
        s.tab_n, s.tab_vlo, s.tab_h = n_nodes, v_lo, (v_hi - v_lo) / (n_nodes - 1)
    return s


_libs = {}


def lib(omp: bool = False):
    """The serial oracle library, or with omp its OpenMP build."""
    if omp not in _libs:
        build()
        L = ctypes.CDLL(_OMP_PATH if omp else _LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64, u32, u64, vp = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p)
        L.ora_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.ora_philox4x32_10.restype = None
        L.ora_noise.argtypes = [u64, u32, i64]
        L.ora_noise.restype = d
        L.ora_event_word.argtypes = [u64, u32, i64]
        L.ora_event_word.restype = u32
        L.ora_rate.argtypes = [i32, P(d), d, P(d)]
        L.ora_rate.restype = d
        L.ora_gate_inf.argtypes = [P(OraModel), vp, i64, i64, i32, d]
        L.ora_gate_inf.restype = d
        L.ora_cable_run.argtypes = [P(OraModel), i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, i64,
                                    i32, i32, vp, d, d, u64, d, vp, vp, vp]
        L.ora_cable_run.restype = i32
        L.ora_gate_pq.argtypes = [P(OraModel), vp, i64, i64, i32, d, P(d), P(d)]
        L.ora_gate_pq.restype = None
        L.ora_init_state.argtypes = [P(OraModel), vp, i64, vp, vp]
        L.ora_init_state.restype = None
        L.ora_n_state.argtypes = [P(OraModel)]
        L.ora_n_state.restype = i32
        L.ora_run.argtypes = [P(OraModel), i64, vp, vp, vp, vp, i64, i32, i32, vp, d, d, u64, d,
                              vp, vp, vp, vp]
        L.ora_run_sine.argtypes = [P(OraModel), i64, vp, vp, vp, i64, i32, vp, vp, vp, vp, vp]
        L.ora_run_sine.restype = i32
        L.ora_sine_rate.argtypes = [d, d]
        L.ora_sine_rate.restype = u32
        L.ora_sine.argtypes = [d, u32, i64]
        L.ora_sine.restype = d
        L.ora_background_count.argtypes = [u32, d]
        L.ora_background_count.restype = i32
        L.ora_background.argtypes = [u64, u32, i64, d, d, d, P(i32)]
        L.ora_background.restype = d
        L.ora_run.restype = i32
        L.ora_net_run.argtypes = [P(OraModel), i64, vp, vp, vp, vp, d, vp, i32, vp, u32, d, u64,
                                  i32, vp, d, d, u64, d, i64, i32, vp]
        L.ora_net_run.restype = i32
        L.ora_syn_deliver.argtypes = [i64, vp, vp, vp, d, vp, vp, vp]
        L.ora_syn_deliver.restype = None
        L.ora_bptt.argtypes = [P(OraModel), i64, vp, vp, i32, vp, vp, vp, i32, d, vp, vp, vp, vp]
        L.ora_bptt.restype = i32
        L.ora_threads.argtypes = []
        L.ora_threads.restype = i32
        _libs[omp] = L
    return _libs[omp]


def threads(omp: bool = False) -> int:
    """Threads the oracle's independent-neuron loop uses."""
    return int(lib(omp).ora_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# random numbers (published definitions)
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def noise(seed: int, nid: int, t: int) -> float:
    return float(lib().ora_noise(seed, nid, t))


def event_word(seed: int, nid: int, t: int) -> int:
    return int(lib().ora_event_word(seed, nid, t))


# --------------------------------------------------------------------------
# single-neuron pieces
# --------------------------------------------------------------------------
def rate(form: str, coefs, V: float):
    """(value, dvalue/dV) of one rate function."""
    k = (ctypes.c_double * 4)(*[float(x) for x in coefs])
    dv = ctypes.c_double()
    r = lib().ora_rate(FORMS[form], k, float(V), ctypes.byref(dv))
    return float(r), float(dv.value)


def gate_pq(model: dict, g: int, V: float):
    """(P, Q) of gate g at V, the terms of the gate update p' = p + (P - p) Q:
    exact, or interpolated when the model carries a "table"."""
    s = model_to_struct(model)
    P, Q = ctypes.c_double(), ctypes.c_double()
    lib().ora_gate_pq(ctypes.byref(s), None, 1, 0, int(g), float(V), ctypes.byref(P), ctypes.byref(Q))
    return P.value, Q.value


def n_state(model: dict) -> int:
    return 1 + len(model["gates"]) + (2 if model.get("syn") else 0)


def init_state(model: dict, v0, coef=None) -> np.ndarray:
    v0 = _f64(np.atleast_1d(v0))
    n = v0.shape[0]
    st = np.zeros((n_state(model), n), dtype=np.float64)
    coef = _f64(coef)
    s = model_to_struct(model)
    lib().ora_init_state(ctypes.byref(s), _p(coef), n, _p(v0), _p(st))
    return st


def _input_mode(T, n, i_const, noise_mu, noise_sigma, i_dense, background):
    """(mode, i_const, i_dense, mu, sigma, lam) of one of the input kinds;
    background = (lam, mu, sigma)."""
    if i_dense is not None:
        i_dense = _f64(i_dense)
        assert i_dense.shape == (T, n)
        return IN_DENSE, None, i_dense, 0.0, 0.0, 0.0
    if background is not None:
        lam, mu, sigma = (float(x) for x in background)
        return IN_BACKGROUND, None, None, mu, sigma, lam
    if noise_mu is not None:
        return IN_NOISE, None, None, float(noise_mu), float(noise_sigma or 0.0), 0.0
    if i_const is not None:
        return IN_CONST, _f64(i_const), None, 0.0, 0.0, 0.0
    return IN_NONE, None, None, 0.0, 0.0, 0.0


def background_count(w0: int, lam: float) -> int:
    """N for Philox word w0 (inverse transform in binary32)."""
    return int(lib().ora_background_count(int(w0), float(lam)))


def background(seed: int, nid: int, t: int, lam: float, mu: float, sigma: float):
    """(current, N) of the background input for (seed, element, step)."""
    N = ctypes.c_int32()
    I = lib().ora_background(int(seed), int(nid), int(t), float(lam), float(mu), float(sigma),
                             ctypes.byref(N))
    return I, N.value


def sine_rate(f: float, dt: float) -> int:
    """R: the frequency f (Hz) as revolutions / 2^32 per step of dt (ms)."""
    return int(lib().ora_sine_rate(float(f), float(dt)))


def sine(amp: float, R: int, t: int) -> float:
    return float(lib().ora_sine(float(amp), int(R), int(t)))


def run(model: dict, state: np.ndarray, T: int, t0: int = 0, *, i_const=None, noise_mu=None,
        noise_sigma=None, seed: int = 0, i_dense=None, coef=None, cm=None, ids=None,
        record_v: bool = False, record_spikes: bool = True, level: bool = False, background=None,
        sine=None, omp: bool = False):
    """Advance independent neurons T steps in place.  Returns dict with
    'spikes' [T][n] uint8 (upward crossings), 'v' [T][n] (optional) and
    'level' [n] (count of steps with V >= v_th, optional).  omp: the OpenMP
    build (same results; used to time the oracle on all host cores)."""
    s = model_to_struct(model)
    n = state.shape[1]
    assert state.dtype == np.float64 and state.flags.c_contiguous
    coef, cm = _f64(coef), _f64(cm)
    spk = np.zeros((T, n), np.uint8) if record_spikes else None
    vr = np.zeros((T, n), np.float64) if record_v else None
    lv = np.zeros(n, np.float64) if level else None
    if sine is not None:  # sine = (amplitudes [n], frequencies [n] in Hz)
        amp, freq = _f64(sine[0]), _f64(sine[1])
        rc = lib().ora_run_sine(ctypes.byref(s), n, _p(coef), _p(cm), _p(state), int(t0), int(T),
                                _p(amp), _p(freq), _p(spk), _p(vr), _p(lv))
        if rc != 0:
            raise ValueError("oracle rejected the model (rc=%d)" % rc)
        return {"spikes": spk, "v": vr, "level": lv}
    mode, i_const, i_dense, mu, sigma, lam = _input_mode(T, n, i_const, noise_mu, noise_sigma,
                                                        i_dense, background)
    ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    rc = lib(omp).ora_run(ctypes.byref(s), n, _p(coef), _p(cm), _p(ids), _p(state), int(t0), int(T),
                       mode, _p(i_const), mu, sigma, int(seed), lam, _p(i_dense), _p(spk), _p(vr),
                       _p(lv))
    if rc != 0:
        raise ValueError("oracle rejected the model (rc=%d)" % rc)
    return {"spikes": spk, "v": vr, "level": lv}


def cable_run(model: dict, state: np.ndarray, T: int, morph: dict, t0: int = 0, *, i_const=None,
              noise_mu=None, noise_sigma=None, seed: int = 0, i_dense=None, coef=None, cm=None,
              ids=None, record_v: bool = False, record_spikes: bool = True, background=None):
    """Advance multi-compartment neurons T steps in place (state [n_state][n],
    n = N*K).  morph = {"K": K, "parent": [K], "g_axial": [K],
    "area": [K] or None, "gbar": [K][n_channels] or None}.  Returns dict with
    'spikes' [T][n] and 'v' [T][n] (optional), as run()."""
    s = model_to_struct(model)
    n = state.shape[1]
    assert state.dtype == np.float64 and state.flags.c_contiguous
    K = int(morph["K"])
    parent = np.ascontiguousarray(morph["parent"], dtype=np.int32)
    g_ax = _f64(np.zeros(K) if morph.get("g_axial") is None else morph["g_axial"])
    area = _f64(morph.get("area"))
    gbar = _f64(morph.get("gbar"))
    mode, i_const, i_dense, mu, sigma, lam = _input_mode(T, n, i_const, noise_mu, noise_sigma,
                                                        i_dense, background)
    coef, cm = _f64(coef), _f64(cm)
    ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    spk = np.zeros((T, n), np.uint8) if record_spikes else None
    vr = np.zeros((T, n), np.float64) if record_v else None
    rc = lib().ora_cable_run(ctypes.byref(s), n, K, _p(parent), _p(g_ax), _p(area), _p(gbar),
                             _p(coef), _p(cm), _p(ids), _p(state), int(t0), int(T), mode, _p(i_const),
                             mu, sigma, int(seed), lam, _p(i_dense), _p(spk), _p(vr))
    if rc != 0:
        raise ValueError("oracle rejected the model or morphology (rc=%d)" % rc)
    return {"spikes": spk, "v": vr}


def net_run(model: dict, state: np.ndarray, csr, w_scale: float, T: int, t0: int = 0, *,
            ext_mask=None, ext_thresh: int = 0, w_ext: float = 0.0, seed: int = 0, i_const=None,
            delay=None, max_delay: int = 1, background=None, in_seed: int = 0, omp: bool = False):
    """Recurrent network, T steps in place; returns spikes [T][n] uint8.
    delay: per-synapse delays in steps [nnz] (None: 1); background =
    (lam, mu, sigma) drawn with in_seed.  omp: the OpenMP build (the neuron
    updates of a step on several threads; same results)."""
    s = model_to_struct(model)
    n = state.shape[1]
    row_ptr = np.ascontiguousarray(csr[0], dtype=np.int64)
    col = np.ascontiguousarray(csr[1], dtype=np.int32)
    w = _f64(csr[2])
    dl = None if delay is None else np.ascontiguousarray(delay, dtype=np.uint8)
    em = None if ext_mask is None else np.ascontiguousarray(ext_mask, dtype=np.uint8)
    ic = _f64(i_const)
    mode, mu, sigma, lam = IN_NONE, 0.0, 0.0, 0.0
    if background is not None:
        mode = IN_BACKGROUND
        lam, mu, sigma = (float(x) for x in background)
    elif ic is not None:
        mode = IN_CONST
    spk = np.zeros((T, n), np.uint8)
    rc = lib(omp).ora_net_run(ctypes.byref(s), n, _p(state), _p(row_ptr), _p(col), _p(w),
                           float(w_scale), _p(dl), int(max_delay), _p(em), int(ext_thresh),
                           float(w_ext), int(seed), mode, _p(ic), mu, sigma, int(in_seed), lam,
                           int(t0), int(T), _p(spk))
    if rc != 0:
        raise ValueError("oracle rejected the network (rc=%d)" % rc)
    return spk


def syn_deliver(csr, w_scale: float, spikes, ge, gi):
    n = len(csr[0]) - 1
    row_ptr = np.ascontiguousarray(csr[0], dtype=np.int64)
    col = np.ascontiguousarray(csr[1], dtype=np.int32)
    w = _f64(csr[2])
    s = np.ascontiguousarray(spikes, dtype=np.uint8)
    assert ge.dtype == np.float64 and gi.dtype == np.float64
    lib().ora_syn_deliver(n, _p(row_ptr), _p(col), _p(w), float(w_scale), _p(s), _p(ge), _p(gi))


def bptt(model: dict, state0: np.ndarray, I: np.ndarray, *, cm=None, dL_dr=None, dL_dV=None,
         smooth: bool = False, beta: float = 0.2):
    """Forward + reverse sweep.  Returns (r, dI, dCm, dx0)."""
    s = model_to_struct(model)
    ns, n = state0.shape
    T = I.shape[0]
    st = _f64(state0)
    I = _f64(I)
    cm, dL_dr, dL_dV = _f64(cm), _f64(dL_dr), _f64(dL_dV)
    r = np.zeros(n)
    dI = np.zeros((T, n))
    dC = np.zeros(n)
    dx0 = np.zeros((ns, n))
    rc = lib().ora_bptt(ctypes.byref(s), n, _p(cm), _p(st), int(T), _p(I), _p(dL_dr), _p(dL_dV),
                        1 if smooth else 0, float(beta), _p(r), _p(dI), _p(dC), _p(dx0))
    if rc != 0:
        raise ValueError("oracle rejected the model (rc=%d)" % rc)
    return r, dI, dC, dx0


# --------------------------------------------------------------------------
# spike bookkeeping
# --------------------------------------------------------------------------
def spike_times(spk: np.ndarray):
    """List of step-index arrays, one per neuron, from a [T][n] 0/1 raster."""
    return [np.nonzero(spk[:, i])[0] for i in range(spk.shape[1])]


def unpack_bits(bits: np.ndarray, n: int) -> np.ndarray:
    """[T][words] uint32 little-endian bit rows -> [T][n] uint8 raster."""
    b = np.ascontiguousarray(bits).view(np.uint8)
    out = np.unpackbits(b.reshape(bits.shape[0], -1), axis=1, bitorder="little")
    return out[:, :n]


# --------------------------------------------------------------------------
# dense pieces of the differentiable layer (plain definitions, FP64)
# --------------------------------------------------------------------------
def projection(S: np.ndarray, W: np.ndarray) -> np.ndarray:
    """I = S W: input projection of the linear layer in front of the HH
    neurons (the Sequential(Linear, HHNode) composition of Fig. 1e)."""
    return np.asarray(S, np.float64) @ np.asarray(W, np.float64)


def projection_weight_grad(S: np.ndarray, dI: np.ndarray) -> np.ndarray:
    """dW = S^T dI."""
    return np.asarray(S, np.float64).T @ np.asarray(dI, np.float64)


def readout_ce(r: np.ndarray, W: np.ndarray, b: np.ndarray, labels: np.ndarray):
    """logits = r W + b; mean cross entropy; gradients wrt r, W, b."""
    r = np.asarray(r, np.float64)
    z = r @ np.asarray(W, np.float64) + np.asarray(b, np.float64)
    zmax = z.max(axis=1, keepdims=True)
    ez = np.exp(z - zmax)
    prob = ez / ez.sum(axis=1, keepdims=True)
    B = r.shape[0]
    loss = float(np.mean(-np.log(prob[np.arange(B), labels])))
    dz = prob.copy()
    dz[np.arange(B), labels] -= 1.0
    dz /= B
    return loss, dz @ np.asarray(W, np.float64).T, r.T @ dz, dz.sum(axis=0), z


# --------------------------------------------------------------------------
# MLP surrogate: x -> act(x W1 + b1) -> act(. W2 + b2) -> . W3 + b3, with
# act SiLU or hard-swish
# --------------------------------------------------------------------------
def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def hardswish(x):
    """x relu6(x + 3) / 6 (Howard et al., 2019, "Searching for MobileNetV3")."""
    return x * np.clip(x + 3.0, 0.0, 6.0) / 6.0


def dhardswish(x):
    """Derivative of hardswish: 0 below -3, 1 above 3, x / 3 + 1/2 between
    (the kinks take the outer side's value)."""
    return np.where(x <= -3.0, 0.0, np.where(x >= 3.0, 1.0, x / 3.0 + 0.5))


ACTIVATIONS = {"silu": (silu, dsilu), "hardswish": (hardswish, dhardswish)}


def bf16_round(x):
    """x rounded to the nearest bfloat16 value (8 significant bits, ties to
    even), from the exact binary64 value."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


def mlp_forward(params, x, act="silu", quantize=False):
    """params = [W1, b1, W2, b2, W3, b3] with Wk [in, out].  quantize: the
    network as the bf16 inference evaluates it -- W1, b1, W2 and W3 rounded
    to bf16, the input split into a bf16 high part and a bf16 low part of
    the remainder, and both hidden activations rounded to bf16; b2, b3 and
    all sums exact."""
    f, _ = ACTIVATIONS[act]
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    x = np.asarray(x, np.float64)
    q = bf16_round if quantize else (lambda v: v)
    if quantize:
        W1, b1, W2, W3 = q(W1), q(b1), q(W2), q(W3)
        hi = q(x)
        x = hi + q(x - hi)
    a1 = x @ W1 + b1
    h1 = q(f(a1))
    a2 = h1 @ W2 + b2
    h2 = q(f(a2))
    y = h2 @ W3 + b3
    return y, (x, a1, h1, a2, h2, act)


def mlp_backward(params, cache, dy):
    """Gradients of sum(dy * y) wrt every parameter, and wrt x."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    x, a1, h1, a2, h2, act = cache
    _, df = ACTIVATIONS[act]
    dy = np.asarray(dy, np.float64)
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dh2 = dy @ W3.T
    da2 = dh2 * df(a2)
    gW2 = h1.T @ da2
    gb2 = da2.sum(0)
    dh1 = da2 @ W2.T
    da1 = dh1 * df(a1)
    gW1 = x.T @ da1
    gb1 = da1.sum(0)
    dx = da1 @ W1.T
    return [gW1, gb1, gW2, gb2, gW3, gb3], dx


def mlp_split(flat):
    """The packed parameter vector (W1 [7][64], b1, W2 [64][64], b2, W3
    [64][6], b3) as the list mlp_forward takes."""
    flat = np.asarray(flat, np.float64)
    out, off = [], 0
    for a, b in ((7, 64), (64, 64), (64, 6)):
        out.append(flat[off: off + a * b].reshape(a, b))
        off += a * b
        out.append(flat[off: off + b])
        off += b
    return out


def mlp_apply(params, norm, x, act="silu", quantize=False):
    """The surrogate's state change for raw inputs x [S][7]: the network on
    (x - mean) / std, its output de-normalized (y std + mean); norm is the
    32-entry normalization (input mean [0:7], std [8:15], output mean
    [16:22], std [24:30])."""
    norm = np.asarray(norm, np.float64)
    xn = (np.asarray(x, np.float64) - norm[0:7]) / norm[8:15]
    y, _ = mlp_forward(params, xn, act=act, quantize=quantize)
    return y * norm[24:30] + norm[16:22]


def surrogate_run(model, state, T, k, params, norm, i_dense, *, act="silu", v_fb=-50.0,
                  check_every=10, check_tol=0.5, quantize=True):
    """The surrogate deployment policy in binary64, step for step as stated:
    for each call of k steps, a neuron is admissible when V <= v_fb; the
    network's prediction x + mlp_apply(x) (gates clamped to [0, 1]) is a
    candidate when the neuron is admissible and the predicted V <= v_fb; the
    neuron takes the prediction when it is a candidate, has not failed the
    last check and the call is not a check call (every check_every-th call);
    otherwise it runs the k plain steps of run().  On a check call a
    candidate whose plain V differs from the predicted V by more than
    check_tol fails the check and stays plain until the next check call.
    Spikes come from plain steps only.  state: [1 + G][n] (V, gates), in
    place.  Returns dict with 'spikes' [T][n], 'stats' (surrogate calls,
    plain calls, failed checks) and 'margin' [n], the smallest distance of
    any decision quantity from its threshold (|V - v_fb| before and after,
    ||V_plain - V_pred| - check_tol|) over the run."""
    G = len(model["gates"])
    assert state.shape[0] == 1 + G and G + 1 == 6 and T % k == 0
    n = state.shape[1]
    I = np.asarray(i_dense, np.float64)
    forced = np.zeros(n, bool)
    spikes = np.zeros((T, n), np.uint8)
    stats = np.zeros(3, np.int64)
    margin = np.full(n, np.inf)
    for c in range(T // k):
        t = c * k
        check = check_every > 0 and (c + 1) % check_every == 0
        V = state[0].copy()
        sub = V <= v_fb
        x = np.concatenate([state.T, I[t:t + k].mean(0)[:, None]], axis=1)
        pred = x[:, :6] + mlp_apply(params, norm, x, act=act, quantize=quantize)
        pred[:, 1:] = np.clip(pred[:, 1:], 0.0, 1.0)
        cand = sub & (pred[:, 0] <= v_fb)
        margin = np.minimum(margin, np.abs(V - v_fb))
        margin[sub] = np.minimum(margin[sub], np.abs(pred[sub, 0] - v_fb))
        use = cand & ~forced & (not check)
        plain = ~use
        if plain.any():
            cols = np.nonzero(plain)[0]
            s = np.ascontiguousarray(state[:, cols])
            r = run(model, s, k, t0=t, i_dense=np.ascontiguousarray(I[t:t + k][:, cols]))
            spikes[t:t + k, cols] = r["spikes"]
            state[:, cols] = s
            if check:
                cc = cols[cand[cols]]
                d = np.abs(state[0, cc] - pred[cc, 0])
                margin[cc] = np.minimum(margin[cc], np.abs(d - check_tol))
                fail = d > check_tol
                forced[cc] = fail
                stats[2] += int(fail.sum())
        state[:, use] = pred[use].T
        stats[0] += int(use.sum())
        stats[1] += int(plain.sum())
    return {"spikes": spikes, "stats": stats, "margin": margin}


def mse_loss_grad(y, target):
    """L = mean over samples of sum over outputs of (y - target)^2; dL/dy."""
    d = np.asarray(y, np.float64) - np.asarray(target, np.float64)
    B = d.shape[0]
    return float(np.sum(d * d) / B), 2.0 * d / B


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, 2015, Algorithm 1), one update; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
