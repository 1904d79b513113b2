"""Python binding of libhh (ctypes).  Argument marshalling only: every step of
the method runs in the HIP kernels behind the C ABI declared in include/hh.h.

Torch tensors serve as device memory; the current torch stream is passed to
every call.  If libhh.so is missing or fails to load, importing this module
raises -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhh.so")

MAX_GATES, MAX_CH, MAX_CH_GATES = 8, 8, 4
FORMS = {"exp": 0, "sigmoid": 1, "linoid": 2, "bell": 3}
KINDS = {"ab": 0, "inftau": 1}
VMETH = {"fe": 0, "ee": 1}
IN_NONE, IN_CONST, IN_NOISE, IN_DENSE, IN_BACKGROUND, IN_SINE = 0, 1, 2, 3, 4, 5
STATUS = {0: "HH_OK", -1: "HH_E_INVALID", -2: "HH_E_SHAPE", -3: "HH_E_HIP",
          -4: "HH_E_NONFINITE", -5: "HH_E_UNSUPPORTED", -6: "HH_E_OOM", -7: "HH_E_TIMEOUT"}


class HHError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(status, "?"), status))
        self.status = status


class Rate(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("A", ctypes.c_float), ("B", ctypes.c_float),
                ("K", ctypes.c_float), ("c", ctypes.c_float)]


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("r", Rate * 2)]


class Channel(ctypes.Structure):
    _fields_ = [("gbar", ctypes.c_float), ("E", ctypes.c_float), ("n_gates", ctypes.c_int32),
                ("gate", ctypes.c_int32 * MAX_CH_GATES), ("expo", ctypes.c_int32 * MAX_CH_GATES)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_gates", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("gates", Gate * MAX_GATES), ("channels", Channel * MAX_CH),
                ("C_m", ctypes.c_float), ("dt", ctypes.c_float), ("v_th", ctypes.c_float),
                ("v_method", ctypes.c_int32), ("has_syn", ctypes.c_int32),
                ("tau_e", ctypes.c_float), ("tau_i", ctypes.c_float),
                ("E_e", ctypes.c_float), ("E_i", ctypes.c_float)]


class Input(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("i_const", ctypes.c_void_p), ("mu", ctypes.c_float),
                ("sigma", ctypes.c_float), ("seed", ctypes.c_uint64), ("i_dense", ctypes.c_void_p),
                ("lam", ctypes.c_float), ("freq", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    _fields_ = [("spikes", ctypes.c_void_p), ("v_rec", ctypes.c_void_p), ("ckpt", ctypes.c_void_p),
                ("ckpt_every", ctypes.c_int32), ("level", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhh.so is not built (%s); run python -m paper_2601_21407_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    i32, i64, u32, u64, f32, sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_float, ctypes.c_size_t)
    sig = {
        "hh_init": ([P(vp), P(ModelDesc), i64, i32, vp, vp], i32),
        "hh_destroy": ([vp], i32),
        "hh_status_string": ([i32], ctypes.c_char_p),
        "hh_n_state": ([vp], i32),
        "hh_set_fusion": ([vp, i32], i32),
        "hh_set_specialize": ([vp, i32], i32),
        "hh_set_rate_table": ([vp, f32, f32, i32, vp], i32),
        "hh_set_morphology": ([vp, i32, vp, vp, vp, vp, vp], i32),
        "hh_init_state": ([vp, vp, vp, f32, vp], i32),
        "hh_step_n": ([vp, vp, i64, i32, P(Input), P(Outputs), vp], i32),
        "hh_attach_csr": ([vp, vp, vp, vp, i64, f32], i32),
        "hh_set_external": ([vp, vp, u32, f32, u64], i32),
        "hh_set_delays": ([vp, vp, i32], i32),
        "hh_set_delivery": ([vp, i32], i32),
        "hh_syn_propagate": ([vp, vp, vp, vp, vp], i32),
        "hh_backward": ([vp, vp, i32, P(Input), i32, vp, vp, f32, vp, vp, vp, vp, sz, vp], i32),
        "hh_backward_part": ([vp, vp, i32, P(Input), i32, i32, i32, vp, vp, f32, vp, vp, vp, vp, sz,
                              vp], i32),
        "hh_backward_workspace": ([vp, i32, i32], sz),
        "hh_check": ([vp, P(i64), vp], i32),
        "hh_proj_forward": ([vp, vp, vp, i32, i32, i32, vp], i32),
        "hh_proj_forward_bits": ([vp, i32, vp, vp, i32, i32, i32, vp], i32),
        "hh_proj_wgrad": ([vp, vp, vp, i32, i32, i32, i32, vp, sz, vp], i32),
        "hh_proj_wgrad_workspace": ([i32, i32, i32], sz),
        "hh_proj_wgrad_bits": ([vp, i32, vp, vp, i32, i32, i32, i32, vp, sz, vp], i32),
        "hh_readout_ce": ([vp, i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "hh_readout_ce_workspace": ([i32, i32], sz),
        "hh_readout_ce_noalloc": ([vp, i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp], i32),
        "hh_level_rate": ([vp, i64, i32, vp, vp], i32),
        "hh_adam_step": ([vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp, vp], i32),
        "hh_mlp_grad": ([vp, vp, vp, vp, i32, i32, i32, vp, vp, vp, sz, vp], i32),
        "hh_mlp_grad_workspace": ([i32], sz),
        "hh_mlp_forward": ([vp, vp, vp, i32, i32, i32, vp, vp], i32),
        "hh_mlp_norm": ([vp, vp, i64, vp, vp, sz, vp], i32),
        "hh_mlp_norm_workspace": ([], sz),
        "hh_surrogate_transitions": ([vp, i32, vp, i64, i32, i32, f32, vp, vp, i64, vp, vp, sz, vp],
                                     i32),
        "hh_surrogate_transitions_workspace": ([i32, i32], sz),
        "hh_mlp_pack": ([vp, vp, vp, vp], i32),
        "hh_mlp_packed_bytes": ([], sz),
        "hh_mlp_infer": ([vp, i32, vp, i32, vp, vp], i32),
        "hh_surrogate_step_n": ([vp, vp, i32, vp, vp, i64, i32, i32, P(Input), f32, i32, f32, vp, vp,
                                 vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def exported_symbols():
    """Names of the C-ABI entry points this binding uses."""
    return [n for n in ("hh_init", "hh_destroy", "hh_status_string", "hh_n_state", "hh_set_fusion",
                        "hh_set_specialize", "hh_set_rate_table", "hh_set_morphology",
                        "hh_init_state", "hh_step_n", "hh_attach_csr", "hh_set_external",
                        "hh_set_delays", "hh_set_delivery",
                        "hh_syn_propagate", "hh_backward", "hh_backward_part",
                        "hh_backward_workspace", "hh_check",
                        "hh_proj_forward", "hh_proj_forward_bits", "hh_proj_wgrad",
                        "hh_proj_wgrad_workspace", "hh_proj_wgrad_bits",
                        "hh_readout_ce", "hh_readout_ce_workspace", "hh_readout_ce_noalloc",
                        "hh_adam_step",
                        "hh_level_rate",
                        "hh_mlp_grad", "hh_mlp_grad_workspace", "hh_mlp_forward", "hh_mlp_pack",
                        "hh_mlp_norm", "hh_mlp_norm_workspace", "hh_surrogate_transitions",
                        "hh_surrogate_transitions_workspace",
                        "hh_mlp_packed_bytes", "hh_mlp_infer", "hh_surrogate_step_n")]


def _ok(status: int, what: str):
    if status != 0:
        raise HHError(status, what)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def desc_from_model(model: dict) -> ModelDesc:
    """Translate a model dictionary (see workloads) into hh_model_desc."""
    d = ModelDesc()
    gates, chans = model["gates"], model["channels"]
    if len(gates) > MAX_GATES or len(chans) > MAX_CH:
        raise ValueError("too many gates or channels")
    d.n_gates, d.n_channels = len(gates), len(chans)
    for g, gate in enumerate(gates):
        d.gates[g].kind = KINDS[gate["kind"]]
        for r, rt in enumerate(gate["rates"]):
            d.gates[g].r[r].form = FORMS[rt[0]]
            d.gates[g].r[r].A, d.gates[g].r[r].B, d.gates[g].r[r].K, d.gates[g].r[r].c = rt[1:5]
    for c, ch in enumerate(chans):
        d.channels[c].gbar, d.channels[c].E = ch["gbar"], ch["E"]
        d.channels[c].n_gates = len(ch["gates"])
        for k, (gi, ex) in enumerate(ch["gates"]):
            d.channels[c].gate[k], d.channels[c].expo[k] = gi, ex
    d.C_m, d.dt, d.v_th = model["C"], model["dt"], model["v_th"]
    d.v_method = VMETH[model["v_method"]]
    syn = model.get("syn")
    d.has_syn = 1 if syn else 0
    if syn:
        d.tau_e, d.tau_i, d.E_e, d.E_i = syn["tau_e"], syn["tau_i"], syn["E_e"], syn["E_i"]
    return d


def _need(t, what, dtype, min_numel, exact=False):
    """A device tensor argument of the given dtype with at least (or, with
    exact, exactly) min_numel elements: the library writes or reads that many
    and cannot check the size behind a raw pointer itself."""
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError("%s: expected a device tensor" % what)
    if t.dtype not in dtype:
        raise ValueError("%s: expected dtype %s, got %s" % (what, dtype, t.dtype))
    if (t.numel() != min_numel) if exact else (t.numel() < min_numel):
        raise ValueError("%s: expected %s%d elements, got %d"
                         % (what, "" if exact else "at least ", min_numel, t.numel()))


def _need_bytes(t, what, nbytes):
    """A device tensor argument of at least nbytes bytes (the library reads it
    as raw bytes, whatever its dtype)."""
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError("%s: expected a device tensor" % what)
    if t.numel() * t.element_size() < nbytes:
        raise ValueError("%s: expected at least %d bytes, got %d"
                         % (what, nbytes, t.numel() * t.element_size()))


_F32 = (torch.float32,)
_I32 = (torch.int32,)

# models still alive at interpreter exit are destroyed by an exit hook that
# runs before torch's and the HIP runtime's own teardown (a profiler attached
# to the process has finalized by the time late finalizers would run)
_LIVE = weakref.WeakSet()


@atexit.register
def _destroy_live_models():
    try:
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for m in list(_LIVE):
        m.close()


class Model:
    """A population of n = N * B HH neurons on the current device."""

    def __init__(self, model: dict, N: int, B: int = 1, coef=None, cm=None, desc=None):
        self.model = model
        self.N, self.B, self.n = int(N), int(B), int(N) * int(B)
        self._keep = [coef, cm]  # the library reads these for the model's lifetime
        self.desc = desc if desc is not None else desc_from_model(model)
        G = len(model["gates"]) if desc is None else int(self.desc.n_gates)
        _need(coef, "coef", _F32, G * 8 * self.N, exact=True)
        _need(cm, "cm", _F32, self.N, exact=True)
        h = ctypes.c_void_p()
        _ok(lib.hh_init(ctypes.byref(h), ctypes.byref(self.desc), self.N, self.B, _ptr(coef),
                        _ptr(cm)), "hh_init")
        self.h = h
        self.n_state = lib.hh_n_state(self.h)
        _LIVE.add(self)

    def close(self, _destroy=lib.hh_destroy):
        """Free the library's model now (also done when the object goes)."""
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    # the library is bound as a default argument: at interpreter exit the
    # module's globals may already be cleared when the last models go
    def __del__(self, _destroy=lib.hh_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    @property
    def words(self) -> int:
        return (self.n + 31) // 32

    def set_fusion(self, k: int):
        _ok(lib.hh_set_fusion(self.h, int(k)), "hh_set_fusion")

    def set_specialize(self, on: bool):
        _ok(lib.hh_set_specialize(self.h, 1 if on else 0), "hh_set_specialize")

    def set_rate_table(self, v_lo: float, v_hi: float, n_nodes: int):
        """Tabulated gate kinetics on [v_lo, v_hi] mV with n_nodes nodes; 0 removes it."""
        _ok(lib.hh_set_rate_table(self.h, float(v_lo), float(v_hi), int(n_nodes), _stream()),
            "hh_set_rate_table")

    def set_morphology(self, K: int, parent=None, g_axial=None, area=None, gbar=None):
        """K compartments per neuron (host arrays of K entries; gbar [K][n_channels]);
        K = 0 removes the morphology."""
        def host(a, dt):
            return None if a is None else np.ascontiguousarray(a, dtype=dt)
        par = host(parent, np.int32)
        gax, ar, gb = host(g_axial, np.float32), host(area, np.float32), host(gbar, np.float32)
        ptr = [None if a is None else a.ctypes.data_as(ctypes.c_void_p) for a in (par, gax, ar, gb)]
        _ok(lib.hh_set_morphology(self.h, int(K), *ptr, _stream()), "hh_set_morphology")

    def new_state(self, device="cuda"):
        return torch.empty((self.n_state, self.n), dtype=torch.float32, device=device)

    def init_state(self, state, v0=None, v0_scalar: float = -65.0):
        _need(state, "state", _F32, self.n_state * self.n, exact=True)
        _need(v0, "v0", _F32, self.n, exact=True)
        _ok(lib.hh_init_state(self.h, _ptr(state), _ptr(v0), float(v0_scalar), _stream()),
            "hh_init_state")
        return state

    def step_n(self, state, n_steps: int, t0: int = 0, *, i_const=None, noise=None, i_dense=None,
               spikes=None, v_rec=None, ckpt=None, ckpt_every: int = 1, level=None,
               background=None, sine=None):
        """noise = (mu, sigma, seed); background = (lam, mu, sigma, seed);
        sine = (amplitudes [n], frequencies [n] in Hz), device tensors."""
        n, T = self.n, max(int(n_steps), 0)
        _need(state, "state", _F32, self.n_state * n, exact=True)
        _need(spikes, "spikes", _I32, T * self.words)
        _need(v_rec, "v_rec", _F32, T * n)
        _need(i_dense, "i_dense", _F32, T * n)
        _need(i_const, "i_const", _F32, n)
        _need(level, "level", _F32, n)
        if ckpt is not None:
            _need(ckpt, "ckpt", _F32, -(-T // max(int(ckpt_every), 1)) * self.n_state * n)
        if sine is not None:
            _need(sine[0], "sine amplitudes", _F32, n)
            _need(sine[1], "sine frequencies", _F32, n)
        inp = Input()
        if i_dense is not None:
            inp.mode, inp.i_dense = IN_DENSE, _ptr(i_dense)
        elif sine is not None:
            inp.mode, inp.i_const, inp.freq = IN_SINE, _ptr(sine[0]), _ptr(sine[1])
        elif background is not None:
            inp.mode = IN_BACKGROUND
            inp.lam, inp.mu, inp.sigma = (float(x) for x in background[:3])
            inp.seed = int(background[3])
        elif noise is not None:
            inp.mode = IN_NOISE
            inp.mu, inp.sigma, inp.seed = float(noise[0]), float(noise[1]), int(noise[2])
        elif i_const is not None:
            inp.mode, inp.i_const = IN_CONST, _ptr(i_const)
        else:
            inp.mode = IN_NONE
        out = Outputs(_ptr(spikes), _ptr(v_rec), _ptr(ckpt), int(ckpt_every), _ptr(level))
        _ok(lib.hh_step_n(self.h, _ptr(state), int(t0), int(n_steps), ctypes.byref(inp),
                          ctypes.byref(out), _stream()), "hh_step_n")

    def attach_csr(self, row_ptr, col, w, w_scale: float):
        """CSR over the N neurons of one copy (shared by the B copies)."""
        _need(row_ptr, "row_ptr", (torch.int64,), self.N + 1, exact=True)
        _need(col, "col", _I32, col.numel())
        _need(w, "w", _F32, col.numel(), exact=True)
        self._keep += [row_ptr, col, w]
        self._nnz = col.numel()
        _ok(lib.hh_attach_csr(self.h, _ptr(row_ptr), _ptr(col), _ptr(w), int(col.numel()),
                              float(w_scale)), "hh_attach_csr")

    def set_external(self, ext_mask, thresh: int, w_ext: float, seed: int):
        """ext_mask: uint8 [N], shared by the copies."""
        _need(ext_mask, "ext_mask", (torch.uint8,), self.N, exact=True)
        self._keep.append(ext_mask)
        _ok(lib.hh_set_external(self.h, _ptr(ext_mask), int(thresh), float(w_ext), int(seed)),
            "hh_set_external")

    def set_delays(self, delay, max_delay: int):
        """Per-synapse delays in steps (device uint8 [nnz]); None: one step."""
        _need(delay, "delay", (torch.uint8,), getattr(self, "_nnz", 0))
        if delay is not None:
            self._keep.append(delay)
        _ok(lib.hh_set_delays(self.h, _ptr(delay), int(max_delay)), "hh_set_delays")

    def set_delivery(self, mode: str):
        """Network time-loop delivery: "auto" (by target range where the
        library can) or "push" (device atomics)."""
        code = {"auto": 0, "push": 1}[mode]
        _ok(lib.hh_set_delivery(self.h, code), "hh_set_delivery")

    def syn_propagate(self, spike_bits, state, n_spikes=None):
        """One delivery of the sources set in spike_bits (one bit per element,
        int32 or uint32 words) into the conductances of state; n_spikes, if
        given, receives the number of spiking sources."""
        _need(spike_bits, "spike_bits", (torch.int32, torch.uint32), self.words)
        _need(state, "state", _F32, self.n_state * self.n, exact=True)
        _need(n_spikes, "n_spikes", _I32, 1)
        _ok(lib.hh_syn_propagate(self.h, _ptr(spike_bits), _ptr(state), _ptr(n_spikes), _stream()),
            "hh_syn_propagate")

    def _check_backward(self, ckpt, ckpt_every, i_dense, T, dI, dL_dlevel, dL_dV, dCm, dx0):
        n, T = self.n, max(int(T), 0)
        _need(ckpt, "ckpt", _F32, -(-T // max(int(ckpt_every), 1)) * self.n_state * n)
        _need(i_dense, "i_dense", _F32, T * n)
        _need(dI, "dI", _F32, T * n)
        _need(dL_dlevel, "dL_dlevel", _F32, n)
        _need(dL_dV, "dL_dV", _F32, T * n)
        _need(dCm, "dCm", _F32, self.N)
        _need(dx0, "dx0", _F32, self.n_state * n)

    def backward_workspace(self, ckpt_every: int, T: int) -> int:
        return int(lib.hh_backward_workspace(self.h, int(ckpt_every), int(T)))

    def backward(self, ckpt, ckpt_every: int, i_dense, T: int, dI, *, dL_dlevel=None, dL_dV=None,
                 beta: float = 0.2, dCm=None, dx0=None, workspace=None):
        self._check_backward(ckpt, ckpt_every, i_dense, T, dI, dL_dlevel, dL_dV, dCm, dx0)
        inp = Input()
        inp.mode, inp.i_dense = IN_DENSE, _ptr(i_dense)
        ws_bytes = self.backward_workspace(ckpt_every, T)
        if workspace is None and ws_bytes:
            workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dI.device)
        _ok(lib.hh_backward(self.h, _ptr(ckpt), int(ckpt_every), ctypes.byref(inp), int(T),
                            _ptr(dL_dlevel), _ptr(dL_dV), float(beta), _ptr(dI), _ptr(dCm),
                            _ptr(dx0), _ptr(workspace), ws_bytes, _stream()), "hh_backward")

    def backward_part(self, ckpt, ckpt_every: int, i_dense, T: int, t_lo: int, t_hi: int, dI, *,
                      workspace, dL_dlevel=None, dL_dV=None, beta: float = 0.2, dCm=None,
                      dx0=None):
        """The adjoint over steps [t_lo, t_hi) (see hh_backward_part); calls go
        backwards over adjacent ranges and share `workspace`."""
        self._check_backward(ckpt, ckpt_every, i_dense, T, dI, dL_dlevel, dL_dV, dCm, dx0)
        inp = Input()
        inp.mode, inp.i_dense = IN_DENSE, _ptr(i_dense)
        ws_bytes = self.backward_workspace(ckpt_every, T)
        assert workspace.numel() * workspace.element_size() >= ws_bytes
        _ok(lib.hh_backward_part(self.h, _ptr(ckpt), int(ckpt_every), ctypes.byref(inp), int(T),
                                 int(t_lo), int(t_hi), _ptr(dL_dlevel), _ptr(dL_dV), float(beta),
                                 _ptr(dI), _ptr(dCm), _ptr(dx0), _ptr(workspace), ws_bytes,
                                 _stream()), "hh_backward_part")

    def check(self):
        """Synchronizes; returns (status, first_bad_index)."""
        fb = ctypes.c_int64(-1)
        st = lib.hh_check(self.h, ctypes.byref(fb), _stream())
        return st, fb.value


def proj_forward(A_bf16, Wt_bf16, out):
    """out [M][N] = A [M][K] . Wt [N][K]^T (bf16 operands, FP32 result)."""
    M, K = A_bf16.shape
    N = Wt_bf16.shape[0]
    assert A_bf16.dtype == torch.bfloat16 and Wt_bf16.dtype == torch.bfloat16
    assert out.dtype == torch.float32 and tuple(out.shape) == (M, N) and Wt_bf16.shape[1] == K
    assert A_bf16.is_contiguous() and Wt_bf16.is_contiguous() and out.is_contiguous()
    _ok(lib.hh_proj_forward(_ptr(A_bf16), _ptr(Wt_bf16), _ptr(out), M, N, K, _stream()),
        "hh_proj_forward")
    return out


def proj_forward_bits(A_bits, K: int, Wt_bf16, out):
    """out [M][N] = A . Wt^T for a binary A given as bits: A_bits int32
    [M][words], bit k%32 of word k/32 = A[m][k]."""
    M, wpr = A_bits.shape
    N = Wt_bf16.shape[0]
    assert A_bits.dtype == torch.int32 and Wt_bf16.dtype == torch.bfloat16
    assert tuple(out.shape) == (M, N) and out.dtype == torch.float32 and Wt_bf16.shape[1] == K
    assert A_bits.is_contiguous() and Wt_bf16.is_contiguous() and out.is_contiguous()
    _ok(lib.hh_proj_forward_bits(_ptr(A_bits), int(wpr), _ptr(Wt_bf16), _ptr(out), M, N, int(K),
                                 _stream()), "hh_proj_forward_bits")
    return out


def proj_wgrad(A_bf16, dOut, dWt, workspace=None, accumulate=False):
    """dWt [N][K] = dOut [M][N]^T . A [M][K] (added to dWt with accumulate)."""
    M, K = A_bf16.shape
    N = dOut.shape[1]
    assert A_bf16.dtype == torch.bfloat16 and dOut.dtype == torch.float32
    assert tuple(dWt.shape) == (N, K) and dWt.dtype == torch.float32 and dOut.shape[0] == M
    assert A_bf16.is_contiguous() and dOut.is_contiguous() and dWt.is_contiguous()
    need = int(lib.hh_proj_wgrad_workspace(M, N, K))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dWt.device)
    _ok(lib.hh_proj_wgrad(_ptr(A_bf16), _ptr(dOut), _ptr(dWt), 1 if accumulate else 0, M, N, K,
                          _ptr(workspace),
                          workspace.numel() * workspace.element_size(), _stream()), "hh_proj_wgrad")
    return dWt


def proj_wgrad_bits(A_bits, M: int, dOut, dWt, workspace=None, accumulate=False, m0: int = 0):
    """dWt [N][K] = dOut [M][N]^T . A for a binary A given as bits in 32-row
    groups: A_bits int32 [ceil(rows/32)][K], bit b of word (w, k) = A[32 w + b][k]
    (see workloads.pack_bits_cols).  With m0 (a multiple of 32) the product
    covers rows m0 .. m0 + M - 1 of A, and dOut holds just those rows;
    accumulate adds to dWt."""
    W_, K = A_bits.shape
    N = dOut.shape[1]
    assert A_bits.dtype == torch.int32 and dOut.dtype == torch.float32
    assert tuple(dWt.shape) == (N, K) and dWt.dtype == torch.float32 and dOut.shape[0] == M
    assert A_bits.is_contiguous() and dOut.is_contiguous() and dWt.is_contiguous()
    assert m0 % 32 == 0 and (m0 + M + 31) // 32 <= W_
    need = int(lib.hh_proj_wgrad_workspace(M, N, K))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dWt.device)
    base = ctypes.c_void_p(A_bits.data_ptr() + (m0 // 32) * K * 4) if A_bits.numel() else None
    _ok(lib.hh_proj_wgrad_bits(base, int(K), _ptr(dOut), _ptr(dWt), 1 if accumulate else 0,
                               int(M), N, K, _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream()),
        "hh_proj_wgrad_bits")
    return dWt


def readout_ce(level, T: int, W, bias, labels, dlevel, dW, db, loss, logits=None, workspace=None):
    """Readout + cross entropy, forward and backward (see hh.h)."""
    B, H = level.shape
    C = W.shape[1]
    assert labels.dtype == torch.int32 and labels.numel() == B
    _need(level, "level", _F32, B * H, exact=True)
    _need(W, "W", _F32, H * C, exact=True)
    _need(bias, "bias", _F32, C, exact=True)
    _need(dlevel, "dlevel", _F32, B * H, exact=True)
    _need(dW, "dW", _F32, H * C, exact=True)
    _need(db, "db", _F32, C, exact=True)
    _need(loss, "loss", _F32, 1)
    _need(logits, "logits", _F32, B * C, exact=True)
    need = int(lib.hh_readout_ce_workspace(B, C))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=level.device)
    _ok(lib.hh_readout_ce(_ptr(level), int(T), _ptr(W), _ptr(bias), _ptr(labels), B, H, C,
                          _ptr(loss), _ptr(dlevel), _ptr(dW), _ptr(db), _ptr(logits),
                          _ptr(workspace), workspace.numel(), _stream()), "hh_readout_ce")


def level_rate(level, T: int, rate):
    """rate = level / T (the differentiable layer's output)."""
    _need(level, "level", _F32, rate.numel())
    _need(rate, "rate", _F32, level.numel(), exact=True)
    _ok(lib.hh_level_rate(_ptr(level), rate.numel(), int(T), _ptr(rate), _stream()),
        "hh_level_rate")
    return rate


def adam_step(param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
              param_bf16=None):
    n = param.numel()
    _need(param, "param", _F32, n)
    for t, what in ((grad, "grad"), (m, "m"), (v, "v")):
        _need(t, what, _F32, n, exact=True)
    _need(param_bf16, "param_bf16", (torch.bfloat16,), n, exact=True)
    _ok(lib.hh_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), float(lr),
                         float(beta1), float(beta2), float(eps), int(step), _ptr(param_bf16),
                         _stream()), "hh_adam_step")


# ---------------------------------------------------------------------------
# learned surrogate
# ---------------------------------------------------------------------------
MLP_NPARAM = 5062
MLP_IN, MLP_H, MLP_OUT = 7, 64, 6


ACT_SILU, ACT_HARDSWISH = 0, 1
_ACTS = {"silu": ACT_SILU, "hardswish": ACT_HARDSWISH}


def act_code(act) -> int:
    """HH_ACT_* of an activation given by name ('silu', 'hardswish') or code."""
    return _ACTS[act] if isinstance(act, str) else int(act)


def _mlp_data(X, Y=None, norm=None):
    _need(X, "X", _F32, X.shape[0] * MLP_IN, exact=True)
    if Y is not None:
        _need(Y, "Y", _F32, X.shape[0] * MLP_OUT, exact=True)
    if norm is not None:
        _need(norm, "norm", _F32, 32, exact=True)


def mlp_grad(params, norm, X, Y, grad, loss=None, quantize=True, act="silu", workspace=None):
    """MSE loss on the normalized targets and its parameter gradient; X [S][7]
    and Y [S][6] are raw samples (see hh.h)."""
    _mlp_data(X, Y, norm)
    S = X.shape[0]
    need = int(lib.hh_mlp_grad_workspace(S))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    _ok(lib.hh_mlp_grad(_ptr(params), _ptr(norm), _ptr(X), _ptr(Y), S, 1 if quantize else 0,
                        act_code(act), _ptr(grad), _ptr(loss), _ptr(workspace), workspace.numel(),
                        _stream()), "hh_mlp_grad")
    return workspace


def mlp_forward(params, norm, X, Y, quantize=True, act="silu"):
    """VALU forward on raw inputs; Y receives the de-normalized outputs."""
    _mlp_data(X, Y, norm)
    _ok(lib.hh_mlp_forward(_ptr(params), _ptr(norm), _ptr(X), X.shape[0], 1 if quantize else 0,
                           act_code(act), _ptr(Y), _stream()), "hh_mlp_forward")


def mlp_norm(X, Y):
    """Feature normalization [32] of a training set (mean and standard
    deviation per feature, computed in the library)."""
    _mlp_data(X, Y)
    norm = torch.empty(32, dtype=torch.float32, device=X.device)
    ws = torch.empty(int(lib.hh_mlp_norm_workspace()), dtype=torch.uint8, device=X.device)
    _ok(lib.hh_mlp_norm(_ptr(X), _ptr(Y), X.shape[0], _ptr(norm), _ptr(ws), ws.numel(), _stream()),
        "hh_mlp_norm")
    return norm


def surrogate_transitions(traj, i_dense, k: int, v_fb: float, cap: int):
    """Training samples from plain trajectories (see hh.h): traj [T][7][n] the
    state before every step, i_dense [T][n].  Returns (X [S][7], Y [S][6]),
    S = min(qualifying samples, cap)."""
    T, ns, n = traj.shape
    _need(traj, "traj", _F32, T * ns * n, exact=True)
    _need(i_dense, "i_dense", _F32, T * n, exact=True)
    X = torch.empty((cap, MLP_IN), dtype=torch.float32, device=traj.device)
    Y = torch.empty((cap, MLP_OUT), dtype=torch.float32, device=traj.device)
    count = torch.zeros(1, dtype=torch.int64, device=traj.device)
    ws = torch.empty(max(int(lib.hh_surrogate_transitions_workspace(T, k)), 1), dtype=torch.uint8,
                     device=traj.device)
    _ok(lib.hh_surrogate_transitions(_ptr(traj), ns, _ptr(i_dense), n, T, int(k), float(v_fb),
                                     _ptr(X), _ptr(Y), int(cap), _ptr(count), _ptr(ws), ws.numel(),
                                     _stream()), "hh_surrogate_transitions")
    S = min(int(count.item()), cap)
    return X[:S], Y[:S]


def mlp_pack(params, norm):
    _need(params, "params", _F32, MLP_NPARAM, exact=True)
    _need(norm, "norm", _F32, 32, exact=True)
    packed = torch.empty(int(lib.hh_mlp_packed_bytes()), dtype=torch.uint8, device=params.device)
    _ok(lib.hh_mlp_pack(_ptr(params), _ptr(norm), _ptr(packed), _stream()), "hh_mlp_pack")
    return packed


def mlp_infer(packed, X, Y, act="silu"):
    _mlp_data(X, Y)
    _ok(lib.hh_mlp_infer(_ptr(packed), act_code(act), _ptr(X), X.shape[0], _ptr(Y), _stream()),
        "hh_mlp_infer")


def surrogate_step_n(model: Model, packed, state, flags, n_steps: int, k: int, t0: int = 0, *,
                     noise=None, i_dense=None, v_fallback=-50.0, check_every=10, check_tol=0.5,
                     spikes=None, stats=None, act="silu"):
    n, T = model.n, max(int(n_steps), 0)
    _need_bytes(packed, "packed", int(lib.hh_mlp_packed_bytes()))
    _need(state, "state", _F32, model.n_state * n, exact=True)
    _need_bytes(flags, "flags", n)
    _need(i_dense, "i_dense", _F32, T * n)
    _need(spikes, "spikes", _I32, T * model.words)
    _need(stats, "stats", (torch.int64,), 3)
    inp = Input()
    if i_dense is not None:
        inp.mode, inp.i_dense = IN_DENSE, _ptr(i_dense)
    else:
        inp.mode = IN_NOISE
        inp.mu, inp.sigma, inp.seed = float(noise[0]), float(noise[1]), int(noise[2])
    _ok(lib.hh_surrogate_step_n(model.h, _ptr(packed), act_code(act), _ptr(state), _ptr(flags), int(t0),
                                int(n_steps), int(k), ctypes.byref(inp), float(v_fallback),
                                int(check_every), float(check_tol), _ptr(spikes), _ptr(stats),
                                _stream()), "hh_surrogate_step_n")
