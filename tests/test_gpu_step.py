"""GPU parity of the fused multi-step kernel (hh_step_n) against the FP64
oracle, through the C ABI.

Tolerances: non-spiking traces within 1e-3 mV of the oracle over the whole
run; spiking neurons with the same number of spikes and every spike within
one dt.  A neuron whose oracle result itself moves by more than that under a
1e-6 relative change of its input, or when the oracle's state is rounded to
binary32 every step, is ill-conditioned: it is counted and reported, not
failed (tests.gpu_util).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import judge, need_gpu, print_case

pytestmark = pytest.mark.gpu


def _run_gpu(model, n, T, *, B=1, i_const=None, noise=None, i_dense=None, coef=None, cm=None,
             v0=-65.0, record_v=False, fusion=32, t0=0, state=None, specialize=True, table=None):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    N = n // B
    dev = "cuda"
    coef_t = None if coef is None else torch.tensor(coef, device=dev)
    cm_t = None if cm is None else torch.tensor(cm, dtype=torch.float32, device=dev)
    M = hh.Model(model, N, B, coef=coef_t, cm=cm_t)
    M.set_fusion(fusion)
    M.set_specialize(specialize)
    if table is not None:
        M.set_rate_table(*table)
    st = M.new_state() if state is None else state
    if state is None:
        if np.isscalar(v0):
            M.init_state(st, v0_scalar=float(v0))
        else:
            M.init_state(st, v0=torch.tensor(np.asarray(v0, np.float32), device=dev))
    spikes = torch.zeros((T, M.words), dtype=torch.int32, device=dev)
    vrec = torch.zeros((T, n), dtype=torch.float32, device=dev) if record_v else None
    ic = None if i_const is None else torch.tensor(np.asarray(i_const, np.float32), device=dev)
    idn = None if i_dense is None else torch.tensor(np.asarray(i_dense, np.float32), device=dev)
    M.step_n(st, T, t0, i_const=ic, noise=noise, i_dense=idn, spikes=spikes, v_rec=vrec)
    status, bad = M.check()
    assert status == 0, (status, bad)
    bits = spikes.cpu().numpy().view(np.uint32)
    return {"raster": O.unpack_bits(bits, n) if n <= 65536 else None, "bits": bits,
            "v": None if vrec is None else vrec.cpu().numpy(),
            "state": st.cpu().numpy(), "model": M, "state_t": st}


def _columns(bits, ids):
    """[T][len(ids)] raster of selected neurons from packed spike words."""
    ids = np.asarray(ids)
    return ((bits[:, ids // 32] >> (ids % 32).astype(np.uint32)) & 1).astype(np.uint8)


def _judge(model, st0, T, g, ro, base_kw, *, max_ill_frac, v_tol=1e-3, label=""):
    """Parity criteria for point neurons (tests.gpu_util.judge)."""
    return judge(O, model, st0, T, g, ro, base_kw, max_excused_frac=max_ill_frac, v_tol=v_tol,
                 label=label)


_ORACLE_CACHE = {}


def _cached(key, fn):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = fn()
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("specialize", [True, False])
def test_validation_workload_full_size(specialize):
    """1,024 classic HH neurons, I ~ U[0, 20), dt = 0.01 ms, 10,000 steps
    (compiled specialization and run-time interpreter)."""
    print_case("classic HH 1024 x 10000 dt=0.01 specialize=%s" % specialize)
    m = W.classic_hh(dt=0.01)
    n, T = 1024, 10000
    I = W.validation_currents(n, seed=1).astype(np.float64)
    g = _run_gpu(m, n, T, i_const=I, record_v=True, specialize=specialize)
    st0 = O.init_state(m, np.full(n, -65.0))
    ro = _cached("validation", lambda: O.run(m, st0.copy(), T, i_const=I, record_v=True))
    assert (ro["spikes"].sum(0) == 0).sum() > 50 and (ro["spikes"].sum(0) > 0).sum() > 500
    _judge(m, st0, T, g, ro, {"i_const": I}, max_ill_frac=0.02, label="validation")


def test_noise_stream_matches_oracle():
    """I = 0 + 1 z: a gate-free, conductance-free neuron started at V = 0 for
    one step with dt = C = 1 reports exactly the drawn normal."""
    torch = need_gpu()
    m = {"gates": [], "channels": [], "C": 1.0, "dt": 1.0, "v_th": 1e9, "v_method": "fe", "syn": None}
    n = 130
    for t0 in (0, 1, 2, 3, 4, 7, 1001):
        g = _run_gpu(m, n, 1, noise=(0.0, 1.0, 12345), v0=0.0, t0=t0)
        z = np.array([O.noise(12345, i, t0) for i in range(n)])
        assert np.max(np.abs(g["state"][0] - z)) < 2e-5, t0
    del torch


@pytest.mark.parametrize("specialize", [True, False])
def test_custom_channels_sampled_full_size(specialize):
    """1,048,576 neurons with jittered cortical channels and noisy input,
    dt = 0.025 ms, 4,000 steps, 32 fused steps per launch; 4,096 sampled
    neurons checked against the oracle."""
    print_case("custom channels 1048576 x 4000 K=32 (sampled 4096) specialize=%s" % specialize)
    m = W.custom_channels(dt=0.025)
    n, T, seed = 1 << 20, 4000, 2
    coef = W.jitter_coef(m, n, seed=seed)
    g = _run_gpu(m, n, T, noise=(5.0, 3.0, seed), coef=coef, fusion=32, specialize=specialize)
    assert np.isfinite(g["state"]).all()
    rng = np.random.default_rng(99)
    ids = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.choice(n, 4091, replace=False)]))
    c64 = coef[:, ids].astype(np.float64)
    st0 = O.init_state(m, np.full(len(ids), -65.0), coef=c64)
    kw = {"noise_mu": 5.0, "noise_sigma": 3.0, "seed": seed, "coef": c64, "ids": ids}
    ro = _cached("custom", lambda: O.run(m, st0.copy(), T, **kw))
    assert ro["spikes"].sum(0).mean() > 1.0
    gs = {"raster": _columns(g["bits"], ids), "v": None}
    _judge(m, st0, T, gs, ro, kw, max_ill_frac=0.02, label="custom-channels")


@pytest.mark.parametrize("v_method", ["fe", "ee"])
@pytest.mark.parametrize("n,B", [(1, 1), (100, 1), (1000, 2), (4097, 1)])
def test_small_populations(v_method, n, B):
    print_case("small n=%d B=%d %s" % (n, B, v_method))
    m = W.classic_hh(dt=0.02, v_method=v_method)
    T = 2500
    rng = np.random.default_rng(n)
    I = (15.0 * rng.random(n)).astype(np.float32).astype(np.float64)
    v0 = (-70.0 + 10.0 * rng.random(n)).astype(np.float32)
    g = _run_gpu(m, n, T, B=B, i_const=I, v0=v0, record_v=True)
    st0 = O.init_state(m, v0.astype(np.float64))
    ro = O.run(m, st0.copy(), T, i_const=I, record_v=True)
    _judge(m, st0, T, g, ro, {"i_const": I}, max_ill_frac=0.05, label="small")


def test_inftau_gate_and_per_neuron_capacitance():
    """Cortical set (with the M-type (p_inf, 1/tau) gate), per-neuron C_m shared
    over a batch of 3."""
    print_case("cortical set, per-neuron C_m, B=3")
    m = W.custom_channels(dt=0.025)
    N, B, T = 300, 3, 3000
    n = N * B
    rng = np.random.default_rng(5)
    cm = (0.7 + 0.6 * rng.random(N)).astype(np.float32)
    I = (1.0 + 8.0 * rng.random(n)).astype(np.float32).astype(np.float64)
    g = _run_gpu(m, n, T, B=B, i_const=I, cm=cm, record_v=True)
    st0 = O.init_state(m, np.full(n, -65.0))
    cmn = np.tile(cm.astype(np.float64), B)
    ro = O.run(m, st0.copy(), T, i_const=I, cm=cmn, record_v=True)
    q = (ro["spikes"].sum(0) == 0).sum()
    assert 0 < q < n
    _judge(m, st0, T, g, ro, {"i_const": I, "cm": cmn}, max_ill_frac=0.05, label="cortical")


def test_leak_only_model_and_zero_steps():
    torch = need_gpu()
    m = W.classic_hh(dt=0.05)
    m["gates"] = []
    m["channels"] = [{"gbar": 0.3, "E": -54.4, "gates": []}]
    g = _run_gpu(m, 70, 200, i_const=np.full(70, 3.0), v0=-80.0, record_v=True)
    vinf = -54.4 + 3.0 / 0.3
    exact = vinf + (-80.0 - vinf) * (1 - 0.05 * 0.3) ** np.arange(1, 201)
    assert np.max(np.abs(g["v"][:, 0] - exact)) < 1e-4
    st = g["state_t"].clone()
    g["model"].step_n(st, 0)
    assert torch.equal(st, g["state_t"])


def test_fusion_depth_and_resume_are_bit_identical():
    """K = 1, K = 7 and K = 32 give bit-identical states, spikes and V; a run
    split at an arbitrary step and resumed from its state matches the
    unsplit run bit for bit (the noise is keyed by the absolute step)."""
    torch = need_gpu()
    m = W.custom_channels(dt=0.025)
    n, T, seed = 3000, 700, 7
    coef = W.jitter_coef(m, n, seed=seed)
    outs = [_run_gpu(m, n, T, noise=(5.0, 3.0, seed), coef=coef, fusion=k, record_v=True)
            for k in (1, 7, 32)]
    for o in outs[1:]:
        assert np.array_equal(o["state"], outs[0]["state"])
        assert np.array_equal(o["raster"], outs[0]["raster"])
        assert np.array_equal(o["v"], outs[0]["v"])
    gen = _run_gpu(m, n, T, noise=(5.0, 3.0, seed), coef=coef, fusion=32, record_v=True,
                   specialize=False)
    assert np.max(np.abs(gen["v"] - outs[0]["v"])[:50]) < 1e-3  # same math, other rounding order
    a = _run_gpu(m, n, 333, noise=(5.0, 3.0, seed), coef=coef)
    b = _run_gpu(m, n, T - 333, noise=(5.0, 3.0, seed), coef=coef, t0=333, state=a["state_t"])
    assert np.array_equal(b["state"], outs[0]["state"])
    assert np.array_equal(np.concatenate([a["raster"], b["raster"]]), outs[0]["raster"])
    del torch


def test_checkpoints_and_level_counts():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.025)
    N, B, T, every = 64, 4, 120, 50
    n = N * B
    rng = np.random.default_rng(8)
    I = (10.0 + 5.0 * rng.standard_normal((T, n))).astype(np.float32)
    M = hh.Model(m, N, B)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    nck = (T + every - 1) // every
    ck = torch.zeros((nck, M.n_state, n), device="cuda")
    lv = torch.zeros(n, device="cuda")
    M.step_n(st, T, i_dense=torch.tensor(I, device="cuda"), ckpt=ck, ckpt_every=every, level=lv)
    assert M.check()[0] == 0
    s = O.init_state(m, np.full(n, -65.0))
    for j in range(nck):
        c = ck[j].cpu().numpy()
        assert np.max(np.abs(c[:-1] - s)) < 2e-3, j
        assert np.max(np.abs(c[-1])) < 1e-4  # low part of V
        steps = min(every, T - j * every)
        O.run(m, s, steps, i_dense=I[j * every: j * every + steps].astype(np.float64), record_spikes=False)
    s = O.init_state(m, np.full(n, -65.0))
    lo = O.run(m, s, T, i_dense=I.astype(np.float64), level=True)["level"]
    assert np.sum(np.abs(lv.cpu().numpy() - lo)) <= 2


def test_nonfinite_state_is_reported():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.01)
    M = hh.Model(m, 500)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    st[0, 321] = float("nan")
    st[0, 400] = float("nan")
    M.step_n(st, 5, i_const=torch.zeros(500, device="cuda"))
    status, first = M.check()
    assert status == -4  # HH_E_NONFINITE
    assert first == 321
    assert M.check() == (0, -1)  # flags are cleared by the check
