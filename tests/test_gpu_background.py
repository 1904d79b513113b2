"""The background input of the cortex model (Methods, cortical network:
drawn directly as N ~ Poisson(lam) events of Gaussian amplitude) on the
device against the oracle: the event counts bit for bit (an integer that
floating point decides, taken in binary32 on both sides), the currents to
FP32 rounding, and whole trajectories under the usual parity criteria."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import need_gpu, print_case
from tests.test_gpu_step import _judge as judge_point

pytestmark = pytest.mark.gpu

# gate-free, conductance-free element: with V0 = 0 and dt = C = 1 one step
# leaves V equal to the drawn current
BARE = {"gates": [], "channels": [], "C": 1.0, "dt": 1.0, "v_th": 1e9, "v_method": "fe",
        "syn": None}


def _one_step(n, t0, bg):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    M = hh.Model(BARE, n)
    st = M.new_state()
    M.init_state(st, v0_scalar=0.0)
    M.step_n(st, 1, t0, background=bg)
    return st.cpu().numpy()[0].astype(np.float64), torch


@pytest.mark.parametrize("lam", [0.05, 1.6, 7.3, 40.0, 80.0])
def test_background_counts_bit_exact(lam):
    """mu = 1, sigma = 0: the element's V after one step is its event count."""
    print_case("background counts lam=%g" % lam)
    n = 50000
    for t0 in (0, 3, 1001):
        v, _ = _one_step(n, t0, (lam, 1.0, 0.0, 21))
        want = np.array([O.background(21, i, t0, lam, 1.0, 0.0)[1] for i in range(n)], np.float64)
        assert np.array_equal(v, want), (t0, np.nonzero(v != want)[0][:5])
        assert abs(want.mean() - lam) < 6 * np.sqrt(lam / n) + 1e-9


def test_background_currents():
    """mu = 0.5, sigma = 2: the current N mu + sqrt(N) sigma z to FP32 rounding of
    the Box-Muller normal."""
    n, lam = 20000, 3.0
    for t0 in (0, 77):
        v, _ = _one_step(n, t0, (lam, 0.5, 2.0, 5))
        want = np.array([O.background(5, i, t0, lam, 0.5, 2.0)[0] for i in range(n)])
        assert np.max(np.abs(v - want) / (1.0 + np.abs(want))) < 2e-5, t0


@pytest.mark.parametrize("which", ["classic", "cortical"])
@pytest.mark.parametrize("table", [None, (-100.0, 60.0, 161)])
def test_background_trajectories(which, table):
    """1,000 neurons x 4,000 steps of 0.025 ms under background input (the
    general-loop kernel, with the rate functions or a rate table), against
    the oracle under the point-neuron criteria."""
    print_case("background trajectories %s table=%s" % (which, table))
    if which == "classic":
        m, bg = W.classic_hh(dt=0.025), (0.8, 3.0, 2.0)
    else:
        m, bg = W.custom_channels(dt=0.025), (1.6, 2.0, 2.0)
    mo = m if table is None else dict(m, table=table)
    n, T, seed = 1000, 4000, 13
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    M = hh.Model(m, n)
    if table is not None:
        M.set_rate_table(*table)
    st = M.init_state(M.new_state(), v0_scalar=-65.0)
    spikes = torch.zeros((T, M.words), dtype=torch.int32, device="cuda")
    vrec = torch.zeros((T, n), dtype=torch.float32, device="cuda")
    M.step_n(st, T, 0, background=bg + (seed,), spikes=spikes, v_rec=vrec)
    status, bad = M.check()
    assert status == 0, (status, bad)
    g = {"raster": O.unpack_bits(spikes.cpu().numpy().view(np.uint32), n),
         "v": vrec.cpu().numpy()}
    st0 = O.init_state(m, np.full(n, -65.0))
    # element ids travel with neuron subsets, so that re-runs of a few
    # neurons draw their own input
    kw = {"background": bg, "seed": seed, "ids": np.arange(n, dtype=np.uint32)}
    ro = O.run(mo, st0.copy(), T, record_v=True, **kw)
    s = ro["spikes"].sum(0)
    assert (s > 0).sum() > 100 and (s == 0).sum() > 50
    judge_point(mo, st0, T, g, ro, kw, max_ill_frac=0.05, label="background-%s" % which)


def test_background_on_the_cable():
    from tests.test_gpu_cable import _judge as judge_cable
    print_case("background on soma3x5 cable")
    m = W.classic_hh(dt=0.025)
    morph = W.soma_dendrites(m, 3, 5)
    N, T, seed = 40, 3000, 4
    n = N * morph["K"]
    bg = (0.8, 2.0, 1.5)
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    M = hh.Model(m, n)
    M.set_morphology(morph["K"], morph["parent"], morph["g_axial"], morph["area"], morph["gbar"])
    st = M.init_state(M.new_state(), v0_scalar=-65.0)
    spikes = torch.zeros((T, M.words), dtype=torch.int32, device="cuda")
    vrec = torch.zeros((T, n), dtype=torch.float32, device="cuda")
    M.step_n(st, T, 0, background=bg + (seed,), spikes=spikes, v_rec=vrec)
    status, bad = M.check()
    assert status == 0
    g = {"raster": O.unpack_bits(spikes.cpu().numpy().view(np.uint32), n),
         "v": vrec.cpu().numpy()}
    st0 = O.init_state(m, np.full(n, -65.0))
    kw = {"background": bg, "seed": seed}
    ro = O.cable_run(m, st0.copy(), T, morph, record_v=True, **kw)
    assert ro["spikes"].sum() > 0
    judge_cable(m, morph, st0, T, g, ro, kw, label="background-cable")


def test_background_errors():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.025)
    M = hh.Model(m, 256)
    st = M.init_state(M.new_state(), v0_scalar=-65.0)
    for lam in (-0.1, 80.5, float("nan"), float("inf")):
        with pytest.raises(hh.HHError) as e:
            M.step_n(st, 4, background=(lam, 1.0, 1.0, 1))
        assert e.value.status == -1, lam
    M.step_n(st, 4, background=(0.0, 1.0, 1.0, 1))  # lam = 0 is valid: no events
    mc = W.custom_channels(dt=0.025)
    Mc = hh.Model(mc, 256)
    stc = Mc.init_state(Mc.new_state(), v0_scalar=-65.0)
    packed = torch.zeros(hh.lib.hh_mlp_packed_bytes() // 4 + 1, dtype=torch.int32, device="cuda")
    flags = torch.zeros(256, dtype=torch.int32, device="cuda")
    inp = hh.Input()
    inp.mode, inp.lam, inp.mu, inp.sigma, inp.seed = hh.IN_BACKGROUND, 1.0, 1.0, 1.0, 1
    import ctypes
    rc = hh.lib.hh_surrogate_step_n(Mc.h, hh._ptr(packed), hh.ACT_SILU, hh._ptr(stc), hh._ptr(flags), 0, 10, 10,
                                    ctypes.byref(inp), -50.0, 10, 0.5, None, None, hh._stream())
    assert rc == -5
