"""Parity of the tabulated gate kinetics (Methods, "Engineering optimization":
cheaper approximations of the rate functions) against the oracle's table
mode: the same straight-line interpolants of p_inf and q = 1 - exp(-dt/tau)
between equally spaced nodes, in FP64.  Criteria as for the exact kernels:
quiet traces within 1e-3 mV, spike trains within one dt up to each neuron's
predictability horizon, ill-conditioned neurons reported."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import need_gpu, print_case
from tests.test_gpu_step import _cached, _columns, _judge, _run_gpu

pytestmark = pytest.mark.gpu


def _tab(model, table):
    return dict(model, table=table)


def test_tabulated_validation_workload():
    """1,024 classic HH neurons, I ~ U[0, 20), dt = 0.01 ms, 10,000 steps,
    321 nodes over [-100, 60] mV (h = 0.5 mV)."""
    print_case("tabulated classic HH 1024 x 10000 dt=0.01 nodes=321")
    table = (-100.0, 60.0, 321)
    m = W.classic_hh(dt=0.01)
    mt = _tab(m, table)
    n, T = 1024, 10000
    I = W.validation_currents(n, seed=1).astype(np.float64)
    g = _run_gpu(m, n, T, i_const=I, record_v=True, table=table)
    st0 = O.init_state(m, np.full(n, -65.0))
    ro = O.run(mt, st0.copy(), T, i_const=I, record_v=True)
    assert (ro["spikes"].sum(0) > 0).sum() > 500
    _judge(mt, st0, T, g, ro, {"i_const": I}, max_ill_frac=0.02, label="tab-validation")


@pytest.mark.parametrize("which", ["classic", "cortical"])
@pytest.mark.parametrize("mode", ["dense", "noise", "const"])
@pytest.mark.parametrize("syn", [False, True])
@pytest.mark.parametrize("nodes", [201, 1601])
def test_tabulated_input_modes(which, mode, syn, nodes):
    """Every launch variant of the tabulated step (dense, noise and
    constant input; with and without synaptic state; the table staged in
    LDS (201 nodes, at most 16 KB) or read from device memory (1,601 nodes,
    77 KB and 128 KB, over the 64 KB a block may stage)) on a ragged
    population of 300 neurons."""
    print_case("tabulated %s mode=%s syn=%s nodes=%d n=300" % (which, mode, syn, nodes))
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    table = (-100.0, 60.0, nodes)
    m = W.classic_hh(dt=0.025) if which == "classic" else W.custom_channels(dt=0.025)
    G = len(m["gates"])
    if syn:
        m = W.with_synapses(m)
    mt = _tab(m, table)
    n, T = 300, 1200
    rng = np.random.default_rng(17)
    v0 = (-70.0 + 10.0 * rng.random(n)).astype(np.float32)
    st0 = O.init_state(m, v0.astype(np.float64))
    state = None
    if syn:  # start with open synaptic conductances, decaying over the run
        Mi = hh.Model(m, n)
        state = Mi.init_state(Mi.new_state(), v0=torch.tensor(v0, device="cuda"))
        state[1 + G] = 0.3
        state[2 + G] = 0.2
        st0[1 + G] = float(np.float32(0.3))
        st0[2 + G] = float(np.float32(0.2))
    kw_g, kw_o = {}, {}
    if mode == "dense":
        mu = 2.0 if which == "classic" else 4.0
        I = (mu + 6.0 * rng.standard_normal((T, n))).astype(np.float32).astype(np.float64)
        kw_g["i_dense"], kw_o["i_dense"] = I, I
    elif mode == "noise":
        kw_g["noise"] = (5.0, 3.0, 7)
        # ids travel with neuron subsets when the judge re-runs a few neurons
        kw_o.update(noise_mu=5.0, noise_sigma=3.0, seed=7, ids=np.arange(n, dtype=np.uint32))
    else:
        I = (12.0 * rng.random(n)).astype(np.float32).astype(np.float64)
        kw_g["i_const"], kw_o["i_const"] = I, I
    g = _run_gpu(m, n, T, v0=v0, record_v=True, table=table, state=state, **kw_g)
    ro = O.run(mt, st0.copy(), T, record_v=True, **kw_o)
    assert ro["spikes"].sum() > 0
    _judge(mt, st0, T, g, ro, kw_o, max_ill_frac=0.05, label="tab-%s-%s" % (which, mode))


@pytest.mark.parametrize("nodes", [161, 641])
def test_tabulated_full_size_sampled(nodes):
    """The benchmark's configuration (1,048,576 cortical neurons, noisy
    input 5 + 3z, dt = 0.025 ms, 4,000 steps, 32 fused steps per launch)
    with 161 nodes (h = 1 mV, 256-lane blocks) and 641 nodes (h = 0.25 mV,
    51 KB in LDS, 512-lane blocks); 2,048 sampled neurons against the
    oracle."""
    print_case("tabulated cortical 1048576 x 4000 nodes=%d (sampled 2048)" % nodes)
    table = (-100.0, 60.0, nodes)
    m = W.custom_channels(dt=0.025)
    mt = _tab(m, table)
    n, T, seed = 1 << 20, 4000, 2
    g = _run_gpu(m, n, T, noise=(5.0, 3.0, seed), fusion=32, table=table)
    assert np.isfinite(g["state"]).all()
    rng = np.random.default_rng(98)
    ids = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.choice(n, 2043, replace=False)]))
    st0 = O.init_state(m, np.full(len(ids), -65.0))
    kw = {"noise_mu": 5.0, "noise_sigma": 3.0, "seed": seed, "ids": ids}
    ro = _cached("tab-full-%d" % nodes, lambda: O.run(mt, st0.copy(), T, **kw))
    assert ro["spikes"].sum(0).mean() > 1.0
    gs = {"raster": _columns(g["bits"], ids), "v": None}
    _judge(mt, st0, T, gs, ro, kw, max_ill_frac=0.02, label="tab-full-size")


@pytest.mark.parametrize("table", [(-80.0, 0.0, 81), (-100.0, 60.0, 2), (-100.0, 60.0, 1 << 20)])
def test_tabulated_range_edges(table):
    """A table narrower than the voltage range (spike peaks clamp to the top
    node), the single-segment table, and the largest node count."""
    print_case("tabulated classic range edges table=%s" % (table,))
    m = W.classic_hh(dt=0.025)
    mt = _tab(m, table)
    n, T = 130, 800
    I = (4.0 + 14.0 * np.random.default_rng(3).random(n)).astype(np.float32).astype(np.float64)
    g = _run_gpu(m, n, T, i_const=I, record_v=True, table=table)
    st0 = O.init_state(m, np.full(n, -65.0))
    ro = O.run(mt, st0.copy(), T, i_const=I, record_v=True)
    if table[2] == 81:
        assert np.max(ro["v"]) > 0.0  # the clamp is exercised
    _judge(mt, st0, T, g, ro, {"i_const": I}, max_ill_frac=0.05, label="tab-edges")


@pytest.mark.parametrize("nodes", [161, 641, 1601])
def test_tabulated_fusion_and_resume_bit_identical(nodes):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.custom_channels(dt=0.025)
    n, T = 70000, 300  # 256-lane blocks (512 with the 641-node table in LDS), ragged last block
    outs = []
    for fusion, splits in ((32, (300,)), (5, (120, 180)), (1, (299, 1))):
        M = hh.Model(m, n)
        M.set_fusion(fusion)
        M.set_rate_table(-100.0, 60.0, nodes)
        st = M.init_state(M.new_state(), v0_scalar=-65.0)
        bits = torch.zeros((T, M.words), dtype=torch.int32, device="cuda")
        t0 = 0
        for k in splits:
            M.step_n(st, k, t0, noise=(5.0, 3.0, 11), spikes=bits[t0:t0 + k])
            t0 += k
        outs.append((st.cpu().numpy(), bits.cpu().numpy()))
    for st, b in outs[1:]:
        assert np.array_equal(st, outs[0][0]) and np.array_equal(b, outs[0][1])


def test_tabulated_errors_and_removal():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.025)
    n, T = 1000, 200
    M = hh.Model(m, n)
    for args, status in (((-100.0, 60.0, 1), -2), ((-100.0, 60.0, (1 << 20) + 1), -2),
                         ((60.0, -100.0, 100), -1), ((0.0, 0.0, 100), -1),
                         ((float("nan"), 60.0, 100), -1), ((-100.0, float("inf"), 100), -1)):
        with pytest.raises(hh.HHError) as e:
            M.set_rate_table(*args)
        assert e.value.status == status, args
    # removal restores the exact kernel bit for bit
    ic = torch.full((n,), 9.0, device="cuda")
    ref = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(ref, T, i_const=ic)
    M.set_rate_table(-100.0, 60.0, 161)
    tab = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(tab, T, i_const=ic)
    assert not torch.equal(tab, ref)
    M.set_rate_table(0.0, 0.0, 0)
    again = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(again, T, i_const=ic)
    assert torch.equal(again, ref)
    # per-neuron coefficients are refused
    coef = torch.tensor(W.jitter_coef(m, n, seed=1), device="cuda")
    with pytest.raises(hh.HHError) as e:
        hh.Model(m, n, coef=coef).set_rate_table(-100.0, 60.0, 161)
    assert e.value.status == -5
    # the interpreter, the adjoint and the surrogate refuse a tabulated model
    M.set_rate_table(-100.0, 60.0, 161)
    M.set_specialize(False)
    st = M.init_state(M.new_state(), v0_scalar=-65.0)
    with pytest.raises(hh.HHError) as e:
        M.step_n(st, 10, i_const=ic)
    assert e.value.status == -5
    M.set_specialize(True)
    M.step_n(st, 10, i_const=ic)
    ck = torch.zeros((2, M.n_state, n), device="cuda")
    Id = torch.zeros((20, n), device="cuda")
    dI = torch.zeros_like(Id)
    with pytest.raises(hh.HHError) as e:
        M.backward(ck, 10, Id, 20, dI)
    assert e.value.status == -5
    mc = W.custom_channels(dt=0.025)
    Mc = hh.Model(mc, 256)
    Mc.set_rate_table(-100.0, 60.0, 161)
    stc = Mc.init_state(Mc.new_state(), v0_scalar=-65.0)
    packed = torch.zeros(hh.lib.hh_mlp_packed_bytes() // 4 + 1, dtype=torch.int32, device="cuda")
    flags = torch.zeros(256, dtype=torch.int32, device="cuda")
    with pytest.raises(hh.HHError) as e:
        hh.surrogate_step_n(Mc, packed, stc, flags, 10, 10, noise=(5.0, 3.0, 1))
    assert e.value.status == -5
