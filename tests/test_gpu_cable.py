"""Parity of multi-compartment neurons (Methods, Eq. (1) with its spatial
term; second-order explicit difference in space) against the oracle's
cable run.  Criteria as for point neurons: compartments that never spike
follow the oracle within 1e-3 mV at every step, spike trains agree in count
and within one dt; a mismatch is excused only when a 1e-6 relative probe of
the input, or the oracle run with its state rounded to binary32 every step,
moves the oracle's own result for that compartment by more than the
tolerance (tests.gpu_util); spike trains agree up to each compartment's
predictability horizon (the first spike such a probe moves by more than one
step), as for point neurons.  Excused cases are counted."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import judge, need_gpu, print_case

pytestmark = pytest.mark.gpu



def _morph(kind, model):
    """Morphologies: soma + 3 dendrites of 5 (areas, dendrites at 30%
    channel density), a 64-compartment unbranched cable, a 32-compartment
    binary tree, a soma with 4 children (the most one compartment may have),
    two compartments, and one (the point neuron)."""
    nch = len(model["channels"])
    if kind == "soma3x5":
        return W.soma_dendrites(model, 3, 5)
    if kind == "chain64":
        return {"K": 64, "parent": [-1] + list(range(63)), "g_axial": [0.0] + [2.0] * 63,
                "area": None, "gbar": None}
    if kind == "tree32":
        return {"K": 32, "parent": [-1] + [(c - 1) // 2 for c in range(1, 32)],
                "g_axial": [0.0] + [1.0 + 0.05 * c for c in range(1, 32)],
                "area": [2.0] + [1.0 - 0.01 * c for c in range(1, 32)], "gbar": None}
    if kind == "star8":
        return {"K": 8, "parent": [-1, 0, 0, 0, 0, 1, 2, 3], "g_axial": [0.0, 1, 2, 3, 4, 1, 1, 1],
                "area": None, "gbar": np.full((8, nch), 1.0) * [c["gbar"] for c in model["channels"]]}
    if kind == "pair":
        return {"K": 2, "parent": [-1, 0], "g_axial": [0.0, 0.8], "area": [1.0, 0.4], "gbar": None}
    return {"K": 1, "parent": [-1], "g_axial": None, "area": None, "gbar": None}


def _run_gpu(model, morph, n, T, *, v0=-65.0, state=None, i_const=None, noise=None, i_dense=None,
             record_v=True, fusion=32, specialize=True, cm=None, table=None):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    dev = "cuda"
    cm_t = None if cm is None else torch.tensor(np.asarray(cm, np.float32), device=dev)
    M = hh.Model(model, n, cm=cm_t)
    M.set_fusion(fusion)
    M.set_specialize(specialize)
    if table is not None:
        M.set_rate_table(*table)
    M.set_morphology(morph["K"], morph["parent"], morph.get("g_axial"), morph.get("area"),
                     morph.get("gbar"))
    if state is None:
        st = M.new_state()
        if np.isscalar(v0):
            M.init_state(st, v0_scalar=float(v0))
        else:
            M.init_state(st, v0=torch.tensor(np.asarray(v0, np.float32), device=dev))
    else:
        st = state
    spikes = torch.zeros((T, M.words), dtype=torch.int32, device=dev)
    vrec = torch.zeros((T, n), dtype=torch.float32, device=dev) if record_v else None
    ic = None if i_const is None else torch.tensor(np.asarray(i_const, np.float32), device=dev)
    idn = None if i_dense is None else torch.tensor(np.asarray(i_dense, np.float32), device=dev)
    M.step_n(st, T, 0, i_const=ic, noise=noise, i_dense=idn, spikes=spikes, v_rec=vrec)
    status, bad = M.check()
    assert status == 0, (status, bad)
    bits = spikes.cpu().numpy().view(np.uint32)
    return {"bits": bits, "raster": O.unpack_bits(bits, n) if n <= 65536 else None,
            "v": None if vrec is None else vrec.cpu().numpy(), "state": st.cpu().numpy(),
            "model": M, "state_t": st}


def _judge(model, morph, st0, T, g, ro, kw, *, v_tol=1e-3, max_ill_frac=0.05, label=""):
    """Parity criteria of tests.gpu_util.judge per compartment; the oracle
    re-runs a compartment together with its whole neuron."""
    return judge(O, model, st0, T, g, ro, kw, max_excused_frac=max_ill_frac, v_tol=v_tol,
                 label=label, morph=morph)


def _inputs(mode, morph, N, T, seed):
    K = morph["K"]
    n = N * K
    rng = np.random.default_rng(seed)
    if mode == "dense":  # one dendrite tip per neuron, amplitude U[0, 10) with 50% noise
        I = np.zeros((T, n))
        tip = K - 1
        amp = 10.0 * rng.random(N)
        for j in range(N):
            I[:, j * K + tip] = amp[j] * (1 + 0.5 * rng.standard_normal(T))
        I = I.astype(np.float32).astype(np.float64)
        return {"i_dense": I}, {"i_dense": I}
    if mode == "noise":
        return {"noise": (2.5, 3.0, seed)}, {"noise_mu": 2.5, "noise_sigma": 3.0, "seed": seed}
    if mode == "noise_quiet":
        return {"noise": (0.5, 1.0, seed)}, {"noise_mu": 0.5, "noise_sigma": 1.0, "seed": seed}
    I = 1.5 * rng.random(n)
    I[::K] = 20.0 * rng.random(N)  # the root compartments get more
    I = I.astype(np.float32).astype(np.float64)
    return {"i_const": I}, {"i_const": I}


@pytest.mark.parametrize("mode", ["const", "noise"])
def test_single_compartment_equals_point_kernel(mode):
    """K = 1: no edges, so the cable kernel must give the point kernel's
    results bit for bit."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.025)
    n, T = 1000, 700
    rng = np.random.default_rng(6)
    ic = torch.tensor((12.0 * rng.random(n)).astype(np.float32), device="cuda")
    outs = []
    for morph in (False, True):
        M = hh.Model(m, n)
        if morph:
            M.set_morphology(1, [-1])
        st = M.init_state(M.new_state(), v0_scalar=-65.0)
        bits = torch.zeros((T, M.words), dtype=torch.int32, device="cuda")
        if mode == "const":
            M.step_n(st, T, 0, i_const=ic, spikes=bits)
        else:
            M.step_n(st, T, 0, noise=(6.0, 3.0, 4), spikes=bits)
        outs.append((st.cpu().numpy(), bits.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][1].any()
    del torch


@pytest.mark.parametrize("kind,mode,N", [
    ("soma3x5", "dense", 37), ("soma3x5", "noise", 37), ("soma3x5", "noise_quiet", 20),
    ("soma3x5", "const", 37), ("chain64", "dense", 6), ("chain64", "const", 5),
    ("tree32", "noise", 9), ("tree32", "const", 9), ("star8", "dense", 41), ("star8", "noise", 41),
    ("pair", "const", 150), ("pair", "noise", 150)])
def test_cable_parity(kind, mode, N):
    """Classic HH channels on several morphologies, 2,000 steps of 0.025 ms;
    N neurons, so that the population ends in a partly filled wavefront."""
    print_case("cable %s mode=%s N=%d" % (kind, mode, N))
    m = W.classic_hh(dt=0.025)
    morph = _morph(kind, m)
    K = morph["K"]
    n, T = N * K, 2000
    kw_g, kw_o = _inputs(mode, morph, N, T, seed=N)
    g = _run_gpu(m, morph, n, T, **kw_g)
    st0 = O.init_state(m, np.full(n, -65.0))
    ro = O.cable_run(m, st0.copy(), T, morph, record_v=True, **kw_o)
    _judge(m, morph, st0, T, g, ro, kw_o, label="cable-%s-%s" % (kind, mode))


@pytest.mark.parametrize("specialize", [True, False])
def test_cable_cortical_channels_and_capacitance(specialize):
    """The cortical set (five gates, the M-type (p_inf, 1/tau) gate) on the
    soma + 3 dendrites morphology with per-compartment C_m, through the
    compiled specialization and through the interpreter."""
    print_case("cable cortical soma3x5 specialize=%s" % specialize)
    m = W.custom_channels(dt=0.025)
    morph = _morph("soma3x5", m)
    K = morph["K"]
    N, T = 24, 2000
    n = N * K
    rng = np.random.default_rng(12)
    cm = (0.8 + 0.4 * rng.random(n)).astype(np.float32).astype(np.float64)
    kw_g, kw_o = _inputs("const", morph, N, T, seed=3)
    g = _run_gpu(m, morph, n, T, cm=cm, specialize=specialize, **kw_g)
    st0 = O.init_state(m, np.full(n, -65.0))
    kw_o = dict(kw_o, cm=cm)
    ro = O.cable_run(m, st0.copy(), T, morph, record_v=True, **kw_o)
    assert ro["spikes"].sum() > 0
    _judge(m, morph, st0, T, g, ro, kw_o, label="cable-cortical")


def test_cable_with_synaptic_state():
    """Synaptic conductances open at the start and decaying (the synaptic
    launch variant)."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.with_synapses(W.classic_hh(dt=0.025))
    G = 3
    morph = _morph("soma3x5", m)
    N, T = 20, 1500
    n = N * morph["K"]
    Mi = hh.Model(m, n)
    state = Mi.init_state(Mi.new_state(), v0_scalar=-65.0)
    state[1 + G] = 0.3
    state[2 + G] = 0.1
    st0 = O.init_state(m, np.full(n, -65.0))
    st0[1 + G] = float(np.float32(0.3))
    st0[2 + G] = float(np.float32(0.1))
    kw_g, kw_o = _inputs("const", morph, N, T, seed=8)
    g = _run_gpu(m, morph, n, T, state=state, **kw_g)
    ro = O.cable_run(m, st0.copy(), T, morph, record_v=True, **kw_o)
    _judge(m, morph, st0, T, g, ro, kw_o, label="cable-syn")


def test_cable_full_size_sampled():
    """The benchmark's configuration: 65,536 neurons of soma + 3 dendrites
    (1,048,576 compartments), noisy input 2.5 + 3z, 4,000 steps of 0.025 ms,
    32 fused steps per launch; 40 sampled neurons against the oracle."""
    print_case("cable soma3x5 65536 neurons x 4000 (sampled 40)")
    m = W.classic_hh(dt=0.025)
    morph = _morph("soma3x5", m)
    K = morph["K"]
    N, T, seed = 65536, 4000, 9
    n = N * K
    g = _run_gpu(m, morph, n, T, noise=(2.5, 3.0, seed), record_v=False)
    assert np.isfinite(g["state"]).all()
    rng = np.random.default_rng(17)
    neurons = np.unique(np.concatenate([[0, 1, 3, N - 1], rng.choice(N, 36, replace=False)]))
    cols = (neurons[:, None] * K + np.arange(K)[None, :]).ravel()
    st0 = O.init_state(m, np.full(len(cols), -65.0))
    kw = {"noise_mu": 2.5, "noise_sigma": 3.0, "seed": seed, "ids": cols.astype(np.uint32)}
    ro = O.cable_run(m, st0.copy(), T, morph, record_v=True, **kw)
    assert ro["spikes"].sum(0).mean() > 1.0
    raster = ((g["bits"][:, cols // 32] >> (cols % 32).astype(np.uint32)) & 1).astype(np.uint8)
    _judge(m, morph, st0, T, {"raster": raster, "v": None}, ro, kw, max_ill_frac=0.05,
           label="cable-full-size")


@pytest.mark.parametrize("nodes,mode", [(321, "const"), (1601, "const"), (321, "noise"),
                                        (1601, "dense")])
def test_cable_with_rate_table(nodes, mode):
    """Tabulated gate kinetics in every compartment of the soma + 3
    dendrites morphology: the table staged in LDS (321 nodes, 15 KB) or
    read from device memory (1,601 nodes, 77 KB), under constant, noisy
    and dense input, against the oracle's cable run with the same table."""
    print_case("cable soma3x5 with table nodes=%d input=%s" % (nodes, mode))
    m = W.classic_hh(dt=0.025)
    morph = _morph("soma3x5", m)
    table = (-100.0, 60.0, nodes)
    mt = dict(m, table=table)
    N, T = 37, 2000
    n = N * morph["K"]
    kw_g, kw_o = _inputs(mode, morph, N, T, seed=N)
    g = _run_gpu(m, morph, n, T, table=table, **kw_g)
    st0 = O.init_state(m, np.full(n, -65.0))
    ro = O.cable_run(mt, st0.copy(), T, morph, record_v=True, **kw_o)
    assert ro["spikes"].sum() > 0
    _judge(mt, morph, st0, T, g, ro, kw_o, label="cable-table-%d-%s" % (nodes, mode))


def test_cable_wide_blocks_bit_identical():
    """A 641-node table (31 KB in LDS) on 72,000 compartments runs in
    512-lane blocks with a ragged last block; its first 65,472 compartments
    equal, bit for bit, a 65,472-compartment run in 64-lane blocks (the
    arithmetic per compartment does not depend on the block size)."""
    print_case("cable wide blocks 641-node table")
    m = W.classic_hh(dt=0.025)
    morph = _morph("soma3x5", m)
    table = (-100.0, 60.0, 641)
    T = 400
    outs = []
    for n in (72000, 65472):
        g = _run_gpu(m, morph, n, T, noise=(2.5, 3.0, 17), table=table)
        outs.append(g)
    big, small = outs
    n = 65472
    assert np.array_equal(big["bits"][:, :n // 32], small["bits"])
    assert np.array_equal(big["v"][:, :n], small["v"])
    assert np.array_equal(big["state"][:, :n], small["state"])
    assert small["raster"].sum() > 0


def test_cable_fusion_and_resume_bit_identical():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.025)
    morph = _morph("soma3x5", m)
    n, T = 70000 // 16 * 16, 300
    outs = []
    for fusion, splits in ((32, (300,)), (7, (120, 180)), (1, (299, 1))):
        M = hh.Model(m, n)
        M.set_fusion(fusion)
        M.set_morphology(morph["K"], morph["parent"], morph["g_axial"], morph["area"], morph["gbar"])
        st = M.init_state(M.new_state(), v0_scalar=-65.0)
        bits = torch.zeros((T, M.words), dtype=torch.int32, device="cuda")
        t0 = 0
        for k in splits:
            M.step_n(st, k, t0, noise=(2.5, 3.0, 5), spikes=bits[t0:t0 + k])
            t0 += k
        outs.append((st.cpu().numpy(), bits.cpu().numpy()))
    for st, b in outs[1:]:
        assert np.array_equal(st, outs[0][0]) and np.array_equal(b, outs[0][1])


def test_cable_errors_and_removal():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.classic_hh(dt=0.025)
    n = 1000
    M = hh.Model(m, n)
    bad = [((3, [-1, 0, 1], [0, 1, 1]), -2),            # not a power of two
           ((128, [-1] + list(range(127)), [0] + [1] * 127), -2),
           ((64, [-1] + list(range(63)), [0] + [1] * 63), -2),  # 1000 is not a multiple of 64
           ((4, [-1, 0, 3, 1], [0, 1, 1, 1]), -1),      # parent after the child
           ((4, [-1, 0, 0, -2], [0, 1, 1, 1]), -1),
           ((4, [-1, 0, 0, 0], [0, 1, -1, 1]), -1),     # negative conductance
           ((4, [-1, 0, 0, 0], None), -1),
           ((8, [-1, 0, 0, 0, 0, 0, 1, 2], [0] + [1] * 7), -5)]  # five children
    for args, status in bad:
        with pytest.raises(hh.HHError) as e:
            M.set_morphology(*args)
        assert e.value.status == status, args
    with pytest.raises(hh.HHError) as e:
        M.set_morphology(4, [-1, 0, 0, 0], [0, 1, 1, 1], area=[1, 1, 0, 1])
    assert e.value.status == -1
    # different inputs per element, so that the coupling moves current
    ic = torch.linspace(0.0, 12.0, n, device="cuda")
    ref = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(ref, 300, i_const=ic)
    M.set_morphology(4, [-1, 0, 0, 0], [0, 1, 1, 1])
    cab = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(cab, 300, i_const=ic)
    # checkpoints, level counts, tables, the adjoint and the surrogate are refused
    ck = torch.zeros((1, M.n_state, n), device="cuda")
    for kw in ({"ckpt": ck, "ckpt_every": 300}, {"level": torch.zeros(n, device="cuda")}):
        with pytest.raises(hh.HHError) as e:
            M.step_n(cab, 10, i_const=ic, **kw)
        assert e.value.status == -5
    Id = torch.zeros((20, n), device="cuda")
    with pytest.raises(hh.HHError) as e:
        M.backward(torch.zeros((2, M.n_state, n), device="cuda"), 10, Id, 20, torch.zeros_like(Id))
    assert e.value.status == -5
    # removal restores the point kernel bit for bit
    M.set_morphology(0)
    again = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(again, 300, i_const=ic)
    assert torch.equal(again, ref) and not torch.equal(cab, ref)
    # a table and a morphology combine, in either order
    M.set_rate_table(-100.0, 60.0, 161)
    M.set_morphology(4, [-1, 0, 0, 0], [0, 1, 1, 1])
    both = M.init_state(M.new_state(), v0_scalar=-65.0)
    M.step_n(both, 300, i_const=ic)
    assert not torch.equal(both, cab)
