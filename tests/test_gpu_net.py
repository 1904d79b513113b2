"""GPU parity of the recurrent-network path (persistent kernel with spike
compaction and CSR scatter) and of hh_syn_propagate, through the C ABI.

Synaptic arrivals are accumulated in 64-bit fixed point on the GPU and in
FP64 (CSR order) in the oracle.  Networks are chaotic: spike-exact parity is
required up to the predictability horizon, the first step at which the
oracle's own raster changes under tiny perturbations (1 FP32 ulp of V0,
1e-6 of the weight scale); past it the comparison is statistical.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import need_gpu, print_case, spike_mismatch

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _net_gpu(m, csr, scale, v0, T, *, ext=None, i_const=None, state=None, t0=0,
             delivery="auto"):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    n = len(csr[0]) - 1
    M = hh.Model(m, n)
    rp, col, w = _dev(csr[0]), _dev(csr[1]), _dev(csr[2].astype(np.float32))
    M.attach_csr(rp, col, w, scale)
    M.set_delivery(delivery)
    if ext is not None:
        M.set_external(_dev(ext[0]), ext[1], ext[2], ext[3])
    st = M.new_state() if state is None else state
    if state is None:
        M.init_state(st, v0=_dev(v0.astype(np.float32)))
    spikes = torch.zeros((max(T, 1), M.words), dtype=torch.int32, device="cuda")
    ic = None if i_const is None else _dev(np.asarray(i_const, np.float32))
    M.step_n(st, T, t0, i_const=ic, spikes=spikes)
    status, bad = M.check()
    assert status == 0, (status, bad)
    bits = spikes[:T].cpu().numpy().view(np.uint32)
    return {"raster": O.unpack_bits(bits, n), "state": st.cpu().numpy(), "state_t": st, "M": M,
            "bufs": (rp, col, w)}


def test_syn_propagate_matches_oracle_and_is_deterministic():
    print_case("syn_propagate n=5003 fan=300")
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    n = 5003
    m = W.net_model()
    csr = W.net_csr(n=n, fan_out=300, seed=11, inh_scale=4.0)
    rng = np.random.default_rng(1)
    s = (rng.random(n) < 0.3).astype(np.uint8)
    words = (n + 31) // 32
    bits = np.zeros(words * 32, np.uint8)
    bits[:n] = s
    packed = np.packbits(bits.reshape(-1, 8), axis=1, bitorder="little").reshape(-1).view(np.uint32)
    M = hh.Model(m, n)
    M.attach_csr(_dev(csr[0]), _dev(csr[1]), _dev(csr[2]), 0.03)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    G = len(m["gates"])
    ge0 = rng.random(n).astype(np.float32) * 0.1
    gi0 = rng.random(n).astype(np.float32) * 0.1
    st[1 + G] = _dev(ge0)
    st[2 + G] = _dev(gi0)
    outs = []
    for rep in range(2):
        s2 = st.clone()
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        M.syn_propagate(_dev(packed), s2, cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == int(s.sum())
        outs.append(s2.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    ge, gi = ge0.astype(np.float64), gi0.astype(np.float64)
    O.syn_deliver(csr, 0.03, s, ge, gi)
    assert np.allclose(outs[0][1 + G], ge, rtol=3e-7, atol=1e-9)
    assert np.allclose(outs[0][2 + G], gi, rtol=3e-7, atol=1e-9)
    # everything else untouched
    assert np.array_equal(outs[0][: 1 + G], st.cpu().numpy()[: 1 + G])


@pytest.mark.parametrize("sorted_rows", [True, False])
def test_syn_propagate_no_spikes_and_empty_rows(sorted_rows):
    """Degenerate one-shot deliveries: with no source spiking the count is 0
    and the state is untouched, bit for bit; on a CSR whose rows are mostly
    empty (only every third row has synapses) with every source spiking, the
    empty rows deliver nothing and the conductances match the oracle.  Rows
    sorted by target take the binned delivery, shuffled rows the per-event
    one."""
    print_case("syn_propagate degenerate sorted=%s" % sorted_rows)
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    n, fan = 2000, 150
    rng = np.random.default_rng(21)
    counts = np.where(np.arange(n) % 3 == 0, fan, 0)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cols, ws = [], []
    for j in range(n):
        if counts[j] == 0:
            continue
        c = rng.choice(n, size=fan, replace=False).astype(np.int32)
        c = np.sort(c) if sorted_rows else rng.permutation(c)
        sign = 1.0 if j < int(0.8 * n) else -4.0
        cols.append(c)
        ws.append((sign * rng.lognormal(-1.0, 0.5, fan)).astype(np.float32))
    csr = (row_ptr, np.concatenate(cols), np.concatenate(ws))
    m = W.net_model()
    G = len(m["gates"])
    M = hh.Model(m, n)
    M.attach_csr(_dev(csr[0]), _dev(csr[1]), _dev(csr[2]), 0.03)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    ge0 = rng.random(n).astype(np.float32) * 0.1
    gi0 = rng.random(n).astype(np.float32) * 0.1
    st[1 + G] = _dev(ge0)
    st[2 + G] = _dev(gi0)
    words = (n + 31) // 32
    # no spikes
    s2 = st.clone()
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    M.syn_propagate(torch.zeros(words, dtype=torch.int32, device="cuda"), s2, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    assert torch.equal(s2, st)
    # every source spikes: the empty rows contribute nothing
    s3 = st.clone()
    allbits = np.zeros(words * 32, np.uint8)
    allbits[:n] = 1
    packed = np.packbits(allbits.reshape(-1, 8), axis=1, bitorder="little").reshape(-1).view(np.uint32)
    M.syn_propagate(_dev(packed), s3, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == n
    out = s3.cpu().numpy()
    ge, gi = ge0.astype(np.float64), gi0.astype(np.float64)
    O.syn_deliver(csr, 0.03, np.ones(n, np.uint8), ge, gi)
    assert np.allclose(out[1 + G], ge, rtol=3e-7, atol=1e-9)
    assert np.allclose(out[2 + G], gi, rtol=3e-7, atol=1e-9)
    assert np.array_equal(out[: 1 + G], st.cpu().numpy()[: 1 + G])


@pytest.mark.parametrize("n,fan_out,p_spike", [(3001, 700, 0.6), (9001, 300, 0.7)])
def test_syn_propagate_binned_equals_per_event_delivery(n, fan_out, p_spike):
    """The binned delivery (rows sorted by target) and the per-event delivery
    (the same CSR with every row's synapses shuffled, which the library
    detects) give identical conductances, bit for bit; so do the B = 2 copies
    of a batch (per-event path) and the single network, copy by copy.  The
    first case has segments longer than one 128-event pass in one chunk of
    rows; the second several chunks of rows and target ranges, both ragged."""
    print_case("syn_propagate binned vs per-event n=%d fan_out=%d" % (n, fan_out))
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.net_model()
    rp, col, w = W.net_csr(n=n, fan_out=fan_out, seed=13, inh_scale=4.0)
    rng = np.random.default_rng(2)
    col_s, w_s = col.copy(), w.copy()
    for j in range(n):
        a, b = rp[j], rp[j + 1]
        p = rng.permutation(b - a)
        col_s[a:b], w_s[a:b] = col[a:b][p], w[a:b][p]
    s = (rng.random(n) < p_spike).astype(np.uint8)
    bits = np.zeros(((n + 31) // 32) * 32, np.uint8)
    bits[:n] = s
    packed = np.packbits(bits.reshape(-1, 8), axis=1, bitorder="little").reshape(-1).view(np.uint32)
    G = len(m["gates"])
    outs = []
    for c_, w_ in ((col, w), (col_s, w_s)):
        M = hh.Model(m, n)
        bufs = [_dev(rp), _dev(c_), _dev(w_)]
        M.attach_csr(bufs[0], bufs[1], bufs[2], 0.05)
        st = M.init_state(M.new_state(), v0_scalar=-65.0)
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        M.syn_propagate(_dev(packed), st, cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == int(s.sum())
        outs.append(st.cpu().numpy())
    assert outs[0][1 + G].sum() > 0
    assert np.array_equal(outs[0], outs[1])
    # two copies: copy 0 spikes as above, copy 1 with the complementary bits
    s2 = np.concatenate([s, 1 - s])
    bits2 = np.zeros(((2 * n + 31) // 32) * 32, np.uint8)
    bits2[:2 * n] = s2
    packed2 = np.packbits(bits2.reshape(-1, 8), axis=1, bitorder="little").reshape(-1).view(np.uint32)
    M2 = hh.Model(m, n, 2)
    bufs = [_dev(rp), _dev(col), _dev(w)]
    M2.attach_csr(bufs[0], bufs[1], bufs[2], 0.05)
    st2 = M2.init_state(M2.new_state(), v0_scalar=-65.0)
    M2.syn_propagate(_dev(packed2), st2)
    g2 = st2.cpu().numpy()
    assert np.array_equal(g2[:, :n], outs[0])
    ge, gi = np.zeros(n), np.zeros(n)
    O.syn_deliver((rp, col, w), 0.05, 1 - s, ge, gi)
    assert np.allclose(g2[1 + G, n:], ge, rtol=3e-7, atol=1e-9)
    assert np.allclose(g2[2 + G, n:], gi, rtol=3e-7, atol=1e-9)


def test_syn_propagate_full_network_all_spiking():
    print_case("syn_propagate full 38000 x 2630 all spiking")
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    n = 38000
    m = W.net_model()
    csr = W.net_csr(n=n, inh_scale=W.NET_INH_SCALE)
    M = hh.Model(m, n)
    M.attach_csr(_dev(csr[0]), _dev(csr[1]), _dev(csr[2]), W.NET_W_SCALE)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    bits = torch.full(((n + 31) // 32,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    M.syn_propagate(bits, st, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == n
    got = st.cpu().numpy()
    ge, gi = np.zeros(n), np.zeros(n)
    O.syn_deliver(csr, W.NET_W_SCALE, np.ones(n, np.uint8), ge, gi)
    G = len(m["gates"])
    assert np.allclose(got[1 + G], ge, rtol=3e-7, atol=0)
    assert np.allclose(got[2 + G], gi, rtol=3e-7, atol=0)


def _horizon(m, csr, scale, v0, T, ext):
    """First step at which the oracle raster changes under the probes (T if
    never), and the reference raster."""
    kw = dict(ext_mask=ext[0], ext_thresh=ext[1], w_ext=ext[2], seed=ext[3])
    ref = O.net_run(m, O.init_state(m, v0), csr, scale, T, **kw)
    h = T
    v32 = v0.astype(np.float32)
    ulp = np.spacing(np.abs(v32)).astype(np.float64)
    for pv0, ps in [(v0 + ulp, scale), (v0 - ulp, scale), (v0, scale * (1 + 1e-6)),
                    (v0, scale * (1 - 1e-6))]:
        r = O.net_run(m, O.init_state(m, pv0), csr, ps, T, **kw)
        d = np.nonzero((r != ref).any(axis=1))[0]
        if len(d):
            h = min(h, int(d[0]))
    return h, ref


@pytest.mark.parametrize("n,fan,T", [(2000, 200, 2000), (513, 40, 1500)])
def test_network_spike_exact_to_horizon(n, fan, T):
    print_case("network n=%d fan=%d T=%d" % (n, fan, T))
    m = W.net_model()
    csr = W.net_csr(n=n, fan_out=fan, seed=5, inh_scale=4.0)
    mask, thr = W.net_external(n=n, frac=0.05, seed=5)
    ext = (mask, thr, 0.5, 5)
    v0 = W.net_v0(n, 5).astype(np.float64)
    scale = 0.3
    g = _net_gpu(m, csr, scale, v0, T, ext=ext)
    h, ref = _horizon(m, csr, scale, v0, T, ext)
    assert ref.sum() > 5 * n * T * 1e-4  # the network is active (> 5 Hz)
    # the comparison must cover most of the run: on these networks the
    # oracle's raster is unchanged by the probes for all T steps
    assert h >= 0.9 * T, h
    upto = max(h - 1, 0)
    bad = spike_mismatch(g["raster"][:upto], ref[:upto])
    print("horizon %d of %d steps, spikes %d, mismatched neurons before horizon %d"
          % (h, T, int(ref.sum()), len(bad)), flush=True)
    assert len(bad) == 0
    # determinism: a second run is bit-identical
    g2 = _net_gpu(m, csr, scale, v0, T, ext=ext)
    assert np.array_equal(g2["raster"], g["raster"])
    assert np.array_equal(g2["state"], g["state"])


@pytest.mark.parametrize("n,fan,T,burst", [(2000, 200, 1000, False), (3001, 300, 120, True),
                                           (513, 40, 400, False), (100003, 60, 150, False)])
def test_network_pull_delivery_equals_push(n, fan, T, burst):
    """The delivery by target range (each block pulls the previous step's
    spiking rows' events for its own 512 neurons) and the push delivery
    (device atomics into arrival accumulators) add the same fixed-point
    increments: rasters and final states are bit-identical, also in a burst
    where thousands of neurons spike in one step (more rows than a block
    stages at once) and with a ragged last block; resumed runs too."""
    print_case("pull vs push n=%d fan=%d T=%d burst=%s" % (n, fan, T, burst))
    m = W.net_model()
    csr = W.net_csr(n=n, fan_out=fan, seed=21, inh_scale=4.0)
    mask, thr = W.net_external(n=n, frac=0.05, seed=21)
    ext = (mask, thr, 0.5, 21)
    v0 = W.net_v0(n, 21).astype(np.float64)
    ic = np.full(n, 40.0) if burst else None
    out = {}
    for d in ("auto", "push"):
        out[d] = _net_gpu(m, csr, 0.3, v0, T, ext=ext, i_const=ic, delivery=d)
    if burst:
        assert out["push"]["raster"].sum(axis=1).max() > 2 * 512
    assert out["push"]["raster"].sum() > 0
    assert np.array_equal(out["auto"]["raster"], out["push"]["raster"])
    assert np.array_equal(out["auto"]["state"], out["push"]["state"])
    a = _net_gpu(m, csr, 0.3, v0, T // 3, ext=ext, i_const=ic)
    b = _net_gpu(m, csr, 0.3, v0, T - T // 3, ext=ext, i_const=ic, state=a["state_t"],
                 t0=T // 3)
    assert np.array_equal(b["state"], out["push"]["state"])


def test_attach_refuses_invalid_csr_and_keeps_the_previous_one():
    """hh_attach_csr checks the CSR on the device before any delivery can use
    it (a bad column or row pointer would send the delivery's writes out of
    bounds): each invalid CSR is refused with HH_E_INVALID, and the model
    keeps running on the connectivity attached before, bit for bit."""
    print_case("attach invalid CSR")
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.net_model()
    n, fan = 600, 40
    rp, col, w = W.net_csr(n=n, fan_out=fan, seed=17, inh_scale=4.0)
    v0 = W.net_v0(n, 17).astype(np.float64)
    ref = _net_gpu(m, (rp, col, w), 0.3, v0, 200, i_const=np.full(n, 8.0))
    M = ref["M"]
    bad = []
    c1 = col.copy(); c1[5] = n; bad.append((rp, c1))            # column = N
    c2 = col.copy(); c2[fan * 7 + 3] = -1; bad.append((rp, c2))  # negative column
    r3 = rp.copy(); r3[10], r3[11] = r3[11], r3[10]; bad.append((r3, col))  # decreasing
    r4 = rp.copy(); r4[-1] -= 3; bad.append((r4, col))           # does not end at nnz
    r5 = rp.copy(); r5[0] = 1; bad.append((r5, col))             # does not start at 0
    for r_, c_ in bad:
        bufs = [_dev(r_), _dev(c_), _dev(w.astype(np.float32))]
        with pytest.raises(hh.HHError) as e:
            M.attach_csr(bufs[0], bufs[1], bufs[2], 0.3)
        assert e.value.status == -1
    st = M.init_state(M.new_state(), v0=_dev(v0.astype(np.float32)))
    spikes = torch.zeros((200, M.words), dtype=torch.int32, device="cuda")
    M.step_n(st, 200, 0, i_const=_dev(np.full(n, 8.0, np.float32)), spikes=spikes)
    assert np.array_equal(O.unpack_bits(spikes.cpu().numpy().view(np.uint32), n), ref["raster"])
    assert np.array_equal(st.cpu().numpy(), ref["state"])


def test_network_resume_and_tiny_cases():
    print_case("network resume / n=1")
    m = W.net_model()
    n, fan = 700, 50
    csr = W.net_csr(n=n, fan_out=fan, seed=8, inh_scale=4.0)
    mask, thr = W.net_external(n=n, frac=0.05, seed=8)
    ext = (mask, thr, 0.5, 8)
    v0 = W.net_v0(n, 8).astype(np.float64)
    full = _net_gpu(m, csr, 0.3, v0, 600, ext=ext)
    a = _net_gpu(m, csr, 0.3, v0, 250, ext=ext)
    b = _net_gpu(m, csr, 0.3, v0, 350, ext=ext, state=a["state_t"], t0=250)
    assert np.array_equal(b["state"], full["state"])
    assert np.array_equal(np.concatenate([a["raster"], b["raster"]]), full["raster"])
    # a single neuron without synapses, driven by a constant current
    one = (np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    g = _net_gpu(m, one, 0.3, np.array([-65.0]), 400, i_const=[12.0])
    ro = O.net_run(m, O.init_state(m, np.array([-65.0])), one, 0.3, 400, i_const=np.array([12.0]))
    assert g["raster"].sum() >= 3
    assert len(spike_mismatch(g["raster"], ro)) == 0
    # zero steps leaves the state untouched
    st = full["state_t"].clone()
    full["M"].step_n(st, 0)
    assert np.array_equal(st.cpu().numpy(), full["state"])


def test_full_network_statistics_and_determinism():
    """The configured network at full size and length: 38,000 neurons, 99.94 M
    synapses, 10,000 steps of 0.1 ms.  Bit-identical reruns; spike-exact
    against the oracle up to the predictability horizon (the first step at
    which the oracle's raster changes under 1 FP32 ulp of V0 or 1e-6 of the
    weight scale); population rates over the whole run within max(2 %, 3x
    the oracle's own spread under the ulp perturbation)."""
    print_case("full network 38000 x 2630, 10000 steps")
    n, T = 38000, 10000
    m = W.net_model()
    csr = W.net_csr(n=n, inh_scale=W.NET_INH_SCALE)
    mask, thr = W.net_external(n=n)
    ext = (mask, thr, W.NET_W_EXT, 3)
    v0 = W.net_v0(n, 3).astype(np.float64)
    g1 = _net_gpu(m, csr, W.NET_W_SCALE, v0, T, ext=ext)
    g2 = _net_gpu(m, csr, W.NET_W_SCALE, v0, T, ext=ext)
    assert np.array_equal(g1["raster"], g2["raster"]) and np.array_equal(g1["state"], g2["state"])
    kw = dict(ext_mask=mask, ext_thresh=thr, w_ext=W.NET_W_EXT, seed=3, omp=True)
    ro = O.net_run(m, O.init_state(m, v0), csr, W.NET_W_SCALE, T, **kw)
    ulp = np.spacing(np.abs(v0.astype(np.float32))).astype(np.float64)
    rp = O.net_run(m, O.init_state(m, v0 + ulp), csr, W.NET_W_SCALE, T, **kw)
    # the horizon: the other probes over the first steps (it is reached well
    # within them on this network)
    Th = 1500
    h = T
    for r in [rp] + [O.net_run(m, O.init_state(m, pv0), csr, ps, Th, **kw)
                     for pv0, ps in ((v0 - ulp, W.NET_W_SCALE), (v0, W.NET_W_SCALE * (1 + 1e-6)),
                                     (v0, W.NET_W_SCALE * (1 - 1e-6)))]:
        d = np.nonzero((r[:min(len(r), T)] != ro[:len(r)]).any(axis=1))[0]
        if len(d):
            h = min(h, int(d[0]))
    assert h < Th
    bad = spike_mismatch(g1["raster"][:max(h - 1, 0)], ro[:max(h - 1, 0)])
    before = int(ro[:h].sum())
    print("full network: horizon %d steps (%d spikes before it), mismatched before %d"
          % (h, before, len(bad)), flush=True)
    assert h >= 20 and before > 100
    assert len(bad) == 0
    ne = int(0.8 * n)

    def rates(r):
        c = r.sum(0) / (T * 0.1e-3)
        return np.array([c[:ne].mean(), c[ne:].mean()])
    rg, rr, rq = rates(g1["raster"]), rates(ro), rates(rp)
    tol = np.maximum(0.02 * rr, 3 * np.abs(rq - rr))
    print("rates GPU %s oracle %s perturbed-oracle %s tol %s" % (rg, rr, rq, tol), flush=True)
    assert np.all(rr > 1.0)
    assert np.all(np.abs(rg - rr) <= tol)


# ---------------------------------------------------------------------------
# synaptic delays of several steps (a ring of arrivals in flight) and the
# background input in the network kernel
# ---------------------------------------------------------------------------
def _net_model_gpu(m, csr, scale, *, delay=None, max_delay=1, ext=None):
    need_gpu()
    from paper_2601_21407_amd import hh
    n = len(csr[0]) - 1
    M = hh.Model(m, n)
    bufs = [_dev(csr[0]), _dev(csr[1]), _dev(csr[2].astype(np.float32))]
    M.attach_csr(bufs[0], bufs[1], bufs[2], scale)
    if delay is not None:
        d = _dev(delay)
        bufs.append(d)
        M.set_delays(d, max_delay)
    if ext is not None:
        em = _dev(ext[0])
        bufs.append(em)
        M.set_external(em, ext[1], ext[2], ext[3])
    return M, bufs


def _run_on(M, v0, T, *, state=None, t0=0, background=None, i_const=None):
    import torch
    st = state
    if st is None:
        st = M.new_state()
        M.init_state(st, v0=_dev(v0.astype(np.float32)))
    spikes = torch.zeros((max(T, 1), M.words), dtype=torch.int32, device="cuda")
    ic = None if i_const is None else _dev(np.asarray(i_const, np.float32))
    M.step_n(st, T, t0, spikes=spikes, background=background, i_const=ic)
    status, bad = M.check()
    assert status == 0, (status, bad)
    return O.unpack_bits(spikes[:T].cpu().numpy().view(np.uint32), M.n), st


def _horizon_kw(m, csr, scale, v0, T, kw):
    ref = O.net_run(m, O.init_state(m, v0), csr, scale, T, **kw)
    h = T
    ulp = np.spacing(np.abs(v0.astype(np.float32))).astype(np.float64)
    for pv0, ps in [(v0 + ulp, scale), (v0 - ulp, scale), (v0, scale * (1 + 1e-6)),
                    (v0, scale * (1 - 1e-6))]:
        r = O.net_run(m, O.init_state(m, pv0), csr, ps, T, **kw)
        d = np.nonzero((r != ref).any(axis=1))[0]
        if len(d):
            h = min(h, int(d[0]))
    return h, ref


@pytest.mark.parametrize("drive", ["external", "background"])
def test_network_pathway_delays_spike_exact_to_horizon(drive):
    """1,500 neurons in 8 populations, 150 targets per source, a delay of 1
    to 15 steps per pathway; spike-exact against the oracle up to the
    horizon, and bit-identical on a rerun."""
    print_case("network delays drive=%s" % drive)
    m = W.net_model()
    n, fan, T = 1500, 150, 2000
    csr = W.net_csr(n=n, fan_out=fan, seed=5, inh_scale=4.0)
    dl, _, _ = W.pathway_delays(csr, 8, 15, 5)
    v0 = W.net_v0(n, 5).astype(np.float64)
    kw = {"delay": dl, "max_delay": 15}
    if drive == "external":
        mask, thr = W.net_external(n=n, frac=0.05, seed=5)
        ext = (mask, thr, 0.5, 5)
        kw.update(ext_mask=mask, ext_thresh=thr, w_ext=0.5, seed=5)
        bg = None
    else:
        ext = None
        bg = (0.5, 3.0, 2.0, 3)
        kw.update(background=bg[:3], in_seed=bg[3])
    # weight scale 0.15: the oracle's raster stays predictable over the whole
    # run under both drives (at 0.3 the external drive's diverges early)
    M, bufs = _net_model_gpu(m, csr, 0.15, delay=dl, max_delay=15, ext=ext)
    g, st = _run_on(M, v0, T, background=bg)
    h, ref = _horizon_kw(m, csr, 0.15, v0, T, kw)
    assert ref.sum() > 5 * n * T * 1e-4
    upto = max(h - 1, 0)
    bad = spike_mismatch(g[:upto], ref[:upto])
    print("horizon %d of %d steps, spikes %d, mismatched neurons before horizon %d"
          % (h, T, int(ref.sum()), len(bad)), flush=True)
    assert h > 200 and len(bad) == 0
    g2, st2 = _run_on(M, v0, T, background=bg)  # t0 = 0 again: nothing left in flight
    assert np.array_equal(g2, g) and np.array_equal(st2.cpu().numpy(), st.cpu().numpy())
    del bufs


def test_network_delays_resume_carries_arrivals_in_flight():
    """Split runs on one model equal the unsplit run: arrivals still in
    flight at the end of a call are delivered by the next."""
    m = W.net_model()
    n, fan = 700, 50
    csr = W.net_csr(n=n, fan_out=fan, seed=8, inh_scale=4.0)
    dl, _, _ = W.pathway_delays(csr, 8, 12, 8)
    mask, thr = W.net_external(n=n, frac=0.05, seed=8)
    ext = (mask, thr, 0.5, 8)
    v0 = W.net_v0(n, 8).astype(np.float64)
    M, bufs = _net_model_gpu(m, csr, 0.3, delay=dl, max_delay=12, ext=ext)
    full, stf = _run_on(M, v0, 600)
    a, st = _run_on(M, v0, 250)
    b, st = _run_on(M, v0, 7, state=st, t0=250)
    c, st = _run_on(M, v0, 343, state=st, t0=257)
    assert full.sum() > 0
    assert np.array_equal(np.concatenate([a, b, c]), full)
    assert np.array_equal(st.cpu().numpy(), stf.cpu().numpy())
    del bufs


def test_network_unit_delays_equal_one_step_kernel():
    m = W.net_model()
    n, fan = 900, 60
    csr = W.net_csr(n=n, fan_out=fan, seed=9, inh_scale=4.0)
    mask, thr = W.net_external(n=n, frac=0.05, seed=9)
    ext = (mask, thr, 0.5, 9)
    v0 = W.net_v0(n, 9).astype(np.float64)
    M0, b0 = _net_model_gpu(m, csr, 0.3, ext=ext)
    M1, b1 = _net_model_gpu(m, csr, 0.3, delay=np.ones(len(csr[1]), np.uint8), max_delay=4,
                            ext=ext)
    r0, s0 = _run_on(M0, v0, 800)
    r1, s1 = _run_on(M1, v0, 800)
    assert r0.sum() > 0 and np.array_equal(r0, r1)
    assert np.array_equal(s0.cpu().numpy(), s1.cpu().numpy())
    del b0, b1


def test_network_delay_errors():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.net_model()
    n = 200
    M = hh.Model(m, n)
    d = _dev(np.ones(10, np.uint8))
    with pytest.raises(hh.HHError) as e:
        M.set_delays(d, 4)  # no connectivity attached
    assert e.value.status == -1
    csr = W.net_csr(n=n, fan_out=10, seed=2, inh_scale=4.0)
    M, bufs = _net_model_gpu(m, csr, 0.3)
    nnz = len(csr[1])
    for arr, mx, status in ((np.full(nnz, 5, np.uint8), 4, -1), (np.zeros(nnz, np.uint8), 4, -1),
                            (np.ones(nnz, np.uint8), 0, -2), (np.ones(nnz, np.uint8), 256, -2)):
        with pytest.raises(hh.HHError) as e:
            M.set_delays(_dev(arr), mx)
        assert e.value.status == status, (mx, status)
    M.set_delays(None, 0)
    # attaching a connectivity drops a delay table set for the previous one
    v0 = W.net_v0(n, 2).astype(np.float64)
    ref, _ = _run_on(M, v0, 300, i_const=np.full(n, 9.0))
    M.set_delays(_dev(np.full(nnz, 7, np.uint8)), 8)
    delayed, _ = _run_on(M, v0, 300, i_const=np.full(n, 9.0))
    M.attach_csr(bufs[0], bufs[1], bufs[2], 0.3)
    again, _ = _run_on(M, v0, 300, i_const=np.full(n, 9.0))
    assert ref.sum() > 0 and not np.array_equal(delayed, ref) and np.array_equal(again, ref)
    del torch, bufs


# ---------------------------------------------------------------------------
# a batch of independent copies of one network sharing the CSR (the paper's
# parallel simulations on one device), and the compiled cortical channel set
# ---------------------------------------------------------------------------
def _block_diagonal(csr, B):
    """The CSR of B disjoint copies of a network (copy b's targets + b N)."""
    rp, col, w = csr
    N = len(rp) - 1
    nnz = len(col)
    rpb = np.concatenate([rp[:-1] + b * nnz for b in range(B)] + [[B * nnz]]).astype(np.int64)
    colb = np.concatenate([col + b * N for b in range(B)]).astype(np.int32)
    return rpb, colb, np.tile(w, B)


def _batch_gpu(m, csr, scale, v0, T, B, *, ext=None, specialize=True, background=None,
               i_const=None, delivery="auto"):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    N = len(csr[0]) - 1
    M = hh.Model(m, N, B)
    M.set_specialize(specialize)
    bufs = [_dev(csr[0]), _dev(csr[1]), _dev(csr[2].astype(np.float32))]
    M.attach_csr(bufs[0], bufs[1], bufs[2], scale)
    M.set_delivery(delivery)
    if ext is not None:
        em = _dev(ext[0])
        bufs.append(em)
        M.set_external(em, ext[1], ext[2], ext[3])
    st = M.new_state()
    M.init_state(st, v0=_dev(v0.astype(np.float32)))
    spikes = torch.zeros((T, M.words), dtype=torch.int32, device="cuda")
    ic = None if i_const is None else _dev(np.asarray(i_const, np.float32))
    M.step_n(st, T, 0, spikes=spikes, background=background, i_const=ic)
    status, bad = M.check()
    assert status == 0, (status, bad)
    return O.unpack_bits(spikes.cpu().numpy().view(np.uint32), M.n), st.cpu().numpy()


@pytest.mark.parametrize("N,B,fan,T,burst", [(700, 3, 80, 600, False), (1000, 6, 100, 400, False),
                                             (3001, 2, 300, 100, True), (600, 5, 60, 300, True),
                                             (4000, 5, 150, 300, False),
                                             (20000, 5, 100, 200, False)])
def test_network_batch_pull_delivery_equals_push(N, B, fan, T, burst):
    """Batches of copies (N >= 512) deliver by target range too: a block's
    512 elements straddle two copies wherever N is not a multiple of 512, and
    it pulls from both copies' lists the spans of rows that cover its window.
    Bit-identical to the push delivery, with external events, and in a burst
    (thousands of spikes in one step, lists longer than one block stages);
    40 blocks synchronize with the flag-array barrier, and 100,000 neurons
    (196 blocks of 512) run in blocks of 1,024, as grids of 128 or more do."""
    print_case("batch pull vs push N=%d B=%d burst=%s" % (N, B, burst))
    m = W.net_model()
    csr = W.net_csr(n=N, fan_out=fan, seed=31, inh_scale=4.0)
    mask, thr = W.net_external(n=N, frac=0.05, seed=31)
    v0 = W.net_v0(N * B, 31).astype(np.float64)
    ic = np.full(N * B, 40.0) if burst else None
    out = {}
    for d in ("auto", "push"):
        out[d] = _batch_gpu(m, csr, 0.3, v0, T, B, ext=(mask, thr, 0.5, 31), i_const=ic,
                            delivery=d)
    r_p, s_p = out["push"]
    if burst:
        assert r_p.sum(axis=1).max() > 2 * 512
    assert r_p.sum() > 0
    assert np.array_equal(out["auto"][0], r_p)
    assert np.array_equal(out["auto"][1], s_p)


def test_network_batch_of_copies_matches_oracle():
    """B = 3 copies of a 1,000-neuron network share one CSR, each with its own
    initial state and its own external-event stream (keyed by the element
    index): spike-exact to the predictability horizon against the oracle's
    run of the block-diagonal network of the three copies."""
    print_case("network batch B=3 N=1000 fan=100")
    m = W.net_model()
    N, B, T = 1000, 3, 1500
    csr = W.net_csr(n=N, fan_out=100, seed=6, inh_scale=4.0)
    mask, thr = W.net_external(n=N, frac=0.05, seed=6)
    v0 = W.net_v0(N * B, 6).astype(np.float64)
    scale = 0.3
    raster, _ = _batch_gpu(m, csr, scale, v0, T, B, ext=(mask, thr, 0.5, 6))
    big = _block_diagonal(csr, B)
    h, ref = _horizon(m, big, scale, v0, T, (np.tile(mask, B), thr, 0.5, 6))
    assert ref.sum() > 5 * N * B * T * 1e-4
    assert h >= 0.9 * T, h
    bad = spike_mismatch(raster[:h - 1], ref[:h - 1])
    print("batch horizon %d of %d, spikes per copy %s, mismatched %d"
          % (h, T, [int(ref[:, b * N:(b + 1) * N].sum()) for b in range(B)], len(bad)), flush=True)
    assert len(bad) == 0
    # the copies differ (own states and streams)
    assert not np.array_equal(raster[:, :N], raster[:, N:2 * N])


def test_network_batch_identical_copies_equal_single_run():
    """Copies with the same initial state and input and no random drive run
    exactly like the single network, bit for bit (fixed-point arrivals do
    not depend on the order of the atomics)."""
    print_case("network batch identical copies B=4")
    m = W.net_model()
    N, B, T = 800, 4, 800
    csr = W.net_csr(n=N, fan_out=80, seed=9, inh_scale=4.0)
    v0 = W.net_v0(N, 9).astype(np.float64)
    r1, s1 = _batch_gpu(m, csr, 0.5, v0, T, 1, background=(1.0, 2.0, 1.0, 4))
    # background keyed by the element index: copy 0 equals the single run
    rB, sB = _batch_gpu(m, csr, 0.5, np.tile(v0, B), T, B, background=(1.0, 2.0, 1.0, 4))
    assert r1.sum() > 0
    assert np.array_equal(rB[:, :N], r1)
    assert np.array_equal(sB[:, :N], s1)
    # and without random drive every copy equals copy 0
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    Mq = hh.Model(m, N, B)
    bufs = [_dev(csr[0]), _dev(csr[1]), _dev(csr[2].astype(np.float32))]
    Mq.attach_csr(bufs[0], bufs[1], bufs[2], 0.5)
    st = Mq.new_state()
    Mq.init_state(st, v0=_dev(np.tile(v0, B).astype(np.float32)))
    spikes = torch.zeros((T, Mq.words), dtype=torch.int32, device="cuda")
    Mq.step_n(st, T, 0, spikes=spikes, i_const=_dev(np.full(N * B, 9.0, np.float32)))
    rq = O.unpack_bits(spikes.cpu().numpy().view(np.uint32), N * B)
    sq = st.cpu().numpy()
    assert rq.sum() > 0
    for b in range(1, B):
        assert np.array_equal(rq[:, b * N:(b + 1) * N], rq[:, :N])
        assert np.array_equal(sq[:, b * N:(b + 1) * N], sq[:, :N])


def test_network_batch_too_large_is_refused():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m = W.net_model()
    N, B = 38000, 64  # 2.4 M neurons: more than one co-resident grid holds
    csr = (np.zeros(N + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    M = hh.Model(m, N, B)
    bufs = [_dev(csr[0]), _dev(np.zeros(1, np.int32)), _dev(np.zeros(1, np.float32))]
    M.attach_csr(bufs[0], bufs[1][:0], bufs[2][:0], 0.1)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    with pytest.raises(hh.HHError) as e:
        M.step_n(st, 5)
    assert e.value.status == -5


@pytest.mark.parametrize("specialize", [True, False])
def test_cortical_network_spike_exact_to_horizon(specialize):
    """The cortical channel set (Na, Kd, M, L-Ca, leak; exponential Euler in
    V at dt = 0.1 ms) in the network kernel: the compiled variant and the
    run-time interpreter, spike-exact to the predictability horizon against
    the oracle, with one-step delays and background input."""
    print_case("cortical network specialize=%s" % specialize)
    m = W.with_synapses(W.custom_channels(dt=0.1, v_method="ee"))
    n, T = 1200, 1500
    csr = W.net_csr(n=n, fan_out=120, seed=14, inh_scale=4.0)
    v0 = W.net_v0(n, 14).astype(np.float64)
    scale = 0.3
    bg = (2.0, 3.0, 2.0)  # about 40 Hz
    raster, _ = _batch_gpu(m, csr, scale, v0, T, 1, specialize=specialize,
                           background=bg + (15,))
    kw = dict(background=bg, in_seed=15)
    h, ref = _horizon_kw(m, csr, scale, v0, T, kw)
    assert ref.sum() > 10 * n * T * 1e-4, ref.sum()
    # the oracle's own raster first changes under the probes near step 600
    # of this faster-firing network: several thousand spikes lie before it
    assert h >= 400, h
    assert ref[:h].sum() > 1000
    bad = spike_mismatch(raster[:h - 1], ref[:h - 1])
    print("cortical horizon %d of %d, spikes %d, mismatched %d" % (h, T, int(ref.sum()), len(bad)),
          flush=True)
    assert len(bad) == 0


@pytest.mark.parametrize("blocks", [8, 75, 149])
def test_barrier_probe_modes_odd_and_even_grids(blocks):
    """The barrier probe in its three modes, on grids whose barrier area is
    not a multiple of 8 bytes long (the accumulators after it must still be
    aligned for the 64-bit atomics of mode 1); every barrier completes."""
    print_case("barrier probe blocks=%d" % blocks)
    torch = need_gpu()
    from paper_2601_21407_amd import probe as PR
    work = None
    flags_at = ((256 + blocks) * 4 + 255) // 256 * 256  # the flags follow the barrier words
    for mode in (0, 1, 2):
        work = PR.probe_barrier(50, blocks, mode, work)
        torch.cuda.synchronize()
        flags = work[flags_at:flags_at + 8].cpu().numpy().view(np.int32)
        assert flags[1] == 0, (mode, flags)  # no barrier timed out
