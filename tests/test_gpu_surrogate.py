"""GPU checks of the learned surrogate: the MLP training kernel's loss and
gradient against the FP64 oracle (and against an FP64 emulation of the bf16
rounding it applies), the MFMA inference against the VALU forward, the
deployment kernel's plumbing against the plain integrator, and a short
end-to-end training run whose deployment is judged by the plain integrator.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import need_gpu, print_case

pytestmark = pytest.mark.gpu


def _rand_params(rng):
    ps = []
    for a, b in ((7, 64), (64, 64), (64, 6)):
        ps += [rng.standard_normal((a, b)) / np.sqrt(a), 0.1 * rng.standard_normal(b)]
    return ps


def _flat(ps):
    return np.concatenate([p.reshape(-1) for p in ps]).astype(np.float32)


def _unflat(v):
    out, off = [], 0
    for a, b in ((7, 64), (64, 64), (64, 6)):
        out.append(v[off: off + a * b].reshape(a, b))
        off += a * b
        out.append(v[off: off + b])
        off += b
    return out


def _bf(x):
    return W.bf16_round(np.asarray(x, np.float32)).astype(np.float64)


@pytest.mark.parametrize("S", [1, 100, 1000, 70001])
def test_mlp_grad_matches_oracle(S):
    print_case("mlp grad S=%d" % S)
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(S)
    flat = _flat(_rand_params(rng))
    X = rng.standard_normal((S, 7)).astype(np.float32)
    Y = rng.standard_normal((S, 6)).astype(np.float32)
    dev = lambda a: torch.tensor(a, device="cuda")
    g = torch.zeros(hh.MLP_NPARAM, device="cuda")
    loss = torch.zeros(1, device="cuda")
    hh.mlp_grad(dev(flat), dev(X), dev(Y), g, loss, quantize=False)
    ps = _unflat(flat.astype(np.float64))
    y, cache = O.mlp_forward(ps, X)
    L, dy = O.mse_loss_grad(y, Y)
    grads, _ = O.mlp_backward(ps, cache, dy)
    ref = np.concatenate([q.reshape(-1) for q in grads])
    got = g.cpu().numpy()
    assert abs(loss.item() - L) <= 1e-5 * L
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    # the plain forward
    Yg = torch.empty((S, 6), device="cuda")
    hh.mlp_forward(dev(flat), dev(X), Yg, quantize=False)
    assert np.allclose(Yg.cpu().numpy(), y, rtol=1e-5, atol=1e-5)


def test_mlp_grad_quantized_matches_emulation():
    """quantize=1: weights, hidden activations and the input split rounded to
    bf16 exactly as the MFMA inference does; compared with an FP64 emulation
    of those roundings (straight-through gradient)."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(3)
    S = 3000
    flat = _flat(_rand_params(rng))
    X = rng.standard_normal((S, 7)).astype(np.float32)
    Y = rng.standard_normal((S, 6)).astype(np.float32)
    dev = lambda a: torch.tensor(a, device="cuda")
    g = torch.zeros(hh.MLP_NPARAM, device="cuda")
    loss = torch.zeros(1, device="cuda")
    hh.mlp_grad(dev(flat), dev(X), dev(Y), g, loss, quantize=True)
    W1, b1, W2, b2, W3, b3 = _unflat(flat.astype(np.float64))
    W1q, W2q, W3q = _bf(W1), _bf(W2), _bf(W3)
    xh = _bf(X)
    xq = xh + _bf(X - xh)
    a1 = xq @ W1q + b1
    h1 = _bf(O.silu(a1))
    a2 = h1 @ W2q + b2
    h2 = _bf(O.silu(a2))
    y = h2 @ W3q + b3
    L, dy = O.mse_loss_grad(y, Y)
    gW3 = h2.T @ dy
    dA2 = (dy @ W3q.T) * O.dsilu(a2)
    gW2 = h1.T @ dA2
    dA1 = (dA2 @ W2q.T) * O.dsilu(a1)
    gW1 = xq.T @ dA1
    ref = np.concatenate([gW1.reshape(-1), dA1.sum(0), gW2.reshape(-1), dA2.sum(0),
                          gW3.reshape(-1), dy.sum(0)])
    got = g.cpu().numpy()
    assert abs(loss.item() - L) <= 1e-4 * L
    # bf16 roundings of activations can differ where FP32 and FP64 straddle a
    # rounding boundary: compare normwise
    assert np.linalg.norm(got - ref) <= 2e-3 * np.linalg.norm(ref)


@pytest.mark.parametrize("S", [64, 1000, 4097])
def test_mfma_inference_matches_valu_forward(S):
    """The register-resident MFMA inference (packed fragments, transposed
    activations) equals the quantized VALU forward up to accumulation order."""
    print_case("mfma infer S=%d" % S)
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(S + 1)
    flat = _flat(_rand_params(rng))
    mu = np.array([-60, 0.05, 0.6, 0.3, 0.05, 0.01, 5], np.float32)
    sd = np.array([5, 0.02, 0.1, 0.1, 0.02, 0.005, 3], np.float32)
    Xraw = (mu + sd * rng.standard_normal((S, 7))).astype(np.float32)
    norm = np.zeros(32, np.float32)
    norm[0:7], norm[8:15] = mu, sd
    norm[16:22] = 0.01 * rng.standard_normal(6)
    norm[24:30] = 0.1 + rng.random(6)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")
    packed = hh.mlp_pack(dev(flat), dev(norm))
    Y = torch.empty((S, 6), device="cuda")
    hh.mlp_infer(packed, dev(Xraw), Y)
    Xn = ((Xraw - mu) / sd).astype(np.float32)
    Yr = torch.empty((S, 6), device="cuda")
    hh.mlp_forward(dev(flat), dev(Xn), Yr, quantize=True)
    ref = Yr.cpu().numpy() * norm[24:30] + norm[16:22]
    got = Y.cpu().numpy()
    err = np.abs(got - ref) / (norm[24:30])
    print("mfma vs valu: max normalized error %.2e" % err.max())
    assert err.max() < 2e-2 and np.median(err) < 2e-3


def _packed_random(torch, hh, scale=1e-3):
    rng = np.random.default_rng(11)
    flat = _flat(_rand_params(rng))
    norm = np.zeros(32, np.float32)
    norm[0:7] = [-62, 0.05, 0.6, 0.3, 0.05, 0.01, 5]
    norm[8:15] = [5, 0.02, 0.1, 0.1, 0.02, 0.005, 3]
    norm[24:30] = scale
    return hh.mlp_pack(torch.tensor(flat, device="cuda"), torch.tensor(norm, device="cuda"))


@pytest.mark.parametrize("n", [1000, 70000])
def test_deployment_all_plain_equals_plain_kernel(n):
    """With the fallback threshold below every V the deployment kernel runs
    only plain steps through its compaction pool: states and spikes equal the
    plain fused kernel bit for bit."""
    print_case("surrogate all-plain n=%d" % n)
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    from paper_2601_21407_amd import surrogate as SG
    packed = _packed_random(torch, hh)
    T = 800
    _, st_s, bits_s, stats = SG.deploy(packed, n, T, noise=(5.0, 3.0, 9), v_fallback=-1000.0,
                                       check_every=0)
    _, st_p, bits_p = SG.plain_run(n, T, noise=(5.0, 3.0, 9))
    torch.cuda.synchronize()
    assert torch.equal(st_s, st_p)
    assert torch.equal(bits_s, bits_p)
    assert stats[0].item() == 0 and stats[1].item() == n * T // 10


def test_deployment_surrogate_step_equals_inference():
    """One surrogate call with dense input: every neuron below the threshold
    takes exactly the MFMA inference result for (state, mean current)."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    from paper_2601_21407_amd import surrogate as SG
    packed = _packed_random(torch, hh, scale=1e-2)
    n, k = 3000, 10
    rng = np.random.default_rng(4)
    I = (5.0 + 3.0 * rng.standard_normal((k, n))).astype(np.float32)
    It = torch.tensor(I, device="cuda")
    M, st, bits, stats = SG.deploy(packed, n, k, i_dense=It, check_every=0, v_fallback=1e6)
    m = W.custom_channels(dt=0.025)
    s0 = O.init_state(m, np.full(n, -65.0))
    X = np.zeros((n, 7), np.float32)
    X[:, 0] = s0[0]
    X[:, 1:6] = s0[1:6].T
    ib = np.zeros(n, np.float32)
    for j in range(k):
        ib = ib + I[j]
    X[:, 6] = ib / np.float32(k)
    # the kernel's initial state is its own p_inf(-65) in FP32
    M2 = hh.Model(m, n)
    s2 = M2.new_state()
    M2.init_state(s2, v0_scalar=-65.0)
    s2n = s2.cpu().numpy()
    X[:, 0] = s2n[0] + s2n[6]
    X[:, 1:6] = s2n[1:6].T
    Y = torch.empty((n, 6), device="cuda")
    hh.mlp_infer(packed, torch.tensor(X, device="cuda"), Y)
    Yn = Y.cpu().numpy()
    got = st.cpu().numpy()
    assert stats[0].item() == n
    assert np.allclose(got[0], X[:, 0] + Yn[:, 0], rtol=0, atol=1e-5)
    assert np.allclose(got[1:6].T, np.clip(X[:, 1:6] + Yn[:, 1:6], 0, 1), rtol=0, atol=1e-6)


def test_train_and_deploy_small():
    """A short training run on trajectories of the plain kernel reduces the
    loss; deployment on 4,096 neurons stays close to the plain integrator."""
    print_case("surrogate train small")
    torch = need_gpu()
    from paper_2601_21407_amd import surrogate as SG
    from paper_2601_21407_amd import hh
    X, dY = SG.generate_transitions(n_traj=400, T=4000, seed=3)
    assert X.shape[0] > 500000
    norm = SG.norm_stats(X, dY)
    params, hist = SG.train(X, dY, norm, epochs=3, batch=8192, lr=3e-3)
    print("loss history", hist)
    assert hist[-1] < 0.5 * hist[0]
    packed = hh.mlp_pack(params, norm)
    n, T = 4096, 2000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(21)
    I = (5.0 + 3.0 * torch.randn((T, n), generator=gen, device="cuda")).contiguous()
    _, _, bits_p = SG.plain_run(n, T, i_dense=I)
    _, _, bits_s, stats = SG.deploy(packed, n, T, i_dense=I)
    torch.cuda.synchronize()
    e = SG.spike_time_error(bits_p.cpu().numpy(), bits_s.cpu().numpy(), n, 0.025, 0.025)
    st = stats.cpu().numpy()
    print("spike-time error", e, "stats", st)
    assert st[0] > st[1]  # most calls use the surrogate
    assert e["unmatched_frac"] < 0.5
