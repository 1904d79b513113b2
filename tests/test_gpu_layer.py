"""GPU parity of the differentiable HH layer: MFMA input projection and its
weight gradient, the BPTT adjoint (hh_backward) with surrogate spike
derivative and checkpoint re-computation, readout + cross entropy and Adam,
each through the C ABI against the FP64 oracle.

Adjoint tolerances (16 neurons x 20 steps against FP64 central finite
differences of the smooth-output loss, whose exact gradient the surrogate
gradient equals because the trajectory does not depend on the output):
normwise relative error <= 1e-4, and per component
|g_gpu - g_fd| <= 1e-3 |g_fd| + 1e-5 max|g_fd|.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_21407_amd import workloads as W
from tests.gpu_util import need_gpu, print_case

pytestmark = pytest.mark.gpu


def _bf16_tensor(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x, np.float32), device="cuda").to(torch.bfloat16)


@pytest.mark.parametrize("M,N,K,binary", [(300, 200, 70, False), (129, 1025, 33, True),
                                          (1, 1, 1, False), (640, 256, 700, True),
                                          (257, 129, 36, False), (0, 5, 7, False),
                                          (3, 4, 0, False), (4100, 300, 701, True)])
def test_projection_forward_and_wgrad_small(M, N, K, binary):
    print_case("proj M=%d N=%d K=%d" % (M, N, K))
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(M + N + K)
    A = (rng.random((M, K)) < 0.05).astype(np.float32) if binary else rng.standard_normal((M, K))
    Wt = rng.standard_normal((K, N))
    A16, W16 = W.bf16_round(A), W.bf16_round(Wt)
    out = torch.empty((M, N), device="cuda")
    # the library takes the weights transposed, Wt [N][K]
    hh.proj_forward(_bf16_tensor(A16), _bf16_tensor(W16.T), out)
    ref = O.projection(A16, W16)
    scale = np.abs(A16.astype(np.float64)) @ np.abs(W16.astype(np.float64))
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-6 * scale + 1e-30)
    dO = rng.standard_normal((M, N)).astype(np.float32)
    dWt = torch.empty((N, K), device="cuda")
    hh.proj_wgrad(_bf16_tensor(A16), torch.tensor(dO, device="cuda"), dWt)
    refw = O.projection_weight_grad(A16, dO)
    scw = np.abs(A16.astype(np.float64)).T @ np.abs(dO.astype(np.float64))
    # dOut enters as bf16 hi + lo parts: ~2^-16 relative per term
    assert np.all(np.abs(dWt.cpu().numpy().T - refw) <= 2e-5 * scw + 1e-30)


@pytest.mark.parametrize("M,N,K", [(300, 200, 70), (129, 1025, 33), (1, 1, 1), (640, 256, 700),
                                   (257, 129, 32), (513, 130, 64), (3, 4, 0), (0, 5, 7)])
def test_projection_forward_bits(M, N, K):
    """Spike input given as bits: the product equals the oracle's on the
    unpacked 0/1 matrix, and the bf16-input kernel's result."""
    print_case("proj bits M=%d N=%d K=%d" % (M, N, K))
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(7 * M + N + K)
    A = (rng.random((M, K)) < 0.1).astype(np.float32)
    W16 = W.bf16_round(rng.standard_normal((K, N)))
    bits = W.pack_bits(A) if M > 0 else np.zeros((0, max(1, (K + 31) // 32)), np.int32)
    if bits.shape[1] == 0:
        bits = np.zeros((M, 1), np.int32)
    # junk in the bits past K must be ignored
    if K % 32:
        bits = bits.copy()
        bits[:, -1] |= np.int32(-1 << (K % 32)) if K % 32 else 0
    out = torch.empty((M, N), device="cuda")
    Wt = _bf16_tensor(W16.T)
    hh.proj_forward_bits(torch.tensor(bits, device="cuda"), K, Wt, out)
    ref = O.projection(A, W16)
    scale = np.abs(A.astype(np.float64)) @ np.abs(W16.astype(np.float64))
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-6 * scale + 1e-30)
    if M > 0 and K > 0:
        out2 = torch.empty((M, N), device="cuda")
        hh.proj_forward(_bf16_tensor(A), Wt, out2)
        # same products, same tile order: identical
        assert torch.equal(out, out2)
    # weight gradient from bits packed along M (junk past M ignored)
    dO = rng.standard_normal((M, N)).astype(np.float32)
    bT = W.pack_bits_cols(A) if M > 0 else np.zeros((1, K), np.int32)
    if M % 32:
        bT = bT.copy()
        bT[-1, :] |= np.int32(-1 << (M % 32))
    dWt = torch.empty((N, K), device="cuda")
    hh.proj_wgrad_bits(torch.tensor(bT, device="cuda"), M, torch.tensor(dO, device="cuda"), dWt)
    refw = O.projection_weight_grad(A, dO)
    scw = np.abs(A.astype(np.float64)).T @ np.abs(dO.astype(np.float64))
    assert np.all(np.abs(dWt.cpu().numpy().T - refw) <= 2e-5 * scw + 1e-30)
    if M > 0 and K > 0:
        dWt2 = torch.empty((N, K), device="cuda")
        hh.proj_wgrad(_bf16_tensor(A), torch.tensor(dO, device="cuda"), dWt2)
        assert torch.equal(dWt, dWt2)


@pytest.mark.parametrize("M,N,K", [(700, 130, 1000), (2100, 64, 1601)])
def test_weight_gradient_wide_K(M, N, K):
    """K wider than one block's column span (768): the column blocks of the
    weight gradient, for spike bits and bf16 input, match the oracle and each
    other exactly."""
    print_case("wgrad wide K M=%d N=%d K=%d" % (M, N, K))
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(M + K)
    A = (rng.random((M, K)) < 0.05).astype(np.float32)
    dO = rng.standard_normal((M, N)).astype(np.float32)
    dWt = torch.empty((N, K), device="cuda")
    hh.proj_wgrad_bits(torch.tensor(W.pack_bits_cols(A), device="cuda"), M,
                       torch.tensor(dO, device="cuda"), dWt)
    refw = O.projection_weight_grad(A, dO)
    scw = np.abs(A.astype(np.float64)).T @ np.abs(dO.astype(np.float64))
    assert np.all(np.abs(dWt.cpu().numpy().T - refw) <= 2e-5 * scw + 1e-30)
    dWt2 = torch.empty((N, K), device="cuda")
    hh.proj_wgrad(_bf16_tensor(A), torch.tensor(dO, device="cuda"), dWt2)
    assert torch.equal(dWt, dWt2)


def test_projection_full_size_sampled():
    """S [250*256 x 700] Bernoulli spikes x W_in [700 x 1024] bf16."""
    print_case("proj full 64000 x 1024 x 700")
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    S, labels = W.layer_inputs()
    T, B, n_in = S.shape
    A = S.reshape(T * B, n_in).astype(np.float32)
    Win, _, _, _ = W.layer_params()
    W16 = W.bf16_round(Win)
    At = _bf16_tensor(A)
    out = torch.empty((T * B, 1024), device="cuda")
    hh.proj_forward(At, _bf16_tensor(W16.T), out)
    rows = np.random.default_rng(0).choice(T * B, 400, replace=False)
    ref = O.projection(A[rows], W16)
    scale = np.abs(A[rows]) @ np.abs(W16.astype(np.float64))
    got = out.cpu().numpy()[rows]
    assert np.all(np.abs(got - ref) <= 1e-6 * scale + 1e-30)
    # the bit-packed spike input gives the identical product
    outb = torch.empty_like(out)
    hh.proj_forward_bits(torch.tensor(W.pack_bits(A), device="cuda"), n_in, _bf16_tensor(W16.T), outb)
    assert torch.equal(out, outb)
    # weight gradient of the same shapes, checked on a column block
    dO = np.random.default_rng(1).standard_normal((T * B, 1024)).astype(np.float32) * 1e-3
    dWt = torch.empty((1024, n_in), device="cuda")
    hh.proj_wgrad(At, torch.tensor(dO, device="cuda"), dWt)
    cols = slice(0, 1024, 37)
    refw = O.projection_weight_grad(A, dO[:, cols])
    scw = np.abs(A).T @ np.abs(dO[:, cols].astype(np.float64))
    assert np.all(np.abs(dWt.cpu().numpy()[cols, :].T - refw) <= 2e-5 * scw + 1e-30)


def _bwd_case(n=16, T=20, seed=0, B=1):
    m = W.classic_hh(dt=0.025)
    rng = np.random.default_rng(seed)
    N = n // B
    I = (8.0 + 6.0 * rng.standard_normal((T, n))).astype(np.float32)
    cm = (0.8 + 0.4 * rng.random(N)).astype(np.float32)
    v0 = (-65.0 + 30.0 * rng.random(n)).astype(np.float32)
    return m, I, cm, v0, rng


def _gpu_bwd(m, I, cm, v0, ckpt_every, dlevel=None, dV=None, B=1, beta=0.2, specialize=True):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    T, n = I.shape
    N = n // B
    cm_t = torch.tensor(cm, device="cuda")
    M = hh.Model(m, N, B, cm=cm_t)
    M.set_specialize(specialize)
    st = M.new_state()
    M.init_state(st, v0=torch.tensor(v0, device="cuda"))
    x0 = st.clone()
    nck = (T + ckpt_every - 1) // ckpt_every
    ck = torch.zeros((nck, M.n_state, n), device="cuda")
    lv = torch.zeros(n, device="cuda")
    It = torch.tensor(I, device="cuda")
    M.step_n(st, T, i_dense=It, ckpt=ck, ckpt_every=ckpt_every, level=lv)
    dI = torch.zeros((T, n), device="cuda")
    dC = torch.zeros(N, device="cuda")
    dx0 = torch.zeros((M.n_state, n), device="cuda")
    M.backward(ck, ckpt_every, It, T, dI,
               dL_dlevel=None if dlevel is None else torch.tensor(dlevel.astype(np.float32), device="cuda"),
               dL_dV=None if dV is None else torch.tensor(dV.astype(np.float32), device="cuda"),
               beta=beta, dCm=dC, dx0=dx0)
    assert M.check()[0] == 0
    return (dI.cpu().numpy(), dC.cpu().numpy(), dx0.cpu().numpy(), lv.cpu().numpy(),
            x0.cpu().numpy())


def _check_grad(g, ref, what):
    g = np.asarray(g, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nrm = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)
    comp = np.abs(g - ref) <= 1e-3 * np.abs(ref) + 1e-5 * np.max(np.abs(ref))
    print("%s: normwise %.2e, components ok %d/%d" % (what, nrm, comp.sum(), comp.size), flush=True)
    assert nrm <= 1e-4, (what, nrm)
    assert comp.all(), (what, np.nonzero(~comp)[0][:10])


@pytest.mark.parametrize("ckpt_every", [1, 7, 20, 50])
@pytest.mark.parametrize("specialize", [True, False])
def test_adjoint_against_finite_differences(ckpt_every, specialize):
    """16 neurons x 20 steps; loss linear in the smooth spike output and in V."""
    print_case("adjoint FD ckpt=%d specialize=%s" % (ckpt_every, specialize))
    m, I, cm, v0, rng = _bwd_case()
    T, n = I.shape
    cr = rng.standard_normal(n)
    cv = rng.standard_normal((T, n)) * 0.01
    dI, dC, dx0, _, x0 = _gpu_bwd(m, I, cm, v0, ckpt_every, dlevel=cr, dV=cv, specialize=specialize)
    st0 = O.init_state(m, v0.astype(np.float64))
    I64 = I.astype(np.float64)
    cm64 = cm.astype(np.float64)

    def loss(I_, cm_, st_):
        r, _, _, _ = O.bptt(m, st_, I_, cm=cm_, dL_dr=cr, smooth=True)
        v = O.run(m, st_.copy(), T, i_dense=I_, cm=cm_, record_v=True, record_spikes=False)["v"]
        return float(cr @ r + np.sum(cv * v))
    h = 1e-5
    fdI = np.zeros((T, n))
    for t in range(T):
        for i in range(n):
            Ip, Im = I64.copy(), I64.copy()
            Ip[t, i] += h
            Im[t, i] -= h
            fdI[t, i] = (loss(Ip, cm64, st0) - loss(Im, cm64, st0)) / (2 * h)
    _check_grad(dI, fdI, "dL/dI")
    fdC = np.zeros(n)
    for i in range(n):
        cp, cmn = cm64.copy(), cm64.copy()
        cp[i] += h
        cmn[i] -= h
        fdC[i] = (loss(I64, cp, st0) - loss(I64, cmn, st0)) / (2 * h)
    _check_grad(dC, fdC, "dL/dC_m")
    # the FP64 oracle adjoint agrees with the same finite differences
    _, oI, oC, ox0 = O.bptt(m, st0, I64, cm=cm64, dL_dr=cr, dL_dV=cv, smooth=True)
    assert np.linalg.norm(oI - fdI) / np.linalg.norm(fdI) < 1e-6
    _check_grad(dx0[:4], ox0, "dL/dx0")


def test_adjoint_against_oracle_batched_two_level():
    """2 x 512 neurons (C_m shared over the batch) x 250 steps, checkpoints
    every 50 steps (two-level replay), level-output surrogate gradient."""
    print_case("adjoint vs oracle 1024 x 250 ckpt 50")
    m, I, cm, v0, rng = _bwd_case(n=1024, T=250, seed=3, B=2)
    T, n = I.shape
    dlevel = rng.standard_normal(n)
    dI, dC, dx0, lv, _ = _gpu_bwd(m, I, cm, v0, 50, dlevel=dlevel, B=2)
    st0 = O.init_state(m, v0.astype(np.float64))
    cmn = np.tile(cm.astype(np.float64), 2)
    r, oI, oC, ox0 = O.bptt(m, st0, I.astype(np.float64), cm=cmn, dL_dr=dlevel, smooth=False)
    # the forward level counts match where the trajectories do
    same = np.abs(lv - r * T) == 0
    assert same.mean() > 0.97
    # per-neuron relative error of the gradient sequence, over neurons whose
    # spike counts agree
    num = np.linalg.norm(dI - oI, axis=0)
    den = np.maximum(np.linalg.norm(oI, axis=0), 1e-12)
    rel = num / den
    good = same & (den > 1e-9)
    print("adjoint rel err median %.2e p99 %.2e max %.2e over %d neurons"
          % (np.median(rel[good]), np.percentile(rel[good], 99), rel[good].max(), good.sum()))
    assert np.percentile(rel[good], 99) < 1e-3
    assert np.median(rel[good]) < 1e-4
    oCs = oC.reshape(2, -1).sum(0)
    relc = np.abs(dC - oCs) / np.maximum(np.abs(oCs), 1e-9)
    assert np.median(relc) < 1e-3


def test_adjoint_full_size_sampled():
    """The configured layer at full size: 256 x 1,024 HH units (262,144
    neurons) x 250 steps, checkpoints every 50 steps, level-output surrogate
    gradient, dense input of the layer's mean drive (10 + 6 z uA/cm^2).  The
    oracle's BPTT runs on every batch copy of 8 hidden units (2,048 neurons):
    their dL/dI sequences per neuron and the 8 units' dL/dC_m (summed over the
    batch) are compared."""
    print_case("adjoint full size 262144 x 250 ckpt 50, 2048 sampled")
    need_gpu()
    m = W.classic_hh(dt=0.025)
    N, B, T = 1024, 256, 250
    n = N * B
    rng = np.random.default_rng(31)
    I = (10.0 + 6.0 * rng.standard_normal((T, n))).astype(np.float32)
    cm = (0.8 + 0.4 * rng.random(N)).astype(np.float32)
    v0 = (-65.0 + 30.0 * rng.random(n)).astype(np.float32)
    dlevel = rng.standard_normal(n)
    dI, dC, dx0, lv, _ = _gpu_bwd(m, I, cm, v0, 50, dlevel=dlevel, B=B)
    units = np.array([0, 1, 137, 400, 511, 512, 777, 1023])
    cols = (np.arange(B)[:, None] * N + units[None, :]).ravel()
    st0 = O.init_state(m, v0[cols].astype(np.float64))
    r, oI, oC, _ = O.bptt(m, st0, np.ascontiguousarray(I[:, cols].astype(np.float64)),
                          cm=cm[cols % N].astype(np.float64), dL_dr=dlevel[cols], smooth=False)
    same = np.abs(lv[cols] - r * T) == 0
    assert same.mean() > 0.97, same.mean()
    g = dI[:, cols]
    rel = np.linalg.norm(g - oI, axis=0) / np.maximum(np.linalg.norm(oI, axis=0), 1e-12)
    good = same & (np.linalg.norm(oI, axis=0) > 1e-9)
    print("full-size adjoint rel err median %.2e p99 %.2e over %d neurons"
          % (np.median(rel[good]), np.percentile(rel[good], 99), good.sum()), flush=True)
    assert good.sum() > 1500
    assert np.percentile(rel[good], 99) < 1e-3 and np.median(rel[good]) < 1e-4
    # dC_m of a unit sums its 256 batch copies (all of them sampled)
    oCu = oC.reshape(B, len(units)).sum(0)
    relc = np.abs(dC[units] - oCu) / np.maximum(np.abs(oCu), 1e-9)
    print("dC_m rel err per unit", relc, flush=True)
    assert np.median(relc) < 1e-3


def test_adjoint_checkpoint_strides_agree():
    """The same gradient from checkpoint strides 1, 10 and 50 (the replay
    reproduces the forward trajectory)."""
    m, I, cm, v0, rng = _bwd_case(n=256, T=120, seed=5)
    dlevel = rng.standard_normal(256)
    outs = [_gpu_bwd(m, I, cm, v0, s, dlevel=dlevel)[0] for s in (1, 10, 50)]
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) <= 1e-6 * np.max(np.abs(outs[0]))


def test_adjoint_in_parts_equals_whole():
    """hh_backward_part over adjacent ranges, from the end backwards, gives
    the single call's dI, dC_m and dx0 bit for bit (the adjoint and the dC_m
    partials carried in the workspace)."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    m, I, cm, v0, rng = _bwd_case(n=300, T=130, seed=9, B=3)
    dlevel = rng.standard_normal(300).astype(np.float32)
    dV = (0.01 * rng.standard_normal(I.shape)).astype(np.float32)
    dI, dC, dx0, _, _ = _gpu_bwd(m, I, cm, v0, 20, dlevel=dlevel, dV=dV, B=3)
    T, n = I.shape
    M = hh.Model(m, n // 3, 3, cm=torch.tensor(cm, device="cuda"))
    st = M.new_state()
    M.init_state(st, v0=torch.tensor(v0, device="cuda"))
    ck = torch.zeros(((T + 19) // 20, M.n_state, n), device="cuda")
    It = torch.tensor(I, device="cuda")
    M.step_n(st, T, i_dense=It, ckpt=ck, ckpt_every=20)
    dI2 = torch.zeros((T, n), device="cuda")
    dC2 = torch.zeros(n // 3, device="cuda")
    dx02 = torch.zeros((M.n_state, n), device="cuda")
    ws = torch.empty(M.backward_workspace(20, T), dtype=torch.uint8, device="cuda")
    kw = dict(workspace=ws, dL_dlevel=torch.tensor(dlevel, device="cuda"),
              dL_dV=torch.tensor(dV, device="cuda"), dCm=dC2, dx0=dx02)
    for lo, hi in ((120, 130), (60, 120), (40, 60), (0, 40)):
        M.backward_part(ck, 20, It, T, lo, hi, dI2, **kw)
    assert M.check()[0] == 0
    assert np.array_equal(dI2.cpu().numpy(), dI)
    assert np.array_equal(dC2.cpu().numpy(), dC)
    assert np.array_equal(dx02.cpu().numpy(), dx0)
    # ranges that are not segment aligned are refused
    with pytest.raises(hh.HHError):
        M.backward_part(ck, 20, It, T, 10, 130, dI2, **kw)


def test_weight_gradient_accumulates_over_row_ranges():
    """The spike-input weight gradient over row ranges with accumulate equals
    one call over all rows (to rounding: the split of the sum differs)."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(12)
    M, N, K = 3000, 300, 100
    A = (rng.random((M, K)) < 0.1).astype(np.float32)
    dO = rng.standard_normal((M, N)).astype(np.float32)
    bT = torch.tensor(W.pack_bits_cols(A), device="cuda")
    dOt = torch.tensor(dO, device="cuda")
    whole = torch.empty((N, K), device="cuda")
    hh.proj_wgrad_bits(bT, M, dOt, whole)
    acc = torch.full((N, K), 123.0, device="cuda")
    for i, (lo, hi) in enumerate(((2048, 3000), (1024, 2048), (0, 1024))):
        hh.proj_wgrad_bits(bT, hi - lo, dOt[lo:hi].contiguous(), acc, accumulate=i > 0, m0=lo)
    ref = O.projection_weight_grad(A, dO)
    scw = np.abs(A).T @ np.abs(dO.astype(np.float64))
    assert np.all(np.abs(acc.cpu().numpy().T - ref) <= 2e-5 * scw + 1e-30)
    assert np.all(np.abs(acc.cpu().numpy() - whole.cpu().numpy()).T <= 2e-5 * scw + 1e-30)


def test_readout_ce_against_oracle():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(7)
    B, H, C, T = 37, 300, 20, 250
    level = rng.integers(0, 40, (B, H)).astype(np.float32)
    Wo = (rng.standard_normal((H, C)) / np.sqrt(H)).astype(np.float32)
    b = (0.1 * rng.standard_normal(C)).astype(np.float32)
    lab = rng.integers(0, C, B).astype(np.int32)
    dev = lambda x: torch.tensor(x, device="cuda")
    dl = torch.empty((B, H), device="cuda")
    dW = torch.empty((H, C), device="cuda")
    db = torch.empty(C, device="cuda")
    loss = torch.empty(1, device="cuda")
    logits = torch.empty((B, C), device="cuda")
    hh.readout_ce(dev(level), T, dev(Wo), dev(b), dev(lab), dl, dW, db, loss, logits)
    L, dr, gW, gb, z = O.readout_ce(level.astype(np.float64) / T, Wo, b, lab)
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    assert np.allclose(logits.cpu().numpy(), z, rtol=1e-5, atol=1e-6)
    # dL/dr, the rate gradient the adjoint takes
    assert np.allclose(dl.cpu().numpy(), dr, rtol=1e-4, atol=1e-9)
    assert np.allclose(dW.cpu().numpy(), gW, rtol=1e-4, atol=1e-8)
    assert np.allclose(db.cpu().numpy(), gb, rtol=1e-4, atol=1e-8)


def test_adam_against_oracle():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    rng = np.random.default_rng(8)
    n = 100003
    p = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n)
    v = np.zeros(n)
    tp, tm, tv = (torch.tensor(x, device="cuda") for x in (p, np.zeros(n, np.float32), np.zeros(n, np.float32)))
    p16 = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    pr = p.astype(np.float64)
    for step in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        hh.adam_step(tp, torch.tensor(g, device="cuda"), tm, tv, step, 1e-2, param_bf16=p16)
        pr, m, v = O.adam_step(pr, g.astype(np.float64), m, v, step, 1e-2)
    assert np.allclose(tp.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    assert np.array_equal(p16.float().cpu().numpy(), W.bf16_round(tp.cpu().numpy()))


def test_autograd_function_routes_the_adjoint():
    """HHFunction: r from the level output, and torch autograd delivers the
    adjoint's dI, dx0 and dC_m, equal to the oracle's BPTT."""
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    from paper_2601_21407_amd.autograd import HHFunction
    print_case("autograd function 2 x 128 x 120 ckpt 40")
    m, I, cm, v0, rng = _bwd_case(n=256, T=120, seed=9, B=2)
    T, n = I.shape
    cm_t = torch.tensor(cm, device="cuda", requires_grad=True)
    M = hh.Model(m, n // 2, 2, cm=cm_t.detach())
    x0 = M.new_state()
    M.init_state(x0, v0=torch.tensor(v0, device="cuda"))
    It = torch.tensor(I, device="cuda", requires_grad=True)
    x0r = x0.clone().requires_grad_(True)
    wvec = torch.tensor(rng.standard_normal(n).astype(np.float32), device="cuda")
    r = HHFunction.apply(It, x0r, cm_t, M, 40, 0.2)
    (r * wvec).sum().backward()
    # the same calls made directly
    dI, dC, dx0, lv, _ = _gpu_bwd(m, I, cm, v0, 40, dlevel=wvec.cpu().numpy(), B=2)
    assert np.allclose(r.detach().cpu().numpy(), lv / T, rtol=1e-6, atol=0)  # r = level / T
    assert np.array_equal(It.grad.cpu().numpy(), dI)
    assert np.array_equal(x0r.grad.cpu().numpy(), dx0)
    assert np.array_equal(cm_t.grad.cpu().numpy(), dC)
    # and against the oracle
    st0 = O.init_state(m, v0.astype(np.float64))
    ro, oI, oC, _ = O.bptt(m, st0, I.astype(np.float64), cm=np.tile(cm.astype(np.float64), 2),
                           dL_dr=wvec.cpu().numpy().astype(np.float64), smooth=False)
    same = np.abs(lv - ro * T) == 0  # neurons whose level counts agree
    assert same.mean() > 0.97
    rel = np.linalg.norm((dI - oI)[:, same]) / max(np.linalg.norm(oI[:, same]), 1e-12)
    assert rel < 1e-3, rel
