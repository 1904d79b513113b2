"""The allocation-free readout entry point (hh_readout_ce_noalloc) against
the workspace entry point (hh_readout_ce): both run the same kernels, so
every output must agree bit for bit, on two calls in a row (the second with
a smaller problem, which reuses the static scratch left by the first), and
a problem larger than the static scratch is refused without a launch."""
import numpy as np
import pytest

from tests.gpu_util import need_gpu, print_case

pytestmark = pytest.mark.gpu


def _problem(torch, B, H, C, T, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    level = torch.randint(0, T + 1, (B, H), generator=g).float().cuda()
    W = (0.1 * torch.randn(H, C, generator=g)).cuda()
    b = (0.1 * torch.randn(C, generator=g)).cuda()
    lab = torch.randint(0, C, (B,), generator=g, dtype=torch.int32).cuda()
    return level, W, b, lab


def _outputs(torch, B, H, C):
    z = lambda *s: torch.full(s, float("nan"), device="cuda")
    return z(1), z(B, H), z(H, C), z(C), z(B, C)


def _call(hh, fn, args, extra):
    level, T, W, b, lab, B, H, C, outs = args
    loss, dl, dW, db, logits = outs
    p = hh._ptr
    return fn(p(level), T, p(W), p(b), p(lab), B, H, C, p(loss), p(dl), p(dW), p(db), p(logits),
              *extra, hh._stream())


@pytest.mark.parametrize("sizes", [[(300, 1024, 20), (37, 100, 7)]])
def test_noalloc_matches_workspace_entry_point(sizes):
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    fn = hh.lib.hh_readout_ce_noalloc
    T = 250
    for k, (B, H, C) in enumerate(sizes):
        print_case("readout noalloc call %d B=%d H=%d C=%d" % (k, B, H, C))
        level, W, b, lab = _problem(torch, B, H, C, T, seed=11 + k)
        ref, got = _outputs(torch, B, H, C), _outputs(torch, B, H, C)
        ws = torch.empty(int(hh.lib.hh_readout_ce_workspace(B, C)), dtype=torch.uint8, device="cuda")
        rc = _call(hh, hh.lib.hh_readout_ce, (level, T, W, b, lab, B, H, C, ref),
                   (hh._ptr(ws), ws.numel()))
        assert rc == 0
        rc = _call(hh, fn, (level, T, W, b, lab, B, H, C, got), ())
        assert rc == 0
        torch.cuda.synchronize()
        for name, a, c in zip(("loss", "dlevel", "dW", "db", "logits"), ref, got):
            assert torch.isfinite(a).all(), name
            assert torch.equal(a, c), name


def test_noalloc_refuses_oversized_problem():
    torch = need_gpu()
    from paper_2601_21407_amd import hh
    fn = hh.lib.hh_readout_ce_noalloc
    B, H, C, T = 16384, 8, 16, 10  # B (C + 1) = 278,528 > 262,144 floats
    # buffers of the full size, so the arguments are valid in every respect
    # but the scratch limit
    level, W, b, lab = _problem(torch, B, H, C, T, seed=3)
    outs = _outputs(torch, B, H, C)
    p = hh._ptr
    rc = fn(p(level), T, p(W), p(b), p(lab), B, H, C, *(p(o) for o in outs), hh._stream())
    assert rc == -2  # HH_E_SHAPE, nothing launched
    assert all(torch.isnan(o).all() for o in outs)
