"""The FP32 issue-rate calibration kernels (jt_calibrate_valu) compute what
they claim: the per-lane sums of their eight chains equal a float32 replay of
the same updates on the host (multiplies and fused multiply-adds) or the fixed
point that the transcendental updates reach; and the kernels' time grows with
the rounds they run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2606_01547_amd import Context
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = Context(0)
    yield c
    c.close()


def _sums(ctx, kind, blocks, iters):
    from ctypes import c_void_p
    from paper_2606_01547_amd._native import _check
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    _check(ctx._lib.jt_calibrate_valu(kind, blocks, iters, c_void_p(out.data_ptr()), c_void_p(s.cuda_stream)))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


_F = np.float32


def _fma(a, b, c):
    # one rounding, as the fused multiply-add: the product of two floats is
    # exact in float64 and the sum rounds to float32 (a double rounding is
    # possible in rare ties, far inside the tolerances below)
    return (a.astype(np.float64) * np.float64(b) + np.float64(c)).astype(_F)


def _replay(kind, iters):
    """The eight chains of one block's 256 lanes, replayed in float32."""
    t = np.arange(256)
    a = np.stack([_F(1.0) + _F(1e-3) * _F((t + 31 * i) & 63) for i in range(8)]).astype(_F)
    b, c = _F(0.999), _F(1e-3)
    lane = (t & 1).astype(_F)
    xv = (_F(1e-7) * (_F(1.0) + lane)).astype(_F)
    bv = (b + _F(1e-9) * lane).astype(_F)
    cv = (c - _F(1e-9) * lane).astype(_F)
    rb = _F(1.0) / b
    for _ in range(iters):
        if kind == 0:
            a = _fma(a, b, c)
        elif kind == 2:
            a = _fma(_fma(a, b, c), b, c)
            a[:2] = (1.0 / np.sqrt(a[:2].astype(np.float64))).astype(_F)
        elif kind == 3:
            a = ((a * b).astype(_F) * rb).astype(_F)
        elif kind == 4:
            for i in range(8):
                a[i] = _fma(a[i], _F(_F(0.999) - _F(1e-4) * _F(i)), _F(_F(1e-3) + _F(1e-7) * _F(i)))
        elif kind == 6:
            a = (xv.astype(np.float64)[None, :] * np.float64(b) + a.astype(np.float64)).astype(_F)
        elif kind == 7:
            a = (a.astype(np.float64) * bv.astype(np.float64)[None, :] + cv.astype(np.float64)[None, :]).astype(_F)
    return a.astype(np.float64).sum(0)


def test_chains_match_a_float32_replay(ctx):
    """Kinds built from multiplies and fused multiply-adds are replayed
    exactly; the transcendental kinds (hardware approximations) are checked
    against their fixed points after enough rounds to reach them."""
    for kind, blocks, iters in ((0, 4, 1024), (2, 2, 512), (3, 1, 1024), (4, 2, 1024), (6, 1, 1024), (7, 2, 1024)):
        got = _sums(ctx, kind, blocks, iters).reshape(blocks, 256)
        want = _replay(kind, iters)
        # kind 4 folds its per-chain constants at compile time, where the
        # multiply-add may be contracted (one rounding) or not: one unit in
        # the last place of a slope near 0.999 moves that chain's limit by
        # about 6e-5 of itself
        tol = 2e-4 if kind == 4 else 2e-6
        for blk in range(blocks):
            np.testing.assert_allclose(got[blk], want, rtol=tol, err_msg=f"kind {kind}")
    # a <- a^(-1/2) halves the distance to 1 each round
    np.testing.assert_allclose(_sums(ctx, 1, 2, 200), 8.0, rtol=1e-6)
    # a <- log2(a) + 2 is attracted to 4 (slope 1 / (4 ln 2) there)
    np.testing.assert_allclose(_sums(ctx, 5, 1, 200), 32.0, rtol=1e-5)
    # the accumulating kind grows by about one unit in the last place a step
    t = np.arange(256)
    start = sum(1.0 + 1e-3 * ((t + 31 * i) & 63) for i in range(8))
    assert np.all(_replay(6, 1024) > start + 8 * 1024 * 0.9e-7)


def test_time_grows_with_rounds(ctx):
    short = ctx.calibrate_valu(0, 1024, 1024)
    long_ = ctx.calibrate_valu(0, 1024, 8192)
    assert long_ > 3.0 * short


def test_rejects_bad_arguments(ctx):
    from ctypes import c_void_p
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    for kind, blocks, iters in ((8, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 1, 0)):
        assert ctx._lib.jt_calibrate_valu(kind, blocks, iters, c_void_p(out.data_ptr()), c_void_p(s.cuda_stream)) != 0
