"""GPU check of sdnn_mse_noalloc, the MSE entry point that allocates nothing (its
per-workgroup partial sums live in a static device array): through the C ABI it
must give exactly what sdnn_mse gives, on two calls in a row, the second on a
smaller input, and both must match the FP64 oracle's MSE."""
import ctypes

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
DEV = "cuda:0"

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2004_10908_amd as P
    P.lib()
    return P


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _call(P, name, y, t, dy, loss):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = getattr(P.lib(), name)(_ptr(y), _ptr(t), ctypes.c_int64(y.numel()), _ptr(dy), _ptr(loss), stream)
    assert st == 0, P.lib().sdnn_last_error()


def test_noalloc_mse_equals_mse_on_two_calls(P):
    rng = np.random.default_rng(11)
    for n in (1_000_003, 777):                     # the second call on a smaller input
        print(f"sdnn_mse_noalloc vs sdnn_mse, n = {n}", flush=True)
        yh = rng.normal(size=n).astype(np.float32)
        th = rng.normal(size=n).astype(np.float32)
        y, t = torch.from_numpy(yh).to(DEV), torch.from_numpy(th).to(DEV)
        dy_a, dy_b = torch.full_like(y, np.nan), torch.full_like(y, np.nan)
        loss_a = torch.full((257,), np.nan, device=DEV)          # sdnn_mse: loss[0] + 256 partials
        loss_b = torch.full((1,), np.nan, device=DEV)            # sdnn_mse_noalloc: loss[0] only
        _call(P, "sdnn_mse", y, t, dy_a, loss_a)
        _call(P, "sdnn_mse_noalloc", y, t, dy_b, loss_b)
        torch.cuda.synchronize()
        assert torch.equal(dy_a, dy_b)
        assert torch.equal(loss_a[:1], loss_b)
        rl, rdy = oracle.mse(yh, th)
        assert abs(float(loss_b.item()) - rl) <= 1e-5 * rl
        np.testing.assert_allclose(dy_b.cpu().numpy(), rdy, rtol=1e-5, atol=1e-9)


def test_noalloc_mse_optional_outputs_and_errors(P):
    y = torch.rand(5000, device=DEV)
    t = torch.rand(5000, device=DEV)
    loss = torch.full((1,), np.nan, device=DEV)
    _call(P, "sdnn_mse_noalloc", y, t, None, loss)             # loss only
    dy = torch.full_like(y, np.nan)
    _call(P, "sdnn_mse_noalloc", y, t, dy, None)               # gradient only
    torch.cuda.synchronize()
    ref = float(((y.double() - t.double()) ** 2).mean())
    assert abs(float(loss.item()) - ref) <= 1e-5 * ref
    assert torch.allclose(dy, 2 * (y - t) / y.numel(), rtol=1e-6, atol=0)
    lib = P.lib()
    assert lib.sdnn_mse_noalloc(None, None, ctypes.c_int64(-1), None, None, None) == P.sdnn.SDNN_EINVAL
    assert lib.sdnn_mse_noalloc(None, None, ctypes.c_int64(10), None, _ptr(loss), None) == P.sdnn.SDNN_EINVAL
