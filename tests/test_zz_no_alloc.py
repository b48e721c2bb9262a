"""The allocation-free network gradient (zema_mlp_grad_noalloc) against zema_mlp_grad.

Two calls in a row through the C-ABI, the second with fewer rows, each compared with
the allocating entry point on the same weights and rows:
  * 40,000 rows (2,500 tiles: the scratch's 256 blocks take 10 tiles each, the
    allocating call 625 blocks of 4): loss within 1e-6 relative, gradient within 1e-5
    of its norm and per entry within 1e-5 of the largest entry (FP32 partial sums in
    another grouping; each of the 9,603 entries sums 40,000 FP32 terms);
  * 3,001 rows (a ragged last tile, the same 4-tile blocks as the allocating call):
    loss and gradient bitwise equal, so no partial of the larger first call leaks into
    the second;
  * a third call at the largest size of the bitwise range (16,384 rows) and an
    oversized request rejected with ZEMA_E_ARG before any launch.
"""
import numpy as np
import pytest

import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(*a):
    print(*a, flush=True)


def test_noalloc_gradient_matches_allocating_call():
    _need_gpu()
    from paper_2311_05945_amd import zema
    th = sg.mlp_init(5)
    th[1024:1088] = 0.05
    M = zema.Mlp(th)
    g_out = torch.zeros(zema.MLP_PARAMS, dtype=torch.float32, device="cuda")
    for n, bitwise in ((40000, False), (3001, True), (16384, True)):
        x, t = sg.mlp_batch(7 + n, n)
        xf = torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()
        tf = torch.as_tensor(np.asarray(t, dtype=np.float32), device="cuda").contiguous()
        g_out.fill_(float("nan"))
        torch.cuda.synchronize()
        log(f"noalloc gradient: n={n}")
        loss_n = M.grad_noalloc(xf, tf, g_out)
        loss_a, g_a = M.grad(xf, tf)
        gn, ga = g_out.cpu().numpy(), g_a.cpu().numpy()
        assert np.all(np.isfinite(gn))
        err = np.abs(gn - ga).max()
        log(f"n={n}: loss {loss_n:.9e} vs {loss_a:.9e}, max |g_noalloc - g| {err:.3e} "
            f"(max |g| {np.abs(ga).max():.3e})")
        if bitwise:
            assert loss_n == loss_a and np.array_equal(gn, ga)
        else:
            assert abs(loss_n - loss_a) <= 1e-6 * abs(loss_a)
            assert np.linalg.norm(gn - ga) <= 1e-5 * np.linalg.norm(ga)
            assert err <= 1e-5 * np.abs(ga).max()
    with pytest.raises(zema.ZemaError) as e:
        big = torch.zeros((1, 16), dtype=torch.float32, device="cuda")
        lib = zema.lib()
        import ctypes as C
        loss = C.c_double()
        rc = lib.zema_mlp_grad_noalloc(M.h, C.c_void_p(big.data_ptr()), C.c_void_p(big.data_ptr()),
                                       (1 << 26) + 1, C.c_void_p(g_out.data_ptr()), C.byref(loss))
        M._chk(rc)
    assert e.value.code == zema.E_ARG
