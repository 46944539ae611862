"""qq_evaluate_static, the evaluation entry point that allocates nothing (its workspace is the library's
fixed device scratch array), through the C ABI: its energies and gradients equal qq_evaluate's on the
same inputs, bit for bit (same kernels and schedule, only the workspace address differs), on two calls
in a row whose second is smaller than the first (the array keeps the first call's contents), with host
and with device parameters and outputs; a request larger than the array is refused before any device
work and leaves the outputs untouched."""
import ctypes

import numpy as np
import pytest

from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def reference(pb, x, flags):
    p, B = x.shape[1] // 2, x.shape[0]
    e, g = np.empty(B), np.empty((B, 2 * p))
    N.qq_evaluate(pb.handle, p, B, x, flags, None, 0, None, e, g if flags & N.QQ_GRAD else None)
    return e, g


def static(pb, x, flags):
    p, B = x.shape[1] // 2, x.shape[0]
    e, g = np.full(B, np.nan), np.full((B, 2 * p), np.nan)
    N.qq_evaluate_static(pb.handle, p, B, x, flags, None, e, g if flags & N.QQ_GRAD else None)
    return e, g


def test_static_matches_evaluate_on_two_calls_second_smaller():
    flags = N.QQ_ENERGY | N.QQ_GRAD
    big = W.dense_integer_symmetric(20, 901)
    small = W.dense_gaussian_upper(14, 902)
    pb_big, pb_small = Problem(big.H, big.f, big.c0), Problem(small.H, small.f, small.c0)
    try:
        x1 = W.random_params(3, 4, 903)   # n = 20, p = 3, 4 sets: 64 MiB of states
        x2 = W.random_params(2, 2, 904)   # n = 14, p = 2, 2 sets
        assert pb_big.workspace_size(3, 4, flags) <= N.QQ_STATIC_SCRATCH_BYTES
        for pb, x in ((pb_big, x1), (pb_small, x2)):
            print(f"n={pb.n} p={x.shape[1] // 2} B={x.shape[0]}", flush=True)
            e_s, g_s = static(pb, x, flags)
            e_r, g_r = reference(pb, x, flags)
            assert np.array_equal(e_s, e_r) and np.array_equal(g_s, g_r), (pb.n, e_s - e_r)
        # energy only, after the larger call: nothing stale is read
        e_s, _ = static(pb_small, x2, N.QQ_ENERGY)
        e_r, _ = reference(pb_small, x2, N.QQ_ENERGY)
        assert np.array_equal(e_s, e_r)
    finally:
        pb_big.close()
        pb_small.close()


def test_static_device_params_and_outputs():
    import torch

    inst = W.dense_integer_symmetric(12, 905)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        x = W.random_params(2, 3, 906)
        flags = N.QQ_ENERGY | N.QQ_GRAD
        e_r, g_r = reference(pb, x, flags)
        dev = torch.device("cuda:0")
        xt = torch.tensor(x, device=dev)
        e = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
        g = torch.full((3, 4), float("nan"), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev)
        N.qq_evaluate_static(pb.handle, 2, 3, xt, flags | N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE, stream, e, g)
        torch.cuda.synchronize()
        assert np.array_equal(e.cpu().numpy(), e_r) and np.array_equal(g.cpu().numpy(), g_r)
    finally:
        pb.close()


def test_static_refuses_requests_beyond_the_array():
    inst = W.dense_integer_symmetric(22, 907)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        flags = N.QQ_ENERGY | N.QQ_GRAD
        x = W.random_params(1, 4, 908)    # 4 sets of psi and lambda at n = 22: 256 MiB
        assert pb.workspace_size(1, 4, flags) > N.QQ_STATIC_SCRATCH_BYTES
        e = np.full(4, 7.0)
        g = np.full((4, 2), 7.0)
        with pytest.raises(N.QQError) as ei:
            N.qq_evaluate_static(pb.handle, 1, 4, x, flags, None, e, g)
        assert ei.value.status == N.QQ_E_WORKSPACE and "scratch" in str(ei.value)
        assert np.all(e == 7.0) and np.all(g == 7.0)
        # a request that fits still works afterwards
        e1, g1 = static(pb, x[:1], flags)
        e_r, g_r = reference(pb, x[:1], flags)
        assert np.array_equal(e1, e_r) and np.array_equal(g1, g_r)
    finally:
        pb.close()


def test_static_rejects_bad_arguments_like_evaluate():
    L = N.lib()
    dp = ctypes.POINTER(ctypes.c_double)
    x = np.array([0.1, 0.2])
    e = np.zeros(1)
    assert L.qq_evaluate_static(None, 1, 1, x.ctypes.data_as(dp), N.QQ_ENERGY, None, e.ctypes.data_as(dp),
                                None) == N.QQ_E_INVALID


def test_static_complex128_and_partitioned():
    inst = W.dense_integer_symmetric(13, 909)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        pb.set_allocation(W.contiguous_allocation(13, [7, 6]), 2, [7, 6])
        x = W.random_params(2, 2, 910)
        for flags in (N.QQ_ENERGY | N.QQ_GRAD | N.QQ_C128, N.QQ_ENERGY | N.QQ_GRAD | N.QQ_PARTITIONED):
            e_s, g_s = static(pb, x, flags)
            e_r, g_r = reference(pb, x, flags)
            assert np.array_equal(e_s, e_r) and np.array_equal(g_s, g_r), flags
    finally:
        pb.close()
