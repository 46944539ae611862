"""The Python binding checks caller buffers before it passes their addresses to the library
(CPU only: every case raises before the library is called).

A buffer shorter than the call needs, of another element type, strided, or on the wrong side of the
PCIe bus for the *_ON_DEVICE flags would otherwise be read or written out of bounds by the library's
copies and kernels.  Out-of-range p or batch are left to the library, which rejects them with its
own status code (tested with a problem on the GPU)."""
import numpy as np
import pytest

from paper_2606_26297_amd import native as N

E = N.QQ_ENERGY


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()


@pytest.mark.parametrize("params,energy,grad,flags,exc", [
    (np.zeros(3), np.zeros(1), None, E, ValueError),                              # params short (2p = 4)
    (np.zeros(4, dtype=np.float32), np.zeros(1), None, E, TypeError),             # params float32
    (np.zeros((4, 2))[:, 0], np.zeros(1), None, E, ValueError),                   # params strided
    (np.zeros(4), np.zeros(0), None, E, ValueError),                              # energy short
    (np.zeros(4), np.zeros(1, dtype=np.int64), None, E, TypeError),               # energy int64
    (np.zeros(4), np.zeros(1), np.zeros(3), E | N.QQ_GRAD, ValueError),           # gradient short
    (np.zeros(4), np.zeros(1), None, E | N.QQ_PARAMS_ON_DEVICE, ValueError),      # host params, device flag
    (np.zeros(4), np.zeros(1), None, E | N.QQ_OUT_ON_DEVICE, ValueError),         # host output, device flag
])
def test_evaluate_rejects_bad_buffers(params, energy, grad, flags, exc):
    with pytest.raises(exc):
        N.qq_evaluate(None, 2, 1, params, flags, None, 0, None, energy, grad)


def test_evaluate_many_rejects_bad_buffers():
    with pytest.raises(ValueError):  # second problem's parameters short
        N.qq_evaluate_many([None, None], [1, 2], [1, 1], [np.zeros(2), np.zeros(2)], E, None, None, 0, None,
                           [np.zeros(1), np.zeros(1)], None)
    with pytest.raises(ValueError):  # one output per problem
        N.qq_evaluate_many([None, None], [1, 1], [1, 1], [np.zeros(2), np.zeros(2)], E, None, None, 0, None,
                           [np.zeros(1)], None)


def test_sample_and_graph_reject_bad_buffers():
    with pytest.raises(ValueError):  # host params for a device call
        N.qq_sample(None, 1, np.zeros(2), np.zeros(4), flags=N.QQ_PARAMS_ON_DEVICE)
    with pytest.raises(ValueError):  # host output for a device call
        N.qq_sample(None, 1, np.zeros(2), np.full(4, 0.5), flags=N.QQ_OUT_ON_DEVICE, out=np.zeros(4, np.uint64))
    with pytest.raises(ValueError):  # params short
        N.qq_sample(None, 2, np.zeros(2), np.full(4, 0.5))
    with pytest.raises(ValueError):  # graph parameters live on the device
        N.qq_graph_create(None, 1, 1, 0, None, np.zeros(2))


def test_packed_guarded_buffers_point_at_each_problems_block():
    # problem i's block starts where block i - 1 ends; the packed wrapper checks each buffer once
    p, batch = np.array([1, 3, 2], dtype=np.int32), np.array([2, 1, 4], dtype=np.int32)
    per2p = N._need_many(p, batch, 2) // 8
    assert per2p.tolist() == [4, 6, 16]
    buf = np.zeros(int(per2p.sum()))
    ptrs = N._packed_ptrs(buf, per2p, 8, "params", N._F64)
    base = buf.__array_interface__["data"][0]
    assert list(ptrs) == [base, base + 8 * 4, base + 8 * 10]
    flags = np.zeros(int(batch.sum()), dtype=np.int32)
    ptrs = N._packed_ptrs(flags, N._need_many(p, batch, 0, 1) // 8, 4, "c128_out", ("int32",))
    base = flags.__array_interface__["data"][0]
    assert list(ptrs) == [base, base + 4 * 2, base + 4 * 3]
    with pytest.raises(ValueError):  # one double short
        N._packed_ptrs(np.zeros(25), per2p, 8, "params", N._F64)
    with pytest.raises(TypeError):
        N._packed_ptrs(np.zeros(26, dtype=np.float32), per2p, 8, "params", N._F64)
    with pytest.raises(ValueError):  # the whole guarded call refuses a short packed output before any library call
        N.qq_evaluate_many_guarded_packed([None] * 3, p, batch, np.zeros(26), E | N.QQ_GRAD, None, 1e-5,
                                          np.zeros(6), np.zeros(26))
