"""The atomic-throughput probe used by the profiling script adds exactly reps to every element."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_atomic_probe_counts():
    import ctypes
    from paper_2112_05598_amd import abi
    lib = abi.load()
    n = (1 << 20) + 37  # a ragged tail past the last full workgroup
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for stride in (1, 32):
        y = torch.zeros(n * stride, dtype=torch.float32, device="cuda:0")
        abi.check(lib.perf_atomic_probe(ctypes.c_void_p(y.data_ptr()), n, 3, stride, st))
        torch.cuda.synchronize()
        hit = y.view(n, stride)[:, 0]
        assert torch.all(hit == 3.0)
        assert int(torch.count_nonzero(y)) == n
