"""The atomic-throughput probe of the profiling tooling (measure/) adds exactly reps to every element."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_atomic_probe_counts():
    from measure import probe
    n = (1 << 20) + 37  # a ragged tail past the last full workgroup
    st = torch.cuda.current_stream().cuda_stream
    for stride in (1, 32):
        y = torch.zeros(n * stride, dtype=torch.float32, device="cuda:0")
        probe.atomic_add(y.data_ptr(), n, 3, stride, st)
        torch.cuda.synchronize()
        hit = y.view(n, stride)[:, 0]
        assert torch.all(hit == 3.0)
        assert int(torch.count_nonzero(y)) == n
