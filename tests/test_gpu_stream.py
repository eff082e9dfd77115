"""GPU test of the streaming-ceiling kernel the bench measures the stage kernels
against: out = (a + b) / 2 element by element (exact in FP64 for these inputs), odd
and even lengths, every launch shape, and argument checks."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5547_amd import amr as A
    A.lib()
    return torch, A


@pytest.mark.parametrize("n", [1, 2, 3, 1023, 2048, 2049, 1 << 20, (1 << 20) + 7])
@pytest.mark.parametrize("wpc", [0, 1, 8])
def test_stream_ceiling_computes_the_average(env, n, wpc):
    torch, A = env
    g = torch.Generator(device="cpu").manual_seed(n)
    a = torch.rand(n, generator=g, dtype=torch.float64).cuda()
    b = torch.rand(n, generator=g, dtype=torch.float64).cuda()
    out = torch.full((n + 1,), -7.0, dtype=torch.float64, device="cuda")
    A.amr_stream_ceiling(a, b, out, n, wpc)
    torch.cuda.synchronize()
    assert torch.equal(out[:n], 0.5 * (a + b))
    assert out[n].item() == -7.0  # nothing written past n


def test_stream_ceiling_rejects_bad_arguments(env):
    torch, A = env
    a = torch.zeros(16, dtype=torch.float64, device="cuda")
    for args in ((a, a, a[1:], 8, 0), (a, a, a, 0, 0), (a, a, a, 8, -1), (a, a, a, 8, 65)):
        with pytest.raises(A.AmrError) as ei:
            A.amr_stream_ceiling(*args)
        assert ei.value.status == A.AMR_EINVAL
