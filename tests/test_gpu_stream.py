"""The streaming kernels of known traffic (stencil_stream): every op, width
and nontemporal flag writes exactly its definition, including a tail that is
not a multiple of the width and the in-place form.  Inputs are small
integers scaled by powers of two, so fma(c, a, 2a - b) is exact and equals
the numpy value computed with separate roundings."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.mark.parametrize("n", [1, 255, 1000003])
@pytest.mark.parametrize("width", [1, 2])
@pytest.mark.parametrize("flags", [(False, False), (True, True), (False, True)])
@pytest.mark.parametrize("grid", [0, 7])
def test_stream_ops(dev, n, width, flags, grid):
    from paper_2306_13002_amd.stencil import stream

    rng = np.random.default_rng(n + width)
    a = rng.integers(-64, 64, n) * 0.25
    b = rng.integers(-64, 64, n) * 0.125
    c = rng.integers(-8, 8, n) * 0.5
    A, B, C = (torch.tensor(x, device=dev) for x in (a, b, c))
    D = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    stream("copy", A, None, None, D, width=width, nt_loads=flags[0], nt_stores=flags[1], grid=grid)
    torch.cuda.synchronize()
    assert np.array_equal(D.cpu().numpy(), a)
    stream("3r1w", A, B, C, D, width=width, nt_loads=flags[0], nt_stores=flags[1], grid=grid)
    torch.cuda.synchronize()
    want = c * a + (2 * a - b)
    assert np.array_equal(D.cpu().numpy(), want)
    stream("3r1w", A, B, C, B, width=width, nt_loads=flags[0], nt_stores=flags[1], grid=grid)  # in place
    torch.cuda.synchronize()
    assert np.array_equal(B.cpu().numpy(), want)


def test_stream_rejects_bad_arguments(dev):
    from paper_2306_13002_amd.stencil import StencilError, E_INVAL, stream

    A = torch.zeros(64, dtype=torch.float64, device=dev)
    B = torch.zeros(64, dtype=torch.float64, device=dev)
    with pytest.raises(StencilError) as e:
        stream("3r1w", A, B, A, A)  # d overlaps a
    assert e.value.status == E_INVAL
    with pytest.raises(StencilError) as e:
        stream("copy", A, None, None, B, width=3)
    assert e.value.status == E_INVAL
    odd = torch.zeros(65, dtype=torch.float64, device=dev)
    with pytest.raises(StencilError) as e:
        stream("copy", odd[1:], None, None, B, width=2)  # not 16-byte aligned
    assert e.value.status == E_INVAL
