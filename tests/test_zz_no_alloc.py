"""rism3d_transform_noalloc (twiddle tables in the library's static device
scratch) against rism3d_transform (caller workspace), through the C ABI: the
same kernels on the same tables, so the results agree bit for bit.  Two calls
in a row, the second on a smaller grid (the scratch keeps the first call's
larger tables, which the second must overwrite where it reads)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2403_01039_amd import rism3d
    return rism3d


def _data(shape, count, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((count,) + shape) + 1j * rng.standard_normal((count,) + shape)
    return torch.tensor(x, dtype=torch.complex64, device="cuda")


@pytest.mark.parametrize("forward", [True, False])
def test_noalloc_transform_equals_workspace_transform(R, forward):
    for shape, count, seed in (((64, 96, 128), 2, 1), ((20, 18, 24), 3, 2)):
        print(f"noalloc transform {shape} x{count} forward={forward}", flush=True)
        a = _data(shape, count, seed)
        b = a.clone()
        R.rism3d_transform(a, forward)
        R.rism3d_transform_noalloc(b, forward)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        # and the transform is the shifted DFT: a round trip returns the input
        R.rism3d_transform_noalloc(b, not forward)
        back = b / float(np.prod(shape))
        ref = _data(shape, count, seed)
        assert (back - ref).abs().max().item() < 2e-6 * ref.abs().max().item()


def test_noalloc_rejects_unsupported_grids(R):
    x = torch.zeros((1, 8, 8, 1024), dtype=torch.complex64, device="cuda")
    with pytest.raises(R.RismError) as e:
        R.rism3d_transform_noalloc(x, True)
    assert e.value.status == 1
    y = torch.zeros((1, 8, 8, 14), dtype=torch.complex64, device="cuda")   # factor 7
    with pytest.raises(R.RismError) as e:
        R.rism3d_transform_noalloc(y, True)
    assert e.value.status == 1
