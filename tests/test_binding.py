"""Argument checks of the Python binding that run before any library call
(CPU tier: no device is touched)."""
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vg():
    import paper_1604_03155_amd as vg
    return vg


def test_workspace_none_means_library_buffer(vg):
    assert vg.check_workspace(None, 1 << 30) is None


def test_undersized_workspace_is_rejected(vg):
    ws = torch.empty(1000, dtype=torch.uint8)
    with pytest.raises(ValueError, match="needs 4096"):
        vg.check_workspace(ws, 4096)
    # element size counts: 1000 float64 values are 8000 bytes
    with pytest.raises(ValueError, match="holds 8000 bytes"):
        vg.check_workspace(torch.empty(1000, dtype=torch.float64), 8001)


def test_host_workspace_is_rejected(vg):
    with pytest.raises(ValueError, match="CUDA"):
        vg.check_workspace(torch.empty(4096, dtype=torch.uint8), 4096)


def test_non_contiguous_workspace_is_rejected(vg):
    ws = torch.empty((64, 128), dtype=torch.uint8).t()
    with pytest.raises(ValueError, match="contiguous"):
        vg.check_workspace(ws, 1024)


def test_non_tensor_workspace_is_rejected(vg):
    with pytest.raises(TypeError):
        vg.check_workspace(bytearray(4096), 16)
