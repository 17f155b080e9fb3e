"""CPU tests of the Python binding's argument checks: a caller-supplied output or workspace
is validated before its pointer reaches a kernel. The checks compare tensor properties
only, so they run here on CPU tensors standing in for one device."""
import pytest

torch = pytest.importorskip("torch")

import paper_1902_00176_amd as gfc  # noqa: E402

DEV = torch.device("cpu")


def _inputs():
    gx = torch.zeros(2, 5, 7)
    gy = torch.zeros(2, 5, 7)
    return gx, gy


def test_check_out_accepts_a_good_output():
    gx, gy = _inputs()
    out = torch.empty(2, 5, 7)
    assert gfc.check_out(out, gx.shape, DEV, (gx, gy)) is out


@pytest.mark.parametrize("bad,exc", [
    (lambda: torch.empty(2, 5, 6), ValueError),                      # wrong shape
    (lambda: torch.empty(2, 5, 7, dtype=torch.float64), TypeError),  # wrong dtype
    (lambda: torch.empty(2, 7, 5).transpose(1, 2), ValueError),      # not contiguous
    (lambda: torch.empty(2, 5, 7, device="meta"), ValueError),       # another device
    (lambda: [0.0], TypeError),                                      # not a tensor
])
def test_check_out_rejects_bad_outputs(bad, exc):
    gx, gy = _inputs()
    with pytest.raises(exc):
        gfc.check_out(bad(), gx.shape, DEV, (gx, gy))


def test_check_out_rejects_an_output_aliasing_an_input():
    buf = torch.zeros(3, 5, 7)
    gx, gy = buf[:2], torch.zeros(2, 5, 7)
    with pytest.raises(ValueError, match="share memory"):
        gfc.check_out(gx, gx.shape, DEV, (gx, gy))
    with pytest.raises(ValueError, match="share memory"):
        gfc.check_out(buf[1:], gx.shape, DEV, (gx, gy))  # overlaps by one image
    gfc.check_out(buf[2:].expand(2, 5, 7).contiguous(), gx.shape, DEV, (gx, gy))


def test_check_workspace_counts_bytes_of_any_dtype():
    ws = torch.empty(25, dtype=torch.float32)  # 100 bytes
    assert gfc.check_workspace(ws, 100, DEV) is ws
    with pytest.raises(ValueError, match="too small"):
        gfc.check_workspace(ws, 101, DEV)


def test_check_workspace_rejects_device_contiguity_and_overlap():
    with pytest.raises(ValueError):
        gfc.check_workspace(torch.empty(64, dtype=torch.uint8, device="meta"), 8, DEV)
    with pytest.raises(ValueError):
        gfc.check_workspace(torch.empty(8, 8)[:, ::2], 8, DEV)
    gx = torch.zeros(64)
    with pytest.raises(ValueError, match="share memory"):
        gfc.check_workspace(gx[8:], 8, DEV, (gx,))
