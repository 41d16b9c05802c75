"""The bandwidth probes do the work they are timed for: the march probe
reads its five fields and writes every output cell of its three fields with
its stated expressions (so none of its traffic is optimised away), the stream
probe writes its bitwise combinations of all five inputs into all three
outputs, and the copy is a copy.
Ragged grids (strips and chunks with partial tails), fixed and automatic
tile heights, both element sizes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1309_1230_amd import swe


def note(msg):
    print(f"[probes] {msg}", flush=True)


def march_reference(f):
    """The march probe's outputs from its five inputs (ny x nx arrays): the
    output row y uses rows y, y+1, y+2 (clamped to the grid) and the
    neighbour columns x+1 and x-1 (clamped)."""
    e, a, b, z, m = f
    ny, nx = e.shape
    y = np.arange(ny)
    y1 = np.minimum(y + 1, ny - 1)
    y2 = np.minimum(y + 2, ny - 1)
    xE = np.minimum(np.arange(nx) + 1, nx - 1)
    xW = np.maximum(np.arange(nx) - 1, 0)
    o0 = e + e[y1][:, xE] * m
    o1 = (a + z * a[y1][:, xW]) + e[y2]
    o2 = ((b + b[y1] * z[y1]) + a[y2] * b[y2]) + z[y2]
    return o0, o1, o2


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nx,ny,rows", [(130, 77, 16), (130, 77, 0), (61, 200, 7), (300, 33, 0)])
def test_march_probe_writes_its_expressions(dtype, nx, ny, rows):
    g = torch.Generator().manual_seed(nx * ny + rows)
    ins = [torch.rand(ny, nx, generator=g, dtype=torch.float64).to(dtype).cuda() for _ in range(5)]
    outs = [torch.full((ny, nx), float("nan"), dtype=dtype, device="cuda") for _ in range(3)]
    note(f"march probe {nx}x{ny} rows={rows or 'auto'} {dtype}")
    used = swe.probe_march(ins, outs, nx, ny, nx, rows)
    torch.cuda.synchronize()
    assert used == rows or rows == 0 and used > 0
    ref = march_reference([t.cpu().numpy() for t in ins])
    for o, r in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), r.astype(o.cpu().numpy().dtype))


def test_stream_and_copy_probes_move_their_bytes():
    n = 1 << 20
    g = torch.Generator().manual_seed(3)
    ins = [torch.rand(n, generator=g, dtype=torch.float64).cuda() for _ in range(5)]
    outs = [torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
    for nt in (False, True):
        for o in outs:
            o.fill_(float("nan"))
        swe.probe_stream(ins, outs, nontemporal=nt)
        torch.cuda.synchronize()
        bits = [t.view(torch.int64) for t in ins]
        # out0 = in0 ^ in3, out1 = in1 ^ in4, out2 = in2, on the raw 16-byte vectors
        assert torch.equal(outs[0].view(torch.int64), bits[0] ^ bits[3])
        assert torch.equal(outs[1].view(torch.int64), bits[1] ^ bits[4])
        assert torch.equal(outs[2].view(torch.int64), bits[2])
    src = torch.rand(n, generator=g, dtype=torch.float64).cuda()
    dst = torch.empty_like(src)
    swe.probe_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_march_probe_rejects_bad_rows():
    ins = [torch.zeros(8, 8, dtype=torch.float64, device="cuda") for _ in range(5)]
    outs = [torch.zeros(8, 8, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(swe.SweError):
        swe.probe_march(ins, outs, 8, 8, 8, -1)
