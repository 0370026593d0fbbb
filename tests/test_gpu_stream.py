"""GPU check of the streaming probe kernels the measured ceilings come from:
the copy and the two-reads-per-write kernels write exactly a and a + b over
sizes with ragged grid-stride tails, and the read kernel leaves its sink
untouched."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n4", [64, 1000, 4097, 1 << 20])
@pytest.mark.parametrize("blocks", [1, 3, 8192])
def test_stream_probe_results(n4, blocks):
    import torch
    from paper_2609_28179_amd import glass
    print(f"stream probe n4={n4} blocks={blocks}", flush=True)
    g = torch.Generator(device="cuda:0").manual_seed(n4)
    a = torch.rand(4 * n4 + 64, generator=g, device="cuda:0")
    b = torch.rand(4 * n4 + 64, generator=g, device="cuda:0")
    c = torch.full((4 * n4 + 64,), -7.0, device="cuda:0")
    assert glass.glass_stream_probe(2, a, b, c, n4, blocks) == glass.OK
    torch.cuda.synchronize()
    assert torch.equal(c[:4 * n4], a[:4 * n4]) and (c[4 * n4:] == -7.0).all()
    assert glass.glass_stream_probe(3, a, b, c, n4, blocks) == glass.OK
    torch.cuda.synchronize()
    assert torch.equal(c[:4 * n4], a[:4 * n4] + b[:4 * n4]) and (c[4 * n4:] == -7.0).all()
    assert glass.glass_stream_probe(1, None, None, c, n4, blocks) == glass.OK
    torch.cuda.synchronize()
    assert (c[:4 * n4] == 1.0).all() and (c[4 * n4:] == -7.0).all()
    c.fill_(-7.0)
    assert glass.glass_stream_probe(0, a, None, c, n4, blocks) == glass.OK
    torch.cuda.synchronize()
    assert (c == -7.0).all()
