"""The HBM probe kernels compute what they claim (so their rates are rates of
real reads and writes): small arrays, every mode."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_hbm_probe_values():
    from paper_2512_16642_amd import ehi
    n = 4096 * 4                        # floats per array (a multiple of 4)
    rng = np.random.default_rng(3)
    a = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
    b = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
    u8 = lambda t: t.view(torch.uint8)
    c = torch.zeros(n, dtype=torch.float32, device="cuda")
    d = torch.zeros_like(c)
    e = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    grid = 4
    sink = torch.zeros(grid * 256 * 4, dtype=torch.float32, device="cuda")
    ehi.hbm_probe(0, u8(a), None, u8(c), grid=grid)
    torch.cuda.synchronize()
    assert torch.equal(c, a + a)
    ehi.hbm_probe(3, u8(a), u8(b), u8(c), u8(d), u8(e), e_frac=1.5, grid=grid)
    torch.cuda.synchronize()
    assert torch.equal(c, a + b) and torch.equal(d, a - b)
    n4e = int(1.5 * (n // 4)) * 4
    ref = torch.cat([a * b, a * a])
    assert torch.equal(e[:n4e], ref[:n4e]) and torch.all(e[n4e:] == 0)
    ehi.hbm_probe(4, u8(a), u8(b), grid=grid, sink=u8(sink))
    torch.cuda.synchronize()
    tot = sink.double().sum().item()
    assert abs(tot - (a.double().sum() + b.double().sum()).item()) < 1e-3 * (a.abs().sum() + b.abs().sum()).item()
