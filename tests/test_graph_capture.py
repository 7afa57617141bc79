"""HIP-graph capture of the single-handle product (hh_matvec / hh_matvec_t with
a workspace sized beforehand by hh_reserve).

The captured product is replayed several times, with new inputs copied into
the captured buffer and ordinary eager work between replays, and every replay
must equal an eager product bit for bit (products are deterministic)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("nrhs,trans", [(1, False), (1, True), (8, False)])
def test_captured_product_replays_equal_eager_products(nrhs, trans):
    torch = _torch()
    from paper_2604_09147_amd import HMatrix
    rng = np.random.default_rng(50 + nrhs)
    n = 6000
    P = rng.random((n, 3))
    print(f"graph capture: N={n} nrhs={nrhs} trans={trans}", flush=True)
    g = HMatrix(P, W.INV_R, 1e-6, 1.5, -1, 64)
    g.reserve(nrhs)
    apply = g.matvec_t if trans else g.matvec
    shape = (n,) if nrhs == 1 else (n, nrhs)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    apply(x, out=y)                                  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):                    # current stream = capture stream
        apply(x, out=y)
    for rep in range(4):
        xv = torch.from_numpy(rng.standard_normal(shape)).cuda()
        x.copy_(xv)
        graph.replay()
        torch.cuda.synchronize()
        ref = apply(xv)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"replay {rep} differs from the eager product"
        float((xv * 2.0).sum())                      # eager work between replays
    g.free()
