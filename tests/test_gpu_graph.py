"""The single-instance path captured in a HIP graph: every entry point of the path only
enqueues kernels on the caller's stream (no allocation, no host synchronisation, fills by
kernel rather than memset), so a caller can capture sprinkle -> matrix -> counter ->
actions once and replay it.  Each replay is checked bit for bit against the eager pass and
the oracle, with eager work and synchronisations between replays.  The allocation-free
counter is captured the same way."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_04463_amd as cs
    cs.lib()
    return cs


@pytest.mark.parametrize("region,n,counter", [(W.MINK2_DIAMOND, 1024, 2), (W.MINK4_DIAMOND, 3000, 1),
                                              (W.MINK3_DIAMOND, 2000, 0)])
def test_path_replays_from_a_graph(cs, orc, region, n, counter):
    seed = 4242 + n
    dim = W.REGION_DIM[region]
    dev = torch.device("cuda")
    L = cs.lib()
    ld = cs.cs_ld_words(n)
    coords = torch.empty((cs.cs_coord_planes(region), n), dtype=torch.float64, device=dev)
    bits = torch.empty((n, ld), dtype=torch.int64, device=dev)
    hist = torch.empty(n - 1, dtype=torch.int64, device=dev)
    acts = torch.empty(2, dtype=torch.float64, device=dev)
    sp_ws = torch.empty(L.cs_sprinkle_workspace_bytes(region, n), dtype=torch.uint8, device=dev)
    h_ws = torch.empty(L.cs_histogram_workspace_bytes(n, counter), dtype=torch.uint8, device=dev)

    def step(st):
        cs.binding._check(L.cs_sprinkle(region, 1.2, seed, n, cs.binding._ptr(coords),
                                        cs.binding._ptr(sp_ws), sp_ws.numel(),
                                        cs.binding._stream(st)), "sprinkle")
        cs.cs_causal_matrix(region, coords, n, ld, out=bits, stream=st)
        cs.cs_interval_histogram(bits, n, counter, out=hist, workspace=h_ws, stream=st)
        cs.cs_action(hist, n, dim, 0.0, out=acts[0:1], stream=st)
        cs.cs_action(hist, n, dim, 0.1, out=acts[1:2], stream=st)

    step(torch.cuda.current_stream())
    torch.cuda.synchronize()
    h0 = hist.cpu().numpy().view(np.uint64).copy()
    a0 = acts.cpu().numpy().copy()
    _, _, want, _ = orc.pipeline(region, n, seed, fast=True)
    assert np.array_equal(h0, want)

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            step(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(4):
        hist.fill_(-1)
        acts.fill_(float("nan"))
        bits.fill_(-1)
        x = torch.randn(4096, device=dev).sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(hist.cpu().numpy().view(np.uint64), h0), rep
        assert np.array_equal(acts.cpu().numpy(), a0), rep
        del x


def test_noalloc_counter_in_a_graph(cs, orc):
    """cs_interval_histogram_noalloc needs no workspace, so a graph of it holds no buffer
    but the caller's matrix and histogram."""
    n = 2500
    coords = orc.sprinkle(W.MINK4_DIAMOND, n, 77)
    want = orc.histogram_fast(orc.causal_matrix(W.MINK4_DIAMOND, coords), n)[0]
    b = cs.cs_causal_matrix(W.MINK4_DIAMOND, torch.from_numpy(coords).cuda())
    out = torch.empty(n - 1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            cs.cs_interval_histogram_noalloc(b, n, out, cs.CS_COUNT_MFMA_FP4, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64), want), rep
