"""The assemble, adjoint and product calls under HIP graph capture: they allocate nothing,
clear nothing with memset and only queue kernels on the given stream, so a captured step
(fused forward, adjoint, matrix-free product) replays.  Every replay, with eager work and
synchronizations in between and fresh inputs copied in before it, must equal the eager
results bit for bit (the kernels are deterministic)."""
import pytest
import torch

import parity_helpers as ph
import synth_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wqa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1710_01048_amd as mod
    return mod


@pytest.mark.parametrize("layout", ["grid", "rows"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_captured_step_replays_bitwise(wqa, dtype, layout):
    p, n_el = 3, (9, 10, 21)
    sp = wqa.Space(3, p, n_el)
    sp.set_sample_layout(layout)                # samples on the grid or stored row by row
    dev = sp.device
    # static buffers of the graph
    f = [torch.empty(sp.buffer_shape, dtype=dtype, device=dev) for _ in range(4)]
    gM = torch.empty(sp.n_rows, sp.slots_per_row, dtype=dtype, device=dev)
    gK = torch.empty_like(gM)
    x = torch.empty(sp.n_rows, dtype=dtype, device=dev)
    M = torch.empty_like(gM)
    K = torch.empty_like(gM)
    dc = torch.empty(sp.buffer_shape, dtype=dtype, device=dev)
    da = [torch.empty_like(dc) for _ in range(3)]
    y = torch.empty(sp.n_rows, dtype=dtype, device=dev)

    def step():
        sp.assemble_fused(f[0], f[1:], M, K)
        sp.adjoint(gM, gK, dc, da)
        sp.apply_stiffness(f[1:], x, y)

    def inputs(seed):
        fs = ph.device_fields(sp, ("random", seed), dtype)
        if layout == "rows":
            fs = [sp.rows_from_grid(t) for t in fs]
        g1 = si.upstream_gradient(n_el, p, seed + 1, dtype, dev)
        g2 = si.upstream_gradient(n_el, p, seed + 2, dtype, dev)
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed + 3)
        xs = torch.randn(sp.n_rows, generator=gen, dtype=torch.float64, device=dev).to(dtype)
        return fs, g1, g2, xs

    def load(inp):
        fs, g1, g2, xs = inp
        for a, b in zip(f, fs):
            a.copy_(b)
        gM.copy_(g1)
        gK.copy_(g2)
        x.copy_(xs)

    def outputs():
        return [t.clone() for t in [M, K, dc] + da + [y]]

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        load(inputs(100))
        step()                                  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for seed in (200, 300, 400):
        inp = inputs(seed)
        load(inp)
        step()                                  # eager reference on the same inputs
        torch.cuda.synchronize()
        want = outputs()
        for t in [M, K, dc, y] + da:            # poison the outputs before the replay
            t.fill_(float("nan"))
        load(inp)
        graph.replay()
        torch.cuda.synchronize()
        got = outputs()
        for g, w in zip(got, want):
            assert torch.equal(g, w)
