"""GPU checks of the row-by-row sample layout (wqa_set_sample_layout, WQA_SAMPLES_ROWS).

Each grid point belongs to exactly one row (row i owns the points (i_k Q + q_k)_k of its
rule, Sec. 3), so the row layout is a permutation of the grid: the same values, row i's
Q^d samples as one block.  Every call must give, bit for bit, what it gives on the grid
for the permuted inputs, write every gradient value (NaN-poisoned buffers), and match
the oracle, whose per-row mode takes exactly this layout.
"""
import numpy as np
import pytest
import torch

import parity_helpers as ph
import structured as st
import synth_inputs as si
from oracle import assembly as oa

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}

# (d, p, n_el): ragged tiles in every case; 3D cubic with interior lines whose middle tiles
# take the banded last-direction path; quadratic cases whose row blocks (27 or 9 values)
# are not a multiple of 16 bytes
CASES = [(3, 3, (6, 7, 40)), (3, 3, (4, 5, 9)), (3, 2, (5, 6, 30)), (2, 3, (7, 45)), (2, 2, (6, 50))]


@pytest.fixture(scope="module")
def wqa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1710_01048_amd as mod
    return mod


def _nan(sp, dtype):
    return torch.full(sp.buffer_shape, float("nan"), dtype=dtype, device=sp.device)


def _everything(sp, fs, gM, gK, x, dtype):
    """Every call that reads or writes samples, with NaN-poisoned gradient buffers."""
    d = sp.dim
    M, K = sp.assemble_fused(fs[0], fs[1:])
    Mo = sp.assemble_mass(fs[0])
    Ko = sp.assemble_stiffness(fs[1:])
    dc, da = sp.adjoint(gM, gK, _nan(sp, dtype), [_nan(sp, dtype) for _ in range(d)])
    dcm, _ = sp.adjoint(gM, None, _nan(sp, dtype), None)
    _, dak = sp.adjoint(None, gK, None, [_nan(sp, dtype) for _ in range(d)])
    outs = [M, K, Mo, Ko, sp.apply_mass(fs[0], x), sp.apply_stiffness(fs[1:], x), sp.load_vector(fs[0])]
    return outs, [dc, *da, dcm, *dak]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "d%d-p%d-%s" % (c[0], c[1], "x".join(map(str, c[2]))))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_rows_layout_gives_the_same_bits(wqa, case, dtype):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    f = [torch.from_numpy(v).to(sp.device, dtype) for v in ph._random_fields(p, n_el, 101)]
    gM = si.upstream_gradient(n_el, p, 102, dtype, sp.device)
    gK = si.upstream_gradient(n_el, p, 103, dtype, sp.device)
    x = torch.randn(sp.n_rows, generator=torch.Generator().manual_seed(104)).to(sp.device, dtype)
    modes = [0, 1, 2] if dtype == torch.float32 else [2]
    for mode in modes:
        sp.set_sample_layout("grid")
        sp.set_final_mode(mode)
        grid_out, grid_grads = _everything(sp, f, gM, gK, x, dtype)
        sp.set_sample_layout("rows")
        assert sp.buffer_shape == (sp.n_rows, sp.points_per_row)
        rows_in = [sp.rows_from_grid(v) for v in f]
        rows_out, rows_grads = _everything(sp, rows_in, gM, gK, x, dtype)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(grid_out, rows_out)):
            assert torch.equal(a, b), f"final mode {mode}, output {k}"
        for k, (a, b) in enumerate(zip(grid_grads, rows_grads)):
            assert not torch.isnan(b).any(), f"final mode {mode}, gradient {k}: values left unwritten"
            assert torch.equal(a, sp.grid_from_rows(b)), f"final mode {mode}, gradient {k}"
    sp.set_sample_layout("grid")
    assert sp.buffer_shape == sp.grid_shape


@pytest.mark.parametrize("case", [(3, 3, (5, 6, 37)), (2, 2, (6, 47))], ids=lambda c: "d%d-p%d" % c[:2])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_rows_layout_against_the_oracle(wqa, case, dtype):
    """The oracle's per-row mode takes samples in the row layout: the forward on every row
    and the adjoint at every point, straight from and into row-layout buffers."""
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    sp.set_sample_layout("rows")
    rows = np.arange(sp.n_rows)
    tabs = oa.rule_tables(p, n_el)
    recipe = ("random", 111)
    per_row = ph.oracle_row_fields(tabs, p, n_el, rows, recipe)      # [rows, Q^d] each
    f = [torch.from_numpy(v).to(sp.device, dtype) for v in per_row]
    M, K = sp.assemble_fused(f[0], f[1:])
    Mw, Kw = oa.assemble(p, n_el, tabs, c=per_row[0], a=per_row[1:], rows=rows, per_row=True)
    assert st.row_scaled_error(M.cpu().numpy(), Mw) <= TOL[dtype]
    assert st.row_scaled_error(K.cpu().numpy(), Kw) <= TOL[dtype]
    rng = np.random.default_rng(112)
    valid = si.slot_valid_mask(n_el, p).numpy()
    gM = np.where(valid, rng.normal(size=valid.shape), 0.0)
    gK = np.where(valid, rng.normal(size=valid.shape), 0.0)
    dc, da = sp.adjoint(torch.from_numpy(gM).to(sp.device, dtype), torch.from_numpy(gK).to(sp.device, dtype))
    torch.cuda.synchronize()
    want, scale = ph.oracle_adjoint(p, n_el, tabs, gM, gK, rows)
    errs = ph.entry_errors([g.cpu().numpy() for g in [dc, *da]], want, scale)
    assert max(errs) <= TOL[dtype], errs


def test_layout_switches(wqa):
    """The pitch belongs to the grid layout, and sample buffers must have the layout's shape."""
    sp = wqa.Space(3, 3, (4, 4, 9))
    Nd = sp.grid_shape[-1]
    sp.set_grid_pitch((Nd + 31) // 32 * 32)
    with pytest.raises(RuntimeError):
        sp.set_sample_layout("rows")
    sp.set_grid_pitch(0)
    sp.set_sample_layout("rows")
    with pytest.raises(RuntimeError):
        sp.set_grid_pitch((Nd + 31) // 32 * 32)
    with pytest.raises(ValueError):
        sp.assemble_mass(torch.ones(sp.grid_shape, device=sp.device))
    with pytest.raises(ValueError):
        sp.set_sample_layout("columns")


def _reverse_interior_nodes(x, w, n, Q, p):
    xr, wr = np.asarray(x).reshape(n, Q).copy(), np.asarray(w).reshape(n, Q).copy()
    xr[p:n - p] = xr[p:n - p, ::-1]
    wr[p:n - p] = wr[p:n - p, ::-1]
    return xr.reshape(-1), wr.reshape(-1)


@pytest.mark.parametrize("setup", ["unbanded_rules", "nonuniform_knots", "split_dispatches"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_rows_layout_other_code_paths(wqa, setup, dtype):
    """The row layout against the grid, bit for bit, on the kernels' other paths: rules
    whose nodes are listed in reverse (the band is broken, every tile takes the full
    loops), graded knots in one direction, and launches split into dispatches of 7 tiles."""
    d, p, n_el = 3, 3, (5, 6, 19)
    Q = p + 1
    breaks = None
    if setup == "nonuniform_knots":
        breaks = [None, [(k / n_el[1]) ** 1.4 for k in range(n_el[1] + 1)], None]
    sp = wqa.Space(d, p, n_el, breaks=breaks)
    if setup == "unbanded_rules":
        n0 = n_el[0] + p
        for kind in (wqa.MASS, wqa.STIFFNESS):
            x, w = sp.rules(kind, 0)
            sp.set_rules(kind, 0, *_reverse_interior_nodes(x, w, n0, Q, p))
    if setup == "split_dispatches":
        sp.set_dispatch_limit(7)
    f = [torch.from_numpy(v).to(sp.device, dtype) for v in ph._random_fields(p, n_el, 121)]
    gM = si.upstream_gradient(n_el, p, 122, dtype, sp.device)
    gK = si.upstream_gradient(n_el, p, 123, dtype, sp.device)
    x = torch.randn(sp.n_rows, generator=torch.Generator().manual_seed(124)).to(sp.device, dtype)
    grid_out, grid_grads = _everything(sp, f, gM, gK, x, dtype)
    sp.set_sample_layout("rows")
    rows_out, rows_grads = _everything(sp, [sp.rows_from_grid(v) for v in f], gM, gK, x, dtype)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(grid_out, rows_out)):
        assert torch.equal(a, b), f"output {k}"
    for k, (a, b) in enumerate(zip(grid_grads, rows_grads)):
        assert not torch.isnan(b).any(), f"gradient {k}: values left unwritten"
        assert torch.equal(a, sp.grid_from_rows(b)), f"gradient {k}"
