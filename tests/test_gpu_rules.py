"""GPU checks of how the kernels follow the rules and launch sizes a caller sets:

* a caller's rule whose nodes are listed in another order (the same exact rule) breaks
  the banded pattern of the tables; the kernels must take the full loops and still match
  the oracle given the same reordered tables, forward, adjoint and products;
* launches split into several dispatches (a low dispatch limit) give bitwise the same
  results as one dispatch;
* a rule change waits for work already queued on another stream: that work sees the
  old tables, work queued after it the new ones.
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


@pytest.fixture(scope="module")
def wqa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1710_01048_amd as mod
    return mod


def _reverse_rows(x, w, n, Q, p):
    xr, wr = np.asarray(x).reshape(n, Q).copy(), np.asarray(w).reshape(n, Q).copy()
    xr[p:n - p] = xr[p:n - p, ::-1]
    wr[p:n - p] = wr[p:n - p, ::-1]
    return xr.reshape(-1), wr.reshape(-1)


CASES = [(2, 2, (5, 21), (0, 1)), (2, 3, (7, 23), (0,)), (3, 2, (4, 6, 21), (1,)),
         (3, 3, (6, 7, 23), (0, 1, 2)), (3, 3, (5, 6, 13), (0,))]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "d%d-p%d-dirs%s" % (c[0], c[1], "".join(map(str, c[3]))))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_reordered_rule_every_row(wqa, case, dtype):
    d, p, n_el, dirs = case
    Q = p + 1
    n = [e + p for e in n_el]
    sp = wqa.Space(d, p, n_el)
    tabs = {k: [np.array(v) for v in vals] for k, vals in oa.rule_tables(p, n_el).items() if k != "breaks"}
    tabs["breaks"] = [None] * d
    for k in dirs:
        for kind, kx, kw in ((wqa.MASS, "xM", "wM"), (wqa.STIFFNESS, "xK", "wK")):
            x, w = sp.rules(kind, k)
            sp.set_rules(kind, k, *_reverse_rows(x, w, n[k], Q, p))
            tabs[kx][k], tabs[kw][k] = _reverse_rows(tabs[kx][k], tabs[kw][k], n[k], Q, p)
    fields = ph._random_fields(p, n_el, 61)
    f = [torch.from_numpy(v).to(sp.device, dtype) for v in fields]
    M, K = sp.assemble_fused(f[0], f[1:])
    Mw, Kw = oa.assemble(p, n_el, tabs, c=fields[0], a=fields[1:])
    assert st.row_scaled_error(M.cpu().numpy(), Mw) <= TOL[dtype]
    assert st.row_scaled_error(K.cpu().numpy(), Kw) <= TOL[dtype]
    rows = np.arange(sp.n_rows)
    valid = si.slot_valid_mask(n_el, p).numpy()
    rng = np.random.default_rng(62)
    gM = np.where(valid, rng.normal(size=valid.shape), 0.0)
    gK = np.where(valid, rng.normal(size=valid.shape), 0.0)
    dc, da = sp.adjoint(torch.from_numpy(gM).to(sp.device, dtype), torch.from_numpy(gK).to(sp.device, dtype))
    want, scale = ph.oracle_adjoint(p, n_el, tabs, gM, gK, rows)
    pts = st.point_offsets(n, p, rows)
    errs = ph.entry_errors([g.reshape(-1).cpu().numpy()[pts] for g in [dc] + list(da)], want, scale)
    assert max(errs) <= TOL[dtype], errs
    # products: y = M x and y = K x against the oracle's rows, error per row over sum |terms|
    from test_gpu_apply import _product_error
    cols = st.columns(n, p, rows)
    xd = torch.from_numpy(rng.standard_normal(sp.n_rows)).to(sp.device, dtype)
    x = xd.double().cpu().numpy()
    assert _product_error(sp.apply_mass(f[0], xd).cpu().numpy(), Mw, cols, x) <= TOL[dtype]
    assert _product_error(sp.apply_stiffness(f[1:], xd).cpu().numpy(), Kw, cols, x) <= TOL[dtype]


@pytest.mark.parametrize("limit", [7, 100])
@pytest.mark.parametrize("case", [(3, 3, (5, 6, 13)), (2, 2, (5, 21))], ids=lambda c: "d%d-p%d" % c[:2])
def test_split_dispatches_give_the_same_bits(wqa, case, limit):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    fields = ph._random_fields(p, n_el, 71)
    f = [torch.from_numpy(v).to(sp.device, torch.float32) for v in fields]
    gM = si.upstream_gradient(n_el, p, 72, torch.float32, sp.device)
    gK = si.upstream_gradient(n_el, p, 73, torch.float32, sp.device)
    x = torch.randn(sp.n_rows, generator=torch.Generator().manual_seed(74)).to(sp.device, torch.float32)

    def run():
        M, K = sp.assemble_fused(f[0], f[1:])
        dc, da = sp.adjoint(gM, gK)
        return [M, K, dc, *da, sp.apply_mass(f[0], x), sp.apply_stiffness(f[1:], x), sp.load_vector(f[0])]

    one = run()
    sp.set_dispatch_limit(limit)
    many = run()
    sp.set_dispatch_limit(0)
    torch.cuda.synchronize()
    for a, b in zip(one, many):
        assert torch.equal(a, b)
    Mw, Kw = oa.assemble(p, n_el, oa.rule_tables(p, n_el), c=fields[0], a=fields[1:])
    assert st.row_scaled_error(many[0].cpu().numpy(), Mw) <= 1e-5
    assert st.row_scaled_error(many[1].cpu().numpy(), Kw) <= 1e-5


def test_rule_change_waits_for_queued_work(wqa):
    sp = wqa.Space(3, 3, (96, 96, 96))
    gen = torch.Generator().manual_seed(81)
    c = (torch.rand(sp.grid_shape, generator=gen, dtype=torch.float32) + 0.5).to(sp.device)
    ref = sp.assemble_mass(c)
    torch.cuda.synchronize()
    x, w = sp.rules(wqa.MASS, 0)
    s = torch.cuda.Stream()
    outs = [torch.empty_like(ref) for _ in range(4)]
    with torch.cuda.stream(s):
        for o in outs:
            sp.assemble_mass(c, o)
        # the host changes the rule while the stream still works through the launches;
        # doubling every weight doubles every table entry and entry of M exactly
        sp.set_rules(wqa.MASS, 0, x, 2 * w, exact_tol=-1)
        after = sp.assemble_mass(c)
    s.synchronize()
    for o in outs:
        assert torch.equal(o, ref)
    assert torch.equal(after, 2 * ref)


@pytest.mark.parametrize("case", [(3, 3, (5, 6, 13)), (2, 2, (5, 21)), (3, 2, (4, 3, 9))],
                         ids=lambda c: "d%d-p%d" % c[:2])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_grid_pitch_gives_the_same_bits(wqa, case, dtype):
    """Grid buffers whose last-direction lines are padded to a pitch: every call reads and
    writes the same values at the same grid points as with dense buffers, and never
    touches the padding (NaN there in the inputs stays out of the results, NaN there in
    the gradient buffers stays NaN)."""
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    fields = ph._random_fields(p, n_el, 91)
    f = [torch.from_numpy(v).to(sp.device, dtype) for v in fields]
    gM = si.upstream_gradient(n_el, p, 92, dtype, sp.device)
    gK = si.upstream_gradient(n_el, p, 93, dtype, sp.device)
    x = torch.randn(sp.n_rows, generator=torch.Generator().manual_seed(94)).to(sp.device, dtype)

    def run(fs):
        M, K = sp.assemble_fused(fs[0], fs[1:])
        dc, da = sp.adjoint(gM, gK, torch.full(sp.buffer_shape, float("nan"), dtype=dtype, device=sp.device),
                            [torch.full(sp.buffer_shape, float("nan"), dtype=dtype, device=sp.device)
                             for _ in range(d)])
        return [M, K, sp.apply_mass(fs[0], x), sp.apply_stiffness(fs[1:], x), sp.load_vector(fs[0])], [dc, *da]

    dense, gdense = run(f)
    Nd = sp.grid_shape[-1]
    pitch = (Nd + 31) // 32 * 32 + 4
    sp.set_grid_pitch(pitch)
    assert sp.buffer_shape == sp.grid_shape[:-1] + (pitch,)
    padded = []
    for v in f:
        buf = torch.full(sp.buffer_shape, float("nan"), dtype=dtype, device=sp.device)
        buf[..., :Nd] = v
        padded.append(buf)
    mats, grads = run(padded)
    torch.cuda.synchronize()
    for a, b in zip(dense, mats):
        assert torch.equal(a, b)
    for a, b in zip(gdense, grads):
        assert torch.equal(a, b[..., :Nd])
        assert torch.isnan(b[..., Nd:]).all()
    with pytest.raises(ValueError):
        wqa.WQAssemble.apply(sp, *padded)
    sp.set_grid_pitch(0)
    assert sp.buffer_shape == sp.grid_shape
