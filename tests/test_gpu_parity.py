"""GPU parity: libwqa's HIP kernels against the FP64 oracle (runs on an MI355X).

Forward and adjoint, every dimension/degree/dtype/final-pass mode on small spaces whose
last direction spans several wave tiles with a ragged tail (full comparison of every
row), and the benchmark workloads at full size on a row sample that covers every
boundary class.  Bars: FP64 within 1e-12, FP32 within 1e-5; matrices by row-scaled
relative error (the largest error in a row over the largest exact entry of that row),
gradients entry by entry (each entry's error over the sum of the magnitudes of the
terms it sums, from the oracle's absolute-value adjoint).
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


def _rows_all(space):
    return np.arange(space.n_rows)


SMALL = [
    (2, 2, (3, 4)), (2, 2, (5, 21)), (2, 3, (4, 4)), (2, 3, (7, 23)),
    (3, 2, (3, 4, 5)), (3, 2, (4, 3, 21)), (3, 3, (4, 4, 4)), (3, 3, (5, 4, 13)),
    (3, 3, (6, 7, 23)),
]


def _ids(v):
    return "d%d-p%d-%s" % (v[0], v[1], "x".join(map(str, v[2])))


@pytest.mark.parametrize("case", SMALL, ids=_ids)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("what", ["mass", "stiffness", "fused"])
def test_forward_small_every_row(wqa, case, dtype, what):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    recipe = ("random", 100 + d * 10 + p)
    f = ph.device_fields(sp, recipe, dtype)
    rows = _rows_all(sp)
    Mw, Kw = ph.oracle_forward(p, n_el, rows, recipe)
    nan = float("nan")
    M = torch.full((sp.n_rows, sp.slots_per_row), nan, dtype=dtype, device=sp.device)
    K = torch.full_like(M, nan)
    if what == "mass":
        sp.assemble_mass(f[0], M)
    elif what == "stiffness":
        sp.assemble_stiffness(f[1:], K)
    else:
        sp.assemble_fused(f[0], f[1:], M, K)
    torch.cuda.synchronize()
    if what in ("mass", "fused"):
        Mh = M.cpu().numpy()
        assert not np.isnan(Mh).any(), "unwritten slots in M"
        assert st.row_scaled_error(Mh, Mw) <= TOL[dtype]
        assert np.all(Mh[Mw == 0] == 0)
    if what in ("stiffness", "fused"):
        Kh = K.cpu().numpy()
        assert not np.isnan(Kh).any(), "unwritten slots in K"
        assert st.row_scaled_error(Kh, Kw) <= TOL[dtype]


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["plain", "compensated", "f64acc"])
@pytest.mark.parametrize("case", [(3, 3, (5, 4, 13)), (2, 2, (5, 21))], ids=_ids)
def test_forward_final_modes_fp32(wqa, case, mode):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    sp.set_final_mode(mode)
    recipe = ("random", 7)
    f = ph.device_fields(sp, recipe, torch.float32)
    M, K = sp.assemble_fused(f[0], f[1:])
    Mw, Kw = ph.oracle_forward(p, n_el, _rows_all(sp), recipe)
    assert st.row_scaled_error(M.cpu().numpy(), Mw) <= 1e-5
    assert st.row_scaled_error(K.cpu().numpy(), Kw) <= 1e-5


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["plain", "compensated", "f64acc"])
@pytest.mark.parametrize("case", [(3, 3, (5, 4, 13)), (3, 2, (4, 3, 21)), (2, 3, (7, 23))], ids=_ids)
def test_adjoint_final_modes_fp32(wqa, case, mode):
    """Every FP32 final pass of the adjoint (running sums, Dot2, FP64 accumulator) against
    the oracle at every point, both matrices at once."""
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    sp.set_final_mode(mode)
    n = list(sp.n_basis)
    rng = np.random.default_rng(57 + 3 * d + p)
    valid = si.slot_valid_mask(n_el, p).numpy()
    gM = np.where(valid, rng.normal(size=valid.shape), 0.0)
    gK = np.where(valid, rng.normal(size=valid.shape), 0.0)
    dc, da = sp.adjoint(torch.from_numpy(gM).to(sp.device, torch.float32),
                        torch.from_numpy(gK).to(sp.device, torch.float32))
    torch.cuda.synchronize()
    rows = _rows_all(sp)
    want, scale = ph.oracle_adjoint(p, n_el, oa.rule_tables(p, n_el), gM, gK, rows)
    pts = st.point_offsets(n, p, rows)
    got = [g.reshape(-1).cpu().numpy()[pts] for g in [dc] + list(da)]
    errs = ph.entry_errors(got, want, scale)
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("case", SMALL, ids=_ids)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("what", ["mass", "stiffness", "both"])
def test_adjoint_small_every_point(wqa, case, dtype, what):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    n = list(sp.n_basis)
    rng = np.random.default_rng(31 + d + p)
    valid = si.slot_valid_mask(n_el, p).numpy()
    # slots outside the space may hold anything, NaN and infinities included: they must
    # be ignored (every such slot meets a zero table factor, and 0 * NaN is NaN)
    junk = np.resize(np.array([np.nan, np.inf, -np.inf]), valid.shape)
    gM = np.where(valid, rng.normal(size=valid.shape), junk)
    gK = np.where(valid, rng.normal(size=valid.shape), junk[:, ::-1])
    use_m, use_k = what in ("mass", "both"), what in ("stiffness", "both")
    dc, da = sp.adjoint(torch.from_numpy(gM).to(sp.device, dtype) if use_m else None,
                        torch.from_numpy(gK).to(sp.device, dtype) if use_k else None)
    torch.cuda.synchronize()
    tabs = oa.rule_tables(p, n_el)
    rows = _rows_all(sp)
    want, scale = ph.oracle_adjoint(p, n_el, tabs, np.where(valid, gM, 0) if use_m else None,
                                    np.where(valid, gK, 0) if use_k else None, rows)
    pts = st.point_offsets(n, p, rows)
    got = ([dc] if use_m else []) + (list(da) if use_k else [])
    errs = ph.entry_errors([g.reshape(-1).cpu().numpy()[pts] for g in got], want, scale)
    assert max(errs) <= TOL[dtype], errs


def test_mass_2d_quadratic_32x32(wqa):
    # 2D C^1 quadratic, 32 x 32 elements, c = 1 + 0.5 sin sin, FP64 mass (every row)
    sp = wqa.Space(2, 2, (32, 32))
    recipe = ("sin_product",)
    f = ph.device_fields(sp, recipe, torch.float64)
    M = sp.assemble_mass(f[0])
    Mw, _ = ph.oracle_forward(2, (32, 32), _rows_all(sp), recipe, want_k=False)
    Mh = M.cpu().numpy()
    assert sp.n_rows == 1156 and sp.slots_per_row == 25
    assert st.row_scaled_error(Mh, Mw) <= 1e-12
    assert st.entry_relative_error(Mh, Mw) <= 1e-12


def _sampled_forward(wqa, d, p, n_el, recipe, dtype, mode=None, count=300):
    sp = wqa.Space(d, p, n_el)
    if mode is not None:
        sp.set_final_mode(mode)
    f = ph.device_fields(sp, recipe, dtype)
    M, K = sp.assemble_fused(f[0], f[1:])
    rows = st.sample_rows(list(sp.n_basis), p, count, seed=hash(n_el) % 1000)
    ridx = torch.from_numpy(rows).to(sp.device)
    Mg, Kg = M[ridx].cpu().numpy(), K[ridx].cpu().numpy()
    del M, K, f
    Mw, Kw = ph.oracle_forward(p, n_el, rows, recipe)
    return st.row_scaled_error(Mg, Mw), st.row_scaled_error(Kg, Kw), st.entry_relative_error(Mg, Mw)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_fused_3d_quadratic_64_cubed(wqa, dtype):
    eM, eK, eMe = _sampled_forward(wqa, 3, 2, (64, 64, 64), ("fourier", 2), dtype)
    print(f"64^3 quadratic {dtype}: row-scaled M {eM:.3e} K {eK:.3e}; entrywise M {eMe:.3e}")
    assert eM <= TOL[dtype] and eK <= TOL[dtype]


@pytest.mark.parametrize("dtype,mode", [(torch.float64, None), (torch.float32, 1),
                                        (torch.float32, 0), (torch.float32, 2)],
                         ids=["f64", "f32-dot2", "f32-plain", "f32-f64acc"])
def test_fused_3d_cubic_deformed_96_cubed(wqa, dtype, mode):
    eM, eK, eMe = _sampled_forward(wqa, 3, 3, (96, 96, 96), ("deformed",), dtype, mode)
    print(f"96^3 deformed cube {dtype} mode {mode}: row-scaled M {eM:.3e} K {eK:.3e}; entrywise M {eMe:.3e}")
    assert eM <= TOL[dtype] and eK <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_adjoint_3d_cubic_64_cubed(wqa, dtype):
    # 64^3 cubic, Fourier coefficients, G ~ N(0,1) (seeds 4001, 4002), gradients through
    # the autograd Function, sampled rows against the oracle's adjoint
    p, n_el = 3, (64, 64, 64)
    sp = wqa.Space(3, p, n_el)
    f = [x.requires_grad_(True) for x in ph.device_fields(sp, ("fourier", 4), dtype)]
    M, K = wqa.WQAssemble.apply(sp, *f)
    gM = si.upstream_gradient(n_el, p, 4001, dtype, sp.device)
    gK = si.upstream_gradient(n_el, p, 4002, dtype, sp.device)
    torch.autograd.backward([M, K], [gM, gK])
    rows = st.sample_rows(list(sp.n_basis), p, 200, seed=4)
    ridx = torch.from_numpy(rows).to(sp.device)
    pts = st.point_offsets(list(sp.n_basis), p, rows)
    tabs = oa.rule_tables(p, n_el)
    want, scale = ph.oracle_adjoint(p, n_el, tabs, gM[ridx].double().cpu().numpy(),
                                    gK[ridx].double().cpu().numpy(), rows)
    errs = ph.entry_errors([x.grad.reshape(-1).cpu().numpy()[pts] for x in f], want, scale)
    print(f"64^3 adjoint {dtype}: per-entry gradient errors {['%.3e' % e for e in errs]}")
    assert max(errs) <= TOL[dtype]


@pytest.mark.parametrize("layout", ["rows", "grid"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_forward_adjoint_160_cubed(wqa, dtype, layout):
    # the benchmark workload at full size, in the launch configuration the benchmark
    # times (default rules and final pass, samples stored row by row; the grid layout
    # too): 160^3 cubic, Fourier c and a_k, fused forward then adjoint with G ~ N(0,1)
    # (seeds 5001, 5002); a row sample covering every boundary class and both ragged tails
    # of the last direction against the oracle
    p, n_el = 3, (160, 160, 160)
    sp = wqa.Space(3, p, n_el)
    recipe = ("fourier", 5)
    f = ph.device_fields(sp, recipe, dtype)
    if layout == "rows":
        sp.set_sample_layout("rows")
        f = [sp.rows_from_grid(v) for v in f]
    M, K = sp.assemble_fused(f[0], f[1:])
    rows = st.sample_rows(list(sp.n_basis), p, 300, seed=5)
    ridx = torch.from_numpy(rows).to(sp.device)
    Mg, Kg = M[ridx].double().cpu().numpy(), K[ridx].double().cpu().numpy()
    del M, K, f
    gM = si.upstream_gradient(n_el, p, 5001, dtype, sp.device)
    gK = si.upstream_gradient(n_el, p, 5002, dtype, sp.device)
    dc, da = sp.adjoint(gM, gK)
    if layout == "rows":
        offs = rows[:, None] * sp.points_per_row + np.arange(sp.points_per_row)[None, :]
    else:
        offs = st.point_offsets(list(sp.n_basis), p, rows)
    pts = torch.from_numpy(offs.reshape(-1)).to(sp.device)
    grads = [g.reshape(-1)[pts].double().cpu().numpy().reshape(rows.size, -1) for g in [dc] + list(da)]
    gm, gk = gM[ridx].double().cpu().numpy(), gK[ridx].double().cpu().numpy()
    del gM, gK, dc, da
    torch.cuda.empty_cache()
    Mw, Kw = ph.oracle_forward(p, n_el, rows, recipe)
    want, scale = ph.oracle_adjoint(p, n_el, oa.rule_tables(p, n_el), gm, gk, rows)
    eM, eK = st.row_scaled_error(Mg, Mw), st.row_scaled_error(Kg, Kw)
    eg = max(ph.entry_errors(grads, want, scale))
    print(f"160^3 {dtype} {layout}: row-scaled M {eM:.3e} K {eK:.3e}; gradients per entry {eg:.3e}")
    assert eM <= TOL[dtype] and eK <= TOL[dtype] and eg <= TOL[dtype]


def test_central_differences_64_cubed(wqa):
    # dL/dtheta at 64 seeded quadrature points (16 per field) against central
    # differences h = 1e-6 in FP64 of L = <G_M, M> + <G_K, K>, evaluated by the oracle
    # on the one row that owns the point; points whose rule weight is 0 are skipped
    p, n_el = 3, (64, 64, 64)
    sp = wqa.Space(3, p, n_el)
    recipe = ("fourier", 4)
    f = ph.device_fields(sp, recipe, torch.float64)
    gM = si.upstream_gradient(n_el, p, 4001, torch.float64, sp.device)
    gK = si.upstream_gradient(n_el, p, 4002, torch.float64, sp.device)
    dc, da = sp.adjoint(gM, gK)
    grads = [dc] + list(da)
    tabs = oa.rule_tables(p, n_el)
    n = list(sp.n_basis)
    rng = np.random.default_rng(4064)
    Q = p + 1
    checked = 0
    h = 1e-6
    while checked < 64:
        field = checked // 16
        row = int(rng.integers(0, sp.n_rows))
        q = int(rng.integers(0, Q ** 3))
        qs = np.unravel_index(q, (Q, Q, Q))
        idx = st.row_multi(n, [row])
        # skip zero-weight (padding) points of the rule that field uses
        zero = False
        for k in range(3):
            key = "wK" if (field >= 1 and k == field - 1) else "wM"
            if tabs[key][k][idx[k][0] * Q + qs[k]] == 0.0:
                zero = True
        if zero:
            continue
        vals = ph.oracle_row_fields(tabs, p, n_el, np.array([row]), recipe)
        gm = gM[row].cpu().numpy()[None]
        gk = gK[row].cpu().numpy()[None]
        Ls = []
        for sign in (1, -1):
            v = [x.copy() for x in vals]
            v[field][0, q] += sign * h
            Mr, Kr = oa.assemble(p, n_el, tabs, c=v[0], a=v[1:], rows=[row], per_row=True)
            Ls.append((gm * Mr).sum() + (gk * Kr).sum())
        fd = (Ls[0] - Ls[1]) / (2 * h)
        off = st.point_offsets(n, p, [row])[0, q]
        got = float(grads[field].reshape(-1)[off])
        # rounding bound of the difference quotient for this row
        Mr, Kr = oa.assemble(p, n_el, tabs, c=vals[0], a=vals[1:], rows=[row], per_row=True)
        bound = 4e-16 * ((np.abs(gm * Mr)).sum() + (np.abs(gk * Kr)).sum()) / h
        assert abs(fd - got) <= 10 * bound + 1e-9 * abs(got), (field, row, q, fd, got, bound)
        checked += 1


def test_deterministic_and_stream_ordered(wqa):
    sp = wqa.Space(3, 3, (8, 9, 10))
    f = ph.device_fields(sp, ("random", 5), torch.float32)
    M1, K1 = sp.assemble_fused(f[0], f[1:])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        M2, K2 = sp.assemble_fused(f[0], f[1:])
    s.synchronize()
    assert torch.equal(M1, M2) and torch.equal(K1, K2)


@pytest.mark.parametrize("flat", [False, True], ids=["grid", "flat"])
def test_autograd_gradcheck_tiny(wqa, flat):
    # fields may come grid-shaped or flat; their gradients take the same shape
    sp = wqa.Space(2, 2, (3, 4))
    rng = np.random.default_rng(2)
    shape = (int(np.prod(sp.grid_shape)),) if flat else sp.grid_shape
    f = [torch.tensor(rng.uniform(0.5, 1.5, shape), device=sp.device, requires_grad=True)
         for _ in range(3)]
    assert torch.autograd.gradcheck(lambda *x: wqa.WQAssemble.apply(sp, *x), f, eps=1e-6, atol=1e-9,
                                    rtol=1e-7, fast_mode=True)


def test_errors_surface(wqa):
    sp = wqa.Space(3, 2, (3, 3, 3))
    c = torch.ones(sp.grid_shape, device=sp.device)
    with pytest.raises(ValueError):
        sp.assemble_mass(c.double(), M=torch.empty(3, device=sp.device))
    with pytest.raises(wqa.WQAError):
        sp.set_final_mode(7)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_properties_every_row_160_cubed(wqa, dtype):
    # 160^3 cubic in the benchmark's launch configuration, properties that hold at any
    # size, checked on all 4.33 M rows: with c = 1 the rows of M sum to the integral of
    # B_i (a product of (t_{i+p+1} - t_i)/(p+1) over directions) and M is symmetric; the
    # rows of K sum to 0 for any A; the adjoint satisfies <G, M(d)> = <adjoint(G), d>
    p, n_el = 3, (160, 160, 160)
    sp = wqa.Space(3, p, n_el)
    dev = sp.device
    n = list(sp.n_basis)
    ones = torch.ones(sp.grid_shape, dtype=dtype, device=dev)
    a = ph.device_fields(sp, ("fourier", 5), dtype)[1:]
    M, K = sp.assemble_fused(ones, a)
    rows = torch.arange(sp.n_rows, device=dev)
    idx = [rows // (n[1] * n[2]), (rows // n[2]) % n[1], rows % n[2]]
    want = torch.ones(sp.n_rows, dtype=torch.float64, device=dev)
    for k, e in enumerate(n_el):
        t = torch.cat([torch.zeros(p, dtype=torch.float64), torch.arange(e + 1, dtype=torch.float64) / e,
                       torch.ones(p, dtype=torch.float64)]).to(dev)
        want *= (t[idx[k] + p + 1] - t[idx[k]]) / (p + 1)
    tol = TOL[dtype]
    rs = M.double().sum(dim=1)
    assert ((rs - want).abs() / want).max().item() <= tol
    Kd = K.double()
    assert (Kd.sum(dim=1).abs() / Kd.abs().sum(dim=1)).max().item() <= tol
    del Kd, K
    # symmetry: slot s of row i is column j = i - p + s; its mirror slot in row j is 2p - s
    S = 2 * p + 1
    sl = torch.arange(S ** 3, device=dev)
    sk = [sl // (S * S), (sl // S) % S, sl % S]
    mirror = (S * S * (S - 1 - sk[0]) + S * (S - 1 - sk[1]) + (S - 1 - sk[2]))
    for r0 in range(0, sp.n_rows, 1 << 19):
        r = rows[r0:r0 + (1 << 19)]
        ik = [x[r0:r0 + (1 << 19)] for x in idx]
        jk = [ik[k][:, None] - p + sk[k][None, :] for k in range(3)]
        ok = (jk[0] >= 0) & (jk[0] < n[0]) & (jk[1] >= 0) & (jk[1] < n[1]) & (jk[2] >= 0) & (jk[2] < n[2])
        col = (jk[0] * n[1] + jk[1]) * n[2] + jk[2]
        mine = M[r]
        theirs = M[col.clamp(0, sp.n_rows - 1), mirror.expand_as(col)]
        scale = mine.abs().amax(dim=1, keepdim=True).double()
        diff = ((mine.double() - theirs.double()).abs() / scale)[ok]
        assert diff.max().item() <= tol
    del M
    # dot-product identity of the adjoint (mass part), in FP64 sums
    c = ph.device_fields(sp, ("fourier", 5), dtype)[0]
    gM = si.upstream_gradient(n_el, p, 5001, dtype, dev)
    Mc = sp.assemble_mass(c)
    lhs = (gM.double() * Mc.double()).sum().item()
    scale = (gM.double() * Mc.double()).abs().sum().item()
    del Mc
    dc, _ = sp.adjoint(gM, None)
    rhs = (dc.double() * c.double()).sum().item()
    assert abs(lhs - rhs) <= tol * scale


_LONG_TABLES = {}


@pytest.mark.parametrize("case", [(2, 2, (3, 2 ** 16)), (2, 3, (2 ** 16, 4))], ids=_ids)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_long_lines(wqa, case, dtype):
    """Long directions: 2^16 elements along the last direction (thousands of wave tiles
    per line) or along the first (65,539 lines).  Fused forward and adjoint on a row
    sample covering both ends of every direction, against the oracle."""
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    recipe = ("fourier", 2)
    f = ph.device_fields(sp, recipe, dtype)
    M, K = sp.assemble_fused(f[0], f[1:])
    rows = st.sample_rows(list(sp.n_basis), p, 200, seed=16)
    ridx = torch.from_numpy(rows).to(sp.device)
    Mg, Kg = M[ridx].double().cpu().numpy(), K[ridx].double().cpu().numpy()
    del M, K, f
    rng = np.random.default_rng(17)
    valid = si.slot_valid_mask(n_el, p).numpy()
    gM = np.where(valid, rng.normal(size=valid.shape), 0.0)
    gK = np.where(valid, rng.normal(size=valid.shape), 0.0)
    dc, da = sp.adjoint(torch.from_numpy(gM).to(sp.device, dtype), torch.from_numpy(gK).to(sp.device, dtype))
    pts = st.point_offsets(list(sp.n_basis), p, rows)
    grads = [g.reshape(-1).cpu().numpy()[pts] for g in [dc] + list(da)]
    if case not in _LONG_TABLES:
        _LONG_TABLES[case] = oa.rule_tables(p, n_el)
    tabs = _LONG_TABLES[case]
    fw = ph.oracle_row_fields(tabs, p, n_el, rows, recipe)
    Mw, Kw = oa.assemble(p, n_el, tabs, c=fw[0], a=fw[1:], rows=rows, per_row=True)
    want, scale = ph.oracle_adjoint(p, n_el, tabs, gM[rows], gK[rows], rows)
    eM, eK = st.row_scaled_error(Mg, Mw), st.row_scaled_error(Kg, Kw)
    eg = max(ph.entry_errors(grads, want, scale))
    print(f"long {case} {dtype}: row-scaled M {eM:.3e} K {eK:.3e}; gradients per entry {eg:.3e}")
    assert eM <= TOL[dtype] and eK <= TOL[dtype] and eg <= TOL[dtype]


def test_beyond_2_31_values_per_matrix(wqa):
    """210^3 cubic: 9,663,597 rows x 343 = 3.3e9 values per matrix, past 2^31 element
    offsets.  FP32 fused forward, then the adjoint with the assembled M and K as upstream
    gradients, on a row sample that includes the last rows, against the oracle."""
    p, n_el = 3, (210, 210, 210)
    sp = wqa.Space(3, p, n_el)
    assert sp.n_rows * sp.slots_per_row > 2 ** 31
    recipe = ("fourier", 5)
    f = ph.device_fields(sp, recipe, torch.float32)
    M, K = sp.assemble_fused(f[0], f[1:])
    del f
    last = sp.n_rows - 1
    rows = np.unique(np.concatenate([st.sample_rows(list(sp.n_basis), p, 200, seed=210),
                                     [last - 213 * 213, last - 213, last - 9, last - 1, last]]))
    ridx = torch.from_numpy(rows).to(sp.device)
    Mg, Kg = M[ridx].double().cpu().numpy(), K[ridx].double().cpu().numpy()
    dc, da = sp.adjoint(M, K)
    pts = torch.from_numpy(st.point_offsets(list(sp.n_basis), p, rows).reshape(-1)).to(sp.device)
    grads = [g.reshape(-1)[pts].double().cpu().numpy().reshape(rows.size, -1) for g in [dc] + list(da)]
    del M, K, dc, da
    torch.cuda.empty_cache()
    tabs = oa.rule_tables(p, n_el)
    fw = ph.oracle_row_fields(tabs, p, n_el, rows, recipe)
    Mw, Kw = oa.assemble(p, n_el, tabs, c=fw[0], a=fw[1:], rows=rows, per_row=True)
    want, scale = ph.oracle_adjoint(p, n_el, tabs, Mg, Kg, rows)
    eM, eK = st.row_scaled_error(Mg, Mw), st.row_scaled_error(Kg, Kw)
    eg = max(ph.entry_errors(grads, want, scale))
    print(f"210^3 f32: row-scaled M {eM:.3e} K {eK:.3e}; gradients per entry {eg:.3e}")
    assert eM <= 1e-5 and eK <= 1e-5 and eg <= 1e-5
