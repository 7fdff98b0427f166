"""GPU parity of the load vector and the matrix-free products (eq:Load, eq:LinSys):
wqa_assemble_load, wqa_apply_mass and wqa_apply_stiffness against the oracle's assembled
rows (b_i = sum_s M_is with c = f; y_i = sum_s M_is x_col(i,s)), on small spaces (every
row) and on the 160^3 cubic workload (sampled rows).  Bar: the error of each row over the
magnitude of its terms, sum_s |M_is x_col| (the products cancel, the rows of K sum to 0):
FP64 1e-12, FP32 1e-5.  Closed forms: b with f = 1 is integral B_i, the product of the
directions' (t_{i+p+1} - t_i)/(p+1); K times a constant vector is 0."""
import numpy as np
import pytest
import torch

import parity_helpers as ph
import structured as st
from oracle import assembly as oa

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}

# 3D: ragged blocks of rows in every direction; the last two also have blocks whose rows
# are all interior along the last direction (its banded loops)
SMALL = [(2, 2, (3, 4)), (2, 2, (5, 21)), (2, 3, (7, 23)), (3, 2, (4, 3, 21)), (3, 3, (4, 4, 4)),
         (3, 3, (6, 7, 23)), (3, 3, (6, 9, 40)), (3, 2, (5, 7, 47))]


@pytest.fixture(scope="module")
def wqa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1710_01048_amd as mod
    return mod


def _ids(v):
    return "d%d-p%d-%s" % (v[0], v[1], "x".join(map(str, v[2])))


def _product_error(y, Mw, cols, x):
    """max_i |y_i - sum_s M_is x_col| / sum_s |M_is x_col| over the rows of Mw."""
    xs = np.where(cols >= 0, x[np.maximum(cols, 0)], 0.0)
    terms = Mw * xs
    want = terms.sum(axis=1)
    scale = np.abs(terms).sum(axis=1)
    scale[scale == 0] = 1.0
    return float((np.abs(np.asarray(y, dtype=np.float64) - want) / scale).max())


@pytest.mark.parametrize("case", SMALL, ids=_ids)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_products_and_load_small_every_row(wqa, case, dtype):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    recipe = ("random", 7 + d + p)
    f = ph.device_fields(sp, recipe, dtype)
    rows = np.arange(sp.n_rows)
    Mw, Kw = ph.oracle_forward(p, n_el, rows, recipe)
    cols = st.columns(list(sp.n_basis), p, rows)
    x = np.random.default_rng(11).standard_normal(sp.n_rows)
    xd = torch.from_numpy(x).to(sp.device, dtype)
    if dtype == torch.float32:
        x = xd.double().cpu().numpy()          # the oracle sees the values the kernel reads
    y = torch.full((sp.n_rows,), float("nan"), dtype=dtype, device=sp.device)
    sp.apply_mass(f[0], xd, y)
    eM = _product_error(y.cpu().numpy(), Mw, cols, x)
    sp.apply_stiffness(f[1:], xd, y)
    eK = _product_error(y.cpu().numpy(), Kw, cols, x)
    sp.load_vector(f[0], y)
    eb = _product_error(y.cpu().numpy(), Mw, cols, np.ones(sp.n_rows))
    print(f"{_ids(case)} {dtype}: M x {eM:.2e}, K x {eK:.2e}, load {eb:.2e}")
    assert max(eM, eK, eb) <= TOL[dtype]


@pytest.mark.parametrize("case", [(2, 3, (7, 9)), (3, 2, (5, 6, 9)), (3, 3, (6, 5, 20))], ids=_ids)
def test_closed_forms(wqa, case):
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    ones = torch.ones(sp.grid_shape, dtype=torch.float64, device=sp.device)
    b = sp.load_vector(ones).cpu().numpy()
    # integral of B_i: product over directions of (t_{i+p+1} - t_i) / (p+1), open knots
    want = np.ones(sp.n_rows)
    idx = st.row_multi(list(sp.n_basis), np.arange(sp.n_rows))
    for k, e in enumerate(n_el):
        t = np.concatenate([np.zeros(p), np.arange(e + 1) / e, np.ones(p)])
        want *= (t[idx[k] + p + 1] - t[idx[k]]) / (p + 1)
    assert np.abs(b - want).max() <= 1e-14 * want.max()
    # K annihilates constants (the rows of K sum to 0 for any A)
    y = sp.apply_stiffness([ones] * d, torch.full((sp.n_rows,), 3.0, dtype=torch.float64, device=sp.device))
    K = sp.assemble_stiffness([ones] * d).cpu().numpy()
    assert np.abs(y.cpu().numpy()).max() <= 1e-13 * 3.0 * np.abs(K).sum(axis=1).max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_products_160_cubed(wqa, dtype):
    p, n_el = 3, (160, 160, 160)
    sp = wqa.Space(3, p, n_el)
    recipe = ("fourier", 5)
    f = ph.device_fields(sp, recipe, dtype)
    g = torch.Generator(device=sp.device)
    g.manual_seed(5003)
    xd = torch.randn(sp.n_rows, generator=g, dtype=torch.float64, device=sp.device).to(dtype)
    yM = sp.apply_mass(f[0], xd)
    yK = sp.apply_stiffness(f[1:], xd)
    b = sp.load_vector(f[0])
    rows = st.sample_rows(list(sp.n_basis), p, 300, seed=6)
    cols = st.columns(list(sp.n_basis), p, rows)
    x = xd.double().cpu().numpy()
    ridx = torch.from_numpy(rows).to(sp.device)
    Mw, Kw = ph.oracle_forward(p, n_el, rows, recipe)
    eM = _product_error(yM[ridx].cpu().numpy(), Mw, cols, x)
    eK = _product_error(yK[ridx].cpu().numpy(), Kw, cols, x)
    eb = _product_error(b[ridx].cpu().numpy(), Mw, cols, np.ones_like(x))
    print(f"160^3 {dtype}: M x {eM:.2e}, K x {eK:.2e}, load {eb:.2e}")
    assert max(eM, eK, eb) <= TOL[dtype]


@pytest.mark.parametrize("case", [(3, 3, (4, 5, 3000)), (3, 3, (3000, 4, 5)), (3, 2, (4, 3000, 5))], ids=_ids)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_products_long_directions(wqa, case, dtype):
    """3D products with one long direction (hundreds of row blocks along it, few across the
    others): sampled rows covering both ends of every direction, against the oracle, in both
    sample layouts (the same bits)."""
    d, p, n_el = case
    sp = wqa.Space(d, p, n_el)
    recipe = ("fourier", 3)
    f = ph.device_fields(sp, recipe, dtype)
    g = torch.Generator(device=sp.device)
    g.manual_seed(5007)
    xd = torch.randn(sp.n_rows, generator=g, dtype=torch.float64, device=sp.device).to(dtype)
    yM = sp.apply_mass(f[0], xd)
    yK = sp.apply_stiffness(f[1:], xd)
    rows = st.sample_rows(list(sp.n_basis), p, 200, seed=8)
    cols = st.columns(list(sp.n_basis), p, rows)
    x = xd.double().cpu().numpy()
    ridx = torch.from_numpy(rows).to(sp.device)
    Mw, Kw = ph.oracle_forward(p, n_el, rows, recipe)
    eM = _product_error(yM[ridx].cpu().numpy(), Mw, cols, x)
    eK = _product_error(yK[ridx].cpu().numpy(), Kw, cols, x)
    print(f"long {_ids(case)} {dtype}: M x {eM:.2e}, K x {eK:.2e}")
    assert max(eM, eK) <= TOL[dtype]
    sp.set_sample_layout("rows")
    fr = [sp.rows_from_grid(v) for v in f]
    assert torch.equal(sp.apply_mass(fr[0], xd), yM)
    assert torch.equal(sp.apply_stiffness(fr[1:], xd), yK)
