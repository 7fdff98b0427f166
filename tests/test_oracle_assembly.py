"""Pins for the oracle's FP64 assembly and adjoint (CPU only).

Constant coefficients on the (affine) unit box: the weighted rules are exact, so the
oracle must reproduce the exact Galerkin matrices, here built independently from
scipy's B-spline basis and numpy's Gauss-Legendre rule (Kronecker products of 1D Gram
matrices).  Variable coefficients: the method is a quadrature, so only its
invariants, linearity and convergence laws are pinned; the adjoint is pinned against
the forward map by the dot-product identity.
"""
import numpy as np
import pytest

import reference_1d as r1
import structured as st
import synth_inputs as si
from oracle import assembly as oa


def _kron(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def _grid_shape(p, n_el):
    return [(e + p) * (p + 1) for e in n_el]


def _all_ones(p, n_el):
    return np.ones(_grid_shape(p, n_el))


@pytest.mark.parametrize("p,n_el", [
    (2, (3,)), (3, (4,)), (2, (3, 4)), (2, (5, 8)), (3, (4, 5)), (3, (7, 6)),
    (2, (3, 4, 5)), (3, (4, 5, 4)),
])
def test_constant_coefficients_equal_exact_galerkin(p, n_el):
    # c = 1, A = I on the unit box: M = kron of 1D mass Grams, K = sum of krons with one
    # 1D stiffness Gram (exactness of the weighted rules on affine maps)
    d = len(n_el)
    tabs = oa.rule_tables(p, n_el)
    one = _all_ones(p, n_el)
    M, K = oa.assemble(p, n_el, tabs, c=one, a=[one] * d)
    n = [e + p for e in n_el]
    Ms = [r1.gram(p, e) for e in n_el]
    Ks = [r1.gram(p, e, deriv=True) for e in n_el]
    M_ref = _kron(Ms)
    K_ref = sum(_kron([Ks[k] if k == kk else Ms[k] for k in range(d)]) for kk in range(d))
    Md, Kd = st.to_dense(M, n, p), st.to_dense(K, n, p)
    assert np.abs(Md - M_ref).max() <= 1e-14 * np.abs(M_ref).max()
    assert np.abs(Kd - K_ref).max() <= 1e-13 * np.abs(K_ref).max()
    # every entry of the exact matrices outside the band is zero, so nothing was lost
    assert np.abs(M_ref[st.to_dense(np.ones_like(M), n, p) == 0]).max(initial=0) == 0


@pytest.mark.parametrize("p", [2, 3])
def test_one_dimensional_thousand_elements_agree_with_standard_gauss(p):
    # Sec. 4, first experiment: 1000 uniform elements, weighted rules vs standard Gauss
    n_el = (1000,)
    tabs = oa.rule_tables(p, n_el)
    one = _all_ones(p, n_el)
    M, K = oa.assemble(p, n_el, tabs, c=one, a=[one])
    n = [1000 + p]
    Mg, Kg = r1.gram(p, 1000), r1.gram(p, 1000, deriv=True)
    dM = np.abs(st.to_dense(M, n, p) - Mg)
    dK = np.abs(st.to_dense(K, n, p) - Kg)
    # Entries are O(h) and O(1/h).  Both sides evaluate the basis at FP64 points of
    # [0, 1], whose absolute resolution near x is ~1.1e-16 x, i.e. up to 1.1e-13 of
    # one element when h = 1e-3: the agreement is at that level, and ten times
    # tighter on the first tenth of the domain.
    assert dM.max() <= 5e-13 * np.abs(Mg).max()
    assert dK.max() <= 5e-13 * np.abs(Kg).max()
    assert dM[:100].max() <= 3e-14 * np.abs(Mg).max()
    assert dK[:100].max() <= 3e-14 * np.abs(Kg).max()


@pytest.mark.parametrize("p,n_el", [(2, (5, 6)), (3, (4, 7)), (3, (4, 5, 6))])
def test_row_sums(p, n_el):
    # c = 1: row sums of M are prod_k int B_{i_k} = prod_k (t_{i_k+p+1} - t_{i_k}) / (p+1);
    # any a_k: row sums of K vanish because sum_j grad B_j = 0
    d = len(n_el)
    tabs = oa.rule_tables(p, n_el)
    rng = np.random.default_rng(7)
    shape = _grid_shape(p, n_el)
    M, K = oa.assemble(p, n_el, tabs, c=np.ones(shape), a=[rng.uniform(0.5, 2, shape) for _ in range(d)])
    n = [e + p for e in n_el]
    idx = st.row_multi(n, np.arange(int(np.prod(n))))
    want = np.ones(len(idx[0]))
    for k in range(d):
        t = r1.knots(p, n_el[k])
        want *= (t[idx[k] + p + 1] - t[idx[k]]) / (p + 1)
    np.testing.assert_allclose(M.sum(axis=1), want, rtol=1e-14)
    assert np.abs(K.sum(axis=1)).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("p,n_el", [(2, (4, 5)), (3, (5, 4, 4))])
def test_symmetry_for_constant_coefficients_and_asymmetry_otherwise(p, n_el):
    d = len(n_el)
    tabs = oa.rule_tables(p, n_el)
    n = [e + p for e in n_el]
    shape = _grid_shape(p, n_el)
    M, K = oa.assemble(p, n_el, tabs, c=np.full(shape, 2.5), a=[np.full(shape, 1.0 + k) for k in range(d)])
    Md, Kd = st.to_dense(M, n, p), st.to_dense(K, n, p)
    assert np.abs(Md - Md.T).max() <= 1e-15 * np.abs(Md).max()
    assert np.abs(Kd - Kd.T).max() <= 1e-14 * np.abs(Kd).max()
    # a varying coefficient breaks the symmetry (each row has its own rule)
    axes = oa.grid_axes(tabs, "c")
    c = si.fourier_grid(axes, si.fourier_modes(99, 0, d)).numpy()
    M2, _ = oa.assemble(p, n_el, tabs, c=c)
    M2d = st.to_dense(M2, n, p)
    assert np.abs(M2d - M2d.T).max() > 1e-6 * np.abs(M2d).max()


def test_linearity():
    p, n_el = 3, (4, 5, 4)
    d = 3
    tabs = oa.rule_tables(p, n_el)
    rng = np.random.default_rng(11)
    shape = _grid_shape(p, n_el)
    c1, c2 = rng.normal(size=shape), rng.normal(size=shape)
    a1 = [rng.normal(size=shape) for _ in range(d)]
    a2 = [rng.normal(size=shape) for _ in range(d)]
    M1, K1 = oa.assemble(p, n_el, tabs, c1, a1)
    M2, K2 = oa.assemble(p, n_el, tabs, c2, a2)
    M3, K3 = oa.assemble(p, n_el, tabs, 2 * c1 - 3 * c2, [2 * x - 3 * y for x, y in zip(a1, a2)])
    np.testing.assert_allclose(M3, 2 * M1 - 3 * M2, atol=1e-14 * np.abs(M3).max())
    np.testing.assert_allclose(K3, 2 * K1 - 3 * K2, atol=1e-13 * np.abs(K3).max())


def test_row_subset_matches_full_assembly():
    p, n_el = 3, (5, 4, 6)
    tabs = oa.rule_tables(p, n_el)
    rng = np.random.default_rng(3)
    shape = _grid_shape(p, n_el)
    c = rng.normal(size=shape)
    a = [rng.normal(size=shape) for _ in range(3)]
    M, K = oa.assemble(p, n_el, tabs, c, a)
    rows = rng.choice(M.shape[0], 40, replace=False)
    Ms, Ks = oa.assemble(p, n_el, tabs, c, a, rows=rows)
    assert np.array_equal(Ms, M[rows]) and np.array_equal(Ks, K[rows])


@pytest.mark.parametrize("p", [2, 3])
def test_variable_coefficient_converges_at_first_order(p):
    # non-constant c: each row's rule integrates c B_i B_j only approximately
    # (Remark on non-affine maps, Sec. 3); the error against the exact integral
    # (dense Gauss) shrinks like h
    errs = []
    for ne in (16, 32, 64):
        n_el = (ne, ne)
        tabs = oa.rule_tables(p, n_el)
        axes = oa.grid_axes(tabs, "c")
        c = si.sin_product_c(axes[0][:, None], axes[1][None, :])
        M, _ = oa.assemble(p, n_el, tabs, c=c)
        # exact: c(x, y) = 1 + 0.5 sin sin is a sum of separable terms
        M1 = r1.gram(p, ne, m=12)
        S1 = r1.gram(p, ne, m=12, coef=lambda x: np.sin(2 * np.pi * x))
        n = [ne + p] * 2
        rows = np.arange(n[0] * n[1])
        i1, i2 = st.row_multi(n, rows)
        cols = st.columns(n, p, rows)
        j1, j2 = np.divmod(np.maximum(cols, 0), n[1])
        ref = M1[i1[:, None], j1] * M1[i2[:, None], j2] + 0.5 * S1[i1[:, None], j1] * S1[i2[:, None], j2]
        ref[cols < 0] = 0.0
        errs.append(np.abs(M - ref).max() / np.abs(ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert all(0.8 < r < 1.6 for r in rates), (errs, rates)


@pytest.mark.parametrize("p,n_el", [(2, (4, 3)), (3, (4, 5)), (2, (3, 4, 3)), (3, (4, 4, 5))])
def test_adjoint_dot_product_identity(p, n_el):
    # <G_M, M(dc)> + <G_K, K(da)> = <dL/dc, dc> + sum_k <dL/da_k, da_k>  (linear maps)
    d = len(n_el)
    tabs = oa.rule_tables(p, n_el)
    shape = _grid_shape(p, n_el)
    rng = np.random.default_rng(5)
    dc = rng.normal(size=shape)
    da = [rng.normal(size=shape) for _ in range(d)]
    M, K = oa.assemble(p, n_el, tabs, dc, da)
    n = [e + p for e in n_el]
    rows = np.arange(int(np.prod(n)))
    valid = si.slot_valid_mask(n_el, p).numpy()
    gM = rng.normal(size=M.shape) * valid
    gK = rng.normal(size=K.shape) * valid
    lhs = (gM * M).sum() + (gK * K).sum()
    gc, ga = oa.adjoint(p, n_el, tabs, gM, gK)
    pts = oa.row_points(p, n_el, rows)
    rhs = (gc * dc.reshape(-1)[pts]).sum() + sum((ga[k] * da[k].reshape(-1)[pts]).sum() for k in range(d))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(gM).sum() * np.abs(M).max())
    # invalid slots of the upstream gradient are ignored
    gM2 = gM + np.where(valid, 0.0, 1e3)
    gc2, _ = oa.adjoint(p, n_el, tabs, gM2, None)
    assert np.array_equal(gc2, gc)


def test_points_partition_the_grid():
    # each coefficient sample belongs to exactly one row (so the adjoint needs no atomics)
    for p, n_el in [(2, (3, 5)), (3, (4, 4, 5))]:
        n = [e + p for e in n_el]
        pts = oa.row_points(p, n_el, np.arange(int(np.prod(n))))
        assert np.array_equal(np.sort(pts.reshape(-1)), np.arange(int(np.prod(_grid_shape(p, n_el)))))


def test_adjoint_matches_central_differences():
    # L is linear in the coefficients, so central differences are exact up to rounding
    p, n_el = 3, (4, 4, 4)
    tabs = oa.rule_tables(p, n_el)
    shape = _grid_shape(p, n_el)
    rng = np.random.default_rng(17)
    c = rng.uniform(0.5, 1.5, shape)
    a = [rng.uniform(0.5, 1.5, shape) for _ in range(3)]
    n = [e + p for e in n_el]
    valid = si.slot_valid_mask(n_el, p).numpy()
    SD = 7 ** 3
    gM = rng.normal(size=(int(np.prod(n)), SD)) * valid
    gK = rng.normal(size=(int(np.prod(n)), SD)) * valid
    gc, ga = oa.adjoint(p, n_el, tabs, gM, gK)
    pts = oa.row_points(p, n_el, np.arange(int(np.prod(n))))
    h = 1e-6
    for trial in range(6):
        r = rng.integers(0, pts.shape[0])
        q = rng.integers(0, pts.shape[1])
        off = pts[r, q]
        field = trial % 4
        arrs = [c] + a
        plus = [x.copy() for x in arrs]
        minus = [x.copy() for x in arrs]
        plus[field].reshape(-1)[off] += h
        minus[field].reshape(-1)[off] -= h
        Mp, Kp = oa.assemble(p, n_el, tabs, plus[0], plus[1:], rows=[r])
        Mm, Km = oa.assemble(p, n_el, tabs, minus[0], minus[1:], rows=[r])
        fd = ((gM[r] * (Mp - Mm)).sum() + (gK[r] * (Kp - Km)).sum()) / (2 * h)
        got = gc[r, q] if field == 0 else ga[field - 1][r, q]
        assert abs(fd - got) <= 1e-7 * max(1.0, abs(got)), (trial, fd, got)


@pytest.mark.parametrize("p,n_el", [(2, (3, 4)), (3, (4, 5)), (2, (3, 4, 3)), (3, (4, 4, 5))])
def test_single_point_coefficient_touches_only_its_row(p, n_el):
    """A coefficient nonzero at one sample point (node q of row i) gives nonzeros in row i
    only, equal to prod_k w_k B_{i_k}(x_k) B_{i_k - p + s_k}(x_k): the weight multiplies
    both functions (eq:GaussQuadSys) and slot s_k is column i_k - p + s_k (Fig. 1).  For
    term k of K the stiffness node, weight and B' stand in direction k and the mass ones
    elsewhere (eq:Decompo).  Basis values from scipy, not the oracle's recursion; a
    transposed product, a shifted slot or a swapped direction fails here."""
    d = len(n_el)
    n = [e + p for e in n_el]
    Q, S = p + 1, 2 * p + 1
    tabs = oa.rule_tables(p, n_el)
    shape = _grid_shape(p, n_el)
    rng = np.random.default_rng(11 + p + d)

    def factor(k, i, q, deriv, xs, ws):
        x, w = xs[k][i[k] * Q + q[k]], ws[k][i[k] * Q + q[k]]
        B = r1.basis_at(p, n_el[k], [x], deriv=deriv)[0]
        out = np.zeros(S)
        for s in range(S):
            col = i[k] - p + s
            if 0 <= col < n[k]:
                out[s] = w * B[i[k]] * B[col]
        return out

    for _ in range(4):
        i = [int(rng.integers(0, nk)) for nk in n]
        q = [int(rng.integers(0, Q)) for _ in range(d)]
        kk = int(rng.integers(0, d))
        point = tuple(i[k] * Q + q[k] for k in range(d))
        c = np.zeros(shape)
        c[point] = 1.0
        a = [np.zeros(shape) for _ in range(d)]
        a[kk][point] = 1.0
        M, K = oa.assemble(p, n_el, tabs, c=c, a=a)
        expM = factor(0, i, q, False, tabs["xM"], tabs["wM"])
        expK = factor(0, i, q, kk == 0, tabs["xK"] if kk == 0 else tabs["xM"], tabs["wK"] if kk == 0 else tabs["wM"])
        for k in range(1, d):
            expM = np.kron(expM, factor(k, i, q, False, tabs["xM"], tabs["wM"]))
            stiff = k == kk
            expK = np.kron(expK, factor(k, i, q, stiff, tabs["xK"] if stiff else tabs["xM"],
                                        tabs["wK"] if stiff else tabs["wM"]))
        row = int(np.ravel_multi_index(i, n))
        others = np.arange(M.shape[0]) != row
        assert not M[others].any() and not K[others].any()
        np.testing.assert_allclose(M[row], expM, rtol=0, atol=1e-14 * max(np.abs(expM).max(), 1e-300))
        np.testing.assert_allclose(K[row], expK, rtol=0, atol=1e-13 * max(np.abs(expK).max(), 1e-300))


def _graded(n):
    return tuple((k / n) ** 1.4 for k in range(n + 1))


def _perturbed(n, seed=3, amp=0.15):
    rng = np.random.default_rng(seed)
    b = np.arange(n + 1) / n + np.concatenate([[0], rng.uniform(-amp, amp, n - 1), [0]]) / n
    return tuple(float(x) for x in b)


def _smooth_field(xyz, field):
    """A smooth test field at points [..., d], different for every field index."""
    d = xyz.shape[-1]
    out = 1.0 + 0.2 * np.prod(xyz, axis=-1)
    for k in range(d):
        out = out + 0.3 * np.cos(2 * np.pi * (k + 1 + field) * xyz[..., k] + 0.7 * k + field)
    return out


@pytest.mark.parametrize("p,n_el,meshes", [
    (2, (4, 5), (None, None)), (3, (5, 6), (None, "graded")),
    (2, (3, 4, 5), (None, None, None)), (2, (6, 3, 6), ("perturbed", None, "graded")),
    (3, (4, 5, 4), (None, None, None)),
])
def test_per_row_samples_equal_full_grid(p, n_el, meshes):
    """The oracle's per-row input mode (samples of the listed rows only, gathered with
    row_points from a grid, or evaluated at row_point_coords) gives the rows the
    full-grid mode gives: every point of a row is the grid point (i_k (p+1) + q_k)_k of
    that field's own grid (the mass nodes, or the stiffness nodes in direction k), in C
    order over q.  A wrong q order, a transposed gather or a field's grid taken for
    another's fails here."""
    d = len(n_el)
    breaks = None
    if any(m is not None for m in meshes):
        breaks = [None if m is None else (_graded(e) if m == "graded" else _perturbed(e))
                  for m, e in zip(meshes, n_el)]
    tabs = oa.rule_tables(p, n_el, breaks)
    n = [e + p for e in n_el]
    rng = np.random.default_rng(23 + p + d)
    rows = np.unique(np.concatenate([[0, int(np.prod(n)) - 1],
                                     rng.integers(0, int(np.prod(n)), size=25)]))
    # random samples: one grid per field, gathered with row_points
    shape = _grid_shape(p, n_el)
    grids = [rng.normal(size=shape) for _ in range(d + 1)]
    pts = oa.row_points(p, n_el, rows)
    assert np.array_equal(pts, st.point_offsets(n, p, rows))
    Mf, Kf = oa.assemble(p, n_el, tabs, c=grids[0], a=grids[1:], rows=rows)
    Mr, Kr = oa.assemble(p, n_el, tabs, c=grids[0].reshape(-1)[pts],
                         a=[g.reshape(-1)[pts] for g in grids[1:]], rows=rows, per_row=True)
    assert np.array_equal(Mf, Mr) and np.array_equal(Kf, Kr)
    # a smooth field of the coordinates: on the full grid of each field's own axes, and at
    # the coordinates row_point_coords gives for the listed rows
    full, per_row = [], []
    for fi, field in enumerate(["c"] + list(range(d))):
        axes = oa.grid_axes(tabs, field)
        mesh = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
        full.append(_smooth_field(mesh, fi))
        per_row.append(_smooth_field(oa.row_point_coords(p, n_el, tabs, rows, field), fi))
    Mf, Kf = oa.assemble(p, n_el, tabs, c=full[0], a=full[1:], rows=rows)
    Mr, Kr = oa.assemble(p, n_el, tabs, c=per_row[0], a=per_row[1:], rows=rows, per_row=True)
    np.testing.assert_allclose(Mr, Mf, rtol=0, atol=1e-14 * np.abs(Mf).max())
    np.testing.assert_allclose(Kr, Kf, rtol=0, atol=1e-14 * np.abs(Kf).max())
    # the fields differ from each other, so a swapped field would not pass the above
    assert np.abs(per_row[1] - per_row[2]).max() > 0.1


@pytest.mark.parametrize("p,n_el", [(2, (3, 4)), (3, (4, 5)), (2, (3, 4, 3)), (3, (4, 4, 5))])
def test_adjoint_and_term_magnitudes_from_scipy_factors(p, n_el):
    """Every gradient entry is sum_s G[s] prod_k f_k(q_k, s_k), with
    f_k = w B_{i_k}(x) B_{i_k - p + s_k}(x) at node q_k of row i_k (B' and the stiffness
    rule in direction k' for da_k', eq:Decompo), and the oracle's absolute variant is
    sum_s |G[s]| prod_k |f_k|.  Factors from scipy's B-splines, sums by einsum over
    every row; slots outside the space hold NaN for the oracle and must be skipped."""
    d = len(n_el)
    n = [e + p for e in n_el]
    Q, S = p + 1, 2 * p + 1
    tabs = oa.rule_tables(p, n_el)

    def factors(k, kind):
        xs, ws = (tabs["xM"][k], tabs["wM"][k]) if kind == "mass" else (tabs["xK"][k], tabs["wK"][k])
        B = r1.basis_at(p, n_el[k], xs, deriv=(kind == "stiffness"))          # [n Q, n]
        F = np.zeros((n[k], Q, S))
        for i in range(n[k]):
            for q in range(Q):
                for s in range(S):
                    col = i - p + s
                    if 0 <= col < n[k]:
                        F[i, q, s] = ws[i * Q + q] * B[i * Q + q, i] * B[i * Q + q, col]
        return F

    FM = [factors(k, "mass") for k in range(d)]
    FK = [factors(k, "stiffness") for k in range(d)]
    rows = np.arange(int(np.prod(n)))
    idx = st.row_multi(n, rows)
    valid = si.slot_valid_mask(n_el, p).numpy()
    rng = np.random.default_rng(41 + p + d)
    gM = np.where(valid, rng.normal(size=valid.shape), 0.0)
    gK = np.where(valid, rng.normal(size=valid.shape), 0.0)
    poisonM = np.where(valid, gM, np.nan)
    poisonK = np.where(valid, gK, np.inf)

    def contract(Fs, G):
        ops = [F[i] for F, i in zip(Fs, idx)]                             # [rows, Q, S] each
        Gs = G.reshape([len(rows)] + [S] * d)
        if d == 2:
            return np.einsum("ras,rbt,rst->rab", *ops, Gs).reshape(len(rows), -1)
        return np.einsum("ras,rbt,rcu,rstu->rabc", *ops, Gs).reshape(len(rows), -1)

    dc, da = oa.adjoint(p, n_el, tabs, poisonM, poisonK)
    ac, aa = oa.adjoint(p, n_el, tabs, poisonM, poisonK, absolute=True)
    want_c = contract(FM, gM)
    want_ac = contract([np.abs(F) for F in FM], np.abs(gM))
    scale = np.abs(want_ac).max()
    np.testing.assert_allclose(dc, want_c, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(ac, want_ac, rtol=0, atol=1e-14 * scale)
    for kk in range(d):
        Fs = [FK[k] if k == kk else FM[k] for k in range(d)]
        want = contract(Fs, gK)
        want_abs = contract([np.abs(F) for F in Fs], np.abs(gK))
        scale = np.abs(want_abs).max()
        np.testing.assert_allclose(da[kk], want, rtol=0, atol=1e-14 * scale)
        np.testing.assert_allclose(aa[kk], want_abs, rtol=0, atol=1e-14 * scale)
        assert np.all(aa[kk] >= np.abs(da[kk]) * (1 - 1e-14))
    # mass factors are non-negative (positive weights, B >= 0): for G >= 0 the two agree
    gpos = np.abs(gM)
    d1, _ = oa.adjoint(p, n_el, tabs, gpos, None)
    a1, _ = oa.adjoint(p, n_el, tabs, gpos, None, absolute=True)
    np.testing.assert_allclose(a1, d1, rtol=1e-14, atol=0)
