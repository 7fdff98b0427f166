"""The HIP kernels on non-uniform knots: forward and adjoint against the oracle on every
row and point of small spaces with graded and perturbed breakpoints, and the Laplace
eigenvalues on graded meshes converging at rate 2p like on uniform ones (Sec. 4)."""
import math

import numpy as np
import pytest
import torch

import parity_helpers as ph
import structured as st
import synth_inputs as si
from oracle import assembly as oa
from test_oracle_nonuniform import MESHES, N

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.fixture(scope="module")
def wqa():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1710_01048_amd as mod
    return mod


CASES = [(2, 2, (N, N), ("graded", "perturbed")), (3, 2, (N, 5, N), ("perturbed", None, "graded")),
         (3, 3, (N, N, N), ("graded", "perturbed", "graded"))]


def _ids(c):
    return "d%d-p%d" % (c[0], c[1])


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_forward_and_adjoint_every_row(wqa, case, dtype):
    d, p, n_el, meshes = case
    breaks = [None if m is None else MESHES[m] for m in meshes]
    sp = wqa.Space(d, p, n_el, breaks=breaks)
    tabs = oa.rule_tables(p, n_el, breaks)
    fields = ph._random_fields(p, n_el, 21)
    f = [torch.from_numpy(x).to(sp.device, dtype) for x in fields]
    M, K = sp.assemble_fused(f[0], f[1:])
    Mw, Kw = oa.assemble(p, n_el, tabs, c=fields[0], a=fields[1:])
    assert st.row_scaled_error(M.cpu().numpy(), Mw) <= TOL[dtype]
    assert st.row_scaled_error(K.cpu().numpy(), Kw) <= TOL[dtype]
    gM = si.upstream_gradient(n_el, p, 31, dtype, sp.device)
    gK = si.upstream_gradient(n_el, p, 32, dtype, sp.device)
    dc, da = sp.adjoint(gM, gK)
    rows = np.arange(sp.n_rows)
    want, scale = ph.oracle_adjoint(p, n_el, tabs, gM.double().cpu().numpy(), gK.double().cpu().numpy(), rows)
    pts = st.point_offsets([e + p for e in n_el], p, rows)
    errs = ph.entry_errors([g.reshape(-1).cpu().numpy()[pts] for g in [dc] + list(da)], want, scale)
    assert max(errs) <= TOL[dtype], errs


@pytest.mark.parametrize("p", [2, 3])
def test_graded_mesh_eigenvalues_converge_at_rate_2p(wqa, p):
    from paper_1710_01048_amd import eigen
    exact = eigen.exact_laplace_eigenvalues(2, 10)[9]
    errs = []
    for n in (16, 32, 64):
        b = np.array([(k / n) ** 1.4 for k in range(n + 1)])
        lam = eigen.laplace_eigenvalues(2, p, (n, n), count=10, breaks=[b, b])
        errs.append((lam[9] - exact) / exact)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(f"graded 2D p={p}: relative errors {['%.3e' % e for e in errs]}, rates {rates}")
    assert all(e > 0 for e in errs)
    assert abs(rates[-1] - 2 * p) < 0.35, (errs, rates)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_products_and_load_vector_on_nonuniform_knots(wqa, dtype):
    from test_gpu_apply import _product_error
    d, p, n_el, meshes = CASES[2]
    breaks = [None if m is None else MESHES[m] for m in meshes]
    sp = wqa.Space(d, p, n_el, breaks=breaks)
    tabs = oa.rule_tables(p, n_el, breaks)
    fields = ph._random_fields(p, n_el, 23)
    f = [torch.from_numpy(v).to(sp.device, dtype) for v in fields]
    Mw, Kw = oa.assemble(p, n_el, tabs, c=fields[0], a=fields[1:])
    cols = st.columns([e + p for e in n_el], p, np.arange(sp.n_rows))
    x = np.random.default_rng(29).standard_normal(sp.n_rows)
    xd = torch.from_numpy(x).to(sp.device, dtype)
    x = xd.double().cpu().numpy()
    eM = _product_error(sp.apply_mass(f[0], xd).cpu().numpy(), Mw, cols, x)
    eK = _product_error(sp.apply_stiffness(f[1:], xd).cpu().numpy(), Kw, cols, x)
    eb = _product_error(sp.load_vector(f[0]).cpu().numpy(), Mw, cols, np.ones_like(x))
    assert max(eM, eK, eb) <= TOL[dtype]
