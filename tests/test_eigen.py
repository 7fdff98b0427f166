"""Laplace eigenvalue experiments (Sec. 4), CPU side: the closed-form spectrum, the band
to CSR conversion, and the solver pipeline on oracle-assembled matrices (the GPU-assembled
runs are in test_gpu_eigen.py)."""
import math

import numpy as np
import pytest

import structured as st
from oracle import assembly as oa


@pytest.fixture(scope="module")
def eig():
    from paper_1710_01048_amd import eigen
    return eigen


def test_exact_spectrum(eig):
    pi2 = math.pi ** 2
    # unit square: |k|^2 = 2, 5, 5, 8, 10, 10, 13, 13, 17, 17, ... (k_i >= 1)
    assert np.allclose(eig.exact_laplace_eigenvalues(2, 10) / pi2, [2, 5, 5, 8, 10, 10, 13, 13, 17, 17])
    # unit cube: 3, 6 (x3), 9 (x3), 11 (x3), 12
    assert np.allclose(eig.exact_laplace_eigenvalues(3, 11) / pi2, [3, 6, 6, 6, 9, 9, 9, 11, 11, 11, 12])


def _oracle_matrices(p, n_el):
    tabs = oa.rule_tables(p, n_el)
    shape = [(e + p) * (p + 1) for e in n_el]
    ones = np.ones(shape)
    return oa.assemble(p, n_el, tabs, c=ones, a=[ones] * len(n_el))


@pytest.mark.parametrize("p,n_el", [(2, (3, 5)), (3, (4, 4, 5))])
def test_band_to_csr_matches_dense(eig, p, n_el):
    M, K = _oracle_matrices(p, n_el)
    n = [e + p for e in n_el]
    for X in (M, K):
        assert np.array_equal(eig.band_to_csr(X, n, p).toarray(), st.to_dense(X, n, p))


def test_interior_indices(eig):
    n = [5, 4, 6]
    inner = eig.interior_indices(n)
    idx = np.array(np.unravel_index(inner, n))
    assert inner.size == 3 * 2 * 4
    assert all(((idx[k] >= 1) & (idx[k] <= n[k] - 2)).all() for k in range(3))


@pytest.mark.parametrize("p", [2, 3])
def test_oracle_spectrum_converges_at_rate_2p(eig, p):
    # 2D, c = 1 and A = I on the identity map: the rules are exact, so the discrete
    # eigenvalues are the Galerkin ones, above the exact ones (min-max), and the 10-th
    # converges at rate 2p (Sec. 4)
    exact = eig.exact_laplace_eigenvalues(2, 10)
    errs = []
    for N in (8, 16, 32):
        M, K = _oracle_matrices(p, (N, N))
        lam = eig.solve_laplace(M, K, [N + p] * 2, p, count=10)
        assert np.all(lam >= exact * (1 - 1e-12))
        errs.append((lam[9] - exact[9]) / exact[9])
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(rates[-1] - 2 * p) < 0.35, (errs, rates)


@pytest.mark.parametrize("p", [2, 3])
def test_gram_1d_and_fast_diagonalization(eig, p):
    # the preconditioner's 1D matrices are the exact Galerkin ones (scipy reference with
    # another Gauss order), and the fast diagonalization inverts the Kronecker sum
    import reference_1d as r1
    n_el = (5, 4, 6)
    Ms, Ks = [], []
    for e in n_el:
        Mk, Kk = eig.gram_1d(p, e)
        np.testing.assert_allclose(Mk, r1.gram(p, e, m=p + 3), rtol=0, atol=1e-15)
        np.testing.assert_allclose(Kk, r1.gram(p, e, deriv=True, m=p + 3), rtol=0, atol=1e-12 * e * e)
        keep = np.arange(1, Mk.shape[0] - 1)
        Ms.append(Mk[np.ix_(keep, keep)])
        Ks.append(Kk[np.ix_(keep, keep)])
    K = (np.kron(np.kron(Ks[0], Ms[1]), Ms[2]) + np.kron(np.kron(Ms[0], Ks[1]), Ms[2])
         + np.kron(np.kron(Ms[0], Ms[1]), Ks[2]))
    x = np.random.default_rng(3).standard_normal(K.shape[0])
    np.testing.assert_allclose(eig.fast_diagonalization(Ms, Ks)(K @ x), x, rtol=0, atol=1e-10)


@pytest.mark.parametrize("p,n_el", [(2, (16, 16)), (3, (6, 6, 6)), (2, (5, 7, 6))])
def test_conjugate_gradient_inner_solves_give_the_same_spectrum(eig, p, n_el):
    M, K = _oracle_matrices(p, n_el)
    n = [e + p for e in n_el]
    direct = eig.solve_laplace(M, K, n, p, count=10, inner_solver="direct")
    pcg = eig.solve_laplace(M, K, n, p, count=10, inner_solver="pcg")
    np.testing.assert_allclose(pcg, direct, rtol=1e-12, atol=0)
