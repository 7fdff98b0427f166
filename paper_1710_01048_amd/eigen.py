"""Laplace eigenvalue experiments on assembled matrices (Sec. 4 of the paper).

The generalized eigenproblem K u = lambda M u of -Laplace u = lambda u on the unit square
or cube with u = 0 on the boundary.  M (c = 1) and K (A = I) come from the library's
kernels on the identity geometry, so the weighted rules are exact (remark on affine maps
closing Sec. 3) and the discrete spectrum is the Galerkin one of the spline space.  The
exact spectrum is pi^2 (k_1^2 + ... + k_d^2), k_i >= 1; the paper reports the 10-th
eigenvalue converging at rate about 2p under refinement (Fig. of Sec. 4).

Homogeneous Dirichlet conditions remove the basis functions that do not vanish on the
boundary: with open knot vectors only the first and the last function of each direction
(eq:Gmap3), so the unknowns are the rows with 1 <= i_k <= n_k - 2 in every direction.

The eigensolver is scipy's shift-invert Lanczos on the host (the assembly is the part
that runs on the GPU).
"""
import itertools
import math

import numpy as np


def band_to_csr(values, n_basis, degree):
    """scipy CSR matrix [rows, rows] from the band layout [rows][(2p+1)^d] (slot s_k of row
    i is column i_k - p + s_k in direction k; slots outside the space are dropped)."""
    import scipy.sparse as sps
    v = np.asarray(values)
    n = [int(x) for x in n_basis]
    d, p = len(n), int(degree)
    S = 2 * p + 1
    rows = int(np.prod(n))
    if v.shape != (rows, S ** d):
        raise ValueError(f"band values of shape {v.shape}, expected {(rows, S ** d)}")
    idx = np.array(np.unravel_index(np.arange(rows), n))                 # [d, rows]
    sl = np.array(np.unravel_index(np.arange(S ** d), [S] * d))          # [d, S^d]
    cols = np.zeros((rows, S ** d), dtype=np.int64)
    ok = np.ones((rows, S ** d), dtype=bool)
    for k in range(d):
        j = idx[k][:, None] - p + sl[k][None, :]
        ok &= (j >= 0) & (j < n[k])
        cols = cols * n[k] + j
    r = np.broadcast_to(np.arange(rows)[:, None], cols.shape)
    return sps.csr_matrix((v[ok], (r[ok], cols[ok])), shape=(rows, rows))


def interior_indices(n_basis):
    """Flat indices of the basis functions that vanish on the boundary."""
    n = [int(x) for x in n_basis]
    grids = np.meshgrid(*[np.arange(1, nk - 1) for nk in n], indexing="ij")
    return np.ravel_multi_index([g.ravel() for g in grids], n)


def exact_laplace_eigenvalues(dim, count):
    """The `count` smallest eigenvalues pi^2 |k|^2 (k_i >= 1) of the Dirichlet Laplacian on
    the unit d-cube, with multiplicity, ascending."""
    kmax = int(math.isqrt(count)) + 3
    vals = sorted(sum(k * k for k in ks) for ks in itertools.product(range(1, kmax + 1), repeat=dim))
    return math.pi ** 2 * np.array(vals[:count], dtype=np.float64)


def gram_1d(degree, n_elem, breaks=None):
    """Dense 1D Galerkin mass and stiffness matrices (int B_i B_j, int B_i' B_j') of the open
    B-spline basis, by element-wise Gauss-Legendre with p + 1 points (exact for these
    polynomial integrands).  Used only to precondition the eigensolver's inner solves."""
    from scipy.interpolate import BSpline
    p, ne = int(degree), int(n_elem)
    b = np.linspace(0.0, 1.0, ne + 1) if breaks is None else np.asarray(breaks, dtype=np.float64)
    t = np.concatenate([np.zeros(p), b, np.ones(p)])
    g, gw = np.polynomial.legendre.leggauss(p + 1)
    h = np.diff(b)
    x = (b[:-1, None] + (g[None, :] + 1) / 2 * h[:, None]).reshape(-1)
    w = (gw[None, :] * h[:, None] / 2).reshape(-1)
    spl = BSpline(t, np.eye(ne + p), p, extrapolate=False)
    B = np.nan_to_num(spl(x))
    D = np.nan_to_num(spl.derivative()(x))
    return (B * w[:, None]).T @ B, (D * w[:, None]).T @ D


def fast_diagonalization(masses, stiffnesses):
    """Exact inverse of the Kronecker sum sum_k M_1 x .. x K_k x .. x M_d, applied through
    the generalized eigenvectors of each direction's pair (K_k V = M_k V L, V^T M_k V = I;
    Lynch, Rice and Thomas' fast diagonalization): a preconditioner for the stiffness
    matrix of constant coefficients on a tensor mesh.  Returns r -> approx K^{-1} r."""
    from scipy.linalg import eigh
    vecs, vals = [], []
    for Mk, Kk in zip(masses, stiffnesses):
        lam, V = eigh(Kk, Mk)
        vecs.append(V)
        vals.append(lam)
    shape = [V.shape[0] for V in vecs]
    d = len(shape)
    denom = np.zeros(shape)
    for k in range(d):
        view = [1] * d
        view[k] = -1
        denom = denom + vals[k].reshape(view)

    def apply(r):
        x = np.asarray(r, dtype=np.float64).reshape(shape)
        for k in range(d):
            x = np.moveaxis(np.tensordot(vecs[k].T, x, axes=(1, k)), 0, k)
        x = x / denom
        for k in range(d):
            x = np.moveaxis(np.tensordot(vecs[k], x, axes=(1, k)), 0, k)
        return x.reshape(-1)

    return apply


def solve_laplace(M_band, K_band, n_basis, degree, count=10, breaks=None, inner_solver="direct"):
    """The `count` smallest eigenvalues of K u = lambda M u restricted to the interior
    functions, from band-layout matrices (host arrays, FP64).

    Shift-invert Lanczos (ARPACK) about 0.  inner_solver="direct" factors K (sparse LU);
    "pcg" solves with K by conjugate gradients to 1e-14, preconditioned by the fast
    diagonalization of the exact 1D Galerkin matrices of the same knots (``breaks`` as
    for ``Space``), which takes a few iterations where a sparse LU of a 3D problem takes
    minutes.  Either way the operator is the given K and M."""
    import scipy.sparse.linalg as spla
    inner = interior_indices(n_basis)
    M = band_to_csr(np.asarray(M_band, dtype=np.float64), n_basis, degree)[inner][:, inner]
    K = band_to_csr(np.asarray(K_band, dtype=np.float64), n_basis, degree)[inner][:, inner]
    # constant coefficients: symmetric up to rounding; the Lanczos solver wants it exact
    M = ((M + M.T) * 0.5).tocsc()
    K = ((K + K.T) * 0.5).tocsc()
    if inner_solver == "direct":
        w = spla.eigsh(K, k=count, M=M, sigma=0.0, which="LM", return_eigenvectors=False)
        return np.sort(w)
    if inner_solver != "pcg":
        raise ValueError(f"inner_solver {inner_solver!r}")
    d = len(n_basis)
    ms, ks = [], []
    for k in range(d):
        n_el = int(n_basis[k]) - int(degree)
        Mk, Kk = gram_1d(degree, n_el, None if breaks is None else breaks[k])
        keep = np.arange(1, Mk.shape[0] - 1)
        ms.append(Mk[np.ix_(keep, keep)])
        ks.append(Kk[np.ix_(keep, keep)])
    pre = fast_diagonalization(ms, ks)
    n = K.shape[0]
    P = spla.LinearOperator((n, n), matvec=pre, dtype=np.float64)
    K = K.tocsr()
    M = M.tocsr()

    def solve(b):
        x, info = spla.cg(K, b, x0=pre(b), rtol=1e-14, atol=0.0, maxiter=200, M=P)
        if info != 0:
            raise RuntimeError(f"inner conjugate gradients did not converge (info {info})")
        return x

    Kinv = spla.LinearOperator((n, n), matvec=solve, dtype=np.float64)
    w = spla.eigsh(K, k=count, M=M, sigma=0.0, which="LM", OPinv=Kinv, return_eigenvectors=False)
    return np.sort(w)


def laplace_eigenvalues(dim, degree, n_elem, count=10, device="cuda:0", breaks=None, inner_solver=None):
    """Assemble M (c = 1) and K (A = I) in FP64 with the library's kernels on `device` and
    return the `count` smallest Dirichlet eigenvalues.  breaks: as for ``Space`` (None:
    uniform knots).  inner_solver: as for ``solve_laplace``; None picks "pcg" above
    20,000 unknowns."""
    import torch

    from .space import Space
    sp = Space(dim, degree, n_elem, device=device, breaks=breaks)
    ones = torch.ones(sp.grid_shape, dtype=torch.float64, device=sp.device)
    M, K = sp.assemble_fused(ones, [ones] * dim)
    if inner_solver is None:
        inner_solver = "pcg" if np.prod([n - 2 for n in sp.n_basis]) > 20000 else "direct"
    return solve_laplace(M.cpu().numpy(), K.cpu().numpy(), sp.n_basis, degree, count, breaks=breaks,
                         inner_solver=inner_solver)
