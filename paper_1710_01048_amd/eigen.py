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


def solve_laplace(M_band, K_band, n_basis, degree, count=10):
    """The `count` smallest eigenvalues of K u = lambda M u restricted to the interior
    functions, from band-layout matrices (host arrays, FP64)."""
    import scipy.sparse.linalg as spla
    inner = interior_indices(n_basis)
    M = band_to_csr(np.asarray(M_band, dtype=np.float64), n_basis, degree)[inner][:, inner]
    K = band_to_csr(np.asarray(K_band, dtype=np.float64), n_basis, degree)[inner][:, inner]
    # constant coefficients: symmetric up to rounding; the Lanczos solver wants it exact
    M = ((M + M.T) * 0.5).tocsc()
    K = ((K + K.T) * 0.5).tocsc()
    w = spla.eigsh(K, k=count, M=M, sigma=0.0, which="LM", return_eigenvectors=False)
    return np.sort(w)


def laplace_eigenvalues(dim, degree, n_elem, count=10, device="cuda:0", breaks=None):
    """Assemble M (c = 1) and K (A = I) in FP64 with the library's kernels on `device` and
    return the `count` smallest Dirichlet eigenvalues.  breaks: as for ``Space`` (None:
    uniform knots)."""
    import torch

    from .space import Space
    sp = Space(dim, degree, n_elem, device=device, breaks=breaks)
    ones = torch.ones(sp.grid_shape, dtype=torch.float64, device=sp.device)
    M, K = sp.assemble_fused(ones, [ones] * dim)
    return solve_laplace(M.cpu().numpy(), K.cpu().numpy(), sp.n_basis, degree, count)
