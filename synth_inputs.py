"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This module holds input recipes only -- coefficient fields, the geometry of the
deformed cube and upstream gradients -- and none of the quadrature or assembly
arithmetic.  Coefficients are evaluated at whatever coordinates the caller passes
(each side passes the nodes of its own rule tables).

Recipes (the paper uses no public data set; its numerical examples are all
synthetic problems on the unit square / cube):

* ``sin_product_c``: c(x, y) = 1 + 0.5 sin(2 pi x) sin(2 pi y).
* ``fourier_modes`` / ``fourier_grid`` / ``fourier_points``: f(x) = 1 + sum_{m<8}
  alpha_m cos(2 pi k_m . x + phi_m), k_m uniform in {0..3}^d without the zero vector,
  phi_m ~ U(0, 2 pi), alpha_m ~ U(0, 0.3), drawn (k, then phi, then alpha) from
  numpy.random.default_rng(1000 * family + field); field 0 is c, fields 1..d are a_k.
* ``deformed_cube``: the map G_k(x) = x_k + 0.05 sin(2 pi x_k) of the unit cube onto
  itself, whose Jacobian J = diag(1 + 0.1 pi cos(2 pi x_k)) is folded into the
  coefficients of the pulled-back forms (eq:Mass and eq:Stiffness with physical c = 1,
  A = I): c = det J, a_k = det J / J_kk^2.
* ``upstream_gradient``: G ~ N(0, 1) on the (2p+1)^d slots of every row (torch
  generator with a fixed seed), slots whose column leaves the space set to zero.
"""
import math

import numpy as np
import torch

N_MODES = 8


def sin_product_c(x, y):
    """c(x, y) = 1 + 0.5 sin(2 pi x) sin(2 pi y) (any broadcastable torch/numpy arrays)."""
    lib = torch if isinstance(x, torch.Tensor) else np
    return 1.0 + 0.5 * lib.sin(2 * math.pi * x) * lib.sin(2 * math.pi * y)


def fourier_modes(family, field, d):
    """(k [8, d] int64, phi [8], alpha [8]) of one random Fourier field."""
    rng = np.random.default_rng(1000 * family + field)
    ks = []
    while len(ks) < N_MODES:
        k = rng.integers(0, 4, size=d)
        if np.any(k != 0):
            ks.append(k)
    phi = rng.uniform(0.0, 2 * math.pi, size=N_MODES)
    alpha = rng.uniform(0.0, 0.3, size=N_MODES)
    return np.array(ks, dtype=np.int64), phi, alpha


def fourier_grid(axes, modes, dtype=torch.float64, device="cpu"):
    """Field on the tensor grid of the 1D coordinate arrays ``axes`` (C order),
    evaluated in float64 and cast to ``dtype``."""
    k, phi, alpha = modes
    d = len(axes)
    xs = [torch.tensor(np.asarray(a, dtype=np.float64), device=device) for a in axes]
    out = torch.ones([x.numel() for x in xs], dtype=torch.float64, device=device)
    for m in range(N_MODES):
        theta = torch.full([1] * d, float(phi[m]), dtype=torch.float64, device=device)
        for j in range(d):
            shape = [1] * d
            shape[j] = -1
            theta = theta + (2 * math.pi * float(k[m, j])) * xs[j].view(shape)
        out += float(alpha[m]) * torch.cos(theta)
        del theta
    return out.to(dtype)


def fourier_points(points, modes):
    """Field at scattered points [n, d] (numpy float64)."""
    k, phi, alpha = modes
    pts = np.asarray(points, dtype=np.float64)
    out = np.ones(pts.shape[0])
    for m in range(N_MODES):
        out += alpha[m] * np.cos(2 * math.pi * (pts @ k[m].astype(np.float64)) + phi[m])
    return out


def deformed_cube_jdiag(x):
    """Diagonal Jacobian entry of G_k(x) = x + 0.05 sin(2 pi x) at coordinate x."""
    lib = torch if isinstance(x, torch.Tensor) else np
    return 1.0 + 0.1 * math.pi * lib.cos(2 * math.pi * x)


def deformed_cube_grid(axes, field, dtype=torch.float64, device="cpu"):
    """Folded coefficient on a tensor grid: field 'c' -> det J, int k -> det J / J_kk^2."""
    d = len(axes)
    js = [deformed_cube_jdiag(torch.tensor(np.asarray(a, dtype=np.float64), device=device))
          for a in axes]
    out = torch.ones([j.numel() for j in js], dtype=torch.float64, device=device)
    for k in range(d):
        shape = [1] * d
        shape[k] = -1
        e = js[k] if field == "c" or k != field else 1.0 / js[k]
        out = out * e.view(shape)
    return out.to(dtype)


def deformed_cube_points(points, field):
    pts = np.asarray(points, dtype=np.float64)
    j = deformed_cube_jdiag(pts)
    det = np.prod(j, axis=1)
    return det if field == "c" else det / j[:, field] ** 2


def slot_valid_mask(n_el, p, rows=None, device="cpu"):
    """Bool [n_rows or len(rows), (2p+1)^d]: slot s of row i is inside the space iff
    every column i_k - p + s_k lies in [0, N_el,k + p)."""
    d = len(n_el)
    S = 2 * p + 1
    n = [int(e) + p for e in n_el]
    if rows is None:
        rows = torch.arange(int(np.prod(n)), device=device, dtype=torch.int64)
    else:
        rows = torch.as_tensor(rows, dtype=torch.int64, device=device)
    idx = []
    rem = rows.clone()
    for k in reversed(range(d)):
        idx.append(rem % n[k])
        rem = rem // n[k]
    idx = idx[::-1]
    s = torch.arange(S ** d, device=device)
    ok = torch.ones(rows.numel(), S ** d, dtype=torch.bool, device=device)
    div = S ** d
    for k in range(d):
        div //= S
        sk = (s // div) % S
        col = idx[k][:, None] - p + sk[None, :]
        ok &= (col >= 0) & (col < n[k])
    return ok


def upstream_gradient(n_el, p, seed, dtype=torch.float64, device="cpu", chunk_rows=1 << 20):
    """G ~ N(0,1) of shape [n_rows, (2p+1)^d] from torch.Generator(seed) on ``device``,
    invalid slots zero.  Generated in row chunks to bound temporary memory."""
    d = len(n_el)
    n_rows = int(np.prod([int(e) + p for e in n_el]))
    SD = (2 * p + 1) ** d
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty(n_rows, SD, dtype=dtype, device=device)
    for r0 in range(0, n_rows, chunk_rows):
        r1 = min(n_rows, r0 + chunk_rows)
        g = torch.randn(r1 - r0, SD, generator=gen, dtype=torch.float64, device=device)
        g *= slot_valid_mask(n_el, p, torch.arange(r0, r1, device=device), device=device)
        out[r0:r1] = g.to(dtype)
    return out
