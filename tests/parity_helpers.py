"""Input recipes for the parity tests, evaluated separately for each side at that
side's own rule nodes (the library's nodes for the device run, the oracle's nodes for
the oracle), plus the error metrics of the comparisons.

recipe:
  ("random", seed)      i.i.d. U(0.5, 1.5) samples on the grid -- one host array, the
                        same values go to both sides (node positions do not matter)
  ("sin_product",)      c = 1 + 0.5 sin(2 pi x) sin(2 pi y), a_k = 1
  ("fourier", family)   random Fourier fields of that seed family (field 0 = c, k+1 = a_k)
  ("deformed",)         deformed-cube coefficients (det J, det J / J_kk^2)
"""
import numpy as np
import torch

import structured as st
import synth_inputs as si
from oracle import assembly as oa


def grid_shape(p, n_el):
    return tuple((e + p) * (p + 1) for e in n_el)


def _random_fields(p, n_el, seed):
    rng = np.random.default_rng(seed)
    shape = grid_shape(p, n_el)
    return [rng.uniform(0.5, 1.5, size=shape) for _ in range(len(n_el) + 1)]


def device_fields(space, recipe, dtype):
    """[c, a_1..a_d] as device tensors of dtype, sampled at the library's nodes."""
    p, n_el, d = space.degree, space.n_elem, space.dim
    dev = space.device
    kind = recipe[0]
    if kind == "random":
        return [torch.from_numpy(f).to(dev, dtype) for f in _random_fields(p, n_el, recipe[1])]
    out = []
    for field in ["c"] + list(range(d)):
        axes = space.grid_axes(field)
        if kind == "sin_product":
            if field == "c":
                x = torch.tensor(axes[0], dtype=torch.float64, device=dev)[:, None]
                y = torch.tensor(axes[1], dtype=torch.float64, device=dev)[None, :]
                out.append(si.sin_product_c(x, y).to(dtype).contiguous())
            else:
                out.append(torch.ones(space.grid_shape, dtype=dtype, device=dev))
        elif kind == "fourier":
            fid = 0 if field == "c" else field + 1
            out.append(si.fourier_grid(axes, si.fourier_modes(recipe[1], fid, d), dtype, dev).contiguous())
        elif kind == "deformed":
            out.append(si.deformed_cube_grid(axes, field, dtype, dev).contiguous())
        else:
            raise ValueError(recipe)
    return out


def oracle_row_fields(tabs, p, n_el, rows, recipe):
    """[c, a_1..a_d] samples of the listed rows, [n_list, (p+1)^d] float64, at the
    oracle's nodes (random recipe: gathered from the shared host array)."""
    d = len(n_el)
    kind = recipe[0]
    n = [e + p for e in n_el]
    if kind == "random":
        pts = st.point_offsets(n, p, rows)
        return [f.reshape(-1)[pts] for f in _random_fields(p, n_el, recipe[1])]
    out = []
    for field in ["c"] + list(range(d)):
        xyz = oa.row_point_coords(p, n_el, tabs, rows, field)          # [n_list, QD, d]
        flat = xyz.reshape(-1, d)
        if kind == "sin_product":
            v = si.sin_product_c(flat[:, 0], flat[:, 1]) if field == "c" else np.ones(len(flat))
        elif kind == "fourier":
            fid = 0 if field == "c" else field + 1
            v = si.fourier_points(flat, si.fourier_modes(recipe[1], fid, d))
        elif kind == "deformed":
            v = si.deformed_cube_points(flat, field)
        else:
            raise ValueError(recipe)
        out.append(v.reshape(xyz.shape[:2]))
    return out


def oracle_forward(p, n_el, rows, recipe, want_m=True, want_k=True):
    tabs = oa.rule_tables(p, n_el)
    f = oracle_row_fields(tabs, p, n_el, rows, recipe)
    M, K = oa.assemble(p, n_el, tabs, c=f[0] if want_m else None, a=f[1:] if want_k else None,
                       rows=rows, per_row=True)
    return M, K


def oracle_adjoint(p, n_el, tabs, gM, gK, rows):
    """The oracle's gradients of the listed rows and, in the same layout, the scale of
    each entry: the sum of the magnitudes of the terms it sums (``absolute=True``).
    Returns ([dc, da_1..da_d], [scale_c, scale_1..scale_d]) with None left out."""
    wc, wa = oa.adjoint(p, n_el, tabs, gM, gK, rows=rows)
    sc, sa = oa.adjoint(p, n_el, tabs, gM, gK, rows=rows, absolute=True)
    want = ([wc] if wc is not None else []) + (list(wa) if wa is not None else [])
    scale = ([sc] if sc is not None else []) + (list(sa) if sa is not None else [])
    return want, scale


def entry_error(got, want, scale):
    """Largest error of any single gradient entry relative to the sum of the magnitudes
    of the terms that entry sums: max |got - want| / sum_s |G_s prod_k T_k|, over arrays
    [rows, points of the row].

    A point whose terms all vanish in exact arithmetic (a stiffness node placed at the
    zero of B'_j, eq:WQquadraticStiff and its traces on non-uniform knots; R6) carries
    only the rounding noise of its table entries, different on either side; such points
    (scale below 1e-10 of the row's largest) are held to the row's largest scale.  Rows
    whose terms are all zero must agree exactly."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    if got.ndim == 1:
        got, want, scale = got[None], want[None], scale[None]
    if np.any(~np.isfinite(got)):
        return float("inf")
    diff = np.abs(got - want)
    row_max = scale.max(axis=1, keepdims=True)
    eff = np.where(scale >= 1e-10 * row_max, scale, row_max)
    zero = eff == 0
    if np.any(diff[zero] != 0):
        return float("inf")
    return float((diff[~zero] / eff[~zero]).max()) if (~zero).any() else 0.0


def entry_errors(got, want, scale):
    """entry_error of each field in turn (lists of arrays)."""
    assert len(got) == len(want) == len(scale)
    return [entry_error(g, w, s) for g, w, s in zip(got, want, scale)]
