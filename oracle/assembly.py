"""Python side of the FP64 oracle (TEST INFRASTRUCTURE ONLY).

``build()`` compiles ``assemble.c`` with gcc and OpenMP; ``assemble`` and ``adjoint``
call it through ctypes on numpy arrays.  ``rule_tables`` gives the per-direction rule
tables (nodes and physical weights of every row) from ``oracle.rules``.

Layouts (shared with the product only through the paper's definitions):
* row i = (i_1..i_d) in C order over n_k = N_el,k + p basis functions;
* slot s = (s_1..s_d) in C order over S = 2p+1, column j_k = i_k - p + s_k;
* coefficient grids are C-ordered [N_1..N_d] with N_k = n_k (p+1); row i owns the
  points (i_k (p+1) + q_k)_k, q_k in [0, p+1).
"""
import ctypes
import functools
import os
import subprocess

import numpy as np

from . import rules

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "assemble.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile the C oracle into oracle/liboracle.so (plain -O2, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall",
                    "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


@functools.lru_cache(maxsize=None)
def _lib():
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    dpp = P(P(ctypes.c_double))
    lib.oracle_assemble.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_int64), dpp,
                                    dpp, dpp, dpp, dpp,
                                    P(ctypes.c_double), dpp,
                                    P(ctypes.c_int64), ctypes.c_int64,
                                    P(ctypes.c_double), P(ctypes.c_double)]
    lib.oracle_assemble.restype = ctypes.c_int
    lib.oracle_assemble_rows.argtypes = lib.oracle_assemble.argtypes
    lib.oracle_assemble_rows.restype = ctypes.c_int
    lib.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_int64), dpp,
                                   dpp, dpp, dpp, dpp,
                                   P(ctypes.c_int64), ctypes.c_int64,
                                   P(ctypes.c_double), P(ctypes.c_double),
                                   P(ctypes.c_double), dpp]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_adjoint_abs.argtypes = lib.oracle_adjoint.argtypes
    lib.oracle_adjoint_abs.restype = ctypes.c_int
    return lib


@functools.lru_cache(maxsize=None)
def _direction(p, n_el, kind):
    xs, ws = rules.direction_table(p, n_el, kind)
    x = np.ascontiguousarray(np.array(xs, dtype=np.float64).reshape(-1))
    w = np.ascontiguousarray(np.array(ws, dtype=np.float64).reshape(-1))
    x.setflags(write=False)
    w.setflags(write=False)
    return x, w


def rule_tables(p, n_el, breaks=None):
    """Per-direction rule tables for elements counts n_el (tuple, one per direction):
    dict with lists xM, wM, xK, wK of flat float64 arrays [n_k * (p+1)], and "breaks"
    (per direction None for uniform knots, else the breakpoints).  breaks: None, or a
    list with one entry per direction, None (uniform) or breakpoints 0 = b_0 < ... < b_N
    = 1 whose rules come from ``oracle.nonuniform`` (homotopy from the uniform rules)."""
    out = {"xM": [], "wM": [], "xK": [], "wK": [], "breaks": []}
    for k, ne in enumerate(n_el):
        b = None if breaks is None else breaks[k]
        for kind, kx, kw in (("mass", "xM", "wM"), ("stiffness", "xK", "wK")):
            if b is None:
                x, w = _direction(p, int(ne), kind)
            else:
                x, w = _direction_breaks(p, tuple(float(v) for v in b), kind)
            out[kx].append(x)
            out[kw].append(w)
        out["breaks"].append(None if b is None else np.ascontiguousarray(np.asarray(b, dtype=np.float64)))
    return out


@functools.lru_cache(maxsize=None)
def _direction_breaks(p, breaks, kind):
    from . import nonuniform
    xs, ws = nonuniform.direction_table(p, breaks, kind)
    x = np.ascontiguousarray(np.array(xs, dtype=np.float64).reshape(-1))
    w = np.ascontiguousarray(np.array(ws, dtype=np.float64).reshape(-1))
    x.setflags(write=False)
    w.setflags(write=False)
    return x, w


def _breaks_ptr(tables, keep):
    brk = tables.get("breaks")
    if brk is None or all(b is None for b in brk):
        return None
    arr = (ctypes.POINTER(ctypes.c_double) * len(brk))()
    for k, b in enumerate(brk):
        if b is not None:
            arr[k] = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            keep.append(b)
    return arr


def grid_axes(tables, field):
    """1D coordinate arrays of the tensor grid a field lives on.  field = 'c' (mass rule
    in every direction) or k (int: the stiffness rule in direction k, mass elsewhere)."""
    d = len(tables["xM"])
    if field == "c":
        return [tables["xM"][k] for k in range(d)]
    return [tables["xK"][k] if k == field else tables["xM"][k] for k in range(d)]


def _ptr_array(arrays):
    arr = (ctypes.POINTER(ctypes.c_double) * len(arrays))()
    for k, a in enumerate(arrays):
        arr[k] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return arr


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


def assemble(p, n_el, tables, c=None, a=None, rows=None, per_row=False):
    """Rows of M (if c is given) and K (if a is given) as float64 [n_list, (2p+1)^d].

    c and a[k] are full grids, or with per_row=True the samples of the listed rows only,
    [n_list, (p+1)^d] in the point order of ``row_points``."""
    d = len(n_el)
    if per_row and rows is None:
        raise ValueError("per_row needs rows")
    lib = _lib()
    ne = np.ascontiguousarray(np.array(n_el, dtype=np.int64))
    n_rows = int(np.prod([n + p for n in n_el]))
    rows_arr = None if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    n_list = n_rows if rows_arr is None else rows_arr.size
    SD = (2 * p + 1) ** d
    keep = []
    c64 = None if c is None else _f64(c)
    a64 = None if a is None else [_f64(x) for x in a]
    M = np.empty((n_list, SD)) if c is not None else None
    K = np.empty((n_list, SD)) if a is not None else None
    xM, wM = _ptr_array(tables["xM"]), _ptr_array(tables["wM"])
    xK, wK = _ptr_array(tables["xK"]), _ptr_array(tables["wK"])
    keep += [xM, wM, xK, wK]
    P = ctypes.POINTER(ctypes.c_double)
    fn = lib.oracle_assemble_rows if per_row else lib.oracle_assemble
    brk = _breaks_ptr(tables, keep)
    rc = fn(
        d, p, ne.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), brk, xM, wM, xK, wK,
        None if c64 is None else c64.ctypes.data_as(P),
        None if a64 is None else _ptr_array(a64),
        None if rows_arr is None else rows_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        n_list,
        None if M is None else M.ctypes.data_as(P),
        None if K is None else K.ctypes.data_as(P))
    if rc != 0:
        raise ValueError(f"oracle_assemble failed with {rc}")
    return M, K


def adjoint(p, n_el, tables, gM=None, gK=None, rows=None, absolute=False):
    """Gradients of <gM, M> + <gK, K> with respect to the coefficient samples of the
    listed rows: dc [n_list, (p+1)^d] and da = list of d such arrays (None where the
    matching upstream gradient is None).  gM, gK are [n_list, (2p+1)^d].

    absolute=True returns, in the same layout, the sum of the magnitudes of the terms
    each gradient entry sums, sum_s |G[s]| prod_k |factor_k(q, s)|: the scale of the
    rounding error any evaluation order of that sum can make."""
    d = len(n_el)
    lib = _lib()
    ne = np.ascontiguousarray(np.array(n_el, dtype=np.int64))
    n_rows = int(np.prod([n + p for n in n_el]))
    rows_arr = None if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    n_list = n_rows if rows_arr is None else rows_arr.size
    QD = (p + 1) ** d
    P = ctypes.POINTER(ctypes.c_double)
    gM64 = None if gM is None else _f64(gM)
    gK64 = None if gK is None else _f64(gK)
    dc = np.empty((n_list, QD)) if gM is not None else None
    da = [np.empty((n_list, QD)) for _ in range(d)] if gK is not None else None
    xM, wM = _ptr_array(tables["xM"]), _ptr_array(tables["wM"])
    xK, wK = _ptr_array(tables["xK"]), _ptr_array(tables["wK"])
    keep = [xM, wM, xK, wK]
    brk = _breaks_ptr(tables, keep)
    fn = lib.oracle_adjoint_abs if absolute else lib.oracle_adjoint
    rc = fn(
        d, p, ne.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), brk, xM, wM, xK, wK,
        None if rows_arr is None else rows_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        n_list,
        None if gM64 is None else gM64.ctypes.data_as(P),
        None if gK64 is None else gK64.ctypes.data_as(P),
        None if dc is None else dc.ctypes.data_as(P),
        None if da is None else _ptr_array(da))
    if rc != 0:
        raise ValueError(f"oracle_adjoint failed with {rc}")
    return dc, da


def row_points(p, n_el, rows):
    """Flat grid offsets of every point of the listed rows, [n_list, (p+1)^d], in the
    same q order as ``adjoint`` returns them."""
    d = len(n_el)
    Q = p + 1
    n = [ne + p for ne in n_el]
    N = [nk * Q for nk in n]
    rows = np.asarray(rows, dtype=np.int64)
    idx = []
    rem = rows.copy()
    for k in reversed(range(d)):
        idx.append(rem % n[k])
        rem //= n[k]
    idx = idx[::-1]
    qs = np.array(np.unravel_index(np.arange(Q ** d), [Q] * d)).T   # [QD, d]
    off = np.zeros((rows.size, Q ** d), dtype=np.int64)
    for k in range(d):
        off = off * N[k] + (idx[k][:, None] * Q + qs[None, :, k])
    return off


def row_point_coords(p, n_el, tables, rows, field):
    """Coordinates [n_list, (p+1)^d, d] of the points of the listed rows on the grid of
    ``field`` ('c' or a direction k), in the point order of ``row_points``."""
    d = len(n_el)
    Q = p + 1
    n = [ne + p for ne in n_el]
    rows = np.asarray(rows, dtype=np.int64)
    axes = grid_axes(tables, field)
    idx = []
    rem = rows.copy()
    for k in reversed(range(d)):
        idx.append(rem % n[k])
        rem //= n[k]
    idx = idx[::-1]
    qs = np.array(np.unravel_index(np.arange(Q ** d), [Q] * d)).T
    out = np.empty((rows.size, Q ** d, d))
    for k in range(d):
        out[:, :, k] = axes[k][idx[k][:, None] * Q + qs[None, :, k]]
    return out
