"""Space: one spline space with its rules on one device; WQAssemble: autograd wrapper.

Argument marshalling only -- shapes, dtypes, devices and contiguity are checked here,
then the device pointers and the current HIP stream go to libwqa.
"""
import ctypes

import numpy as np
import torch

from ._lib import F32, F64, MASS, STIFFNESS, check, lib

_DTYPES = {torch.float32: F32, torch.float64: F64}


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Space:
    """Open tensor-product B-spline space of degree 2 or 3 in 2 or 3 dimensions, uniform
    knots unless ``breaks`` says otherwise (Sec. 2.2), with its weighted Gaussian row
    rules (Sec. 3).  Each direction takes degree + 1 to 2^24 elements.

    device: a torch CUDA (HIP) device, or None for a host-only space (rules and tables
    only; the assemble calls then fail).  rules: "default" installs the library's
    rules; None leaves them to ``set_rules``.  breaks: None (uniform knots), or one
    entry per direction, None or the breakpoints 0 = b_0 < ... < b_N = 1 of that
    direction (the default rules are then traced from the uniform ones by homotopy).
    """

    def __init__(self, dim, degree, n_elem, device="cuda:0", rules="default", breaks=None):
        self.dim, self.degree = int(dim), int(degree)
        self.n_elem = tuple(int(e) for e in n_elem)
        if len(self.n_elem) != self.dim:
            raise ValueError("n_elem needs one entry per direction")
        self.device = None if device is None else torch.device(device)
        dev_index = -1 if self.device is None else (self.device.index or 0)
        handle = ctypes.c_void_p()
        check(lib.wqa_create(ctypes.byref(handle), dev_index))
        self._ctx = handle
        ne = (ctypes.c_int64 * self.dim)(*self.n_elem)
        check(lib.wqa_set_space(self._ctx, self.dim, self.degree, ne))
        self.breaks = [None] * self.dim
        if breaks is not None:
            if len(breaks) != self.dim:
                raise ValueError("breaks needs one entry per direction")
            dp = ctypes.POINTER(ctypes.c_double)
            for k, b in enumerate(breaks):
                if b is None:
                    continue
                arr = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
                if arr.shape != (self.n_elem[k] + 1,):
                    raise ValueError(f"breaks[{k}] needs n_elem[{k}] + 1 = {self.n_elem[k] + 1} values")
                check(lib.wqa_set_knots(self._ctx, k, arr.ctypes.data_as(dp)))
                self.breaks[k] = arr
        if rules == "default":
            check(lib.wqa_set_default_rules(self._ctx))
        elif rules is not None:
            raise ValueError("rules must be 'default' or None")
        rows, slots, pts = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        dims = (ctypes.c_int64 * 3)()
        check(lib.wqa_query(self._ctx, ctypes.byref(rows), ctypes.byref(slots), ctypes.byref(pts), dims))
        self.n_rows, self.slots_per_row, self.points_per_row = rows.value, slots.value, pts.value
        self.grid_shape = tuple(dims[k] for k in range(self.dim))
        self.buffer_shape = self.grid_shape           # sample buffers: grid lines padded to the pitch,
        self.pitch = 0                                # or [rows, points_per_row] stored row by row
        self.sample_layout = "grid"
        self.n_basis = tuple(e + self.degree for e in self.n_elem)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            lib.wqa_destroy(ctx)
            self._ctx = None

    # --- rules ------------------------------------------------------------------------
    def set_rules(self, kind, direction, nodes, weights, exact_tol=1e-12):
        x = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1))
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib.wqa_set_rules(self._ctx, kind, direction, self.degree + 1, x.ctypes.data_as(dp),
                                w.ctypes.data_as(dp), float(exact_tol)))

    def rules(self, kind, direction):
        """(nodes, weights) of one kind and direction, each [n_dir, p+1] float64."""
        if not 0 <= direction < self.dim:
            raise ValueError(f"direction {direction} of a {self.dim}-dimensional space")
        n = self.n_basis[direction]
        x = np.empty((n, self.degree + 1))
        w = np.empty((n, self.degree + 1))
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib.wqa_get_rules(self._ctx, kind, direction, x.ctypes.data_as(dp), w.ctypes.data_as(dp)))
        return x, w

    def tables(self, kind, direction):
        """FP64 contraction table [n_dir, p+1, 2p+1] used by the kernels."""
        if not 0 <= direction < self.dim:
            raise ValueError(f"direction {direction} of a {self.dim}-dimensional space")
        n = self.n_basis[direction]
        t = np.empty((n, self.degree + 1, 2 * self.degree + 1))
        check(lib.wqa_get_tables(self._ctx, kind, direction, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return t

    def grid_axes(self, field):
        """1D coordinates of a field's tensor grid: field 'c' (mass nodes everywhere) or
        k (stiffness nodes in direction k, mass nodes elsewhere)."""
        out = []
        for k in range(self.dim):
            kind = STIFFNESS if field != "c" and k == field else MASS
            out.append(self.rules(kind, k)[0].reshape(-1))
        return out

    def set_final_mode(self, mode):
        check(lib.wqa_set_final_mode(self._ctx, int(mode)))

    def set_grid_pitch(self, pitch):
        """Grid buffers (fields and gradients) hold lines of `pitch` values along the last
        direction, the first N_d of them the grid (0: dense).  buffer_shape follows."""
        check(lib.wqa_set_grid_pitch(self._ctx, int(pitch)))
        self.pitch = int(pitch)
        if self.sample_layout == "grid":        # by row only pitch 0 is accepted; the shape stays
            self.buffer_shape = self.grid_shape[:-1] + (self.pitch or self.grid_shape[-1],)

    def set_sample_layout(self, layout):
        """'grid' (the default) or 'rows': every sample buffer (fields, gradients, f)
        then holds [n_rows, points_per_row], the points each row owns as one block
        (see rows_from_grid).  buffer_shape follows."""
        code = {"grid": 0, "rows": 1}.get(layout)
        if code is None:
            raise ValueError("layout must be 'grid' or 'rows'")
        check(lib.wqa_set_sample_layout(self._ctx, code))
        self.sample_layout = layout
        if code:
            self.buffer_shape = (self.n_rows, self.points_per_row)
        else:
            self.buffer_shape = self.grid_shape[:-1] + (self.pitch or self.grid_shape[-1],)

    def rows_from_grid(self, t):
        """A dense grid-shaped tensor's values in the row layout: row i's block holds its
        points (i_k Q + q_k)_k, q_1 slowest (a permutation, made with torch)."""
        Q = self.degree + 1
        split = []
        for n in self.n_basis:
            split += [n, Q]
        v = t.reshape(split)
        v = v.permute(*range(0, 2 * self.dim, 2), *range(1, 2 * self.dim, 2))
        return v.reshape(self.n_rows, self.points_per_row).contiguous()

    def grid_from_rows(self, t):
        """The inverse of rows_from_grid: a [n_rows, points_per_row] tensor on the grid."""
        Q = self.degree + 1
        v = t.reshape(*self.n_basis, *([Q] * self.dim))
        order = []
        for k in range(self.dim):
            order += [k, self.dim + k]
        return v.permute(*order).reshape(self.grid_shape).contiguous()

    def set_dispatch_limit(self, max_tasks):
        """Wave tasks per kernel dispatch (0: the default); larger launches are split."""
        check(lib.wqa_set_dispatch_limit(self._ctx, int(max_tasks)))

    # --- buffers ------------------------------------------------------------------------
    def _field(self, t, name, dtype=None):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if t.dtype not in _DTYPES or (dtype is not None and t.dtype != dtype):
            raise ValueError(f"{name}: dtype {t.dtype} (need float32 or float64, all alike)")
        if tuple(t.shape) != self.buffer_shape and tuple(t.shape) != (int(np.prod(self.buffer_shape)),):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, grid buffers are {self.buffer_shape}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.data_ptr() % 16:
            raise ValueError(f"{name} must start on a 16-byte boundary")
        return t

    def _matrix(self, t, name, dtype):
        if t is None:
            return torch.empty(self.n_rows, self.slots_per_row, dtype=dtype, device=self.device)
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous() or \
                t.numel() != self.n_rows * self.slots_per_row or t.data_ptr() % 16:
            raise ValueError(f"{name}: need contiguous, 16-byte aligned {dtype} [{self.n_rows}, "
                             f"{self.slots_per_row}] on {self.device}")
        return t

    def _need_device(self):
        if self.device is None:
            raise RuntimeError("host-only Space: create it with a device to assemble")

    # --- assembly -------------------------------------------------------------------------
    def assemble_mass(self, c, M=None):
        self._need_device()
        c = self._field(c, "c")
        M = self._matrix(M, "M", c.dtype)
        check(lib.wqa_assemble_mass(self._ctx, _DTYPES[c.dtype], ctypes.c_void_p(c.data_ptr()),
                                    ctypes.c_void_p(M.data_ptr()), _stream_handle(self.device)))
        return M

    def _ptrs(self, ts):
        arr = (ctypes.c_void_p * self.dim)()
        for k, t in enumerate(ts):
            arr[k] = t.data_ptr()
        return arr

    def assemble_stiffness(self, a, K=None):
        self._need_device()
        a = [self._field(x, f"a[{k}]", a[0].dtype) for k, x in enumerate(a)]
        if len(a) != self.dim:
            raise ValueError("need one coefficient per direction")
        K = self._matrix(K, "K", a[0].dtype)
        check(lib.wqa_assemble_stiffness(self._ctx, _DTYPES[a[0].dtype], self._ptrs(a),
                                         ctypes.c_void_p(K.data_ptr()), _stream_handle(self.device)))
        return K

    def assemble_fused(self, c, a, M=None, K=None):
        self._need_device()
        c = self._field(c, "c")
        a = [self._field(x, f"a[{k}]", c.dtype) for k, x in enumerate(a)]
        if len(a) != self.dim:
            raise ValueError("need one coefficient per direction")
        M = self._matrix(M, "M", c.dtype)
        K = self._matrix(K, "K", c.dtype)
        check(lib.wqa_assemble_fused(self._ctx, _DTYPES[c.dtype], ctypes.c_void_p(c.data_ptr()), self._ptrs(a),
                                     ctypes.c_void_p(M.data_ptr()), ctypes.c_void_p(K.data_ptr()),
                                     _stream_handle(self.device)))
        return M, K

    def adjoint(self, gM=None, gK=None, dc=None, da=None):
        """dL/dc (if gM) and dL/da_k (if gK) for L = <gM, M> + <gK, K>."""
        self._need_device()
        ref = gM if gM is not None else gK
        if ref is None:
            raise ValueError("need gM or gK")
        dtype = ref.dtype
        for g, name in ((gM, "gM"), (gK, "gK")):
            if g is not None:
                self._matrix(g, name, dtype)
        if gM is not None:
            dc = torch.empty(self.buffer_shape, dtype=dtype, device=self.device) if dc is None else self._field(dc, "dc", dtype)
        else:
            dc = None
        if gK is not None:
            da = [torch.empty(self.buffer_shape, dtype=dtype, device=self.device) for _ in range(self.dim)] \
                if da is None else [self._field(x, f"da[{k}]", dtype) for k, x in enumerate(da)]
        else:
            da = None
        check(lib.wqa_assemble_adjoint(
            self._ctx, _DTYPES[dtype],
            None if gM is None else ctypes.c_void_p(gM.data_ptr()),
            None if gK is None else ctypes.c_void_p(gK.data_ptr()),
            None if dc is None else ctypes.c_void_p(dc.data_ptr()),
            None if da is None else self._ptrs(da),
            _stream_handle(self.device)))
        return dc, da

    # --- load vector and matrix-free products -------------------------------------------
    def _vector(self, t, name, dtype):
        if t is None:
            return torch.empty(self.n_rows, dtype=dtype, device=self.device)
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous() or \
                t.numel() != self.n_rows or t.data_ptr() % 16:
            raise ValueError(f"{name}: need contiguous, 16-byte aligned {dtype} [{self.n_rows}] on {self.device}")
        return t

    def load_vector(self, f, b=None):
        """b_i = integral f B_i with the mass rules (f on the all-mass grid, like c)."""
        self._need_device()
        f = self._field(f, "f")
        b = self._vector(b, "b", f.dtype)
        check(lib.wqa_assemble_load(self._ctx, _DTYPES[f.dtype], ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(b.data_ptr()), _stream_handle(self.device)))
        return b

    def apply_mass(self, c, x, y=None):
        """y = M x without forming M (M as assemble_mass(c) would give)."""
        self._need_device()
        c = self._field(c, "c")
        x = self._vector(x, "x", c.dtype)
        y = self._vector(y, "y", c.dtype)
        check(lib.wqa_apply_mass(self._ctx, _DTYPES[c.dtype], ctypes.c_void_p(c.data_ptr()),
                                 ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 _stream_handle(self.device)))
        return y

    def apply_stiffness(self, a, x, y=None):
        """y = K x without forming K (K as assemble_stiffness(a) would give)."""
        self._need_device()
        a = [self._field(t, f"a[{k}]", a[0].dtype) for k, t in enumerate(a)]
        if len(a) != self.dim:
            raise ValueError("need one coefficient per direction")
        x = self._vector(x, "x", a[0].dtype)
        y = self._vector(y, "y", a[0].dtype)
        check(lib.wqa_apply_stiffness(self._ctx, _DTYPES[a[0].dtype], self._ptrs(a), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), _stream_handle(self.device)))
        return y


class WQAssemble(torch.autograd.Function):
    """(M, K) = WQAssemble.apply(space, c, a_1, ..., a_d), differentiable in c and a_k.

    Forward is the fused assembly; backward is the library's adjoint kernel, which
    recomputes the per-row tables instead of storing intermediates."""

    @staticmethod
    def forward(ctx, space, c, *a):
        if space.pitch != 0:
            raise ValueError("WQAssemble needs dense sample buffers (grid pitch 0): padding would get no gradient")
        ctx.space = space
        ctx.shapes = (c.shape,) + tuple(x.shape for x in a)     # grid-shaped or flat
        c = c.contiguous()
        a = [x.contiguous() for x in a]
        M, K = space.assemble_fused(c, a)
        return M, K

    @staticmethod
    def backward(ctx, gM, gK):
        space = ctx.space
        gM = None if gM is None else gM.contiguous()
        gK = None if gK is None else gK.contiguous()
        if gM is None and gK is None:
            return (None, None) + (None,) * space.dim
        dc, da = space.adjoint(gM, gK)
        # gradients take the shape each input had
        dc = None if dc is None else dc.view(ctx.shapes[0])
        da = (None,) * space.dim if da is None else tuple(g.view(s) for g, s in zip(da, ctx.shapes[1:]))
        return (None, dc) + da
