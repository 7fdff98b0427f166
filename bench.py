"""Benchmark: weighted-quadrature row-wise assembly on one MI355X.

One step = one pass of the whole path over the workload: the fused mass + stiffness
forward assembly followed by its adjoint, on the 3D C^2 cubic space with 160^3
elements (4,330,747 rows, 343 slots per row), random-Fourier c and anisotropic
diagonal A, FP32 values in the implicit-column band layout, the final directional pass
accumulated in FP64 (the all-FP32 compensated Dot2 pass is timed beside it).  Inputs (coefficients and upstream gradients) are resident in HBM
before timing; outputs are preallocated.

value = slots processed per second over the step: 2 x rows x 343 assembled (M and K)
plus 2 x rows x 343 upstream-gradient slots consumed by the adjoint.  Also reported:
the forward under every FP32 final-pass mode, the same workload in FP64, the memory-
pattern probes of libwqa_probes.so (the ceiling of each kernel's byte pattern) and
plain streaming, and (cpu_baseline) the FP64 CPU oracle timed on a row sample, which
also states the error of every GPU result on that sample.

Sample buffers (coefficient samples and gradients) are stored row by row by default
(wqa_set_sample_layout: each row's (p+1)^3 points as one block; the same values and
bytes as the grid, and bit-identical results).  --layout grid puts them on the grid with
the last-direction lines padded to a multiple of 32 values (wqa_set_grid_pitch), so that
every line starts on a 128-byte boundary; the padding is never read or written.  The
other layout's forward and adjoint are timed beside the headline.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--layout rows|grid]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth_inputs as si  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
P, NEL = 3, (160, 160, 160)
SEED_FAMILY = 5                # seeds of the 160^3 workload's Fourier fields and upstream gradients
METRIC = "assembled nnz/s (3D C2 cubic M+K) FP32 vs FP64 at stated err; adjoint nnz/s"
MODES = (("plain", 0), ("dot2", 1), ("f64_accumulate", 2))
HEADLINE_MODE = 2              # final pass accumulated in FP64 (mixed precision; every other stage FP32)
LINE_ALIGN = 32                # grid lines padded to a multiple of this many values
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_160cubed.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1710_01048_amd", "csrc", "wqa_kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time of the cpu_baseline sample")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-modes", action="store_true", help="time only the headline final pass")
    ap.add_argument("--headline-only", action="store_true",
                    help="leave out the other workloads (matrix-free products, 96^3 forward): profiler runs")
    ap.add_argument("--cube96-only", action="store_true",
                    help="run only the 96^3 deformed-cube forward and print its figures (profiler runs)")
    ap.add_argument("--products-only", action="store_true",
                    help="run only the load vector and matrix-free products and print their figures "
                         "(profiler runs)")
    ap.add_argument("--no-probes", action="store_true", help="leave out the memory-pattern probes")
    ap.add_argument("--layout", choices=("rows", "grid"), default="rows",
                    help="sample buffers stored row by row (default) or on the grid with padded lines")
    ap.add_argument("--probe-sweep", type=int, default=0, metavar="N_EL",
                    help="only time the memory-pattern probe variants on the N_EL^3 cubic space (the layout "
                         "experiments behind the kernels' design) and print them")
    ap.add_argument("--profile-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter calibration under rocprofv3)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ev():
    return torch.cuda.Event(enable_timing=True)


def padded_pitch(sp):
    return (sp.grid_shape[-1] + LINE_ALIGN - 1) // LINE_ALIGN * LINE_ALIGN


def padded(sp, dense):
    """`dense` (grid-shaped) copied into a buffer of sp.buffer_shape (padding left as is)."""
    buf = torch.empty(sp.buffer_shape, dtype=dense.dtype, device=dense.device)
    buf[..., :sp.grid_shape[-1]] = dense
    return buf


def use_layout(sp, layout):
    """Samples stored row by row, or on the grid with lines padded to LINE_ALIGN values."""
    if layout == "rows":
        sp.set_sample_layout("rows")
    else:
        sp.set_grid_pitch(padded_pitch(sp))


def place(sp, dense):
    """A dense grid-shaped field in the space's sample layout."""
    return sp.rows_from_grid(dense) if sp.sample_layout == "rows" else padded(sp, dense)


def make_inputs(sp, dtype):
    dev = sp.device
    fields = []
    for field in ["c", 0, 1, 2]:
        fid = 0 if field == "c" else field + 1
        dense = si.fourier_grid(sp.grid_axes(field), si.fourier_modes(SEED_FAMILY, fid, 3), dtype, dev)
        fields.append(place(sp, dense))
        del dense
    gM = si.upstream_gradient(NEL, P, 1000 * SEED_FAMILY + 1, dtype, dev)
    gK = si.upstream_gradient(NEL, P, 1000 * SEED_FAMILY + 2, dtype, dev)
    return fields, gM, gK


def hbm_probe(dev, gib=2, reps=5):
    """Achievable HBM bandwidth on this machine from plain PyTorch kernels on `gib` GiB
    buffers: write-only (fill), read-only (sum) and copy; GB/s of bytes moved."""
    n = (gib << 30) // 4
    a = torch.empty(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    out = {}
    for name, fn, nbytes in (("write", lambda: a.fill_(2.0), 4 * n),
                             ("read", lambda: a.sum(), 4 * n),
                             ("copy", lambda: b.copy_(a), 8 * n)):
        fn()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_GBs"] = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return out


class Sample:
    """Rows whose results the oracle checks: a contiguous block in the middle of the row
    range, with the buffer offsets of their points (in the space's sample layout)."""

    def __init__(self, sp, n_rows):
        n = [e + P for e in NEL]
        start = sp.n_rows // 2 - n_rows // 2
        self.rows = np.arange(start, start + n_rows, dtype=np.int64)
        Q = P + 1
        if sp.sample_layout == "rows":
            off = self.rows[:, None] * Q ** 3 + np.arange(Q ** 3)[None, :]
        else:
            idx = [self.rows // (n[1] * n[2]), (self.rows // n[2]) % n[1], self.rows % n[2]]
            qs = np.array(np.unravel_index(np.arange(Q ** 3), [Q] * 3))
            off = np.zeros((self.rows.size, Q ** 3), dtype=np.int64)
            dims = list(sp.buffer_shape)            # the last direction's lines may be padded
            for k in range(3):
                off = off * dims[k] + idx[k][:, None] * Q + qs[k][None, :]
        self.ridx = torch.from_numpy(self.rows).to(sp.device)
        self.pidx = torch.from_numpy(off.reshape(-1)).to(sp.device)

    def matrices(self, M, K):
        return M[self.ridx].double().cpu().numpy(), K[self.ridx].double().cpu().numpy()

    def grads(self, grads):
        return [g.reshape(-1)[self.pidx].double().cpu().numpy().reshape(self.rows.size, -1) for g in grads]

    def upstream(self, gM, gK):
        return gM[self.ridx].double().cpu().numpy(), gK[self.ridx].double().cpu().numpy()


def time_forward(sp, fields, M, K, reps=10):
    sp.assemble_fused(fields[0], fields[1:], M, K)
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(reps):
        sp.assemble_fused(fields[0], fields[1:], M, K)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_steps(sp, fields, gM, gK, steps, warmup):
    """`steps` timed steps (forward + adjoint): HIP events on the launch stream around
    every kernel, wall clock around the whole loop with synchronizations on both sides."""
    M = torch.empty(sp.n_rows, sp.slots_per_row, dtype=fields[0].dtype, device=sp.device)
    K = torch.empty_like(M)
    dc = torch.empty(sp.buffer_shape, dtype=fields[0].dtype, device=sp.device)
    da = [torch.empty_like(dc) for _ in range(3)]
    for _ in range(warmup):
        sp.assemble_fused(fields[0], fields[1:], M, K)
        sp.adjoint(gM, gK, dc, da)
    torch.cuda.synchronize()
    evs = [[ev() for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        evs[s][0].record()
        sp.assemble_fused(fields[0], fields[1:], M, K)
        evs[s][1].record()
        sp.adjoint(gM, gK, dc, da)
        evs[s][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = [evs[s][0].elapsed_time(evs[s][1]) for s in range(steps)]
    adj = [evs[s][1].elapsed_time(evs[s][2]) for s in range(steps)]
    stats = {name: {"mean": float(np.mean(v)), "median": float(np.median(v)), "min": float(np.min(v))}
             for name, v in (("forward", fwd), ("adjoint", adj))}
    return {"wall_s": wall, "fwd_ms": float(np.mean(fwd)), "adj_ms": float(np.mean(adj)), "stats": stats,
            "out": (M, K, dc, da)}


def product_macs(p, b1, what, b2=4):
    """Multiply-adds per row of the blocked 3D product kernel on banded rows: the last
    direction over the block's (b1 + 2p)(b2 + 2p) window pairs (one table for M, mass and
    stiffness for K), the second direction over b1 + 2p first-direction columns (one
    table, or three), the first direction and the samples (one term, or three)."""
    q = p + 1
    n3, n2, terms = (1, 1, 1) if what == "M" else (2, 3, 3)
    d3 = n3 * (b1 + 2 * p) * (b2 + 2 * p) * q * (p + 1) / (b1 * b2)
    d2 = n2 * q * (b1 + 2 * p) * (p + 1) * q / b1
    return d3 + d2 + terms * q ** 3 * (p + 1) + terms * q ** 3


def matrix_free(sp, args):
    """Load vector and matrix-free products y = M x, y = K x on the same workload (FP32
    and FP64): event-timed per call, with algorithmic HBM bytes per row -- the samples of
    the fields read (Q^d each), x and y (one value each; x's band is re-read from cache)
    -- and the multiply-adds the products' kernel issues per row (blocks of 4 x 4 x R rows,
    banded rows), in `product_macs`."""
    out = {}
    Q, rows = P + 1, sp.n_rows
    for dtype in ((torch.float32,) if args.skip_fp64 else (torch.float32, torch.float64)):
        b = 4 if dtype == torch.float32 else 8
        macs = {1: product_macs(P, 4, "M"), 3: product_macs(P, 4, "K")}
        fields, _, _ = make_inputs_fields(sp, dtype)
        g = torch.Generator(device=sp.device)
        g.manual_seed(5003)
        x = torch.randn(rows, generator=g, dtype=torch.float64, device=sp.device).to(dtype)
        y = torch.empty_like(x)
        res = {}
        for name, fn, nf, terms in (("load_vector", lambda: sp.load_vector(fields[0], y), 1, 0),
                                    ("apply_mass", lambda: sp.apply_mass(fields[0], x, y), 1, 1),
                                    ("apply_stiffness", lambda: sp.apply_stiffness(fields[1:], x, y), 3, 3)):
            fn()
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(10):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            nbytes = rows * (nf * Q ** 3 + (2 if terms else 1)) * b
            flops = 2.0 * rows * (macs[terms] if terms else Q ** 3)
            gbs = nbytes / (ms * 1e-3) / 1e9
            res[name] = {"ms": ms, "GB_s": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                         "TFLOP_s": flops / (ms * 1e-3) / 1e12, "rows_per_s": rows / (ms * 1e-3)}
        out["fp32" if b == 4 else "fp64"] = res
        del fields, x, y
        torch.cuda.empty_cache()
    return out


def deformed_cube_forward(wqa, dev, reps=20, layout="grid"):
    """The 3D C2 cubic forward on 96^3 elements (970,299 rows) with the deformed-cube
    coefficients (det J, det J / J_kk^2 folded into c and a_k): fused M+K, FP32 under every
    final pass and FP64, event-timed, with the fraction of the 8 TB/s HBM peak.  layout:
    the samples on the grid with lines padded to 32 values, or stored row by row."""
    sp = wqa.Space(3, P, (96, 96, 96), device=dev)
    if layout == "grid":
        sp.set_grid_pitch(padded_pitch(sp))
        out = {"rows": sp.n_rows, "sample_layout": "grid", "grid_pitch": sp.buffer_shape[-1]}
        place = lambda t: padded(sp, t)
    else:
        sp.set_sample_layout("rows")
        out = {"rows": sp.n_rows, "sample_layout": "rows"}
        place = sp.rows_from_grid
    runs = [(torch.float32, f"fp32_{name}", mode) for name, mode in MODES] + [(torch.float64, "fp64", None)]
    for dtype, tag, mode in runs:
        b = 4 if dtype == torch.float32 else 8
        f = [place(si.deformed_cube_grid(sp.grid_axes(field), field, dtype, dev)) for field in ["c", 0, 1, 2]]
        M = torch.empty(sp.n_rows, sp.slots_per_row, dtype=dtype, device=dev)
        K = torch.empty_like(M)
        if mode is not None:
            sp.set_final_mode(mode)
        for _ in range(3):
            sp.assemble_fused(f[0], f[1:], M, K)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            sp.assemble_fused(f[0], f[1:], M, K)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = sp.n_rows * (2 * sp.slots_per_row + 4 * sp.points_per_row) * b
        out[tag] = {"forward_ms": ms, "assembled_nnz_per_s": 2 * sp.n_rows * sp.slots_per_row / (ms * 1e-3),
                    "achieved_GB_s": nbytes / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del f, M, K
        torch.cuda.empty_cache()
    for name, _ in MODES:
        out[f"fp32_{name}"]["speedup_vs_fp64"] = out["fp64"]["forward_ms"] / out[f"fp32_{name}"]["forward_ms"]
    sp.set_final_mode(HEADLINE_MODE)
    return out


def other_layout(wqa, dev, args, layout, reps=10):
    """The headline space's forward and adjoint in another sample layout: FP32 (headline
    final pass) and FP64, event-timed, mean per call, with the fraction of the 8 TB/s HBM
    peak (the algorithmic bytes do not depend on the layout)."""
    def timed(fn):
        fn()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    sp = wqa.Space(3, P, NEL, device=dev)
    use_layout(sp, layout)
    out = {"sample_layout": layout}
    for dtype in ((torch.float32,) if args.skip_fp64 else (torch.float32, torch.float64)):
        b = 4 if dtype == torch.float32 else 8
        nbytes = sp.n_rows * (2 * sp.slots_per_row + 4 * sp.points_per_row) * b
        f = [place(sp, si.fourier_grid(sp.grid_axes(fl), si.fourier_modes(SEED_FAMILY, fid, 3), dtype, dev))
             for fid, fl in enumerate(["c", 0, 1, 2])]
        M = torch.empty(sp.n_rows, sp.slots_per_row, dtype=dtype, device=dev)
        K = torch.empty_like(M)
        r = {"forward_ms": timed(lambda: sp.assemble_fused(f[0], f[1:], M, K))}
        r["forward_frac_of_hbm_peak"] = nbytes / (r["forward_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        gM = si.upstream_gradient(NEL, P, 1000 * SEED_FAMILY + 1, dtype, dev)
        gK = si.upstream_gradient(NEL, P, 1000 * SEED_FAMILY + 2, dtype, dev)
        d = [torch.empty(sp.buffer_shape, dtype=dtype, device=dev) for _ in range(4)]
        r["adjoint_ms"] = timed(lambda: sp.adjoint(gM, gK, d[0], d[1:]))
        r["adjoint_frac_of_hbm_peak"] = nbytes / (r["adjoint_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        out["fp32" if b == 4 else "fp64"] = r
        del f, M, K, gM, gK, d
        torch.cuda.empty_cache()
    return out


def pattern_probes(sp, fields, M, K, gM, gK, grads, reps=10):
    """Memory-pattern probes (libwqa_probes.so) on the step's own buffers: each moves the
    bytes one kernel moves, in its tiles and work-group order, without arithmetic -- the
    ceiling of that kernel's data layout on this GPU -- plus plain streaming at 2 GiB."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1710_01048_amd", "libwqa_probes.so"))
    vp = ctypes.c_void_p
    lib.wqap_stream.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int64, vp]
    lib.wqap_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(vp), vp, vp, vp]
    lib.wqap_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int64), vp, vp, ctypes.POINTER(vp), vp]
    stream = lambda: vp(torch.cuda.current_stream().cuda_stream)
    ne = (ctypes.c_int64 * 3)(*NEL)
    # the probe variant of each kernel's layout and order: forward tiles in runs of 8 per
    # XCD on the grid, of 128 with samples by row; the FP32 adjoint's tiles in runs of 8 per
    # XCD (order bits 128)
    if sp.sample_layout == "rows":
        fwd_code, adj_layout = 3 | 512 | (3 << 4), 512 | 128     # forward: runs of 128 tiles per XCD
    else:
        pad = 256 if sp.buffer_shape[-1] == padded_pitch(sp) != sp.grid_shape[-1] else 0
        fwd_code, adj_layout = 3 | pad, pad | 128

    def timed(fn):
        rc = fn()
        assert rc == 0, f"probe refused ({rc})"
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    fp = (vp * 4)(*[t.data_ptr() for t in fields])
    gp = (vp * 4)(*[t.data_ptr() for t in grads])
    out["forward_pattern_ms"] = timed(lambda: lib.wqap_forward(fwd_code, 0, P, ne, fp, vp(M.data_ptr()),
                                                               vp(K.data_ptr()), stream()))
    out["adjoint_pattern_ms"] = timed(lambda: lib.wqap_adjoint(3, adj_layout, 0, P, ne, vp(gM.data_ptr()),
                                                               vp(gK.data_ptr()), gp, stream()))
    nb = 2 << 30
    a = torch.empty(nb // 4, dtype=torch.float32, device=sp.device)
    b = torch.empty_like(a)
    a.fill_(1.0)
    for name, what, moved in (("write", 0, nb), ("read", 1, nb), ("copy", 2, 2 * nb)):
        ms = timed(lambda: lib.wqap_stream(what, vp(b.data_ptr()), vp(a.data_ptr()), nb, stream()))
        out[f"stream_{name}_GBs"] = moved / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def probe_sweep(wqa, dev, n_el, reps=10):
    """Every variant of the memory-pattern probes on the n_el^3 cubic space, FP32: the
    forward's pattern (loads, stores, both) in three work-group orders, with ordinary or
    nontemporal stores, padded lines or row-by-row samples; the adjoint's pattern in its
    tile layout under three orders, with padded lines, row-by-row gradients (one block per
    matrix, or q_1 by q_1, or 4-byte stores, or blocks in the lanes' order), line-q_1
    blocks, line-wide
    work-groups, whole-tile loads, stores after each matrix, a ring of 3 slabs and at most 8
    waves per CU; streaming and k concurrent write fronts.  Milliseconds per
    call and fractions of 8 TB/s for the whole pattern."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1710_01048_amd", "libwqa_probes.so"))
    vp = ctypes.c_void_p
    lib.wqap_stream.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int64, vp]
    lib.wqap_fronts.argtypes = [vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, vp]
    lib.wqap_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(vp), vp, vp, vp]
    lib.wqap_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int64), vp, vp, ctypes.POINTER(vp), vp]
    stream = lambda: vp(torch.cuda.current_stream().cuda_stream)

    def timed(fn):
        rc = fn()
        if rc != 0:
            return None
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) / reps, 4)

    sp = wqa.Space(3, P, (n_el,) * 3, device=dev, rules=None)
    ne = (ctypes.c_int64 * 3)(n_el, n_el, n_el)
    N = sp.grid_shape
    cells = N[0] * N[1] * ((N[2] + LINE_ALIGN - 1) // LINE_ALIGN * LINE_ALIGN)
    alg = sp.n_rows * (2 * sp.slots_per_row + 4 * sp.points_per_row) * 4
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    M = torch.randn(sp.n_rows, sp.slots_per_row, device=dev, generator=g)
    K = torch.randn(sp.n_rows, sp.slots_per_row, device=dev, generator=g)
    f = [torch.rand(cells, device=dev, generator=g) + 0.5 for _ in range(4)]
    d = [torch.empty(cells, device=dev) for _ in range(4)]
    fp = (vp * 4)(*[t.data_ptr() for t in f])
    dp = (vp * 4)(*[t.data_ptr() for t in d])
    out = {"space": f"{n_el}^3 cubic", "algorithmic_GB": alg / 1e9}
    fwd = {}
    for oname, order in (("xcd_runs_of_8", 0), ("xcd_shares", 1), ("dispatch", 2)):
        for parts, pname in ((1, "loads"), (2, "stores"), (3, "both")):
            fwd[f"{oname}/{pname}"] = timed(lambda: lib.wqap_forward(parts | (order << 4), 0, P, ne, fp, vp(M.data_ptr()),
                                                                     vp(K.data_ptr()), stream()))
    for name, code in (("ordinary_stores/stores", 2 | 64), ("ordinary_stores/both", 3 | 64),
                       ("M_only/stores", 2 | 128), ("padded_lines/both", 3 | 256), ("row_samples/loads", 1 | 512),
                       ("row_samples/both", 3 | 512), ("row_samples_xcd_runs_of_128/both", 3 | 512 | (3 << 4)),
                       ("whole_output_lines/stores", 2 | 192), ("whole_output_lines_row_samples/both", 3 | 192 | 512),
                       ("whole_output_lines_row_samples_xcd_runs_of_128/both", 3 | 192 | 512 | (3 << 4)),
                       ("line_aligned_stores/stores", 2 | 1024),
                       ("line_aligned_stores_row_samples_xcd_runs_of_128/both", 3 | 512 | (3 << 4) | 1024),
                       ("stores_of_constants/stores", 2 | 2048),
                       ("stores_of_constants_row_samples_xcd_runs_of_128/both", 3 | 512 | (3 << 4) | 2048)):
        fwd[name] = timed(lambda: lib.wqap_forward(code, 0, P, ne, fp, vp(M.data_ptr()), vp(K.data_ptr()), stream()))
    out["forward_ms"] = fwd
    adj = {}
    for name, layout, parts_list in (("tiles", 0, (1, 2, 3)), ("tiles_dispatch_order", 64, (2, 3)),
                                     ("tiles_xcd_runs_of_8", 128, (2, 3)), ("tiles_padded_lines", 256, (2, 3)),
                                     ("tiles_padded_lines_xcd_runs_of_8", 256 | 128, (2, 3)),
                                     ("row_gradients_block", 512, (2, 3)), ("row_gradients_per_q1", 1024, (2, 3)),
                                     ("row_gradients_4byte", 2048, (2, 3)), ("stores_after_each_matrix", 49, (2, 3)),
                                     ("line_workgroups", 16 + 15, (2, 3)), ("whole_tile_loads", 48, (1, 2, 3)),
                                     ("tiles_padded_lines_xcd_runs_of_8_ring3", 256 | 128 | 4096, (3,)),
                                     ("tiles_padded_lines_xcd_runs_of_8_8_waves_per_cu", 256 | 128 | 8192, (3,)),
                                     ("row_gradients_block_xcd_runs_of_8", 512 | 128, (2, 3)),
                                     ("row_gradients_block_8_waves_per_cu", 512 | 8192, (3,)),
                                     ("row_gradients_block_xcd_runs_of_8_8_waves_per_cu", 512 | 128 | 8192, (3,)),
                                     ("row_gradients_lane_order", 16384, (2, 3)),
                                     ("row_gradients_lane_order_xcd_runs_of_8", 16384 | 128, (2, 3)),
                                     ("row_gradients_lane_order_xcd_runs_of_8_8_waves_per_cu", 16384 | 128 | 8192,
                                      (3,)),
                                     ("line_q1_blocks", 32768, (2, 3)),
                                     ("line_q1_blocks_xcd_runs_of_8", 32768 | 128, (2, 3))):
        for parts in parts_list:
            pname = {1: "loads", 2: "stores", 3: "both"}[parts]
            adj[f"{name}/{pname}"] = timed(lambda: lib.wqap_adjoint(parts, layout, 0, P, ne, vp(M.data_ptr()),
                                                                    vp(K.data_ptr()), dp, stream()))
    out["adjoint_ms"] = adj
    out["frac_of_hbm_peak"] = {k: {n: (alg / (v * 1e-3) / 1e9 / HBM_PEAK_GBS if v and n.endswith("both") else None)
                                   for n, v in out[k].items()} for k in ("forward_ms", "adjoint_ms")}
    del M, K, f, d
    torch.cuda.empty_cache()
    nb = 2 << 30
    a = torch.empty(nb // 4, device=dev)
    b = torch.empty(nb // 4 + (64 << 20), device=dev)
    a.fill_(1.0)
    st = {}
    for name, what, moved in (("write", 0, nb), ("read", 1, nb), ("copy", 2, 2 * nb)):
        ms = timed(lambda: lib.wqap_stream(what, vp(b.data_ptr()), vp(a.data_ptr()), nb, stream()))
        st[f"{name}_TBs"] = moved / (ms * 1e-3) / 1e12 if ms else None
    for k in (1, 16, 128):
        per = (nb // k) // 4096 * 4096
        ms = timed(lambda: lib.wqap_fronts(vp(b.data_ptr()), k, per, per, stream()))
        st[f"fronts_{k}_write_TBs"] = per * k / (ms * 1e-3) / 1e12 if ms else None
    out["stream"] = st
    return out


def make_inputs_fields(sp, dtype):
    fields = []
    for field in ["c", 0, 1, 2]:
        fid = 0 if field == "c" else field + 1
        fields.append(place(sp, si.fourier_grid(sp.grid_axes(field), si.fourier_modes(SEED_FAMILY, fid, 3), dtype,
                                                 sp.device)))
    return fields, None, None


def oracle_inputs(rows):
    from oracle import assembly as oa
    tabs = oa.rule_tables(P, NEL)
    vals = []
    for field in ["c", 0, 1, 2]:
        fid = 0 if field == "c" else field + 1
        xyz = oa.row_point_coords(P, NEL, tabs, rows, field)
        vals.append(si.fourier_points(xyz.reshape(-1, 3), si.fourier_modes(SEED_FAMILY, fid, 3)).reshape(xyz.shape[:2]))
    return tabs, vals


def oracle_run(rows, gm, gk):
    """FP64 oracle (OpenMP over rows, all host cores) on the listed rows: forward then
    adjoint.  Returns (seconds, tables, M, K, dc, da)."""
    from oracle import assembly as oa
    tabs, vals = oracle_inputs(rows)
    t0 = time.perf_counter()
    M, K = oa.assemble(P, NEL, tabs, c=vals[0], a=vals[1:], rows=rows, per_row=True)
    dc, da = oa.adjoint(P, NEL, tabs, gm, gk, rows=rows)
    return time.perf_counter() - t0, tabs, M, K, dc, da


def rowscaled(got, want):
    s = np.abs(want).max(axis=1, keepdims=True)
    s[s == 0] = 1
    return float((np.abs(got - want) / s).max())


def per_entry(got, want, scale):
    """Largest gradient error over the sum of the magnitudes of the terms the entry sums
    ([rows, points]); points whose terms vanish in exact arithmetic (a node at a zero of
    B'_j) hold rounding noise only and are measured against their row's largest scale."""
    row_max = scale.max(axis=1, keepdims=True)
    eff = np.where(scale >= 1e-10 * row_max, scale, row_max)
    return float((np.abs(got - want) / np.where(eff == 0, 1, eff)).max())


def traffic_for(kernel, layout):
    """HBM bytes per launch of `kernel` from the committed counter summary, provided it
    was taken on the current kernel source and in the same sample layout (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            src = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    entry = data.get("kernels", {}).get(kernel)
    if not entry or data.get("kernel_source_sha256") != src or data.get("sample_layout", "grid") != layout:
        return None
    return entry["fetch_bytes"] + entry["write_bytes"]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); rows are independent, see the "
              "sharding note of the design document", file=sys.stderr)
        sys.exit(2)
    import paper_1710_01048_amd as wqa
    from paper_1710_01048_amd import counts
    assert torch.cuda.is_available(), "needs a HIP device"
    dev = torch.device("cuda:0")
    if args.cube96_only:
        print(json.dumps({"forward_96cubed_deformed_cube": deformed_cube_forward(wqa, dev),
                          "forward_96cubed_deformed_cube_rows": deformed_cube_forward(wqa, dev, layout="rows")}),
              flush=True)
        return
    if args.probe_sweep:
        print(json.dumps({"probe_sweep": probe_sweep(wqa, dev, args.probe_sweep)}), flush=True)
        return
    if args.profile_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 3 x 1 GiB read + 1 GiB written")
    sp = wqa.Space(3, P, NEL, device=dev)
    use_layout(sp, args.layout)
    nnz_mat = sp.n_rows * sp.slots_per_row
    nnz_step = 4 * nnz_mat
    log(f"space: {sp.n_rows} rows x {sp.slots_per_row} slots, grid {sp.grid_shape}, buffers {sp.buffer_shape}")
    if args.products_only:
        print(json.dumps({"matrix_free": matrix_free(sp, args)}), flush=True)
        return

    sample = None
    if not args.no_cpu_baseline:
        n_cal = 8192
        cal = Sample(sp, n_cal)
        zero = np.zeros((n_cal, sp.slots_per_row))
        dt = oracle_run(cal.rows, zero, zero)[0]
        n_sample = int(min(600000, max(n_cal, n_cal * args.cpu_seconds / max(dt, 1e-3))))
        sample = Sample(sp, n_sample)
        log(f"oracle: {n_cal} rows in {dt:.3f} s -> sample of {n_sample} rows")

    # ---- FP32 ------------------------------------------------------------------------
    fields, gM, gK = make_inputs(sp, torch.float32)
    torch.cuda.synchronize()
    mode_ms, mode_rows = {}, {}
    if not args.skip_modes:
        M = torch.empty(sp.n_rows, sp.slots_per_row, dtype=torch.float32, device=dev)
        K = torch.empty_like(M)
        for name, mode in MODES:
            sp.set_final_mode(mode)
            mode_ms[name] = time_forward(sp, fields, M, K)
            if sample is not None:
                mode_rows[name] = sample.matrices(M, K)
        del M, K
        log(f"fp32 forward by final pass (ms): {mode_ms}")
    sp.set_final_mode(HEADLINE_MODE)
    r32 = run_steps(sp, fields, gM, gK, args.steps, args.warmup)
    step_ms = r32["wall_s"] * 1e3 / args.steps
    log(f"fp32: forward {r32['fwd_ms']:.3f} ms, adjoint {r32['adj_ms']:.3f} ms, step {step_ms:.3f} ms")
    g32 = None
    if sample is not None:
        mode_rows["headline"] = sample.matrices(r32["out"][0], r32["out"][1])
        g32 = (sample.upstream(gM, gK), sample.grads([r32["out"][2]] + list(r32["out"][3])))
    patterns = None
    if not args.no_probes:
        M, K, dc, da = r32["out"]
        patterns = pattern_probes(sp, fields, M, K, gM, gK, [dc] + list(da))
        del M, K, dc, da
        log(f"pattern probes: {patterns}")
    del r32["out"], fields, gM, gK
    torch.cuda.empty_cache()

    # ---- FP64 ------------------------------------------------------------------------
    r64, g64, m64 = None, None, None
    if not args.skip_fp64:
        f64, gM64, gK64 = make_inputs(sp, torch.float64)
        torch.cuda.synchronize()
        r64 = run_steps(sp, f64, gM64, gK64, args.fp64_steps, 1)
        log(f"fp64: forward {r64['fwd_ms']:.3f} ms, adjoint {r64['adj_ms']:.3f} ms")
        if sample is not None:
            m64 = sample.matrices(r64["out"][0], r64["out"][1])
            g64 = (sample.upstream(gM64, gK64), sample.grads([r64["out"][2]] + list(r64["out"][3])))
        del r64["out"], f64, gM64, gK64
        torch.cuda.empty_cache()

    mfree, cube96, cube96_rows, alt = None, None, None, None
    alt_layout = "grid" if args.layout == "rows" else "rows"
    if not args.headline_only:
        mfree = matrix_free(sp, args)
        log(f"matrix-free: {mfree}")
        cube96 = deformed_cube_forward(wqa, dev)
        log(f"96^3 deformed cube forward: {cube96}")
        cube96_rows = deformed_cube_forward(wqa, dev, layout="rows")
        log(f"96^3 deformed cube forward, samples by row: {cube96_rows}")
        alt = other_layout(wqa, dev, args, alt_layout)
        log(f"{alt_layout} layout: {alt}")

    probe = hbm_probe(dev)
    log(f"hbm probe: {probe}")

    # algorithmic HBM bytes per launch, forward and adjoint alike: per row 2 x S^3 matrix
    # values (written by the forward, read by the adjoint) + 4 x Q^3 field samples
    # (read by the forward, written by the adjoint), 4 bytes each in FP32
    alg_bytes = sp.n_rows * (2 * sp.slots_per_row + 4 * sp.points_per_row) * 4

    # the writes alone: the forward writes the two matrices, the adjoint the four gradients
    write_bytes = {"forward_fp32_mk": sp.n_rows * 2 * sp.slots_per_row * 4,
                   "adjoint_fp32_mk": sp.n_rows * 4 * sp.points_per_row * 4}
    best_probe = max(probe.values())

    def roof(ms, kernel, pattern_ms):
        achieved = alg_bytes / (ms * 1e-3) / 1e9
        traffic = traffic_for(kernel, args.layout)
        wb = write_bytes[kernel]
        out = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": alg_bytes,
               "write_bytes": wb, "write_frac": wb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "frac_of_best_probe": achieved / best_probe}
        if pattern_ms is not None:
            # the same bytes in the same pattern without arithmetic (libwqa_probes.so)
            out["pattern_ceiling"] = alg_bytes / (pattern_ms * 1e-3) / 1e9
            out["frac_of_pattern_ceiling"] = pattern_ms / ms
        return out

    roof_fwd = roof(r32["fwd_ms"], "forward_fp32_mk", patterns and patterns["forward_pattern_ms"])
    roof_adj = roof(r32["adj_ms"], "adjoint_fp32_mk", patterns and patterns["adjoint_pattern_ms"])
    line = {
        "metric": METRIC,
        "value": nnz_step / (step_ms * 1e-3),
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D C2 cubic, 160^3 elements (4,330,747 rows x 343 slots), fused M+K forward "
                               "then adjoint, random-Fourier c and diagonal A, FP32 values and stages; the final "
                               "directional pass accumulated in FP64 (Dot2-compensated FP32 pass reported beside it)",
                   "final_pass": "f64_accumulate",
                   "rows": sp.n_rows, "slots_per_row": sp.slots_per_row, "nnz_per_step": nnz_step,
                   "sample_layout": args.layout,
                   "grid_pitch": sp.buffer_shape[-1] if args.layout == "grid" else None,
                   "parallelism": "single GPU"},
        "forward_ms": r32["fwd_ms"],
        "adjoint_ms": r32["adj_ms"],
        "kernel_ms_per_call": r32["stats"],
        "assembled_nnz_per_s_fp32": 2 * nnz_mat / (r32["fwd_ms"] * 1e-3),
        "adjoint_nnz_per_s_fp32": 2 * nnz_mat / (r32["adj_ms"] * 1e-3),
        "forward_ms_by_final_pass": mode_ms,
        "roofline": roof_fwd if r32["fwd_ms"] >= r32["adj_ms"] else roof_adj,
        "roofline_by_kernel": {"forward": roof_fwd, "adjoint": roof_adj},
        "hbm_probe_torch": probe,
        "pattern_probes": patterns,
        "matrix_free": mfree,
        "forward_96cubed_deformed_cube": cube96,
        "forward_96cubed_deformed_cube_rows": cube96_rows,
        f"sample_layout_{alt_layout}": alt,
        "rule_counts": counts.report(P, NEL),
    }
    if r64 is not None:
        line["fp64"] = {"forward_ms": r64["fwd_ms"], "adjoint_ms": r64["adj_ms"],
                        "assembled_nnz_per_s": 2 * nnz_mat / (r64["fwd_ms"] * 1e-3),
                        "adjoint_nnz_per_s": 2 * nnz_mat / (r64["adj_ms"] * 1e-3),
                        "forward_frac_of_hbm_peak": 2 * alg_bytes / (r64["fwd_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "adjoint_frac_of_hbm_peak": 2 * alg_bytes / (r64["adj_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "kernel_ms_per_call": r64["stats"]}
        line["fp32_vs_fp64_speedup"] = {"forward": r64["fwd_ms"] / r32["fwd_ms"],
                                        "adjoint": r64["adj_ms"] / r32["adj_ms"],
                                        "step": (r64["fwd_ms"] + r64["adj_ms"]) / (r32["fwd_ms"] + r32["adj_ms"])}
    # every FP32 final pass of the forward: its time, its fraction of the HBM peak and its
    # speedup over the FP64 forward (errors against the oracle in accuracy_vs_oracle)
    line["final_pass_modes"] = {
        name: {"forward_ms": ms, "frac_of_hbm_peak": alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "speedup_vs_fp64_forward": (r64["fwd_ms"] / ms) if r64 is not None else None,
               "arithmetic": {"plain": "FP32 fused multiply-adds",
                              "dot2": "compensated summation in FP32 (Ogita-Rump-Oishi Dot2)",
                              "f64_accumulate": "FP32 stage results times FP64 table entries, summed in FP64 "
                                                "(mixed precision; the headline)"}[name]}
        for name, ms in mode_ms.items()}
    if sample is not None:
        from oracle import assembly as oa
        up = g64[0] if g64 is not None else g32[0]
        dt, tabs, Mw, Kw, wc, wa = oracle_run(sample.rows, *up)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        line["cpu_baseline"] = {
            "value": 4 * sample.rows.size * sp.slots_per_row / dt, "unit": "nnz/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample.rows.size} contiguous rows (of {sp.n_rows}) of the same workload: FP64 direct-sum "
                      f"forward + adjoint in {dt:.1f} s"}
        acc = {}
        for name, (Mg, Kg) in mode_rows.items():
            acc[f"fp32_{name}"] = {"M_rowscaled": rowscaled(Mg, Mw), "K_rowscaled": rowscaled(Kg, Kw)}
        wc32, wa32 = oa.adjoint(P, NEL, tabs, *g32[0], rows=sample.rows)
        sc32, sa32 = oa.adjoint(P, NEL, tabs, *g32[0], rows=sample.rows, absolute=True)
        acc["fp32_grad_per_entry"] = max(per_entry(g, w, sc) for g, w, sc in
                                         zip(g32[1], [wc32] + list(wa32), [sc32] + list(sa32)))
        if m64 is not None:
            sc, sa = oa.adjoint(P, NEL, tabs, *up, rows=sample.rows, absolute=True)
            acc["fp64"] = {"M_rowscaled": rowscaled(m64[0], Mw), "K_rowscaled": rowscaled(m64[1], Kw),
                           "grad_per_entry": max(per_entry(g, w, x) for g, w, x in
                                                 zip(g64[1], [wc] + list(wa), [sc] + list(sa)))}
        acc["tolerance"] = {"fp32": 1e-5, "fp64": 1e-12,
                            "measure": "row-scaled (matrices); gradients per entry, over the sum of the "
                                       "magnitudes of the terms each entry sums"}
        line["accuracy_vs_oracle"] = acc
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
