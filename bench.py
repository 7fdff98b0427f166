"""Benchmark: weighted-quadrature row-wise assembly on one MI355X.

One step = one pass of the whole path over the workload: the fused mass + stiffness
forward assembly followed by its adjoint, on the 3D C^2 cubic space with 160^3
elements (4,330,747 rows, 343 slots per row), random-Fourier c and anisotropic
diagonal A, FP32 values in the implicit-column band layout, compensated final pass.
Inputs (coefficients and upstream gradients) are resident in HBM before timing.

value = slots processed per second over the step: 2 x rows x 343 assembled (M and K)
plus 2 x rows x 343 upstream-gradient slots consumed by the adjoint.  The same
workload in FP64 is timed afterwards for the FP32-vs-FP64 comparison, and the FP64
CPU oracle is timed on a row sample (cpu_baseline) and checks the GPU results there.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
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
CONFIG_ID = 5
FINAL_MODE = 1                 # compensated final pass (wqa.FINAL_COMPENSATED)
METRIC = "assembled nnz/s (3D C2 cubic M+K) FP32 vs FP64 at stated err; adjoint nnz/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample size (0: calibrate to ~15 s)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--profile-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter calibration under rocprofv3)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(sp, dtype):
    dev = sp.device
    fields = []
    for field in ["c", 0, 1, 2]:
        fid = 0 if field == "c" else field + 1
        fields.append(si.fourier_grid(sp.grid_axes(field), si.fourier_modes(CONFIG_ID, fid, 3), dtype, dev).contiguous())
    gM = si.upstream_gradient(NEL, P, 1000 * CONFIG_ID + 1, dtype, dev)
    gK = si.upstream_gradient(NEL, P, 1000 * CONFIG_ID + 2, dtype, dev)
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
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_GBs"] = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return out


def run_steps(sp, fields, gM, gK, steps, warmup):
    """Times `steps` steps (forward + adjoint) with HIP events on the launch stream."""
    M = torch.empty(sp.n_rows, sp.slots_per_row, dtype=fields[0].dtype, device=sp.device)
    K = torch.empty_like(M)
    dc = torch.empty_like(fields[0])
    da = [torch.empty_like(fields[0]) for _ in range(3)]
    for _ in range(warmup):
        sp.assemble_fused(fields[0], fields[1:], M, K)
        sp.adjoint(gM, gK, dc, da)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record()
        sp.assemble_fused(fields[0], fields[1:], M, K)
        ev[s][1].record()
        sp.adjoint(gM, gK, dc, da)
        ev[s][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = [ev[s][0].elapsed_time(ev[s][1]) for s in range(steps)]
    adj = [ev[s][1].elapsed_time(ev[s][2]) for s in range(steps)]
    return {"wall_s": wall, "fwd_ms": fwd, "adj_ms": adj, "out": (M, K, dc, da)}


def _rows_g(g, ridx):
    return None if g is None else g[ridx].double().cpu().numpy()


def cpu_baseline(sp, out32, out64, g32, g64, n_rows_sample):
    """FP64 oracle (OpenMP over rows, all host cores) on a contiguous block of rows of the
    same workload: forward then adjoint.  Also states the GPU errors on those rows
    (each precision against the oracle fed with that run's own upstream gradient)."""
    from oracle import assembly as oa
    tabs = oa.rule_tables(P, NEL)
    n = [e + P for e in NEL]
    start = sp.n_rows // 2 - n_rows_sample // 2
    rows = np.arange(start, start + n_rows_sample, dtype=np.int64)
    vals = []
    for field in ["c", 0, 1, 2]:
        fid = 0 if field == "c" else field + 1
        xyz = oa.row_point_coords(P, NEL, tabs, rows, field)
        vals.append(si.fourier_points(xyz.reshape(-1, 3), si.fourier_modes(CONFIG_ID, fid, 3)).reshape(xyz.shape[:2]))
    ridx = torch.from_numpy(rows).to(sp.device)
    g_rows = {tag: (_rows_g(g[0], ridx), _rows_g(g[1], ridx)) for tag, g in (("fp32", g32), ("fp64", g64))
              if g is not None}
    timed_tag = "fp64" if "fp64" in g_rows else "fp32"
    t0 = time.perf_counter()
    Mw, Kw = oa.assemble(P, NEL, tabs, c=vals[0], a=vals[1:], rows=rows, per_row=True)
    grads_want = {timed_tag: oa.adjoint(P, NEL, tabs, *g_rows[timed_tag], rows=rows)}
    dt = time.perf_counter() - t0
    for tag in g_rows:
        if tag not in grads_want:
            grads_want[tag] = oa.adjoint(P, NEL, tabs, *g_rows[tag], rows=rows)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def rowscaled(got, want):
        s = np.abs(want).max(axis=1, keepdims=True)
        s[s == 0] = 1
        return float((np.abs(got - want) / s).max())

    # points of the sampled rows in grid order
    Q = P + 1
    idx = [rows // (n[1] * n[2]), (rows // n[2]) % n[1], rows % n[2]]
    qs = np.array(np.unravel_index(np.arange(Q ** 3), [Q] * 3))
    off = np.zeros((rows.size, Q ** 3), dtype=np.int64)
    for k in range(3):
        off = off * (n[k] * Q) + idx[k][:, None] * Q + qs[k][None, :]
    offt = torch.from_numpy(off.reshape(-1)).to(sp.device)
    acc = {}
    for tag, out in (("fp32", out32), ("fp64", out64)):
        if out is None:
            continue
        M, K, dc, da = out
        e = {"M_rowscaled": rowscaled(M[ridx].double().cpu().numpy(), Mw),
             "K_rowscaled": rowscaled(K[ridx].double().cpu().numpy(), Kw)}
        wc, wa = grads_want[tag]
        grads = [dc] + list(da)
        wants = [wc] + list(wa)
        e["grad_normwise"] = max(
            float(np.abs(g.reshape(-1)[offt].double().cpu().numpy().reshape(rows.size, -1) - w).max()
                  / np.abs(w).max()) for g, w in zip(grads, wants))
        acc[tag] = e
    slots = 4 * rows.size * (2 * P + 1) ** 3
    return {"value": slots / dt, "unit": "nnz/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows.size} contiguous rows (of {sp.n_rows}) of the same workload, fused forward + adjoint, "
                      f"FP64 direct sums, {dt:.1f} s"}, acc, dt


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); rows are independent, see the "
              "sharding note of the design document", file=sys.stderr)
        sys.exit(2)
    import paper_1710_01048_amd as wqa
    assert torch.cuda.is_available(), "needs a HIP device"
    dev = torch.device("cuda:0")
    if args.profile_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 3 x 1 GiB read + 1 GiB written")
    sp = wqa.Space(3, P, NEL, device=dev)
    sp.set_final_mode(FINAL_MODE)
    nnz_mat = sp.n_rows * sp.slots_per_row
    nnz_step = 4 * nnz_mat
    log(f"space: {sp.n_rows} rows x {sp.slots_per_row} slots, grid {sp.grid_shape}")

    fields, gM, gK = make_inputs(sp, torch.float32)
    torch.cuda.synchronize()
    log("fp32 inputs ready; timing")
    r32 = run_steps(sp, fields, gM, gK, args.steps, args.warmup)
    fwd32, adj32 = float(np.mean(r32["fwd_ms"])), float(np.mean(r32["adj_ms"]))
    step_ms = r32["wall_s"] * 1e3 / args.steps
    log(f"fp32: forward {fwd32:.3f} ms, adjoint {adj32:.3f} ms, step {step_ms:.3f} ms")

    # forward time of each FP32 final-pass mode (same inputs and outputs)
    mode_ms = {}
    M, K = r32["out"][0], r32["out"][1]
    for name, mode in (("plain", wqa.FINAL_PLAIN), ("compensated", wqa.FINAL_COMPENSATED),
                       ("f64_accumulate", wqa.FINAL_F64)):
        sp.set_final_mode(mode)
        sp.assemble_fused(fields[0], fields[1:], M, K)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        for i in range(5):
            evs[i].record()
            sp.assemble_fused(fields[0], fields[1:], M, K)
        evs[5].record()
        torch.cuda.synchronize()
        mode_ms[name] = evs[0].elapsed_time(evs[5]) / 5
    sp.set_final_mode(FINAL_MODE)
    sp.assemble_fused(fields[0], fields[1:], M, K)   # leave the headline mode's results in M, K
    log(f"fp32 forward by final pass: {mode_ms}")

    b = 4  # bytes per FP32 value
    fwd_bytes = sp.n_rows * (2 * sp.slots_per_row + 4 * sp.points_per_row) * b
    adj_bytes = fwd_bytes
    dominant = "forward" if fwd32 >= adj32 else "adjoint"
    dom_ms = max(fwd32, adj32)
    achieved = (fwd_bytes if dominant == "forward" else adj_bytes) / (dom_ms * 1e-3) / 1e9

    keep32 = None
    r64 = None
    g64 = None
    if not args.skip_fp64:
        # keep a sample of the fp32 results for the accuracy statement, then free
        keep32 = r32["out"]
        f64, gM64, gK64 = make_inputs(sp, torch.float64)
        torch.cuda.synchronize()
        log("fp64 inputs ready; timing")
        r64 = run_steps(sp, f64, gM64, gK64, args.fp64_steps, 1)
        log(f"fp64: forward {np.mean(r64['fwd_ms']):.3f} ms, adjoint {np.mean(r64['adj_ms']):.3f} ms")
        g64 = (gM64, gK64)
        del f64

    probe = hbm_probe(dev)
    log(f"hbm probe: {probe}")
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
                               "then adjoint, random-Fourier c and diagonal A, FP32 with compensated final pass",
                   "rows": sp.n_rows, "slots_per_row": sp.slots_per_row, "nnz_per_step": nnz_step,
                   "parallelism": "single GPU"},
        "forward_ms": fwd32,
        "forward_ms_by_final_pass": mode_ms,
        "adjoint_ms": adj32,
        "assembled_nnz_per_s_fp32": 2 * nnz_mat / (fwd32 * 1e-3),
        "adjoint_nnz_per_s_fp32": 2 * nnz_mat / (adj32 * 1e-3),
        "roofline": {"bound": "hbm", "kernel": f"{dominant} (fused M+K, FP32)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes": fwd_bytes},
        "hbm_probe_torch": probe,
    }
    if r64 is not None:
        fwd64, adj64 = float(np.mean(r64["fwd_ms"])), float(np.mean(r64["adj_ms"]))
        line["fp64"] = {"forward_ms": fwd64, "adjoint_ms": adj64,
                        "assembled_nnz_per_s": 2 * nnz_mat / (fwd64 * 1e-3),
                        "adjoint_nnz_per_s": 2 * nnz_mat / (adj64 * 1e-3),
                        "step_nnz_per_s": nnz_step / ((fwd64 + adj64) * 1e-3)}
        line["fp32_vs_fp64_speedup"] = {"forward": fwd64 / fwd32, "adjoint": adj64 / adj32,
                                        "step": (fwd64 + adj64) / (fwd32 + adj32)}
    if not args.no_cpu_baseline:
        n_sample = args.cpu_rows
        if n_sample <= 0:
            _, _, dt = cpu_baseline(sp, None, None, (gM, gK), None, 512)
            n_sample = int(min(200000, max(1024, 512 * 15.0 / max(dt, 1e-3))))
            log(f"oracle calibration: 512 rows in {dt:.2f} s -> sample {n_sample} rows")
        out64 = r64["out"] if r64 is not None else None
        cb, acc, dt = cpu_baseline(sp, keep32 if keep32 is not None else r32["out"], out64, (gM, gK), g64,
                                   n_sample)
        line["cpu_baseline"] = cb
        line["accuracy_vs_oracle"] = acc
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
