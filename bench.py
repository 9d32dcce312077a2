"""Benchmark of the fused phi + mu step on one MI355X.

Workload: 2D 4096 x 4096 directional eutectic (3 phases, ternary: 2 mu fields),
x periodic / y no-flux, seeded synthetic initial state (lamellae slab in melt).
A benchmark step is one forward-Euler time step of the whole field (one launch
of the fused kernel).  The timed region runs exactly --steps steps in FP64
(``value``) and, separately, in FP32 (``fp32``), with the state resident in HBM.

Prints one JSON line.  Options: --gpus (only 1 is supported), --steps, --warmup,
--no-cpu (skip the CPU oracle leg), --no-fp32, --n (grid side, default 4096).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--tile", type=str, default="", help="bx,seg override")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of one FP64 state buffer instead")
    return ap.parse_args()


def copy_calibration(n, steps):
    """Plain device-to-device copy of one FP64 C2 state buffer (5 fields x n x n):
    the practical HBM ceiling, and the known-size reference for traffic counters."""
    import torch

    nbytes = 5 * n * n * 8
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"copy_bytes_each_way": nbytes, "ms_per_copy": ms, "GBs_read_plus_write": gbs,
                      "frac_of_8TBs": gbs / HBM_PEAK_GBS}), flush=True)


def time_precision(precision, n, steps, warmup, tile):
    import torch

    from paper_2404_01035_amd import inputs
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(precision=precision, n=(n, n, 1))
    s = Solver(p)
    if tile:
        bx, seg = (int(v) for v in tile.split(","))
        s.set_tile(bx, seg)
    s.load(phi, mu)
    del phi, mu
    s.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = s.diagnostics()
    s.close()
    ncells = p.ncells
    elem = 8 if precision == "f64" else 4
    bytes_per_step = ncells * p.nfields * 2 * elem  # read + write of every field once
    ms_step = ms / steps
    gbs = bytes_per_step / (ms_step * 1e-3) / 1e9
    return {
        "value": ncells * steps / (ms * 1e-3),
        "ms_per_step": ms_step,
        "roofline": {
            "bound": "hbm",
            "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
        "bytes_per_cell_update": p.nfields * 2 * elem,
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
    }


def cpu_baseline(n):
    """The FP64 oracle (numpy, one thread) on one full-grid step of the same workload."""
    from oracle import gp
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c2(precision="f64", n=(n, n, 1))
    t0 = time.perf_counter()
    gp.step(phi, mu, 0, p)
    dt = time.perf_counter() - t0
    return {
        "value": p.ncells / dt,
        "unit": "cell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"1 step of the full {n}x{n} grid, FP64 numpy oracle ({dt:.1f} s)",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.copy_calibration:
        copy_calibration(a.n, a.steps)
        return
    print(f"[bench] FP64 {a.n}x{a.n}: warmup {a.warmup}, timed {a.steps} steps", file=sys.stderr,
          flush=True)
    r64 = time_precision("f64", a.n, a.steps, a.warmup, a.tile)
    r32 = None
    if not a.no_fp32:
        print(f"[bench] FP32 {a.n}x{a.n}", file=sys.stderr, flush=True)
        r32 = time_precision("f32", a.n, a.steps, a.warmup, a.tile)
    cpu = None
    if not a.no_cpu:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.n)
    out = {
        "metric": "cell-updates/s of fused phi+mu step (FP64 vs FP32), % HBM peak, adjoint/fwd cost",
        "value": r64["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded eutectic lamellae slab in melt, seeded parabolic coefficients",
        "config": {
            "workload": f"2D {a.n}x{a.n} directional eutectic, 3 phases, ternary (2 mu), "
                        "x periodic / y no-flux, FP64",
            "grid": [a.n, a.n],
            "phases": 3,
            "components": 3,
            "parallelism": "single GPU",
        },
        "roofline": r64["roofline"],
        "cpu_baseline": cpu,
    }
    if r32:
        out["fp32"] = {
            "value": r32["value"],
            "ms_per_step": r32["ms_per_step"],
            "roofline": r32["roofline"],
            "dtype": "f32 (FP64 Lagrange multiplier and reductions)",
        }
        out["speedup_fp32_over_fp64"] = r32["value"] / r64["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
