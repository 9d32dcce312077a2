"""Benchmark of the fused phi + mu step on one MI355X.

Headline workload: 2D 4096 x 4096 directional eutectic (3 phases, ternary: 2 mu
fields), x periodic / y no-flux, seeded synthetic initial state (lamellae slab
in melt).  A benchmark step is one forward-Euler time step of the whole field
(the fused phi + mu update); the 2D kernels perform two steps per launch, so
the state crosses HBM once per two steps (bitwise the same result as single
steps).  The timed region runs exactly --steps steps in FP64 (``value``) and,
separately, in FP32 (``fp32``), with the state resident in HBM, at the
library's default tiles (the autotuner's picks for this workload; --tune
re-tunes).

Further legs, each a block of the same JSON line:
  dendrite_3d  3D 512^3 binary dendrite with cubic anisotropy, FP32
  batched      256 uneven 2D instances in one persistent launch per two
               steps, replayed as HIP graphs, FP32
  adjoint      512^2 three-phase ternary run, FP32: checkpointed forward run
               (every 100 steps) and the adjoint sweep; their cost ratio
cpu_baseline   the FP64 oracle on two full 4096^2 steps, on the host.

Prints one JSON line.  Options: --gpus (only 1 is supported), --steps,
--warmup, --legs, --no-cpu, --n (2D grid side), --tune, --tile / --tile32 /
--tile3d bx,seg,vec and --tile-batch seg,vec (fixed tiles).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# MI355X vector ALU peaks, TFLOP/s (an FMA counts 2): 256 CUs x 4 SIMDs x 2.4 GHz
# x 16 FP64 lanes (78.6) or x 32 FP32 lanes (157.3), x 2
ALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
CSRC = os.path.join(ROOT, "paper_2404_01035_amd", "csrc")

# HBM bytes per launch of each leg's step kernel, from rocprofv3 counter runs:
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB), the factors being what the same
# counters read for a plain device copy of known size.  A figure holds only
# for the tile and steps per launch it was taken at and for the device sources
# it was taken on (LEG_SOURCES); otherwise the leg reports traffic null.
TRAFFIC = {
    # profiles/k_step2d_eutectic_4096_f64_f32.md
    "c2_f64": {"tile": [256, 31, 1], "fuse": 2, "src": "6e2eeb30c1003a7d",
               "bytes": (2.0 * 388809.3 + 665712.5) * 1024},
    "c2_f32": {"tile": [256, 14, 1], "fuse": 2, "src": "54c91d5dca69cf03",
               "bytes": (2.0 * 224223.4 + 333893.5) * 1024},
    # profiles/k_step3d_dendrite_512_f32.md
    "c3": {"tile": [512, 64, -1], "fuse": 1, "src": "81371fb33d083eef",
           "bytes": (2.0 * 1094183.8 + 1572864.0) * 1024},
    # profiles/k_batch2d_ensemble_256_f32.md
    "c4": {"tile": [256, 32, 1], "fuse": 2, "src": "112d348f54601712",
           "bytes": (2.0 * 705130.6 + 1235434.8) * 1024},
    # profiles/k_antitrap2d_eutectic_4096_f64_f32.md
    "at_f64": {"tile": [62, 12, 1], "fuse": 1, "src": "7f724703195dd7d3",
               "bytes": (2.0 * 867775.7 + 269022.1) * 1024},
    "at_f32": {"tile": [62, 12, 1], "fuse": 1, "src": "7f724703195dd7d3",
               "bytes": (2.0 * 459730.5 + 137750.1) * 1024},
    # profiles/k_antitrap3d_dendrite_512_f32.md
    "at3d_f32": {"tile": [64, 4, 1], "fuse": 1, "src": "7f724703195dd7d3",
                 "bytes": (2.0 * 2646601.9 + 524288.0) * 1024},
}
METRIC = "cell-updates/s of fused phi+mu step (FP64 vs FP32), % HBM peak, adjoint/fwd cost"
ALL_LEGS = ("c2", "c3", "c4", "c5", "at")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--legs", type=str, default=",".join(ALL_LEGS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the legs instead of using the library's default tiles")
    ap.add_argument("--tile", type=str, default="", help="bx,seg,vec of the FP64 leg")
    ap.add_argument("--tile32", type=str, default="", help="bx,seg,vec of the FP32 leg")
    ap.add_argument("--tile3d", type=str, default="", help="bx,seg,vec of the 3D leg (no tuning)")
    ap.add_argument("--tile-batch", type=str, default="",
                    help="seg,vec of the batched leg (no tuning)")
    ap.add_argument("--steps3d", type=int, default=100)
    ap.add_argument("--n3d", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=400)
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of one FP64 state buffer instead")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The device sources each leg's step kernel is built from.
_COMMON = ["mp_internal.hpp", "gp_device.hpp"]
LEG_SOURCES = {
    "c2_f64": _COMMON + ["step2d.hpp", "step3d.hpp", "step_dispatch.hpp", "step_f64_2d.hip"],
    "c2_f32": _COMMON + ["step2d.hpp", "step3d.hpp", "step_dispatch.hpp", "step_f32_2d.hip"],
    "c3": _COMMON + ["step2d.hpp", "step3d.hpp", "step_dispatch.hpp", "step_f32_3d.hip"],
    "c4": _COMMON + ["step2d.hpp", "batch2d.hpp", "batch_f32.hip"],
    "at_f64": ["mp_internal.hpp", "antitrap2d.hpp", "antitrap.hip"],
    "at_f32": ["mp_internal.hpp", "antitrap2d.hpp", "antitrap.hip"],
    "at3d_f32": ["mp_internal.hpp", "antitrap2d.hpp", "antitrap.hip"],
}
# The 3D correction kernel's fixed block shape (x cells, y rows, cells per lane).
AT3D_TILE = [64, 4, 1]
# The correction kernel's fixed strip shape (columns written per wave, rows per wave, cells per lane).
AT_TILE = [62, 12, 1]


def source_hash(leg):
    """sha256 (16 hex digits) over the device sources of one leg's kernel."""
    h = hashlib.sha256()
    for name in LEG_SOURCES[leg]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_of(leg, tile, fuse):
    t = TRAFFIC.get(leg)
    if not t or list(t["tile"]) != list(tile) or t["fuse"] != fuse or t["src"] != source_hash(leg):
        return None
    return t["bytes"]


def roofline(bytes_per_step, ms_step, traffic=None):
    """Algorithmic bytes per launch / launch time (= per step / step time, whatever the
    steps per launch); traffic = counter HBM bytes per launch."""
    gbs = bytes_per_step / (ms_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic)}


def flops_per_cell_update(nphases, ncomp, dim=2, aniso=False):
    """Floating-point operations (an FMA counts 2) of one cell update of the
    multi-well step as the kernels evaluate it, each face once: the cell
    record (h, mobility), one face per axis, the face sums, h of the old phi,
    and the cell update (doubled psi, driving force, Lagrange multiplier, new
    phi and its h, mu with its reciprocal and two Newton steps).  An
    anisotropic pair adds the tangential differences and q components and the
    normal component of d(a_c^2 |q|^2)/dq (one reciprocal square root)."""
    n, m, d = nphases, ncomp - 1, dim
    pairs = n * (n - 1) // 2
    h = 5 * n + 3 if n == 3 else 4 * n
    record = h + m * (2 * n - 1)
    if aniso:
        t = d - 1  # tangential axes
        # per face: sigma sums (n), tangential sums of the two cells' central
        # differences (3 per phase and axis); per pair: q_n (4), q_t (4 per
        # axis), |q|^2 (1 + 2t), rsqrt and the normalised components (5 + 4t),
        # a_c (4), G_n (11), its small-|q| limit (5), the pair factor (1) and
        # the U/W updates (8)
        face = n + 3 * n * t + pairs * (4 + 4 * t + (1 + 2 * t) + (5 + 4 * t) + 4 + 11 + 5 + 1 + 8) + 3 * m
        faces = d * face
    else:
        faces = d * (12 * pairs + 3 * m)
    sums = (n + m) * (2 * d - 1)
    cell = (4 * n * m + (6 if n == 3 else 0)
            + n * (2 * n + 6 if n == 3 else 2 * n + 4)
            + n + 3 * n + h + n + m * (4 * n + 10))
    return record + faces + sums + h + cell


def alu_roofline(flops_per_step, ms_step, precision, traffic=None):
    """Algorithmic flops per launch / launch time against the vector ALU peak."""
    tf = flops_per_step / (ms_step * 1e-3) / 1e12
    peak = ALU_PEAK_TFLOPS[precision]
    return {"bound": "alu", "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(tf / peak, 4), "traffic": None if traffic is None else round(traffic)}


def parse_tile(text):
    return [int(v) for v in text.split(",")] if text else None


class Timer:
    """HIP events on torch's current stream, the stream every library call here runs on."""

    def __init__(self):
        import torch

        self.torch = torch
        self.stream = torch.cuda.current_stream()
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.e0.record(self.stream)
        return self

    def __exit__(self, *exc):
        self.e1.record(self.stream)
        self.torch.cuda.synchronize()
        self.ms = self.e0.elapsed_time(self.e1)


def copy_bandwidth(n, reps=10):
    """Read + write GB/s of a plain device copy of one FP64 C2-sized state buffer:
    the practical HBM ceiling, a second denominator beside the 8 TB/s peak."""
    import torch

    nbytes = 5 * n * n * 8
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    with Timer() as t:
        for _ in range(reps):
            dst.copy_(src)
    gbs = 2 * nbytes / (t.ms / reps * 1e-3) / 1e9
    del src, dst
    return {"achieved": round(gbs, 1), "unit": "GB/s", "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_each_way": nbytes}


def copy_calibration(n, steps):
    """Plain device-to-device copy of one FP64 C2-sized state buffer (5 fields x n x n):
    the practical HBM ceiling, and the known-size reference for traffic counters."""
    import torch

    nbytes = 5 * n * n * 8
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    with Timer() as t:
        for _ in range(steps):
            dst.copy_(src)
    ms = t.ms / steps
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"copy_bytes_each_way": nbytes, "ms_per_copy": ms, "GBs_read_plus_write": gbs,
                      "frac_of_8TBs": gbs / HBM_PEAK_GBS}), flush=True)


def leg_c2(precision, n, steps, warmup, tile, tune):
    from paper_2404_01035_amd import abi, inputs
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c2(precision=precision, n=(n, n, 1))
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    if tile:
        s.set_tile(*tile)
        source = "fixed"
    elif tune:
        s.autotune(reps=10, force=True)
        source = "tuned"
    else:
        source = "default"
    used = list(abi.mp_get_tile(s.st))
    fuse = abi.mp_get_fusion(s.st)
    s.step(warmup)
    with Timer() as t:
        s.step(steps)
    d = s.diagnostics()
    s.close()
    elem = 8 if precision == "f64" else 4
    bpc = p.nfields * 2 * elem  # read + write of every field once
    fpc = flops_per_cell_update(p.nphases, p.ncomp)
    ms_step = t.ms / steps
    traffic = traffic_of(f"c2_{precision}", used, fuse)
    return {
        "value": p.ncells * steps / (t.ms * 1e-3),
        "ms_per_step": ms_step,
        # two steps per launch from registers: the vector ALU, not HBM, bounds it
        "roofline": alu_roofline(p.ncells * fpc, ms_step, precision, traffic),
        "hbm_equivalent": roofline(p.ncells * bpc, ms_step, traffic),
        "flops_per_cell_update": fpc,
        "bytes_per_cell_update": bpc,
        "steps_per_launch": fuse,
        "algorithmic_bytes_per_launch": fuse * p.ncells * bpc,
        "tile": {"bx": used[0], "seg": used[1], "vec": used[2], "source": source},
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
    }


def leg_at3d(n, steps, warmup):
    """The 3D dendrite (FP32) with the anti-trapping current: one 3D step launch and
    the 3D correction kernel per step, against the same run without the current."""
    from paper_2404_01035_amd.solver import Solver
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c3(n=(n, n, n))
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    s.step(warmup)
    with Timer() as t0:
        s.step(steps)
    s.set_antitrapping(True)
    s.step(warmup)
    with Timer() as t1:
        s.step(steps)
    d = s.diagnostics()
    s.close()
    bpc = (2 * p.nphases + 3 * (p.ncomp - 1)) * 4
    ms_plain, ms_at = t0.ms / steps, t1.ms / steps
    ms_corr = ms_at - ms_plain
    return {
        "value": p.ncells * steps / (t1.ms * 1e-3),
        "unit": "cell-updates/s",
        "ms_per_step": ms_at,
        "ms_per_step_without_current": ms_plain,
        "correction_ms_per_step": ms_corr,
        "correction_bytes_per_cell": bpc,
        "roofline": roofline(p.ncells * bpc, ms_corr, traffic_of("at3d_f32", AT3D_TILE, 1))
        if ms_corr > 0 else None,
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
    }


def leg_at(precision, n, steps, warmup):
    """The C2 step with the anti-trapping current: one step per launch followed by the
    correction kernel.  The same run without the current (one step per launch) is
    timed first; the difference is the correction kernel's time per step."""
    from paper_2404_01035_amd.solver import Solver
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c2(precision=precision, n=(n, n, 1))
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    s.set_fusion(1)
    s.step(warmup)
    with Timer() as t0:
        s.step(steps)
    s.set_antitrapping(True)
    s.step(warmup)
    with Timer() as t1:
        s.step(steps)
    d = s.diagnostics()
    s.close()
    elem = 8 if precision == "f64" else 4
    nm = p.ncomp - 1
    # phi^n, phi^{n+1}, mu^n and mu^{n+1} read, mu^{n+1} written, once per cell
    bpc = (2 * p.nphases + 3 * nm) * elem
    ms_plain, ms_at = t0.ms / steps, t1.ms / steps
    ms_corr = ms_at - ms_plain
    return {
        "value": p.ncells * steps / (t1.ms * 1e-3),
        "unit": "cell-updates/s",
        "ms_per_step": ms_at,
        "ms_per_step_without_current": ms_plain,
        "correction_ms_per_step": ms_corr,
        "correction_bytes_per_cell": bpc,
        # the correction kernel: time = step with the current - step without
        "roofline": roofline(p.ncells * bpc, ms_corr, traffic_of(f"at_{precision}", AT_TILE, 1))
        if ms_corr > 0 else None,
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
    }


def leg_c3(n, steps, warmup, tile, tune):
    from paper_2404_01035_amd import abi, inputs
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu = inputs.config_c3(n=(n, n, n))
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    if tile:
        s.set_tile(*tile)
    elif tune:
        s.autotune(reps=5, force=True)
    used = list(abi.mp_get_tile(s.st))
    s.step(warmup)
    with Timer() as t:
        s.step(steps)
    d = s.diagnostics()
    s.close()
    bpc = p.nfields * 2 * 4
    fpc = flops_per_cell_update(p.nphases, p.ncomp, dim=3, aniso=True)
    ms_step = t.ms / steps
    return {
        "workload": f"3D {n}^3 binary dendrite, cubic anisotropy delta=0.02, no-flux, FP32",
        "value": p.ncells * steps / (t.ms * 1e-3),
        "unit": "cell-updates/s",
        "steps": steps,
        "ms_per_step": ms_step,
        "roofline": roofline(p.ncells * bpc, ms_step, traffic_of("c3", used, 1)),
        # the flop side of the same kernel (neither side is saturated: LDS and
        # latency bound)
        "alu": alu_roofline(p.ncells * fpc, ms_step, "f32"),
        "flops_per_cell_update": fpc,
        "bytes_per_cell_update": bpc,
        "steps_per_launch": 1,
        "algorithmic_bytes_per_launch": p.ncells * bpc,
        "tile": {"bx": used[0], "seg": used[1], "vec": used[2]},
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
    }


def leg_c4(steps, warmup, tile, tune, graph_chunk=50):
    from paper_2404_01035_amd import abi, inputs
    from paper_2404_01035_amd.solver import BatchSolver

    members = inputs.config_c4()
    b = BatchSolver([m[0] for m in members])
    for i, (_, phi, mu) in enumerate(members):
        b.load(i, phi, mu)
    b.start(0)
    cells = sum(m[0].ncells for m in members)
    bytes_step = sum(m[0].ncells * m[0].nfields * 2 * 4 for m in members)
    flops_step = sum(m[0].ncells * flops_per_cell_update(m[0].nphases, m[0].ncomp) for m in members)
    del members
    if tile:
        b.set_tile(*tile)
    elif tune:
        b.autotune(reps=5, force=True)
    used = list(abi.mp_get_tile(b.st))
    fuse = abi.mp_get_fusion(b.st)
    b.set_graph(graph_chunk)
    b.step(warmup)
    with Timer() as t:
        b.step(steps)
    diags = b.diagnostics()
    b.close()
    ms_step = t.ms / steps
    return {
        "workload": "256 independent 2D instances, sides U{64..1024}, N in {2,3}, 1-2 mu fields, "
                    f"periodic, FP32, one persistent launch per {fuse} step(s), HIP graphs of "
                    f"{graph_chunk} steps",
        "value": cells * steps / (t.ms * 1e-3),
        "unit": "cell-updates/s",
        "steps": steps,
        "cells": cells,
        "ms_per_step": ms_step,
        "roofline": alu_roofline(flops_step, ms_step, "f32", traffic_of("c4", used, fuse)),
        "hbm_equivalent": roofline(bytes_step, ms_step, traffic_of("c4", used, fuse)),
        "steps_per_launch": fuse,
        "algorithmic_bytes_per_launch": fuse * bytes_step,
        "tile": {"seg": used[1], "vec": used[2]},
        "nonfinite_instances": sum(1 for d in diags if d["nonfinite"]),
    }


def leg_c5(nsteps, every=100, n=512):
    """Checkpointed forward run and adjoint sweep at nominal theta; loss = 1/2 |phi^N - phi*|^2."""
    import numpy as np
    import torch

    from paper_2404_01035_amd import inputs
    from paper_2404_01035_amd.solver import Solver

    p, phi, mu, theta_star = inputs.config_c5(n=n)
    # target from the hidden parameters (untimed)
    s = Solver(inputs.theta_into(p, theta_star))
    s.load(phi, mu)
    s.step(nsteps)
    target = s.current()[: p.nphases].clone()
    s.close()

    s = Solver(p)
    s.load(phi, mu)
    tuned = s.autotune(reps=10, force=True)  # a small grid: the tiles differ from 4096^2's
    ckpt = s.checkpoint_buffer(nsteps, every)
    s.step_ckpt(2, 1, s.checkpoint_buffer(2, 1))  # warm the kernels
    s.load(phi, mu)
    with Timer() as tf:
        s.step_ckpt(nsteps, every, ckpt)
    lam = torch.zeros_like(s.current())
    lam[: p.nphases] = s.current()[: p.nphases] - target
    loss = 0.5 * float((lam[: p.nphases].double() ** 2).sum())
    s.adjoint(lam, ckpt, 2 * every, every, 0)  # warm
    with Timer() as ta:
        _, g = s.adjoint(lam, ckpt, nsteps, every, 0)
    s.close()
    grads = [g["gamma01"], g["gamma02"], g["gamma12"], g["D20"], g["D21"], g["tau"]]
    return {
        "workload": f"2D {n}x{n}, 3 phases, ternary, periodic, FP32 forward + FP32 adjoint, "
                    f"{nsteps} steps, checkpoints every {every}",
        "tile": {k: tuned[k] for k in ("bx", "seg", "vec", "fuse")},
        "forward_ms": tf.ms,
        "adjoint_ms": ta.ms,
        "adjoint_over_forward": ta.ms / tf.ms,
        "forward_cell_updates_per_s": p.ncells * nsteps / (tf.ms * 1e-3),
        "loss": loss,
        "grad_theta": dict(zip(["gamma01", "gamma02", "gamma12", "Dliq1", "Dliq2", "tau"],
                               [float(v) for v in grads])),
        "theta_star": [float(v) for v in np.asarray(theta_star)],
    }


def cpu_baseline(n, nsteps=2):
    """The FP64 oracle (numpy: elementwise array passes, one thread) on ``nsteps``
    full-grid steps of the headline workload."""
    from oracle import gp
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c2(precision="f64", n=(n, n, 1))
    t0 = time.perf_counter()
    gp.run(phi, mu, 0, nsteps, p)
    dt = time.perf_counter() - t0
    return {
        "value": p.ncells * nsteps / dt,
        "unit": "cell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nsteps} steps of the full {n}x{n} grid, FP64 numpy oracle ({dt:.1f} s)",
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
    legs = [x for x in a.legs.split(",") if x]
    log(f"FP64 {a.n}x{a.n}: warmup {a.warmup}, timed {a.steps} steps")
    r64 = leg_c2("f64", a.n, a.steps, a.warmup, parse_tile(a.tile), a.tune)
    out = {
        "metric": METRIC,
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
        "hbm_equivalent": r64["hbm_equivalent"],
        "flops_per_cell_update": r64["flops_per_cell_update"],
        "steps_per_launch": r64["steps_per_launch"],
        "algorithmic_bytes_per_launch": r64["algorithmic_bytes_per_launch"],
        "tile": r64["tile"],
        "diag": r64["diag"],
        "cpu_baseline": None,
    }
    if "c2" in legs:
        log(f"FP32 {a.n}x{a.n}")
        r32 = leg_c2("f32", a.n, a.steps, a.warmup, parse_tile(a.tile32), a.tune)
        out["fp32"] = dict(r32, dtype="f32 (FP64 Lagrange multiplier and reductions)")
        out["speedup_fp32_over_fp64"] = r32["value"] / r64["value"]
    if "c3" in legs:
        log(f"3D {a.n3d}^3 FP32")
        out["dendrite_3d"] = leg_c3(a.n3d, a.steps3d, 5, parse_tile(a.tile3d), a.tune)
    if "c4" in legs:
        log("batched ensemble FP32")
        out["batched"] = leg_c4(a.batch_steps, 50, parse_tile(a.tile_batch), a.tune)
    if "c5" in legs:
        log("checkpointed forward + adjoint FP32")
        out["adjoint"] = leg_c5(a.adjoint_steps)
    if "at" in legs:
        at_steps = min(a.steps, 200)
        log(f"anti-trapping current {a.n}x{a.n}, FP64 and FP32, {at_steps} steps")
        out["antitrapping"] = {"workload": f"2D {a.n}x{a.n} directional eutectic with the anti-trapping "
                                           "current, one step per launch + correction",
                               "f64": leg_at("f64", a.n, at_steps, 5),
                               "f32": leg_at("f32", a.n, at_steps, 5),
                               "dendrite_3d_f32": dict(leg_at3d(a.n3d, min(a.steps3d, 50), 3),
                                                       workload=f"3D {a.n3d}^3 binary dendrite with the current")}
    out["copy_bandwidth"] = copy_bandwidth(a.n)
    if not a.no_cpu:
        log("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(a.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
