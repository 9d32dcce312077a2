"""Benchmark of the fused phi + mu step on one MI355X.

Headline workload: 2D 4096 x 4096 directional eutectic (3 phases, ternary: 2 mu
fields), x periodic / y no-flux, seeded synthetic initial state (lamellae slab
in melt).  A benchmark step is one forward-Euler time step of the whole field
(the fused phi + mu update); the 2D kernels perform two steps per launch, so
the state crosses HBM once per two steps (bitwise the same result as single
steps).  Each leg is timed as the median of five regions of exactly --steps
steps, after --warmup steps and untimed steps until 150 ms have passed, with
the state resident in HBM: FP64 (``value``) and FP32 (``fp32``), at the
library's default tiles (the autotuner's picks for this workload; --tune
re-tunes).  ``roofline`` takes the bound by the max(bytes / bandwidth,
flops / peak) rule over the algorithmic bytes (one read and one write of the
state per step) and flops, and carries the HBM fraction of the real (counter)
traffic and the vector-ALU issue fraction beside it.

Further legs, each a block of the same JSON line:
  dendrite_3d  3D 512^3 binary dendrite with cubic anisotropy, FP32
  batched      256 uneven 2D instances in one persistent launch per two
               steps, replayed as HIP graphs, FP32
  adjoint      512^2 three-phase ternary run, FP32: checkpointed forward run
               (every 100 steps) and the adjoint sweep; their cost ratio
  antitrapping the 4096^2 eutectic with the anti-trapping current formed
               inside the step kernel (and, beside it, the step followed by
               the separate correction kernel), and the 512^3 dendrite with
               the 3D correction kernel after each step
  extended     the 4096^2 eutectic with temperature-dependent coefficients
               (the general kernels), FP64 and FP32
cpu_baseline   the FP64 oracle on the full 4096^2 grid, on the host's cores: two
               steps split into row bands over the usable CPUs (at most 16),
               and one step in a single process; lscpu's model and counts.

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
    "c2_f64": {"tile": [256, 31, 1], "fuse": 2, "src": "4a474857c5ff4d5f",
               "bytes": (2.0 * 369660.8 + 667176.8) * 1024},
    "c2_f32": {"tile": [256, 14, 1], "fuse": 2, "src": "5d7d2c7608a102ff",
               "bytes": (2.0 * 190450.6 + 337887.8) * 1024},
    # profiles/k_step2d_x2_gen_eutectic_4096_f64_f32.md
    "c2ext_f64": {"tile": [256, 31, 1], "fuse": 2, "src": "74a41cb44a9264f6",
                  "bytes": (2.0 * 384876.0 + 656564.4) * 1024},
    "c2ext_f32": {"tile": [256, 14, 1], "fuse": 2, "src": "dedc49bcd4c6aefc",
                  "bytes": (2.0 * 224329.2 + 329085.2) * 1024},
    # profiles/k_step3d_dendrite_512_f32.md
    "c3": {"tile": [512, 64, -1], "fuse": 1, "src": "cd5215f0b01a0136",
           "bytes": (2.0 * 1151502.1 + 1572864.0) * 1024},
    # profiles/k_step2d_at_eutectic_4096_f64_f32.md
    "atf_f64": {"tile": [256, 31, 1], "fuse": 1, "src": "a1969566f127ef6b",
                "bytes": (2.0 * 416826.7 + 659186.5) * 1024},
    "atf_f32": {"tile": [256, 14, 1], "fuse": 1, "src": "a1969566f127ef6b",
                "bytes": (2.0 * 247552.7 + 331791.2) * 1024},
    # profiles/k_antitrap2d_eutectic_4096_f64_f32.md
    "at_f64": {"tile": [62, 12, 1], "fuse": 1, "src": "2bbd3f220a9e5ebc",
               "bytes": (2.0 * 870583.4 + 270298.6) * 1024},
    "at_f32": {"tile": [62, 12, 1], "fuse": 1, "src": "2bbd3f220a9e5ebc",
               "bytes": (2.0 * 462431.8 + 140617.0) * 1024},
    # profiles/k_antitrap3d_dendrite_512_f32.md
    "at3d_f32": {"tile": [62, 2, 1], "fuse": 1, "src": "827edfbe96172ad2",
                 "bytes": (2.0 * 2125895.1 + 581596.0) * 1024},
    # profiles/k_batch2d_ensemble_256_f32.md
    "c4": {"tile": [256, 32, 1], "fuse": 2, "src": "4a2ddb4fb8f20f42",
           "bytes": (2.0 * 706252.1 + 1235989.5) * 1024},
}
METRIC = "cell-updates/s of fused phi+mu step (FP64 vs FP32), % HBM peak, adjoint/fwd cost"
ALL_LEGS = ("c2", "c3", "c4", "c5", "at", "ext", "kks")


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
    ap.add_argument("--settle-ms", type=float, default=None,
                    help="untimed settle time before the timed regions (default 150 ms; 0 for counter runs)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only the host-CPU oracle timing (prints its record; no GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of one FP64 state buffer instead")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The device sources each leg's step kernel is built from.
_COMMON = ["mp_internal.hpp", "gp_device.hpp"]
LEG_SOURCES = {
    "c2_f64": _COMMON + ["diag_cell.hpp", "step2d.hpp", "step_dispatch.hpp", "step_f64_2d.hip"],
    "c2_f32": _COMMON + ["diag_cell.hpp", "step2d.hpp", "step_dispatch.hpp", "step_f32_2d.hip"],
    "c2ext_f64": _COMMON + ["diag_cell.hpp", "step2d.hpp", "step_dispatch.hpp", "step_gen_f64_2d.hip"],
    "c2ext_f32": _COMMON + ["diag_cell.hpp", "step2d.hpp", "step_dispatch.hpp", "step_gen_f32_2d.hip"],
    "c3": _COMMON + ["diag_cell.hpp", "step3d.hpp", "step_dispatch.hpp", "step_f32_3d.hip"],
    "c4": _COMMON + ["diag_cell.hpp", "step2d.hpp", "batch2d.hpp", "batch_f32.hip"],
    "at_f64": _COMMON + ["antitrap2d.hpp", "antitrap.hip"],
    "at_f32": _COMMON + ["antitrap2d.hpp", "antitrap.hip"],
    "at3d_f32": _COMMON + ["antitrap2d.hpp", "antitrap3d.hpp", "antitrap.hip"],
    "atf_f64": _COMMON + ["diag_cell.hpp", "step2d.hpp", "antitrap2d.hpp", "step2d_at.hpp", "step_at.hip"],
    "atf_f32": _COMMON + ["diag_cell.hpp", "step2d.hpp", "antitrap2d.hpp", "step2d_at.hpp", "step_at.hip"],
}
# The 3D correction kernel's FP32 strip shape (columns written per wave, rows per wave, cells per lane).
AT3D_TILE = [62, 2, 1]
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


def flops_per_cell_update(nphases, ncomp, dim=2, aniso=False, ext=False, well1=False):
    """Floating-point operations (an FMA counts 2) of one cell update of the
    multi-well step as the kernels evaluate it, each face once: the cell
    record (h, mobility), one face per axis, the face sums, h of the old phi,
    and the cell update (doubled psi, driving force, Lagrange multiplier, new
    phi and its h, mu with its reciprocal and two Newton steps).  An
    anisotropic pair adds the tangential differences and q components and the
    normal component of d(a_c^2 |q|^2)/dq (one reciprocal square root).  The
    extended model's general cell (ext) adds B(T) and the quadratic C(T), the
    dT/dt term, for two mu fields the off-diagonal susceptibility terms, the
    mobility matrix with its face products and the 2 x 2 solve, and tau(phi).
    The KKS potential of Eq. Well1 (well1, general cell) adds per phase
    2 Theta_a (1 - phi_a)(1 - 2 phi_a) (6) and, for N = 3, 2 Theta_abd phi_b^2 phi_d^2 (3)."""
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
    extra = 0
    if ext:
        extra = 3 * n * m + 2 * n + 2 * n * m + 14  # B(T), C(T)^2 term, Theta, tau(phi)
        if m == 2:
            extra += 4 * n + 6 * d + 2 * (2 * n - 1) + 4  # cross chi, face J products, M matrix, solve
    if well1:
        extra += n * (6 + (3 if n == 3 else 0))
    return record + faces + sums + h + cell + extra


def alu_roofline(flops_per_step, ms_step, precision, traffic=None):
    """Algorithmic flops per launch / launch time against the vector ALU peak."""
    tf = flops_per_step / (ms_step * 1e-3) / 1e12
    peak = ALU_PEAK_TFLOPS[precision]
    return {"bound": "alu", "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(tf / peak, 4), "traffic": None if traffic is None else round(traffic)}


# Vector-ALU issue of each leg's step kernel, from rocprofv3 SQ counter runs:
# VALU instructions per launch (SQ_INSTS_VALU summed over the launch's waves),
# keyed like TRAFFIC (tile, steps per launch, source hash).  A wave64 FP64
# instruction occupies its SIMD for 4 cycles, an FP32 one for 2 (the vector
# peaks above: 16 FP64 or 32 FP32 lanes per SIMD per cycle).
VALU = {
    # profiles/k_step2d_eutectic_4096_f64_f32.md
    "c2_f64": {"tile": [256, 31, 1], "fuse": 2, "src": "4a474857c5ff4d5f", "insts": 153843513.0},
    "c2_f32": {"tile": [256, 14, 1], "fuse": 2, "src": "5d7d2c7608a102ff", "insts": 138091296.0},
    # profiles/k_step2d_x2_gen_eutectic_4096_f64_f32.md
    "c2ext_f64": {"tile": [256, 31, 1], "fuse": 2, "src": "74a41cb44a9264f6", "insts": 229763385.0},
    "c2ext_f32": {"tile": [256, 14, 1], "fuse": 2, "src": "dedc49bcd4c6aefc", "insts": 176406168.0},
    # profiles/k_step3d_dendrite_512_f32.md
    "c3": {"tile": [512, 64, -1], "fuse": 1, "src": "cd5215f0b01a0136", "insts": 545827325.3},
    # profiles/k_step2d_at_eutectic_4096_f64_f32.md
    "atf_f64": {"tile": [256, 31, 1], "fuse": 1, "src": "a1969566f127ef6b", "insts": 203122347.0},
    "atf_f32": {"tile": [256, 14, 1], "fuse": 1, "src": "a1969566f127ef6b", "insts": 145416750.0},
    # profiles/k_antitrap2d_eutectic_4096_f64_f32.md
    "at_f64": {"tile": [62, 12, 1], "fuse": 1, "src": "2bbd3f220a9e5ebc", "insts": 106811674.0},
    "at_f32": {"tile": [62, 12, 1], "fuse": 1, "src": "2bbd3f220a9e5ebc", "insts": 78199324.0},
    # profiles/k_antitrap3d_dendrite_512_f32.md
    "at3d_f32": {"tile": [62, 2, 1], "fuse": 1, "src": "827edfbe96172ad2", "insts": 654686208.0},
    # profiles/k_batch2d_ensemble_256_f32.md
    "c4": {"tile": [256, 32, 1], "fuse": 2, "src": "4a2ddb4fb8f20f42", "insts": 468028690.0},
}
VALU_CYCLES = {"f64": 4, "f32": 2}
SIMDS = 1024         # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9     # MI355X peak engine clock


def valu_of(leg, tile, fuse):
    t = VALU.get(leg)
    if not t or list(t["tile"]) != list(tile) or t["fuse"] != fuse or t["src"] != source_hash(leg):
        return None
    return t["insts"]


def bound_record(bytes_per_step, flops_per_step, ms_step, precision, traffic=None, valu_insts=None,
                 steps_per_launch=1):
    """Roofline of a step kernel by the max(bytes / bandwidth, flops / peak) rule:
    the side whose ideal time is the larger bounds it, and ``roofline``/
    ``alu_roofline`` of that side is returned.  Beside it: ``ideal_ms`` of both
    sides; ``counter_frac``, the HBM rate of the real (counter) traffic against
    the peak, and ``valu_issue_frac``, the share of the launch time the VALU
    instructions occupy their SIMDs -- both null without a counter figure for
    this exact kernel and tile.  Two-step kernels read and write the state once
    per two steps, so their algorithmic-bytes rate (one read and one write per
    step) can exceed the HBM peak; the counter and issue fractions are then
    the limits that bind."""
    t_hbm = bytes_per_step / (HBM_PEAK_GBS * 1e9) * 1e3
    t_alu = flops_per_step / (ALU_PEAK_TFLOPS[precision] * 1e12) * 1e3
    if t_hbm >= t_alu:
        rec = roofline(bytes_per_step, ms_step, traffic)
    else:
        rec = alu_roofline(flops_per_step, ms_step, precision, traffic)
    rec["ideal_ms_per_step"] = {"hbm": round(t_hbm, 6), "alu": round(t_alu, 6)}
    return with_counter_fracs(rec, ms_step * steps_per_launch, precision, traffic, valu_insts)


def with_counter_fracs(rec, ms_launch, precision, traffic=None, valu_insts=None):
    """rec plus ``counter_frac`` (counter traffic per launch / launch time / HBM peak) and
    ``valu_issue_frac`` (VALU instructions x cycles each / SIMDs / clock / launch time),
    each null without a counter figure for this exact kernel and tile."""
    rec["counter_frac"] = None if traffic is None else round(traffic / (ms_launch * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
    rec["valu_issue_frac"] = None if valu_insts is None else round(
        valu_insts * VALU_CYCLES[precision] / SIMDS / CLOCK_HZ / (ms_launch * 1e-3), 4)
    return rec


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


REGIONS = 5          # timed regions per leg; the median is reported
SETTLE_MS = 150.0    # untimed steps after the warm-up until this much wall time has passed


def measure(step, steps, warmup, regions=REGIONS, settle_ms=None):
    """Time ``step(steps)``: ``warmup`` untimed steps, then untimed steps in
    chunks of ``steps`` until ``settle_ms`` of wall time has passed (clocks and
    caches settle; short runs such as 20 steps otherwise time a cold GPU), then
    ``regions`` regions of exactly ``steps`` steps, each bracketed by a device
    synchronisation and HIP events on the stream the kernels run on.  Returns
    the median region's milliseconds, every region's, and the settle steps."""
    import torch

    if settle_ms is None:
        settle_ms = SETTLE_MS
    if warmup > 0:
        step(warmup)
    torch.cuda.synchronize()
    settle = 0
    t0 = time.perf_counter()
    while steps > 0 and (time.perf_counter() - t0) * 1e3 < settle_ms and settle < 50 * max(steps, 1):
        step(steps)
        torch.cuda.synchronize()
        settle += steps
    ms = []
    for _ in range(regions):
        with Timer() as t:
            step(steps)
        ms.append(t.ms)
    return sorted(ms)[len(ms) // 2], ms, settle


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


def diag_timing(s, fuse, reps=REGIONS):
    """One launch of ``fuse`` steps followed by the diagnostics of the state
    reached: the separate reduction pass (mp_step + mp_diagnostics) against the
    partial sums formed inside the step launch (mp_step_diag).  Both end in the
    same host synchronisation and copy; median of ``reps`` event-timed calls."""
    def separate():
        s.step(fuse)
        s.diagnostics()

    def fused():
        s.step_diag(fuse)

    out = {"steps": fuse}
    for name, fn in (("separate_ms", separate), ("fused_ms", fused)):
        fn()
        ms = []
        for _ in range(reps):
            with Timer() as t:
                fn()
            ms.append(t.ms)
        out[name] = round(sorted(ms)[reps // 2], 4)
    return out


def leg_c2(precision, n, steps, warmup, tile, tune, slopes=False, kks=None):
    """The 4096^2 eutectic; slopes: with temperature-dependent coefficients
    (the general kernels of the extended model); kks: the KKS variant with the
    potential of Eq. Well's form ("well", the plain kernels) or Eq. Well1
    ("theta", the general kernels)."""
    from paper_2404_01035_amd import abi, inputs
    from paper_2404_01035_amd.solver import Solver

    cfg = inputs.config_c2_slopes if slopes else inputs.config_c2
    p, phi, mu = cfg(precision=precision, n=(n, n, 1))
    if kks:
        p = inputs.kks_from(p, potential=kks, theta=[0.3, 0.2, 0.4] if kks == "theta" else None,
                            theta3=0.6 if kks == "theta" else 0.0)
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
    ms, regions, settle = measure(s.step, steps, warmup)
    d = s.diagnostics()
    dt = None if (slopes or kks) else diag_timing(s, fuse)
    s.close()
    elem = 8 if precision == "f64" else 4
    bpc = p.nfields * 2 * elem  # read + write of every field once
    fpc = flops_per_cell_update(p.nphases, p.ncomp, ext=slopes or kks == "theta", well1=kks == "theta")
    ms_step = ms / steps
    leg = f"c2{'ext' if slopes else ''}{'kks' + kks if kks else ''}_{precision}"
    traffic = traffic_of(leg, used, fuse)
    return {
        "value": p.ncells * steps / (ms * 1e-3),
        "ms_per_step": ms_step,
        "region_ms": [round(x, 4) for x in regions],
        "settle_steps": settle,
        "roofline": bound_record(p.ncells * bpc, p.ncells * fpc, ms_step, precision, traffic,
                                 valu_of(leg, used, fuse), fuse),
        "alu": alu_roofline(p.ncells * fpc, ms_step, precision),
        "flops_per_cell_update": fpc,
        "bytes_per_cell_update": bpc,
        "steps_per_launch": fuse,
        "algorithmic_bytes_per_launch": fuse * p.ncells * bpc,
        "tile": {"bx": used[0], "seg": used[1], "vec": used[2], "source": source},
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
        **({"diag_timing": dt} if dt else {}),
    }


def leg_at3d(n, steps, warmup):
    """The 3D dendrite (FP32) with the anti-trapping current: one 3D step launch and
    the 3D correction kernel per step, against the same run without the current
    (median regions of each; their difference is the correction kernel's time)."""
    from paper_2404_01035_amd.solver import Solver
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c3(n=(n, n, n))
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    ms0, _, _ = measure(s.step, steps, warmup)
    s.set_antitrapping(True)
    ms1, regions, _ = measure(s.step, steps, warmup)
    d = s.diagnostics()
    s.close()
    bpc = (2 * p.nphases + 3 * (p.ncomp - 1)) * 4
    ms_plain, ms_at = ms0 / steps, ms1 / steps
    ms_corr = ms_at - ms_plain
    return {
        "value": p.ncells * steps / (ms1 * 1e-3),
        "unit": "cell-updates/s",
        "ms_per_step": ms_at,
        "region_ms": [round(x, 4) for x in regions],
        "ms_per_step_without_current": ms_plain,
        "correction_ms_per_step": ms_corr,
        "correction_bytes_per_cell": bpc,
        "roofline": with_counter_fracs(roofline(p.ncells * bpc, ms_corr, traffic_of("at3d_f32", AT3D_TILE, 1)),
                                       ms_corr, "f32", traffic_of("at3d_f32", AT3D_TILE, 1),
                                       valu_of("at3d_f32", AT3D_TILE, 1))
        if ms_corr > 0 else None,
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
    }


def leg_at(precision, n, steps, warmup):
    """The C2 step with the anti-trapping current, one step per launch: the current
    formed inside the step kernel (the leg's rate), and the step followed by the
    separate correction kernel.  The same run without the current (one step per
    launch) is timed first; the difference of the separate path's and the plain
    step's median regions is the correction kernel's time per step."""
    from paper_2404_01035_amd import abi
    from paper_2404_01035_amd.solver import Solver
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c2(precision=precision, n=(n, n, 1))
    s = Solver(p)
    s.load(phi, mu)
    del phi, mu
    s.set_fusion(1)
    ms0, _, _ = measure(s.step, steps, warmup)
    s.set_antitrapping(2)
    ms2, regions2, _ = measure(s.step, steps, warmup)
    s.set_antitrapping(1)
    ms1, regions, _ = measure(s.step, steps, warmup)
    bx, seg, _ = abi.mp_get_tile(s.st)
    d = s.diagnostics()
    s.close()
    elem = 8 if precision == "f64" else 4
    nm = p.ncomp - 1
    # folded: the state read and written once per cell
    bpc = 2 * (p.nphases + nm) * elem
    # correction kernel: phi^n, phi^{n+1}, mu^n and mu^{n+1} read, mu^{n+1} written, once per cell
    bpc_corr = (2 * p.nphases + 3 * nm) * elem
    ms_plain, ms_at, ms_sep = ms0 / steps, ms1 / steps, ms2 / steps
    ms_corr = ms_sep - ms_plain
    tile = [bx, seg, 1]
    return {
        "value": p.ncells * steps / (ms1 * 1e-3),
        "unit": "cell-updates/s",
        "ms_per_step": ms_at,
        "region_ms": [round(x, 4) for x in regions],
        "bytes_per_cell_update": bpc,
        "tile": {"bx": bx, "seg": seg, "vec": 1},
        "roofline": with_counter_fracs(roofline(p.ncells * bpc, ms_at, traffic_of(f"atf_{precision}", tile, 1)),
                                       ms_at, precision, traffic_of(f"atf_{precision}", tile, 1),
                                       valu_of(f"atf_{precision}", tile, 1)),
        "ms_per_step_without_current": ms_plain,
        "separate_correction": {
            "ms_per_step": ms_sep,
            "region_ms": [round(x, 4) for x in regions2],
            "correction_ms_per_step": ms_corr,
            "correction_bytes_per_cell": bpc_corr,
            # the correction kernel: time = step then correction - step without the current
            "roofline": with_counter_fracs(
                roofline(p.ncells * bpc_corr, ms_corr, traffic_of(f"at_{precision}", AT_TILE, 1)), ms_corr,
                precision, traffic_of(f"at_{precision}", AT_TILE, 1), valu_of(f"at_{precision}", AT_TILE, 1))
            if ms_corr > 0 else None,
        },
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
    ms, regions, settle = measure(s.step, steps, warmup)
    d = s.diagnostics()
    dt = diag_timing(s, 1)
    s.close()
    bpc = p.nfields * 2 * 4
    fpc = flops_per_cell_update(p.nphases, p.ncomp, dim=3, aniso=True)
    ms_step = ms / steps
    return {
        "workload": f"3D {n}^3 binary dendrite, cubic anisotropy delta=0.02, no-flux, FP32",
        "value": p.ncells * steps / (ms * 1e-3),
        "unit": "cell-updates/s",
        "steps": steps,
        "ms_per_step": ms_step,
        "region_ms": [round(x, 4) for x in regions],
        "roofline": bound_record(p.ncells * bpc, p.ncells * fpc, ms_step, "f32", traffic_of("c3", used, 1),
                                 valu_of("c3", used, 1), 1),
        # the flop side of the same kernel
        "alu": alu_roofline(p.ncells * fpc, ms_step, "f32"),
        "flops_per_cell_update": fpc,
        "bytes_per_cell_update": bpc,
        "steps_per_launch": 1,
        "algorithmic_bytes_per_launch": p.ncells * bpc,
        "tile": {"bx": used[0], "seg": used[1], "vec": used[2]},
        "diag": {"max_sum_dev": d["max_sum_dev"], "nonfinite": d["nonfinite"]},
        "diag_timing": dt,
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
    ms, regions, _ = measure(b.step, steps, warmup)
    diags = b.diagnostics()
    # the same ensemble with the anti-trapping current folded into the batched
    # step (one step per launch), from the state the run above left
    b.set_antitrapping(True)
    ms_at, regions_at, _ = measure(b.step, steps, warmup)
    b.close()
    ms_step = ms / steps
    return {
        "workload": "256 independent 2D instances, sides U{64..1024}, N in {2,3}, 1-2 mu fields, "
                    f"periodic, FP32, one persistent launch per {fuse} step(s), HIP graphs of "
                    f"{graph_chunk} steps",
        "value": cells * steps / (ms * 1e-3),
        "unit": "cell-updates/s",
        "steps": steps,
        "cells": cells,
        "ms_per_step": ms_step,
        "region_ms": [round(x, 4) for x in regions],
        "roofline": bound_record(bytes_step, flops_step, ms_step, "f32", traffic_of("c4", used, fuse),
                                 valu_of("c4", used, fuse), fuse),
        "alu": alu_roofline(flops_step, ms_step, "f32"),
        "steps_per_launch": fuse,
        "algorithmic_bytes_per_launch": fuse * bytes_step,
        "tile": {"seg": used[1], "vec": used[2]},
        "nonfinite_instances": sum(1 for d in diags if d["nonfinite"]),
        "with_current": {"value": cells * steps / (ms_at * 1e-3), "unit": "cell-updates/s",
                         "ms_per_step": ms_at / steps, "region_ms": [round(x, 4) for x in regions_at],
                         "steps_per_launch": 1},
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
    fwd = []
    for _ in range(REGIONS):  # each region: the whole checkpointed run from the initial state
        s.load(phi, mu)
        with Timer() as tf:
            s.step_ckpt(nsteps, every, ckpt)
        fwd.append(tf.ms)
    lam = torch.zeros_like(s.current())
    lam[: p.nphases] = s.current()[: p.nphases] - target
    loss = 0.5 * float((lam[: p.nphases].double() ** 2).sum())
    s.adjoint(lam, ckpt, 2 * every, every, 0)  # warm
    adj = []
    for _ in range(REGIONS):
        with Timer() as ta:
            _, g = s.adjoint(lam, ckpt, nsteps, every, 0)
        adj.append(ta.ms)
    s.close()
    ms_f = sorted(fwd)[len(fwd) // 2]
    ms_a = sorted(adj)[len(adj) // 2]
    grads = [g["gamma01"], g["gamma02"], g["gamma12"], g["D20"], g["D21"], g["tau"]]
    return {
        "workload": f"2D {n}x{n}, 3 phases, ternary, periodic, FP32 forward + FP32 adjoint, "
                    f"{nsteps} steps, checkpoints every {every}",
        "tile": {k: tuned[k] for k in ("bx", "seg", "vec", "fuse")},
        "forward_ms": ms_f,
        "adjoint_ms": ms_a,
        "forward_region_ms": [round(x, 3) for x in fwd],
        "adjoint_region_ms": [round(x, 3) for x in adj],
        "adjoint_over_forward": ms_a / ms_f,
        "forward_cell_updates_per_s": p.ncells * nsteps / (ms_f * 1e-3),
        "loss": loss,
        "grad_theta": dict(zip(["gamma01", "gamma02", "gamma12", "Dliq1", "Dliq2", "tau"],
                               [float(v) for v in grads])),
        "theta_star": [float(v) for v in np.asarray(theta_star)],
    }


def host_cpu():
    """The host CPU as lscpu reports it, and the CPUs this process may run on."""
    import subprocess

    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    info["usable_cpus"] = len(os.sched_getaffinity(0))
    return info


_BAND = {}


def _band_step(args):
    """Worker: the oracle's windowed step over rows [lo, hi) of the state in _BAND."""
    from oracle import gp

    lo, hi, n = args
    p = _BAND["p"]
    return lo, gp.step_window(_BAND["phi"], _BAND["mu"], n, p, (lo, 0), (hi, p.n[0]))


def oracle_band_steps(phi, mu, n0, nsteps, p, workers):
    """``nsteps`` oracle steps of a 2D state, each split into ``workers`` row bands
    stepped in parallel processes by the oracle's windowed step (equal to the
    full step: it gathers the same ghosts).  Forks, so it runs only in a process
    that has not touched the GPU."""
    import multiprocessing

    import numpy as np

    ny = phi.shape[1]
    bands = [(ny * i // workers, ny * (i + 1) // workers) for i in range(workers)]
    ctx = multiprocessing.get_context("fork")
    for k in range(nsteps):
        _BAND.update(phi=phi, mu=mu, p=p)
        with ctx.Pool(workers) as pool:
            res = pool.map(_band_step, [(lo, hi, n0 + k) for lo, hi in bands])
        nphi, nmu = np.empty_like(phi), np.empty_like(mu)
        for lo, (f, m) in res:
            nphi[:, lo:lo + f.shape[1]] = f
            nmu[:, lo:lo + m.shape[1]] = m
        phi, mu = nphi, nmu
    return phi, mu


def cpu_baseline_run(n, steps_one=1, steps_all=2, max_workers=16):
    """The FP64 oracle on the headline workload, on the host's cores: one process
    (numpy's elementwise passes run on one thread) for ``steps_one`` full-grid
    steps, and ``workers`` processes (the usable CPUs, at most ``max_workers``)
    stepping row bands for ``steps_all`` steps."""
    from oracle import gp
    from paper_2404_01035_amd import inputs

    p, phi, mu = inputs.config_c2(precision="f64", n=(n, n, 1))
    host = host_cpu()
    t0 = time.perf_counter()
    gp.run(phi, mu, 0, steps_one, p)
    t_one = time.perf_counter() - t0
    workers = max(1, min(max_workers, host["usable_cpus"]))
    t0 = time.perf_counter()
    oracle_band_steps(phi, mu, 0, steps_all, p, workers)
    t_all = time.perf_counter() - t0
    return {
        "value": p.ncells * steps_all / t_all,
        "unit": "cell-updates/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{steps_all} steps of the full {n}x{n} FP64 grid, each split into {workers} row bands "
                  f"stepped by the oracle's windowed step in {workers} processes ({t_all:.1f} s)",
        "single_thread": {"value": p.ncells * steps_one / t_one, "cores": 1,
                          "sample": f"{steps_one} full-grid step(s) in one process ({t_one:.1f} s)"},
        "host": host,
    }


def cpu_baseline(n):
    """cpu_baseline_run in a child process that never touches the GPU (it forks
    workers, which a process holding a GPU context must not do)."""
    import subprocess

    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--n", str(n)],
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        log(f"CPU baseline failed: {r.stderr[-500:]}")
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    a = parse()
    global SETTLE_MS
    if a.settle_ms is not None:
        SETTLE_MS = a.settle_ms
    if a.cpu_baseline_only:
        print(json.dumps(cpu_baseline_run(a.n)), flush=True)
        return
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
        "alu": r64["alu"],
        "region_ms": r64["region_ms"],
        "settle_steps": r64["settle_steps"],
        "timing": f"median of {REGIONS} timed regions of exactly --steps steps each, after --warmup "
                  f"steps and untimed steps until {SETTLE_MS:.0f} ms had passed",
        "flops_per_cell_update": r64["flops_per_cell_update"],
        "steps_per_launch": r64["steps_per_launch"],
        "algorithmic_bytes_per_launch": r64["algorithmic_bytes_per_launch"],
        "tile": r64["tile"],
        "diag": r64["diag"],
        "diag_timing": r64.get("diag_timing"),
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
                                           "current, one step per launch (current formed inside the step; "
                                           "the step + separate correction kernel beside it)",
                               "f64": leg_at("f64", a.n, at_steps, 5),
                               "f32": leg_at("f32", a.n, at_steps, 5),
                               "dendrite_3d_f32": dict(leg_at3d(a.n3d, min(a.steps3d, 50), 3),
                                                       workload=f"3D {a.n3d}^3 binary dendrite with the current")}
    if "ext" in legs:
        log(f"extended model: {a.n}x{a.n} eutectic with temperature-dependent coefficients")
        out["extended"] = {
            "workload": f"2D {a.n}x{a.n} directional eutectic with B(T), C(T) from coexistence-line slopes "
                        "and the dT/dt term (general kernels, two steps per launch)",
            "f64": leg_c2("f64", a.n, a.steps, a.warmup, None, False, slopes=True),
            "f32": dict(leg_c2("f32", a.n, a.steps, a.warmup, None, False, slopes=True),
                        dtype="f32 (FP64 Lagrange multiplier and reductions)"),
        }
    if "kks" in legs:
        log(f"KKS variant: {a.n}x{a.n} eutectic, Eq. Well's form and Eq. Well1")
        out["kks"] = {
            "workload": f"2D {a.n}x{a.n} directional eutectic, KKS variant (Eq. aceq), FP64, two steps per "
                        "launch: the potential of Eq. Well's form (plain kernels) and Eq. Well1 (general kernels)",
            "well_f64": leg_c2("f64", a.n, a.steps, a.warmup, None, False, kks="well"),
            "theta_f64": leg_c2("f64", a.n, a.steps, a.warmup, None, False, kks="theta"),
        }
    out["copy_bandwidth"] = copy_bandwidth(a.n)
    if not a.no_cpu:
        log("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(a.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
