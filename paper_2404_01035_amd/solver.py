"""Torch-owned device buffers bound to one library state.

PyTorch only allocates device memory and supplies the stream; every step runs
in libmpstep.so's kernels through the C ABI (``abi``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi


class Solver:
    """One simulation on cuda:0: two ping-pong state buffers plus the reduction workspace."""

    def __init__(self, p, device: str = "cuda:0"):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (torch.cuda.is_available() is False)")
        self.p = p
        self.device = torch.device(device)
        self.dtype = torch.float64 if p.precision == "f64" else torch.float32
        self.st = abi.mp_create(p)
        shape = (p.nfields,) + tuple(p.spatial)
        self.bufs = [torch.empty(shape, dtype=self.dtype, device=self.device) for _ in range(2)]
        nws = abi.mp_workspace_bytes(self.st)
        self.ws = torch.empty(nws, dtype=torch.uint8, device=self.device)
        assert abi.mp_state_bytes(self.st) == self.bufs[0].numel() * self.bufs[0].element_size()
        abi.mp_bind(self.st, self.bufs[0].data_ptr(), self.bufs[1].data_ptr(), self.ws.data_ptr())

    @staticmethod
    def stream() -> int:
        return torch.cuda.current_stream().cuda_stream

    def load(self, phi, mu, step: int = 0):
        """Upload (phi, mu) host arrays into buffer 0 and declare it the state at ``step``."""
        host = np.concatenate([np.asarray(phi), np.asarray(mu)], axis=0)
        self.bufs[0].copy_(torch.from_numpy(np.ascontiguousarray(host)).to(self.dtype))
        torch.cuda.synchronize()
        abi.mp_set_step(self.st, step, 0)

    def step(self, nsteps: int):
        abi.mp_step(self.st, nsteps, self.stream())

    def current(self) -> torch.Tensor:
        w, _ = abi.mp_current(self.st)
        return self.bufs[w]

    @property
    def time_level(self) -> int:
        return abi.mp_current(self.st)[1]

    def fields(self):
        """(phi, mu) of the current state as float64 numpy arrays."""
        torch.cuda.synchronize()
        a = self.current().double().cpu().numpy()
        return a[: self.p.nphases], a[self.p.nphases:]

    def diagnostics(self, allow_nonfinite: bool = False) -> dict:
        return abi.mp_diagnostics(self.st, self.stream(), allow_nonfinite)

    def step_diag(self, nsteps: int, allow_nonfinite: bool = False) -> dict:
        """nsteps steps and the diagnostics of the state reached, reduced from
        partial sums the last step launch forms as it stores the state."""
        return abi.mp_step_diag(self.st, nsteps, self.stream(), allow_nonfinite)[0]

    def set_tile(self, bx: int = 0, seg: int = 0, vec: int = 0):
        abi.mp_set_tile(self.st, bx, seg, vec)

    # ---- moving frame (SHIFT) ------------------------------------------------
    def front_row(self) -> int:
        """Highest row holding a cell whose liquid fraction is below 1/2 (-1 if none)."""
        return abi.mp_front_row(self.st, self.stream())

    def shift(self, rows: int, mu_melt) -> int:
        """Move the frame up by ``rows``: solid rows leave at the bottom, melt at
        ``mu_melt`` enters at the top.  Returns the total frame offset in rows."""
        return abi.mp_shift(self.st, rows, mu_melt, self.stream())

    def step_moving_frame(self, nsteps: int, shiftj: int, every: int, mu_melt) -> int:
        """``nsteps`` steps; every ``every`` steps (and at the end) the front row is
        found and, when it lies above row ``shiftj``, the frame is shifted by the
        difference (the SHIFT / Shiftj keys).  Returns the total frame offset."""
        done, offset = 0, abi.mp_shift(self.st, 0, mu_melt, self.stream())
        while done < nsteps:
            n = min(every, nsteps - done)
            self.step(n)
            done += n
            front = self.front_row()
            if front > shiftj:
                offset = self.shift(front - shiftj, mu_melt)
        return offset

    def set_graph(self, chunk: int):
        """Replay steps as HIP graphs of ``chunk`` steps (0: launch kernel by kernel)."""
        abi.mp_set_graph(self.st, chunk)

    def set_fusion(self, steps: int):
        """Steps per kernel launch (1, or 2 for 2D grids: the state crosses HBM once per two steps)."""
        abi.mp_set_fusion(self.st, steps)

    def set_antitrapping(self, on=True):
        """Anti-trapping current of Eq. jatr in the mu update (2D and 3D, one step per launch): True/1
        forms it inside the 2D step kernel, 2 in a separate correction kernel after each step (the
        only form in 3D); both give the same bits."""
        abi.mp_set_antitrapping(self.st, on)

    def autotune(self, reps: int = 10, cache: str | None = None, force: bool = False) -> dict:
        """Pick the fastest tile for this workload (cached on disk); the state is unchanged."""
        from . import autotune

        return autotune.tune(self.st, [self.p], self.stream(), torch.cuda.get_device_name(self.device),
                             reps, cache, force)

    # ---- checkpointed run and adjoint -------------------------------------
    def checkpoint_buffer(self, nsteps: int, every: int) -> torch.Tensor:
        """Device buffer for ceil(nsteps / every) checkpoints (256-byte slots)."""
        slot = (abi.mp_state_bytes(self.st) + 255) // 256 * 256
        nslots = max(1, -(-int(nsteps) // int(every)))
        return torch.empty(slot * nslots, dtype=torch.uint8, device=self.device)

    def step_ckpt(self, nsteps: int, every: int, ckpt: torch.Tensor):
        abi.mp_step_ckpt(self.st, nsteps, every, ckpt.data_ptr(), self.stream())

    def adjoint(self, lam_final: torch.Tensor, ckpt: torch.Tensor, nsteps: int, every: int, n0: int):
        """dL/d(initial state) and dL/dtheta from dL/d(final state) (state layout)."""
        lam0 = torch.empty_like(self.bufs[0])
        work = torch.empty(abi.mp_adjoint_work_bytes(self.st, every), dtype=torch.uint8,
                           device=self.device)
        lam_final = lam_final.to(self.dtype).contiguous()
        g = abi.mp_adjoint(self.st, ckpt.data_ptr(), nsteps, every, n0, lam_final.data_ptr(),
                           lam0.data_ptr(), work.data_ptr(), self.stream())
        return lam0, g

    def close(self):
        if self.st:
            abi.mp_destroy(self.st)
            self.st = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Many independent 2D simulations stepped together (one persistent launch per step).

    Every instance lives in the same pair of state buffers at the offsets the
    library reports; ``load``/``fields`` move one instance at a time.
    """

    def __init__(self, plist, device: str = "cuda:0"):
        if not torch.cuda.is_available():
            raise RuntimeError("BatchSolver needs a GPU (torch.cuda.is_available() is False)")
        self.plist = list(plist)
        self.device = torch.device(device)
        self.dtype = torch.float64 if self.plist[0].precision == "f64" else torch.float32
        self.esize = 8 if self.dtype == torch.float64 else 4
        self.st = abi.mp_create_batch(self.plist)
        nbytes = abi.mp_state_bytes(self.st)
        self.bufs = [torch.empty(nbytes // self.esize, dtype=self.dtype, device=self.device)
                     for _ in range(2)]
        self.ws = torch.empty(abi.mp_workspace_bytes(self.st), dtype=torch.uint8, device=self.device)
        abi.mp_bind(self.st, self.bufs[0].data_ptr(), self.bufs[1].data_ptr(), self.ws.data_ptr())
        self.offsets = [abi.mp_instance_offset(self.st, i) for i in range(len(self.plist))]

    def _view(self, buf, i):
        off, nb = self.offsets[i]
        p = self.plist[i]
        return buf[off // self.esize:(off + nb) // self.esize].view((p.nfields,) + tuple(p.spatial))

    def load(self, i, phi, mu):
        host = np.concatenate([np.asarray(phi), np.asarray(mu)], axis=0)
        self._view(self.bufs[0], i).copy_(torch.from_numpy(np.ascontiguousarray(host)).to(self.dtype))

    def start(self, step: int = 0):
        """Declare buffer 0 (as filled by ``load``) the state at ``step``."""
        torch.cuda.synchronize()
        abi.mp_set_step(self.st, step, 0)

    def step(self, nsteps: int):
        abi.mp_step(self.st, nsteps, Solver.stream())

    def fields(self, i):
        torch.cuda.synchronize()
        w, _ = abi.mp_current(self.st)
        a = self._view(self.bufs[w], i).double().cpu().numpy()
        n = self.plist[i].nphases
        return a[:n], a[n:]

    def diagnostics(self, allow_nonfinite: bool = False):
        return abi.mp_diagnostics_batch(self.st, Solver.stream(), allow_nonfinite)

    def step_diag(self, nsteps: int, allow_nonfinite: bool = False):
        """nsteps steps, then the diagnostics of every instance (one dict each)."""
        return abi.mp_step_diag(self.st, nsteps, Solver.stream(), allow_nonfinite)

    def set_tile(self, seg: int, vec: int = 0):
        abi.mp_set_tile(self.st, 0, seg, vec)

    def set_antitrapping(self, on=True):
        """Anti-trapping current of Eq. jatr, formed inside the batched step kernel."""
        abi.mp_set_antitrapping(self.st, on)

    def set_graph(self, chunk: int):
        abi.mp_set_graph(self.st, chunk)

    def autotune(self, reps: int = 10, cache: str | None = None, force: bool = False) -> dict:
        """Pick the fastest strip segment for this ensemble (cached on disk)."""
        from . import autotune

        return autotune.tune(self.st, self.plist, Solver.stream(),
                             torch.cuda.get_device_name(self.device), reps, cache, force)

    @property
    def time_level(self) -> int:
        return abi.mp_current(self.st)[1]

    def close(self):
        if self.st:
            abi.mp_destroy(self.st)
            self.st = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
