"""Torch-facing wrapper of the batched persistent sweep (include/lbm_batch.h)."""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from .inputs import MODEL_CODES


class Batch:
    """Independent periodic simulations advanced together by one persistent launch.

    instances: list of dicts with nx, ny, model (name or code), eq_order, omega (5 rates),
    optional rho0; fields: list of (rho, ux, uy) arrays [ny, nx], one per instance."""

    def __init__(self, instances, fields, prec: str = "f64", device="cuda",
                 stream: torch.cuda.Stream | None = None):
        self.device = torch.device(device)
        descs = []
        for d in instances:
            m = d["model"]
            descs.append({**d, "model": MODEL_CODES[m] if isinstance(m, str) else int(m)})
        self.shapes = [(int(d["nx"]), int(d["ny"])) for d in descs]
        self.n = len(descs)
        self.descs = B.make_descs(descs)
        self.prec = B.PRECISIONS[prec]
        cat = [np.concatenate([np.asarray(f[k], dtype=np.float64).ravel() for f in fields]) for k in range(3)]
        dev = [torch.from_numpy(c).to(self.device) for c in cat]
        nbytes = B.lbm_batch_population_bytes(self.descs, self.prec)
        if nbytes == 0:
            raise ValueError("invalid batch description")
        self.pop = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.handle = B.lbm_batch_create(self.descs, self.prec, *(t.data_ptr() for t in dev),
                                         self.pop.data_ptr(), nbytes, self.stream.cuda_stream)
        self.stream.synchronize()

    def run(self, nsteps: int, rebalance_every: int = 0):
        """Advance nsteps; with rebalance_every > 0 the run is cut into pieces of that many steps
        and the live instances are re-dealt over the XCDs between pieces (synchronising)."""
        if rebalance_every <= 0:
            B.lbm_batch_run(self.handle, nsteps)
            return
        done = 0
        while done < nsteps:
            k = min(rebalance_every, nsteps - done)
            B.lbm_batch_run(self.handle, k)
            done += k
            if done < nsteps:
                B.lbm_batch_rebalance(self.handle)

    def rebalance(self):
        """Re-deal the live instances over the XCDs (synchronises)."""
        B.lbm_batch_rebalance(self.handle)

    def status(self):
        """(step, [blow-up step per instance, -1 if none])"""
        return B.lbm_batch_status(self.handle, self.n)

    def state(self, j: int) -> torch.Tensor:
        nx, ny = self.shapes[j]
        f = torch.empty((9, ny, nx), dtype=torch.float64, device=self.device)
        B.lbm_batch_get_state(self.handle, j, f.data_ptr())
        self.stream.synchronize()
        return f

    def mean_u2(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """Domain mean of |u|^2 per instance (FP64 device tensor, asynchronous)."""
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        B.lbm_batch_mean_u2(self.handle, out.data_ptr())
        return out

    def set_active(self, active: torch.Tensor):
        """Retire (for good) the instances whose flag is 0; active: int32 device tensor of n
        flags.  Asynchronous."""
        if active.dtype != torch.int32 or active.numel() != self.n or active.device != self.device:
            raise ValueError("active must be an int32 device tensor with one flag per instance")
        B.lbm_batch_set_active(self.handle, active.contiguous().data_ptr())

    def set_launch(self, nodes_per_thread: int, groups_per_cu: int = 0):
        B.lbm_batch_set_launch(self.handle, nodes_per_thread, groups_per_cu)

    def set_fusion(self, strip_rows: int):
        """Two steps per pass over strips of strip_rows rows (a multiple of 8); 0 turns it off."""
        B.lbm_batch_set_fusion(self.handle, strip_rows)

    def fusion(self) -> int:
        """Strip height of two steps per pass, 0 when off."""
        return B.lbm_batch_get_fusion(self.handle)

    def set_fusion_depth(self, steps: int):
        """Steps per fused pass: 2 or 3 (FP64, FP32)."""
        B.lbm_batch_set_fusion_depth(self.handle, steps)

    def fusion_depth(self) -> int:
        return B.lbm_batch_get_fusion_depth(self.handle)

    def autotune(self, trials: int = 5):
        """Fastest launch shape (nodes per thread, groups per CU, us per step); also decides
        whether two or three steps per pass are used (see fusion(), fusion_depth())."""
        return B.lbm_batch_autotune(self.handle, trials)

    def residency(self, shape: int):
        """(groups per CU from the kernel's resources, runtime occupancy figure, confirmed figure,
        probes that had to lower a figure) of launch shape 0-4 (lbm_batch_residency)."""
        return B.lbm_batch_residency(self.handle, shape)

    def close(self):
        if getattr(self, "handle", None):
            B.lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
