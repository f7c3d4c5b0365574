"""Thin torch-facing wrapper over the C ABI: device memory and the stream come from torch,
every step of the method runs in liblbm's HIP kernels."""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from .inputs import MODEL_CODES


def _model_code(model) -> int:
    return MODEL_CODES[model] if isinstance(model, str) else int(model)


def _dev_f64(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.array(a, dtype=np.float64, order="C")).to(device)


class Sim:
    """One periodic nx x ny D2Q9 simulation on the current HIP device.

    rho, ux, uy: initial macroscopic fields [ny, nx] (numpy or torch, converted to FP64).
    prec: 'f64' | 'f32' | 'f16' (shifted storage for the last two).  eq_order: 2, 3 or 4.
    ref_velocity: reference velocity U of the shifted storage (h = f - f^eq(rho0, U))."""

    def __init__(self, rho, ux, uy, prec: str = "f64", eq_order: int = 4, rho0: float = 1.0,
                 device: str | torch.device = "cuda", stream: torch.cuda.Stream | None = None,
                 ref_velocity=(0.0, 0.0)):
        self.device = torch.device(device)
        rho, ux, uy = (_dev_f64(a, self.device) for a in (rho, ux, uy))
        self.ny, self.nx = rho.shape
        self.prec = B.PRECISIONS[prec]
        self.eq_order = eq_order
        nbytes = B.lbm_population_bytes(self.nx, self.ny, self.prec)
        if nbytes == 0:
            raise ValueError(f"invalid grid {self.nx} x {self.ny}")
        self.pop = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.ctx = B.lbm_init_shifted(self.nx, self.ny, self.prec, eq_order, rho0,
                                      float(ref_velocity[0]), float(ref_velocity[1]), rho.data_ptr(),
                                      ux.data_ptr(), uy.data_ptr(), self.pop.data_ptr(), nbytes,
                                      self.stream.cuda_stream)
        # the init kernel reads rho/ux/uy asynchronously: keep them alive until it has run
        self.stream.synchronize()

    def step(self, model, omega, nsteps: int = 1):
        B.lbm_step(self.ctx, _model_code(model), omega, nsteps)

    def set_launch(self, model, rows: int, xcd: int):
        B.lbm_set_launch(self.ctx, _model_code(model), rows, xcd)

    def set_fusion(self, model, ring_rows: int, strip_rows: int = 0):
        """Two steps per launch (ring_rows 4, 8 or 16, strip_rows a multiple of it); 0 turns it off."""
        B.lbm_set_fusion(self.ctx, _model_code(model), ring_rows, strip_rows)

    def set_fusion_depth(self, model, steps: int):
        """Steps per fused launch of `model`: 2 or 3 (FP32, FP64; with ring_rows 4 or 8)."""
        B.lbm_set_fusion_depth(self.ctx, _model_code(model), steps)

    def fusion_depth(self, model) -> int:
        return B.lbm_get_fusion_depth(self.ctx, _model_code(model))

    def fusion(self, model):
        """(ring_rows, strip_rows) of `model`'s fused launches, (0, 0) when off (fusion_depth() gives
        the steps per launch)."""
        return B.lbm_get_fusion(self.ctx, _model_code(model))

    def autotune(self, model, omega, trials: int = 10):
        """Pick the fastest launches for `model` (state unchanged); returns the single-step shape
        (rows, xcd) and the best microseconds per step; fusion() and fusion_depth() give the fused
        choice."""
        return B.lbm_autotune(self.ctx, _model_code(model), omega, trials)

    def moments(self):
        """(rho, ux, uy) FP64 device tensors [ny, nx] and the totals list
        [mass, px, py, kinetic energy, mean |u|^2, step]."""
        out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(3)]
        tot = B.lbm_moments(self.ctx, *(t.data_ptr() for t in out))
        return out[0], out[1], out[2], tot

    def totals(self):
        return B.lbm_moments(self.ctx, None, None, None)

    def state(self) -> torch.Tensor:
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        B.lbm_get_state(self.ctx, f.data_ptr())
        self.stream.synchronize()
        return f

    def set_state(self, f, step: int):
        t = _dev_f64(f, self.device)
        B.lbm_set_state(self.ctx, t.data_ptr(), step)
        self.stream.synchronize()

    def status(self):
        return B.lbm_status(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            B.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
