"""Gradients of a vortex-transport loss through the stream-and-collide scheme.

``transport_loss(u0, omega, ...)`` runs the forward simulation in liblbm and returns
L = || u(f_T) - u_target ||_2; its backward pass runs the hand-written discrete adjoint
(``lbm_adjoint_step``, include/lbm_adjoint.h) and returns dL/du0 (the initial velocity field)
and dL/domega (all five rates; the four higher-order ones are omega[1:]).

The forward states needed in reverse order are rebuilt from checkpoints of the raw device
state (``lbm_save_state``):
  "sqrt"       ceil(sqrt(n)) evenly spaced checkpoints, each segment recomputed once into a
               ring of at most ceil(sqrt(n)) states (about n extra steps, 2 sqrt(n) states)
  "revolve"    binomial checkpointing with `slots` state buffers (Griewank's schedule: the
               split of each chain uses the binomial bound beta(c, r) = C(c + r, c))
  "store_all"  every state kept (n states, no recomputation)
All three give bit-identical gradients (same kernels, deterministic reductions).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as B
from .inputs import MODEL_CODES
from .sim import Sim


def _binom(n: int, k: int) -> int:
    return math.comb(n, k)


def revolve_split(length: int, free: int) -> int:
    """First checkpoint offset for reversing `length` steps with `free` spare slots: with c
    slots and r recomputations a chain of beta(c, r) = C(c + r, c) steps can be reversed, and
    beta(c, r) = beta(c, r - 1) + beta(c - 1, r) splits it into a left part handled with one
    recomputation less and a right part handled with one slot less."""
    r = 0
    while _binom(free + r, free) < length:
        r += 1
    right_max = _binom(free - 1 + r, free - 1) if free >= 1 else 0
    return max(1, length - right_max)


def sqrt_interval(n: int) -> int:
    return max(1, math.isqrt(max(n - 1, 0)) + 1) if n > 1 else 1


def forward_actions(n: int, schedule: str):
    """Actions of the forward sweep: ("save", key) stores the current state under key,
    ("advance", k) runs k steps."""
    if schedule == "store_all":
        for s in range(n):
            yield ("save", ("s", s))
            yield ("advance", 1)
    elif schedule == "sqrt":
        K = sqrt_interval(n)
        for s in range(0, n, K):
            yield ("save", ("c", s))
            yield ("advance", min(K, n - s))
    elif schedule == "revolve":
        yield ("save", ("r", 0))
        yield ("advance", n)
    else:
        raise ValueError(f"unknown schedule {schedule}")


def backward_actions(n: int, schedule: str, slots: int):
    """Actions of the reverse sweep, after forward_actions: ("load", key, step) restores a
    saved state, ("adjoint", key) runs one reverse step at the saved state `key` (None: the
    current state), ("free", key) releases a saved state.  Reverse steps come for states
    n - 1, ..., 0, in that order."""
    if schedule == "store_all":
        for s in range(n - 1, -1, -1):
            yield ("adjoint", ("s", s))
    elif schedule == "sqrt":
        K = sqrt_interval(n)
        for s0 in reversed(range(0, n, K)):
            s1 = min(s0 + K, n)
            yield ("load", ("c", s0), s0)
            for t in range(s0, s1):
                if t > s0:
                    yield ("advance", 1)
                yield ("save", ("ring", t - s0))
            for t in range(s1 - 1, s0 - 1, -1):
                yield ("adjoint", ("ring", t - s0))
    elif schedule == "revolve":
        if slots < 1:
            raise ValueError("revolve needs at least one slot")
        yield from _revolve(0, n, ("r", 0), slots - 1)
    else:
        raise ValueError(f"unknown schedule {schedule}")


def _revolve(a: int, b: int, key, free: int):
    # the state at step a is saved under key; the adjoint holds lambda_b
    if b - a == 1:
        yield ("adjoint", key)
        return
    if free == 0:
        for t in range(b - 1, a - 1, -1):
            yield ("load", key, a)
            yield ("advance", t - a)
            yield ("adjoint", None)
        return
    m = a + revolve_split(b - a, free)
    yield ("load", key, a)
    yield ("advance", m - a)
    yield ("save", ("r", m))
    yield from _revolve(m, b, ("r", m), free - 1)
    yield ("free", ("r", m))
    yield from _revolve(a, m, key, free)


class _Run:
    def __init__(self, u0, omega, rho0, target, model, nsteps, prec, eq_order, schedule, slots,
                 ref_velocity):
        self.model = MODEL_CODES[model] if isinstance(model, str) else int(model)
        self.omega = [float(w) for w in omega]
        self.nsteps = int(nsteps)
        self.schedule = schedule
        self.slots = int(slots)
        dev = u0.device
        self.rho0 = torch.as_tensor(rho0, dtype=torch.float64, device=dev).contiguous()
        self.ux0 = u0[0].detach().to(torch.float64).contiguous()
        self.uy0 = u0[1].detach().to(torch.float64).contiguous()
        self.tx = torch.as_tensor(target[0], dtype=torch.float64, device=dev).contiguous()
        self.ty = torch.as_tensor(target[1], dtype=torch.float64, device=dev).contiguous()
        self.sim = Sim(self.rho0, self.ux0, self.uy0, prec=prec, eq_order=eq_order, device=dev,
                       ref_velocity=ref_velocity)
        self.ctx = self.sim.ctx
        self.sbytes = B.lbm_state_bytes(self.ctx)
        self.abytes = B.lbm_adjoint_bytes(self.ctx)
        self.dev = dev
        self.saved = {}
        self.steps_run = 0       # forward steps, including recomputation
        self.peak_states = 0     # most raw states held at once

    def _do(self, act):
        kind = act[0]
        if kind == "save":
            b = self.saved.get(act[1])
            if b is None:
                b = torch.empty(self.sbytes, dtype=torch.uint8, device=self.dev)
                self.saved[act[1]] = b
                self.peak_states = max(self.peak_states, len(self.saved))
            B.lbm_save_state(self.ctx, b.data_ptr())
        elif kind == "advance":
            if act[1] > 0:
                B.lbm_step(self.ctx, self.model, self.omega, act[1])
                self.steps_run += act[1]
        elif kind == "load":
            B.lbm_load_state(self.ctx, self.saved[act[1]].data_ptr(), act[2])
        elif kind == "free":
            del self.saved[act[1]]
        elif kind == "adjoint":
            st = None if act[1] is None else self.saved[act[1]].data_ptr()
            B.lbm_adjoint_step(self.ctx, self.model, self.omega, st, self.lam[0].data_ptr(),
                               self.lam[1].data_ptr(), self.domega.data_ptr())
            self.lam.reverse()
        else:
            raise ValueError(kind)

    def forward(self):
        for act in forward_actions(self.nsteps, self.schedule):
            self._do(act)
        self.final = torch.empty(self.sbytes, dtype=torch.uint8, device=self.dev)
        B.lbm_save_state(self.ctx, self.final.data_ptr())
        self.lam = [torch.empty(self.abytes, dtype=torch.uint8, device=self.dev) for _ in range(2)]
        self.loss = B.lbm_adjoint_seed_velocity_l2(self.ctx, self.tx.data_ptr(), self.ty.data_ptr(),
                                                   self.lam[0].data_ptr())
        return self.loss

    def backward(self):
        self.domega = torch.zeros(5, dtype=torch.float64, device=self.dev)
        for act in backward_actions(self.nsteps, self.schedule, self.slots):
            self._do(act)
        dux = torch.empty_like(self.ux0)
        duy = torch.empty_like(self.uy0)
        B.lbm_eq_vjp(self.ctx, self.rho0.data_ptr(), self.ux0.data_ptr(), self.uy0.data_ptr(),
                     self.lam[0].data_ptr(), dux.data_ptr(), duy.data_ptr())
        # leave the context at the final state
        B.lbm_load_state(self.ctx, self.final.data_ptr(), self.nsteps)
        torch.cuda.current_stream(self.dev).synchronize()
        return torch.stack([dux, duy]), self.domega.clone()

    def close(self):
        self.saved.clear()
        self.sim.close()


class TransportLoss(torch.autograd.Function):
    @staticmethod
    def forward(actx, u0, omega, rho0, target, model, nsteps, prec, eq_order, schedule, slots,
                ref_velocity):
        run = _Run(u0, omega.detach().cpu().numpy(), rho0, target, model, nsteps, prec, eq_order,
                   schedule, slots, ref_velocity)
        loss = run.forward()
        actx.run = run
        actx.omega_device = omega.device
        return torch.tensor(loss, dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(actx, g):
        du, dw = actx.run.backward()
        actx.run.close()
        return (g * du, (g * dw).to(actx.omega_device), None, None, None, None, None, None, None, None,
                None)


def transport_loss(u0: torch.Tensor, omega: torch.Tensor, rho0, target, model="CM", nsteps: int = 2000,
                   prec: str = "f32", eq_order: int = 4, schedule: str = "sqrt", slots: int = 8,
                   ref_velocity=(0.0, 0.0)) -> torch.Tensor:
    """L = || u(f_T) - target ||_2 after nsteps of stream-and-collide from f^eq(rho0, u0).

    u0: (2, ny, nx) velocity field (device tensor); omega: (5,) rates (FP64 tensor);
    rho0: (ny, nx) density; target: (2, ny, nx) velocity.  Differentiable in u0 and omega."""
    return TransportLoss.apply(u0, omega, rho0, target, model, nsteps, prec, eq_order, schedule, slots,
                               ref_velocity)
