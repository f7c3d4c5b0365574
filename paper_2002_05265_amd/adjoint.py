"""Gradients of a vortex-transport loss through the stream-and-collide scheme.

``transport_loss(u0, omega, ...)`` runs the forward simulation in liblbm and returns
L = || u(f_T) - u_target ||_2; its backward pass runs the hand-written discrete adjoint
(``lbm_adjoint_step``, include/lbm_adjoint.h) and returns dL/du0 (the initial velocity field)
and dL/domega (all five rates; the four higher-order ones are omega[1:]).

The forward states needed in reverse order are rebuilt from checkpoints of the raw device
state; steps between checkpoints run out-of-place (``lbm_step_raw``, or pairs of them as one
two-step launch, ``lbm_step2_raw_many``, when the context runs the model two or three steps per
launch) straight into the buffer that keeps their result, so no state is ever copied:
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
    """Executes the schedule on raw state buffers without copying them: "save" pins the buffer
    that holds the current state, "load" makes a pinned buffer current, "advance" steps
    out-of-place (lbm_step_raw) into a free buffer of a pool, "adjoint" reads a pinned or the
    current buffer."""

    def __init__(self, u0, omega, rho0, target, model, nsteps, prec, eq_order, schedule, slots,
                 ref_velocity, reverse_depth: int = 2):
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
        # reverse steps in pairs, one launch each (the adjoint between them stays on chip); the
        # gradients are bit-identical to one reverse step per launch
        B.lbm_set_adjoint_depth(self.ctx, reverse_depth)
        self.reverse_depth = reverse_depth
        self.s = {"f64": 8, "f32": 4, "f16": 2}[prec]  # bytes per stored population
        self.a = 8 if prec == "f64" else 4              # bytes per adjoint value
        self.sbytes = B.lbm_state_bytes(self.ctx)
        self.abytes = B.lbm_adjoint_bytes(self.ctx)
        self.dev = dev
        self.saved = {}          # key -> buffer
        self.refs = {}           # id(buffer) -> number of keys pinning it
        # every state buffer the schedule needs, carved out of one allocation up front so that
        # no device allocation happens inside either sweep
        n = self.nsteps
        if schedule == "store_all":
            need = n + 1
        elif schedule == "sqrt":
            K = sqrt_interval(n)
            need = -(-n // K) + (K - 1) + 4
        else:
            need = self.slots + 3
        self.arena = torch.empty((need, self.sbytes), dtype=torch.uint8, device=dev)
        self.pool = [self.arena[i] for i in range(need - 1, -1, -1)]  # free buffers
        self.nbuf = 0
        self.cur = None          # buffer holding the current state
        self.cur_step = 0
        self.q_src, self.q_dst, self.q_step0 = [], [], 0   # queued raw steps
        self.a_states, self.a_keep = [], []                # queued reverse steps
        self.steps_run = 0       # forward steps, including recomputation
        self.peak_states = 0     # most state buffers allocated at once
        self.node_bytes = 0      # bytes per node read and written by the sweeps' step launches

    def _free_buffer(self):
        self.nbuf += 1
        self.peak_states = max(self.peak_states, self.nbuf)
        if self.pool:
            return self.pool.pop()
        return torch.empty(self.sbytes, dtype=torch.uint8, device=self.dev)

    def _release_if_unused(self, b):
        if b is not None and self.refs.get(id(b), 0) == 0 and b is not self.cur:
            self.pool.append(b)
            self.nbuf -= 1

    def _pin(self, key, b):
        old = self.saved.get(key)
        if old is b:
            return
        self.saved[key] = b
        self.refs[id(b)] = self.refs.get(id(b), 0) + 1
        if old is not None:
            self.refs[id(old)] -= 1
            self._release_if_unused(old)

    def _unpin(self, key):
        b = self.saved.pop(key)
        self.refs[id(b)] -= 1
        self._release_if_unused(b)

    def _do(self, act):
        kind = act[0]
        if kind == "save":
            self._pin(act[1], self.cur)
        elif kind == "advance":
            self._flush_adjoints()
            for _ in range(act[1]):
                dst = self._free_buffer()
                if not self.q_src:
                    self.q_step0 = self.cur_step
                self.q_src.append(self.cur.data_ptr())
                self.q_dst.append(dst.data_ptr())
                prev, self.cur = self.cur, dst
                self._release_if_unused(prev)
                self.cur_step += 1
                self.steps_run += 1
        elif kind == "load":
            prev, self.cur = self.cur, self.saved[act[1]]
            self.cur_step = act[2]
            self._release_if_unused(prev)
        elif kind == "free":
            self._unpin(act[1])
        elif kind == "adjoint":
            self._flush_steps()
            st = self.cur if act[1] is None else self.saved[act[1]]
            self.a_states.append(st.data_ptr())
            self.a_keep.append(st)
        else:
            raise ValueError(kind)

    # Steps and reverse steps are queued and issued in batches (one host call each); buffers
    # released meanwhile may be reused by later queued work because everything runs in stream
    # order on one stream.
    def _flush_steps(self):
        if self.q_src:
            B.lbm_step_raw_many(self.ctx, self.model, self.omega, self.q_src, self.q_dst, self.q_step0)
            self.node_bytes += 18 * self.s * len(self.q_src)
            self.q_src, self.q_dst = [], []

    def _reverse(self, states):
        """Reverse steps at the raw states `states` (device pointers, in reverse-step order) from
        the adjoint in self.lam[0], which then holds the result.  Three buffers in rotation let
        lbm_adjoint_many take the steps in pairs; gradients stay pending in the per-strip sums
        until the end of the sweep, so every schedule sums them in the same (step) order."""
        m = len(states)
        ptrs = [self.lam[k % 3].data_ptr() for k in range(m + 1)]
        B.lbm_adjoint_many(self.ctx, self.model, self.omega, states, ptrs, None)
        # a pair reads both states, gathers lambda_{n+1} and writes lambda_{n-1}; a single step
        # reads one state, gathers lambda_{n+1} and writes lambda_n
        pairs = m // 2 if self.reverse_depth == 2 else 0
        self.node_bytes += pairs * 18 * (self.s + self.a) + (m - 2 * pairs) * (9 * self.s + 18 * self.a)
        r = m % 3
        self.lam = self.lam[r:] + self.lam[:r]

    def _flush_adjoints(self):
        if self.a_states:
            self._reverse(self.a_states)
            self.a_states, self.a_keep = [], []

    def _flush(self):
        self._flush_steps()
        self._flush_adjoints()

    # Fast paths: the sqrt(n) and store-all sweeps issue whole segments with two host calls
    # (lbm_step_raw_many / lbm_adjoint_many); they compute, bit for bit, what the generic action
    # executor (used for "revolve") would: the same forward steps in the same order, and the same
    # reverse steps, whose grouping into one- and two-step launches changes no value.
    def _two_step(self) -> bool:
        """Whether the context runs this model fused, two or three steps per launch (then pairs of
        forward steps go through lbm_step2_raw_many; the states written are the same bit for bit)."""
        return B.lbm_get_fusion(self.ctx, self.model)[0] > 0

    def _three_step(self) -> bool:
        """Whether the context runs this model three steps per launch (then three forward steps
        whose first two states are not kept go through lbm_step3_raw_many)."""
        return (B.lbm_get_fusion_depth(self.ctx, self.model) == 3 and
                B.lbm_get_fusion(self.ctx, self.model)[0] in (4, 8))

    def _run_chain(self, chain, step0: int):
        """Advance along chain = [b_0, b_1, ..., b_m] (b_t receives state step0 + t; None = not
        kept, a scratch buffer is used): three steps as one three-step launch where the two states
        between are not kept, pairs of steps as one two-step launch (writing the state between
        them only when it is kept), the rest one step per launch.  Returns the buffer holding the
        last state."""
        ops = []  # ("1", src, dst, step), ("2", src, mid, dst, step) or ("3", src, dst, step)
        cur = chain[0]
        scratch = self._scratch
        t, m = 1, len(chain) - 1
        pairs = self._two_step()
        triples = self._three_step()

        def place(b):
            if b is not None:
                return b
            return scratch[0] if cur is not scratch[0] else scratch[1]

        while t <= m:
            if triples and t + 2 <= m and chain[t] is None and chain[t + 1] is None:
                dst = place(chain[t + 2])
                ops.append(("3", cur, dst, step0 + t - 1))
                cur, t = dst, t + 3
            elif pairs and t + 1 <= m:
                dst = place(chain[t + 1])
                ops.append(("2", cur, chain[t], dst, step0 + t - 1))
                cur, t = dst, t + 2
            else:
                dst = place(chain[t])
                ops.append(("1", cur, dst, step0 + t - 1))
                cur, t = dst, t + 1
        for o in ops:  # every launch reads and writes each population once; a pair may also write
            self.node_bytes += (27 if o[0] == "2" and o[2] is not None else 18) * self.s
        # issue consecutive ops of one kind with one host call
        k = 0
        while k < len(ops):
            j = k
            while j < len(ops) and ops[j][0] == ops[k][0]:
                j += 1
            run = ops[k:j]
            if run[0][0] == "1":
                B.lbm_step_raw_many(self.ctx, self.model, self.omega, [o[1].data_ptr() for o in run],
                                    [o[2].data_ptr() for o in run], run[0][3])
            elif run[0][0] == "3":
                B.lbm_step3_raw_many(self.ctx, self.model, self.omega, [o[1].data_ptr() for o in run],
                                     [o[2].data_ptr() for o in run], run[0][3])
            else:
                B.lbm_step2_raw_many(self.ctx, self.model, self.omega, [o[1].data_ptr() for o in run],
                                     [0 if o[2] is None else o[2].data_ptr() for o in run],
                                     [o[3].data_ptr() for o in run], run[0][4])
            k = j
        self.steps_run += m
        return cur

    def _forward_fast(self):
        n = self.nsteps
        K = n if self.schedule == "store_all" else sqrt_interval(n)
        bufs = [self.cur]
        for t in range(1, n + 1):
            bufs.append(self._free_buffer() if (self.schedule == "store_all" or t % K == 0 or t == n)
                        else None)
        # scratch for states that are not kept
        self._scratch = [self._free_buffer(), self._free_buffer()] if self.schedule == "sqrt" else [None, None]
        self._run_chain(bufs, 0)
        keep = {}
        if self.schedule == "store_all":
            for t in range(n):
                keep[("s", t)] = bufs[t]
        else:
            for t in range(0, n, K):
                keep[("c", t)] = bufs[t]
            self.pool.extend(self._scratch)
            self.nbuf -= len(self._scratch)
        for k, b in keep.items():
            self._pin(k, b)
        self.cur = bufs[n]

    def _backward_fast(self):
        n = self.nsteps
        if self.schedule == "store_all":
            self._reverse([self.saved[("s", t)].data_ptr() for t in range(n - 1, -1, -1)])
            return
        K = sqrt_interval(n)
        ring = [self._free_buffer() for _ in range(K - 1)]
        self._scratch = [None, None]
        for s0 in reversed(range(0, n, K)):
            m = min(s0 + K, n) - s0
            seg = [self.saved[("c", s0)]] + ring[:m - 1]
            if m > 1:
                self._run_chain(seg, s0)
            self._reverse([b.data_ptr() for b in reversed(seg)])
        self.pool.extend(ring)
        self.nbuf -= len(ring)

    def forward(self):
        self.cur = self._free_buffer()
        B.lbm_save_state(self.ctx, self.cur.data_ptr())  # the initial state f^eq(rho0, u0)
        self.cur_step = 0
        if self.schedule in ("sqrt", "store_all"):
            self._forward_fast()
        else:
            for act in forward_actions(self.nsteps, self.schedule):
                self._do(act)
            self._flush()
        self.final = self.cur
        self.refs[id(self.final)] = self.refs.get(id(self.final), 0) + 1  # keep it
        B.lbm_load_state(self.ctx, self.final.data_ptr(), self.nsteps)
        self.lam = [torch.empty(self.abytes, dtype=torch.uint8, device=self.dev) for _ in range(3)]
        self.loss = B.lbm_adjoint_seed_velocity_l2(self.ctx, self.tx.data_ptr(), self.ty.data_ptr(),
                                                   self.lam[0].data_ptr())
        return self.loss

    def backward(self):
        self.domega = torch.zeros(5, dtype=torch.float64, device=self.dev)
        if self.schedule in ("sqrt", "store_all"):
            self._backward_fast()
        else:
            for act in backward_actions(self.nsteps, self.schedule, self.slots):
                self._do(act)
            self._flush()
        B.lbm_adjoint_flush(self.ctx, self.domega.data_ptr())
        dux = torch.empty_like(self.ux0)
        duy = torch.empty_like(self.uy0)
        B.lbm_eq_vjp(self.ctx, self.rho0.data_ptr(), self.ux0.data_ptr(), self.uy0.data_ptr(),
                     self.lam[0].data_ptr(), dux.data_ptr(), duy.data_ptr())
        torch.cuda.current_stream(self.dev).synchronize()
        return torch.stack([dux, duy]), self.domega.clone()

    def close(self):
        self.saved.clear()
        self.pool.clear()
        self.cur = self.final = self.arena = None
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
