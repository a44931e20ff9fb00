"""Differentiable sweeps: a ``torch.autograd.Function`` over many steps of the
HIP sweep, with the hand-written adjoint (``csh_adjoint_step``) in backward.

Forward: primitive fields W0 -> conserved U0 (``csh_init_state``), then
``nsteps`` steps with the CFL timestep chosen on the device (``csh_run_cfl``),
keeping the state every ``checkpoint_every`` steps and the timesteps taken;
with ``checkpoint_every=1`` one ``csh_run_cfl_states`` launch keeps every
state (nsteps states in device memory, no recomputation in backward).
Backward: the timesteps are frozen (the gradient is that of the map with the
recorded dt list); segment by segment from the last, the states of the segment
are recomputed from its checkpoint with those timesteps (``csh_step``) and the
adjoint steps run in reverse; finally ``csh_init_state_adjoint`` carries the
gradient from U0 back to W0.  All arithmetic runs in the library's kernels;
this module only sequences the calls and holds the checkpoints.
"""
from __future__ import annotations

from collections import OrderedDict

import torch

from . import BC_PERIODIC, Grid

# Grid handles reused by consecutive sweeps with the same geometry (the usual
# pattern of an optimisation loop): the handle's captured graph, reduction
# slots and adjoint workspace are then set up once.  At most _CACHE_SIZE
# handles are kept (least recently used dropped); clear_cache() frees them.
_CACHE_SIZE = 2
_cache: OrderedDict = OrderedDict()


def clear_cache() -> None:
    """Drop the grid handles kept for reuse."""
    _cache.clear()


def _grid(W0: torch.Tensor, dx: float, dy: float, bc, potential, checkpoint_every: int) -> Grid:
    # a handle runs on the stream that was current when it was made: the
    # stream is part of the key, so a sweep under another stream gets its own
    key = (tuple(W0.shape), W0.dtype, str(W0.device), float(dx), float(dy), tuple(int(b) for b in bc),
           None if potential is None else tuple(float(x) for x in potential),
           torch.cuda.current_stream(W0.device).cuda_stream)
    g = _cache.pop(key, None)
    if g is None:
        g = Grid(W0, dx, dy, bc)
        if potential is not None:
            g.set_potential(*potential)
    else:
        g.set_state(W0)
    _cache[key] = g
    while len(_cache) > _CACHE_SIZE:
        _cache.popitem(last=False)
    # one timestep log buffer per handle: the graph captured for a segment
    # length is reused as long as its buffers are the same
    if getattr(g, "_seg_log", None) is None or g._seg_log.numel() < checkpoint_every:
        g._seg_log = torch.empty(checkpoint_every, dtype=torch.float64, device=W0.device)
    return g


class AdjointSweep(torch.autograd.Function):
    """U_n = S_{dt_{n-1}} o ... o S_{dt_0} (U(W0)); differentiable in W0."""

    @staticmethod
    def forward(ctx, W0: torch.Tensor, dx: float, dy: float, bc, nsteps: int, checkpoint_every: int,
                cfl: float = 0.8, potential=None, dts=None):
        K = max(1, int(checkpoint_every))
        g = _grid(W0.detach().contiguous(), dx, dy, bc, potential, K)
        U = g.U
        log = g._seg_log
        ckpts, seg_dts = [], []
        if dts is not None:  # replay a given timestep list
            dts = [float(d) for d in dts]
            assert len(dts) == nsteps
        else:
            dts_dev = torch.empty(max(nsteps, 1), dtype=torch.float64, device=U.device)
        if K == 1 and dts is None and nsteps > 0:
            # every state kept (nsteps states in device memory): one graph launch
            # writes the whole trajectory and the reverse pass recomputes nothing
            states, _ = g.run_cfl_states(nsteps, cfl, U0=U, dt_log=dts_dev)
            ckpts = [U.clone()] + [states[k] for k in range(nsteps - 1)]
            U = states[nsteps - 1]
            done = nsteps
        else:
            done = 0
        while done < nsteps:
            k = min(K, nsteps - done)
            ckpts.append(U.clone())
            if dts is None:
                dts_dev[done:done + k].copy_(g.run_cfl(k, cfl, U=U, dt_log=log))  # stays on the device
            else:
                V = U
                for dt in dts[done:done + k]:
                    V = g.step(dt, V)
                U.copy_(V)
            done += k
        if dts is None:
            dts = dts_dev[:nsteps].cpu().tolist()  # one host synchronisation for the whole run
        g.last_signal_speed()  # raises NonPhysicalState if a state of the run was not physical
        seg_dts = [dts[i:i + K] for i in range(0, nsteps, K)]
        ctx.grid = g
        ctx.ckpts = ckpts
        ctx.seg_dts = seg_dts
        ctx.save_for_backward(W0)
        all_dts = torch.tensor([d for seg in seg_dts for d in seg], dtype=torch.float64)
        ctx.mark_non_differentiable(all_dts)
        return U.clone(), all_dts

    @staticmethod
    def backward(ctx, gU: torch.Tensor, _gdts=None):
        (W0,) = ctx.saved_tensors
        g = ctx.grid
        lam = gU.contiguous().to(torch.float64)
        for ck, seg in zip(reversed(ctx.ckpts), reversed(ctx.seg_dts)):
            states = [ck]
            for dt in seg[:-1]:
                states.append(g.step(dt, states[-1]))
            for U, dt in zip(reversed(states), reversed(seg)):
                lam = g.adjoint_step(dt, U, lam)
        lamW = g.init_state_adjoint(W0.detach().contiguous(), lam)
        return lamW, None, None, None, None, None, None, None, None


def sweep(W0: torch.Tensor, dx: float, dy: float = 1.0, bc=(BC_PERIODIC, BC_PERIODIC), nsteps: int = 1,
          checkpoint_every: int = 20, cfl: float = 0.8, potential=None, dts=None) -> torch.Tensor:
    """Differentiable ``nsteps``-step sweep of the primitive fields ``W0``;
    returns (final conserved state, timesteps taken as a CPU float64 tensor)."""
    return AdjointSweep.apply(W0, dx, dy, bc, nsteps, checkpoint_every, cfl, potential, dts)


def run_frozen(W0: torch.Tensor, dx: float, dy: float, bc, dts, potential=None) -> torch.Tensor:
    """Forward only, with a given timestep list (for finite-difference checks):
    one graph launch of len(dts) steps reading the timesteps on the device."""
    g = Grid(W0.contiguous(), dx, dy, bc)
    if potential is not None:
        g.set_potential(*potential)
    d = torch.as_tensor(dts, dtype=torch.float64).to(g.U.device).contiguous()
    return g.run_dts(d).clone()


class FrozenRunner:
    """Repeated forward runs with one timestep list on one grid handle (the
    captured graph is reused across runs): run(W0) -> final conserved state."""

    def __init__(self, W_like: torch.Tensor, dx: float, dy: float, bc, dts, potential=None):
        self.g = Grid(W_like.contiguous(), dx, dy, bc)
        if potential is not None:
            self.g.set_potential(*potential)
        self.dts = torch.as_tensor(dts, dtype=torch.float64).to(W_like.device).contiguous()
        self.W = torch.empty_like(W_like)

    def run(self, W0: torch.Tensor) -> torch.Tensor:
        self.W.copy_(W0)
        self.g.set_state(self.W)
        return self.g.run_dts(self.dts)
