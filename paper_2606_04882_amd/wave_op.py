"""Differentiable wave modelling: traces(c) as a torch.autograd.Function.

forward(vel) runs fd_forward for every shot and returns the traces stacked
as [nshots, nt, nrec]; with segment checkpointing it keeps the checkpoints
(d^{jK}, u^{jK}) every K = `ckpt_every` steps that the forward pass writes
(2 ceil(nt/K) window fields per shot).  backward(dJ/dtraces) runs
fd_adjoint_gradient on them (exact discrete adjoint; no second forward
pass), or, with ckpt == "revolve", the binomial plan with `nsnap` snapshots,
and returns dJ/dc.  With the L2 misfit J = 1/2 ||d - d_obs||^2 computed in torch, the
incoming gradient is d - d_obs.  The FWI use of the stencils is the one the
paper points to in its conclusions (Sec. 7).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import torch

from . import fdwave as F


@dataclass
class Survey:
    """Acquisition shared by every call: grid, stencil, sources, receivers."""
    grid: F.Grid
    stencil_id: int
    sources: Sequence[Tuple[int, ...]]
    wavelet: torch.Tensor          # [nt] float32 on the device
    rec: torch.Tensor              # [nrec, ndim] int32 on the device
    ckpt_every: int = 100
    ckpt: str = "segment"          # or "revolve" (binomial, nsnap snapshots)
    nsnap: int = 0

    def shots(self, traces: torch.Tensor = None, adj: torch.Tensor = None,
              ckpt: torch.Tensor = None) -> List[F.Shot]:
        out = []
        for i, src in enumerate(self.sources):
            out.append(F.Shot(stencil_id=self.stencil_id, src=tuple(src), wavelet=self.wavelet,
                              rec=self.rec, traces=None if traces is None else traces[i],
                              trace_adj=None if adj is None else adj[i],
                              ckpt=None if ckpt is None else ckpt[i]))
        return out

    def keeps_checkpoints(self) -> bool:
        return self.ckpt == "segment"


class WaveOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vel: torch.Tensor, survey: Survey) -> torch.Tensor:
        vel = vel.detach().contiguous()
        nt, nrec = survey.grid.nt, int(survey.rec.shape[0])
        traces = torch.zeros(len(survey.sources), nt, nrec, device=vel.device, dtype=torch.float32)
        ckpt, K = None, 0
        if survey.keeps_checkpoints():
            K = int(survey.ckpt_every)
            n = F.ckpt_numel(survey.grid, survey.shots()[0], K)
            ckpt = torch.empty(len(survey.sources), n, device=vel.device, dtype=torch.float32)
        F.fd_forward(survey.grid, vel, survey.shots(traces, ckpt=ckpt), ckpt_every=K)
        ctx.survey = survey
        ctx.ckpt = ckpt
        ctx.save_for_backward(vel)
        return traces

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        (vel,) = ctx.saved_tensors
        survey = ctx.survey
        adj = grad_traces.detach().to(torch.float32).contiguous()
        scratch = torch.zeros_like(adj)      # traces, rewritten only when the forward pass reruns
        grad = torch.zeros_like(vel)
        F.fd_adjoint_gradient(survey.grid, vel, survey.shots(scratch, adj, ctx.ckpt), survey.ckpt_every, grad,
                              ckpt=survey.ckpt, nsnap=survey.nsnap)
        ctx.ckpt = None
        return grad, None


def model_traces(vel: torch.Tensor, survey: Survey) -> torch.Tensor:
    return WaveOp.apply(vel, survey)
