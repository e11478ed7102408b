"""Differentiable run of the N-phase LBM: a torch.autograd.Function over the C ABI.

    phiT = run_differentiable(cfg, phi0, sigma_pairs, steps, ckpt_every=50, precision="fp64")

forward: init from phi0 [N, *grid] (FP64), run `steps` fused steps on the GPU with the
pair tensions sigma_pairs (p < q, lexicographic), keep a checkpoint of the state every
`ckpt_every` steps, return the N phase fields at the end.  With precision "fp32" the
forward runs the FP32 deviation-storage form and the backward applies the (FP64) adjoint
step along that FP32 trajectory: each recomputed state is exported as the FP64
populations it stands for.
backward: seed the state adjoint from dL/dphiT, then for each checkpoint segment from the
last: restore the checkpoint, recompute the segment's states with the forward kernel, and
run the hand-written adjoint step backwards through them; finally map the adjoint of the
initial state to dL/dphi0 and read dL/dsigma_pq.  All arithmetic runs in the library's
HIP kernels; torch only holds the buffers.
"""
import torch

from . import binding as B
from . import inputs


class NPhaseRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, sigma_pairs, cfg, steps, ckpt_every, precision):
        cfg_s = inputs.with_sigma_pairs(cfg, sigma_pairs.detach().cpu().numpy())
        sim = B.Sim(cfg_s, precision, device=str(phi0.device))
        sim.init(phi0.detach())
        ckpts = []
        t = 0
        while t < steps:
            ckpts.append((t, sim.save_state()))
            n = min(ckpt_every, steps - t)
            sim.step(n)
            t += n
        phiT = sim.fields()[0]
        ctx.sim, ctx.ckpts, ctx.steps = sim, ckpts, steps
        ctx.N = cfg["n_phases"]
        # the gradient of the pair tensions goes back where they came from
        ctx.sigma_device, ctx.sigma_dtype = sigma_pairs.device, sigma_pairs.dtype
        return phiT

    @staticmethod
    def backward(ctx, g_phiT):
        sim, ckpts = ctx.sim, ctx.ckpts
        ws = sim.adjoint_workspace()
        sim.adjoint_sigma(ws, reset=True, read=False)
        lam = sim.adjoint_seed(g_phiT)
        lam2 = torch.empty_like(lam)
        for idx in reversed(range(len(ckpts))):
            t0, buf = ckpts[idx]
            t1 = ckpts[idx + 1][0] if idx + 1 < len(ckpts) else ctx.steps
            n = t1 - t0
            sim.load_state(buf)
            states = []
            for _ in range(n):
                states.append(sim.save_state64())
                sim.step(1)
            for st in reversed(states):
                sim.adjoint_step(st, lam, lam2, ws)
                lam, lam2 = lam2, lam
        dphi0 = sim.adjoint_init(lam, ws)
        dsig = sim.adjoint_sigma(ws, reset=True)
        N = ctx.N
        pairs = [dsig[p, q] for p in range(N) for q in range(p + 1, N)]
        dpairs = torch.tensor(pairs, dtype=torch.float64).to(device=ctx.sigma_device,
                                                              dtype=ctx.sigma_dtype)
        return dphi0, dpairs, None, None, None, None


def run_differentiable(cfg, phi0, sigma_pairs, steps, ckpt_every=50, precision="fp64"):
    """Phase fields [N, *grid] after `steps` steps, differentiable w.r.t. phi0 and the pair
    tensions sigma_pairs (on phi0's CUDA device; sigma_pairs may live on the host or on
    the device, and its gradient is returned there).  Walls and gravity are covered (the
    gravity reference density depends on phi0 and enters dL/dphi0).  precision "fp64" or
    "fp32" (the forward's storage and arithmetic; the adjoint steps are FP64)."""
    return NPhaseRun.apply(phi0, sigma_pairs, cfg, int(steps), int(ckpt_every), precision)
