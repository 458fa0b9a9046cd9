"""Device plumbing from PyTorch: the arena (one uint8 tensor in HBM) and two
HIP streams.  Every computation runs in libcdagx.so; this module only hands it
memory and streams, and refuses to run without a GPU."""
from __future__ import annotations

from typing import Optional

from .binding import Context


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the contraction engine has no CPU path")
    return torch


class DeviceRunner:
    """Binds a Context to cuda:<device> with a torch-allocated arena sized from the plan."""

    def __init__(self, ctx: Context, device: int = 0):
        torch = require_gpu()
        self.torch = torch
        self.ctx = ctx
        self.device = device
        self.dev = torch.device("cuda", device)
        with torch.cuda.device(device):
            self.compute = torch.cuda.Stream(device=self.dev)
            self.copy = torch.cuda.Stream(device=self.dev)
        self.arena: Optional["torch.Tensor"] = None
        ctx.bind_device(device, self.compute.cuda_stream, self.copy.cuda_stream)

    def ensure_arena(self, nbytes: int):
        if self.arena is None or self.arena.numel() < nbytes:
            self.arena = None
            self.torch.cuda.empty_cache()
            self.arena = self.torch.empty(max(256, nbytes), dtype=self.torch.uint8, device=self.dev)
            self.ctx.bind_arena(self.arena.data_ptr(), self.arena.numel())

    def autotune(self, prec="fp64", batched=True, reps=3, in_situ=False, uniform=False):
        """Size the arena for the plan (with room for every variant's workspace),
        then let the library pick kernel variants."""
        plan = self.ctx.plan(prec, batched)
        self.ensure_arena(int(plan["arena_bytes"] * 1.25) + (1 << 20))
        return self.ctx.autotune(prec, batched, reps, in_situ, uniform)

    def run(self, prec="fp64", batched=False):
        plan = self.ctx.plan(prec, batched)
        self.ensure_arena(plan["arena_bytes"])
        return self.ctx.execute(prec, batched)
