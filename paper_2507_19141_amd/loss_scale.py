"""Dynamic loss scaling for the BF16 form of the deformation path.

The upstream gradient of the decoder output is multiplied by the scale S inside the
backward kernels (before any BF16 rounding), and every FP32 gradient the path
accumulates (table, decoder parameters) is multiplied by 1/S when it is written.
After a backward, `observe` enqueues the library's non-finite count on those
gradients; `update` reads it once per step: on overflow the step is to be skipped
and S halves, after `growth_interval` clean steps S doubles.
"""
from __future__ import annotations


class DynamicLossScaler:
    def __init__(self, init_scale: float = 2.0 ** 12, growth_interval: int = 2000, factor: float = 2.0,
                 min_scale: float = 1.0, max_scale: float = 2.0 ** 24, device: str = "cuda"):
        import torch
        self.scale = float(init_scale)
        self.growth_interval = int(growth_interval)
        self.factor = float(factor)
        self.min_scale = float(min_scale)
        self.max_scale = float(max_scale)
        self.good_steps = 0
        self.skipped = 0
        self.counter = torch.zeros(1, dtype=torch.int32, device=device)

    def observe(self, *grads) -> None:
        """Enqueue the non-finite count of each FP32 gradient tensor (no host sync)."""
        from . import _lib
        for g in grads:
            if g is not None and g.numel():
                _lib.h4d_count_nonfinite(g, g.numel(), self.counter)

    def update(self) -> bool:
        """Consume the count of this step: True if the step may be applied."""
        bad = int(self.counter.item())
        self.counter.zero_()
        if bad:
            self.scale = max(self.scale / self.factor, self.min_scale)
            self.good_steps = 0
            self.skipped += 1
            return False
        self.good_steps += 1
        if self.good_steps >= self.growth_interval:
            self.scale = min(self.scale * self.factor, self.max_scale)
            self.good_steps = 0
        return True

    def state_dict(self) -> dict:
        return {"scale": self.scale, "good_steps": self.good_steps, "skipped": self.skipped}

    def load_state_dict(self, d: dict) -> None:
        self.scale = float(d["scale"])
        self.good_steps = int(d["good_steps"])
        self.skipped = int(d.get("skipped", 0))
