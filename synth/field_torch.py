"""The synthetic-field recipe of ``synth.field`` on a torch device.

Same steps (Gaussian field with P = A |m|^n_s, quadratic term, Kaiser factor
along z) in float64, with torch's Philox generator seeded per realisation
instead of numpy's PCG64, so fields are statistically identical to
``make_field`` but not bit-identical.  Used where many large realisations are
needed (ensemble statistics), where generating them on the host would
dominate the run time.
"""
from __future__ import annotations

import torch

from .field import FieldRecipe, power_amplitude


def make_field_torch(recipe: FieldRecipe, device="cuda", dtype=torch.float64) -> torch.Tensor:
    ng = recipe.ng
    vol = recipe.length ** 3
    gen = torch.Generator(device=device)
    gen.manual_seed(int(recipe.seed))
    white = torch.randn((ng, ng, ng), generator=gen, device=device, dtype=torch.float64)
    f = torch.fft.fftfreq(ng, d=1.0 / ng, device=device, dtype=torch.float64).round()
    fz = f[: ng // 2 + 1]
    m2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
    zero = m2 == 0.0
    m2s = torch.where(zero, torch.ones_like(m2), m2)
    amp = power_amplitude(recipe)
    pk = amp * torch.sqrt(m2s) ** recipe.n_s
    pk = torch.where(zero, torch.zeros_like(pk), pk)
    g = torch.fft.irfftn(torch.fft.rfftn(white) * torch.sqrt(pk * ng ** 3 / vol), s=(ng, ng, ng))
    del white
    delta_r = g + recipe.f_ng * (g * g - torch.mean(g * g))
    del g
    kaiser = 1.0 + recipe.beta * (fz[None, None, :] ** 2) / m2s
    kaiser = torch.where(zero, torch.zeros_like(kaiser), kaiser)
    delta_s = torch.fft.irfftn(torch.fft.rfftn(delta_r) * kaiser, s=(ng, ng, ng))
    return delta_s.to(dtype).contiguous()
