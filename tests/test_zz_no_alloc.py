"""The allocation-free entry point hfsi_mass_norm_noalloc against
hfsi_mass_norm, through the C ABI: two calls in a row on the same GPU (they
share the scratch array), the second on a smaller mesh; and the result left
in device memory by a call that the host does not wait for."""
import numpy as np
import pytest

import synth
from gpu_helpers import context_for, torch_dev

pytestmark = pytest.mark.gpu


def _norms(lib, prob, seed):
    import torch
    ctx = context_for(lib, prob)
    dv = torch_dev(synth.random_state(prob, seed, u_scale=0.05, p_scale=0.3).ravel())
    ref = ctx.mass_norm(dv)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.mass_norm_noalloc(dv, out)
    torch.cuda.synchronize()
    return ref, float(out.item()), ctx


def test_mass_norm_noalloc_matches_the_allocating_call(lib):
    print("[noalloc] cube10 then cube4", flush=True)
    big = synth.cube_problem(10, jitter=0.1, seed=1)
    small = synth.cube_problem(4, jitter=0.1, seed=2)
    r1, g1, c1 = _norms(lib, big, 3)
    r2, g2, c2 = _norms(lib, small, 4)
    print(f"[noalloc] {g1!r} vs {r1!r}; {g2!r} vs {r2!r}", flush=True)
    assert abs(g1 - r1) <= 1e-14 * r1
    assert abs(g2 - r2) <= 1e-14 * r2
    assert abs(g1 - g2) > 1e-6 * r1  # different inputs, no stale partials
    # back to the larger mesh's context: the scratch now holds the smaller
    # mesh's partials, which the next call overwrites
    import torch
    dv = torch_dev(synth.random_state(big, 3, u_scale=0.05, p_scale=0.3).ravel())
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    c1.mass_norm_noalloc(dv, out)
    torch.cuda.synchronize()
    assert abs(float(out.item()) - r1) <= 1e-14 * r1


def test_mass_norm_noalloc_checks_arguments(lib):
    import torch
    ctx = lib.Context(0)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.HfsiError):
        ctx.mass_norm_noalloc(out, out)  # no mesh yet
    prob = synth.cube_problem(2)
    ctx.set_problem(prob)
    with pytest.raises(lib.HfsiError):
        ctx.mass_norm_noalloc(None, out)
