"""The non-allocating mass reduction (swe_mass_noalloc) against swe_mass: the
same FP64 value, bit for bit, on two calls in a row through the C ABI, the
second on a smaller mesh (the fixed array keeps the first call's partial
sums, which the second must not read), in both precisions; a mesh beyond the
array's size is refused before anything is enqueued."""
import sys

import numpy as np
import pytest

from paper_2311_11348_amd import inputs as I
from paper_2311_11348_amd import swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mass_both(prob, precision, steps):
    import torch
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    with swe.context_for(prob, precision=precision) as ctx:
        ctx.set_state_fn(prob.ic)
        ctx.step(steps, prob.dt())
        ctx.mass_noalloc(out.data_ptr())
        ctx.sync()
        torch.cuda.synchronize()
        got = float(out.item())
        ref = ctx.mass()
    return got, ref


@pytest.mark.parametrize("precision", [swe.SWE_FP64, swe.SWE_FP32_WB])
def test_mass_noalloc_equals_mass(precision):
    big = I.config_c3(n=160)                      # 51,200 elements: 200 partial sums
    small = I.config_c1(n=20, p=2)                # 800 elements: 4 partial sums
    for name, prob, steps in (("larger", big, 3), ("smaller", small, 5)):
        got, ref = _mass_both(prob, precision, steps)
        say(f"precision {precision} {name} mesh ({prob.mesh.ne} elements): noalloc {got!r}, swe_mass {ref!r}")
        assert np.isfinite(got)
        assert got == ref


def test_mass_noalloc_refuses_a_mesh_beyond_its_array():
    n = 1449                                      # 2 * 1449^2 = 4,199,202 > 4,194,304 elements
    mesh = I.structured_mesh(n)
    prob = I._problem("big", mesh, I.bathy_flat(10.0), I.ic_rest(0.0), 1, 1, 1)
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with swe.context_for(prob) as ctx:
        with pytest.raises(swe.SweError) as ei:
            ctx.mass_noalloc(out.data_ptr())
    assert ei.value.status == swe.SWE_EINVAL and "4194304" in str(ei.value)
