"""Plan instrumentation through the C ABI: per-launch HIP-event timing and
its name filter (only matching launches record events)."""
import pytest
import torch

from gpu_util import make_inputs, say
from paper_2507_02420_amd import gtt as G

pytestmark = pytest.mark.gpu


def test_timing_filter_selects_launches():
    b, n, batch, dtype = 4, 9, 3, torch.complex64
    say("timing filter c64 b=4 n=9")
    x, W, _, _ = make_inputs(b, n, batch, dtype, seed=77)
    plan = G.Plan(b, n, batch, dtype)
    y = torch.empty_like(x)
    plan.timing(True)
    for _ in range(3):
        plan.forward(W, x, y)
    everything = plan.timing_read()
    assert len(everything) == len(plan.describe()["groups"]) >= 2, everything
    first = sorted(everything)[0]
    plan.timing_filter(first)
    for _ in range(4):
        plan.forward(W, x, y)
    only = plan.timing_read()
    assert list(only) == [first] and only[first]["launches"] == 4, only
    plan.timing_filter("no launch has this name")
    plan.forward(W, x, y)
    assert plan.timing_read() == {}
    plan.timing_filter(None)
    plan.forward(W, x, y)
    plan.timing(False)
    assert set(plan.timing_read()) == set(everything)
