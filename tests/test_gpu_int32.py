"""Bit-exact int32 transforms (arithmetic mod 2^32) against the exact oracle."""
import numpy as np
import pytest
import torch

from gpu_util import say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import hadamard2, int_uniform

pytestmark = pytest.mark.gpu


# n = 5..10 run the wave form (digits in registers and across lanes)
@pytest.mark.parametrize("n,batch", [(1, 3), (5, 2), (6, 5), (8, 3), (9, 1), (10, 7), (13, 2), (16, 3), (20, 2)])
def test_hadamard_int32_bit_exact(n, batch):
    say(f"int32 hadamard n={n} batch={batch}")
    H = hadamard2(False).astype(np.int64)
    x = int_uniform((batch, 1 << n), seed=33 + n, lo=-100, hi=100)
    xt = torch.from_numpy(x).to(torch.int32).cuda()
    Wt = torch.from_numpy(H).to(torch.int32).cuda()
    plan = G.Plan(2, n, batch, torch.int32)
    y = plan.forward(Wt, xt)
    back = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    ref = O.staged_int32(H, x, n)
    assert np.array_equal(y.cpu().numpy(), ref)
    assert np.array_equal(back.cpu().numpy().astype(np.int64), x * (1 << n))


@pytest.mark.parametrize("b,n", [(2, 7), (2, 10), (3, 7), (4, 6), (5, 4), (7, 4), (11, 3)])
def test_general_int32_wraparound(b, n):
    say(f"int32 general b={b} n={n}")
    rng = np.random.default_rng(b * 100 + n)
    W = rng.integers(-70000, 70000, size=(b, b))
    x = rng.integers(-2 ** 31, 2 ** 31, size=(2, b ** n))
    xt = torch.from_numpy(x).to(torch.int32).cuda()
    Wt = torch.from_numpy(W).to(torch.int32).cuda()
    y = G.Plan(b, n, 2, torch.int32).forward(Wt, xt)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), O.staged_int32(W, x, n))
