"""Natural-order filter (§4.3, Alg. 3 without the ancilla qubit): GPU against
the oracle, including the paper's printed N = 16 example."""
import numpy as np
import pytest
import torch

from conftest import read_golden
from gpu_util import COMPLEX, TOL, host64, make_inputs, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import u3

pytestmark = pytest.mark.gpu


def test_filter_paper_example_on_gpu():
    d = read_golden("filter_example.txt")
    W = u3(np.pi / 4, 0.0, np.pi).real
    psi = np.array(d["psi"])
    psi = psi / np.linalg.norm(psi)
    x = torch.from_numpy(psi).cuda().reshape(1, 16)
    Wt = torch.from_numpy(W).cuda()
    plan = G.Plan(2, 4, 1, torch.float64)
    lo, hi = plan.filter(Wt, x, 4)
    torch.cuda.synchronize()
    np.testing.assert_allclose(lo.cpu().numpy()[0], d["low"], atol=6e-5)
    np.testing.assert_allclose(hi.cpu().numpy()[0], d["high"], atol=6e-5)
    np.testing.assert_allclose(plan.forward(Wt, x).cpu().numpy()[0], d["spectrum"], atol=6e-5)


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.float64], ids=str)
@pytest.mark.parametrize("b,n,batch,cut", [(2, 12, 3, 100), (3, 9, 2, 5000), (4, 8, 2, 1), (8, 5, 2, 32767),
                                           (2, 16, 2, 1 << 15), (4, 8, 1, 0), (4, 8, 1, 1 << 30)])
def test_filter_matches_oracle(b, n, batch, cut, dtype):
    say(f"filter b={b} n={n} cut={cut} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=1300 + b + n)
    plan = G.Plan(b, n, batch, dtype)
    lo, hi = plan.filter(W, x, cut)
    torch.cuda.synchronize()
    for i in range(batch):
        rlo, rhi = O.natural_filter(W64, x64[i], n, cut)
        scale = np.linalg.norm(x64[i])
        assert np.linalg.norm(host64(lo[i]) - rlo) / scale < 3 * TOL[dtype]
        assert np.linalg.norm(host64(hi[i]) - rhi) / scale < 3 * TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16, torch.float32], ids=str)
@pytest.mark.parametrize("b,n,batch,cut", [(16, 3, 2, 1000), (32, 2, 3, 1), (16, 4, 1, 40000), (32, 3, 1, 0),
                                           (32, 2, 2, 1 << 20)])
def test_filter_matrix_core(b, n, batch, cut, dtype):
    # radix 16 / 32: the natural-order mask is applied while the first
    # inverse group loads its tile on the matrix-core path
    say(f"filter mfma b={b} n={n} cut={cut} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=1400 + b + n)
    plan = G.Plan(b, n, batch, dtype)
    assert all(g["kind"] == "mfma" for g in plan.describe()["groups"])
    lo, hi = plan.filter(W, x, cut)
    torch.cuda.synchronize()
    for i in range(batch):
        rlo, rhi = O.natural_filter(W64, x64[i], n, cut)
        scale = np.linalg.norm(x64[i])
        assert np.linalg.norm(host64(lo[i]) - rlo) / scale < 3 * TOL[dtype]
        assert np.linalg.norm(host64(hi[i]) - rhi) / scale < 3 * TOL[dtype]
