"""Classical transmission protocol (§4.1.1) on the GPU: the k dominant
coefficients (ascending indices, ties to the lower index) and the
reconstruction, against the oracle."""
import numpy as np
import pytest
import torch

from conftest import read_golden
from gpu_util import COMPLEX, TOL, host64, make_inputs, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import hadamard2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.float64, torch.complex128,
                                   torch.bfloat16], ids=str)
@pytest.mark.parametrize("b,n,batch,k", [(2, 10, 3, 1), (2, 10, 3, 17), (4, 7, 2, 300), (3, 8, 2, 6561),
                                         (8, 5, 2, 1000), (2, 16, 1, 4096)])
def test_topk_and_reconstruction(b, n, batch, k, dtype):
    say(f"compress b={b} n={n} k={k} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=1500 + b + n + k)
    plan = G.Plan(b, n, batch, dtype)
    idx, val, recon = plan.compress(W, x, k)
    y = plan.forward(W, x)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy()
    val64 = host64(val)
    y64 = host64(y)
    for i in range(batch):
        ii = idx[i]
        assert np.all(np.diff(ii) > 0)                       # ascending, unique
        np.testing.assert_array_equal(val64[i], y64[i][ii])  # values are the coefficients
        mag = np.abs(y64[i].astype(np.complex128)) ** 2
        rest = np.setdiff1d(np.arange(b ** n), ii)
        if rest.size:
            assert mag[ii].min() >= mag[rest].max() * (1 - 1e-6)  # a valid top-k
        # kept energy against the oracle's coefficients (independent of near-ties)
        ref = O.staged(W64, x64[i], n)
        _, kept_ref, _ = O.topk_compress(W64, x64[i], n, k)
        e_gpu = np.sum(np.abs(ref[ii]) ** 2)
        e_ref = np.sum(np.abs(kept_ref) ** 2)
        assert abs(e_gpu - e_ref) <= 10 * TOL[dtype] * np.sum(np.abs(ref) ** 2)
        # reconstruction = adjoint of the kept coefficients
        sparse = np.zeros(b ** n, dtype=np.complex128 if dtype in COMPLEX else np.float64)
        sparse[ii] = val64[i]
        rr = O.adjoint(W64, sparse, n)
        assert rel_err(host64(recon[i]), rr) < 3 * TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.int32, torch.float64], ids=str)
def test_ties_go_to_lower_index(dtype):
    # x = e_0 under the Hadamard: every coefficient has the same magnitude
    n, k = 9, 37
    W = hadamard2(dtype != torch.int32)
    x = np.zeros((2, 1 << n))
    x[:, 0] = 1 if dtype == torch.int32 else 3.0
    xt = torch.from_numpy(x).to(dtype).cuda()
    Wt = torch.from_numpy(W).to(G.W_DTYPE[dtype]).cuda()
    idx, val, _ = G.Plan(2, n, 2, dtype).compress(Wt, xt, k, reconstruct=False)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.tile(np.arange(k), (2, 1)))


# few large instances: the selection runs on many work-groups per instance
# (chunks of 4096 elements); ties across chunk boundaries, k = 1 and k = N
@pytest.mark.parametrize("dtype", [torch.float32, torch.int32, torch.float64], ids=str)
@pytest.mark.parametrize("n,k", [(15, 37), (16, 5000), (16, 1), (14, 1 << 14)])
def test_chunked_selection_ties_and_extremes(dtype, n, k):
    say(f"chunked top-k ties n={n} k={k} dtype={dtype}")
    W = hadamard2(dtype != torch.int32)
    x = np.zeros((3, 1 << n))
    x[:, 0] = 1 if dtype == torch.int32 else 3.0
    xt = torch.from_numpy(x).to(dtype).cuda()
    Wt = torch.from_numpy(W).to(G.W_DTYPE[dtype]).cuda()
    idx, val, _ = G.Plan(2, n, 3, dtype).compress(Wt, xt, k, reconstruct=False)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.tile(np.arange(k), (3, 1)))


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.bfloat16], ids=str)
def test_chunked_selection_full_size(dtype):
    # 16 x 2^20 with k = N / 64 (the transmission workload's shape): indices
    # against the oracle's on two instances, every instance a valid top-k
    b, n, batch, k = 2, 20, 16, (1 << 20) // 64
    say(f"chunked top-k 16 x 2^20 k={k} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=1700)
    plan = G.Plan(b, n, batch, dtype)
    idx, val, _ = plan.compress(W, x, k, reconstruct=False)
    y = plan.forward(W, x)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy()
    y64 = host64(y)
    for i in range(batch):
        ii = idx[i]
        assert np.all(np.diff(ii) > 0)
        mag = np.abs(y64[i]) ** 2
        thr = np.sort(mag)[-k]
        assert np.all(mag[ii] >= thr) and np.count_nonzero(mag > thr) <= k
    if dtype == torch.float32:
        for i in (0, 15):
            ridx, _, _ = O.topk_compress(W64, x64[i], n, k)
            ref = O.staged(W64, x64[i], n)
            # identical up to near-ties at the threshold (compare the kept energy)
            e_gpu, e_ref = np.sum(np.abs(ref[idx[i]]) ** 2), np.sum(np.abs(ref[ridx]) ** 2)
            assert abs(e_gpu - e_ref) <= 1e-5 * np.sum(np.abs(ref) ** 2)


def test_table1_hadamard_fidelity_on_gpu():
    d = read_golden("table1_hadamard.txt")
    H = torch.from_numpy(hadamard2(True)).to(torch.complex128).cuda()
    for lab in ("S1", "S2", "S3"):
        vals = d[lab]
        psi = np.array(vals[:8])
        x = torch.from_numpy(psi).cuda().reshape(1, 8)
        idx, val, recon = G.Plan(2, 3, 1, torch.complex128).compress(H, x, 2)
        torch.cuda.synchronize()
        F = O.fidelity(psi, recon.cpu().numpy()[0])
        assert abs(F - vals[8].real) < 1.5e-3, (lab, F)
