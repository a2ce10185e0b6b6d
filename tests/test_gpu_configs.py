"""The benchmark's secondary workloads at their full sizes and in the launch
configuration the benchmark times, every instance checked against the FP64
oracle (computed in chunks of instances): 64 x complex64 radix 4 (forward
and inverse), 16 x float32 radix 3 with n = 13 (odd strides), 16 x int32
unnormalised Hadamard radix 2 with n = 20 (bit-exact), and the plain-FP32
form of the 1024-instance ragged batch (sampled instances)."""
import numpy as np
import pytest
import torch

from gpu_util import TOL, host64, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import gaussian, hadamard2, haar_unitary, int_uniform, ragged_shapes, uniform

pytestmark = pytest.mark.gpu


def test_c64_radix4_n10_batch64_forward_inverse():
    b, n, batch = 4, 10, 64
    say("64 x c64 b=4 n=10")
    x = torch.from_numpy(gaussian((batch, b ** n), seed=21, complex_=True).astype(np.complex64)).cuda()
    W = torch.from_numpy(haar_unitary(4, 22).astype(np.complex64)).cuda()
    plan = G.Plan(b, n, batch, torch.complex64)
    y = plan.forward(W, x)
    xr = plan.inverse(W, y)
    torch.cuda.synchronize()
    W64 = host64(W)
    for c0 in range(0, batch, 8):
        x64 = host64(x[c0:c0 + 8])
        assert rel_err(host64(y[c0:c0 + 8]), O.staged(W64, x64, n)) < TOL[torch.complex64], c0
        assert rel_err(host64(xr[c0:c0 + 8]), O.adjoint(W64, host64(y[c0:c0 + 8]), n)) < TOL[torch.complex64], c0
    assert rel_err(host64(xr), host64(x)) < 3 * TOL[torch.complex64]


def test_f32_radix3_n13_batch16():
    b, n, batch = 3, 13, 16
    say("16 x f32 b=3 n=13")
    x = torch.from_numpy(uniform((batch, b ** n), seed=31).astype(np.float32)).cuda()
    W = torch.from_numpy(haar_unitary(3, 32, complex_=False).astype(np.float32)).cuda()
    plan = G.Plan(b, n, batch, torch.float32)
    y = plan.forward(W, x)
    xr = plan.inverse(W, y)
    torch.cuda.synchronize()
    for c0 in range(0, batch, 4):
        x64 = host64(x[c0:c0 + 4])
        assert rel_err(host64(y[c0:c0 + 4]), O.staged(host64(W), x64, n)) < TOL[torch.float32], c0
    assert rel_err(host64(xr), host64(x)) < 3 * TOL[torch.float32]


def test_int32_hadamard_radix2_n20_batch16_exact():
    b, n, batch = 2, 20, 16
    say("16 x int32 Hadamard b=2 n=20")
    x = torch.from_numpy(int_uniform((batch, b ** n), seed=33, lo=-100, hi=100)).to(torch.int32).cuda()
    H = torch.from_numpy(hadamard2(False)).to(torch.int32).cuda()
    plan = G.Plan(b, n, batch, torch.int32)
    y = plan.forward(H, x)
    xr = plan.inverse(H, y)
    torch.cuda.synchronize()
    # every instance against the exact integer oracle (|y| <= 100 * 2^20)
    H64 = hadamard2(False).astype(np.int64)
    for r in range(batch):
        ref = O.staged_int32(H64, x[r].cpu().numpy().astype(np.int64), n)
        assert np.array_equal(y[r].cpu().numpy(), ref), r
    assert torch.equal(xr, x * (1 << n))


def test_ragged_1024_plain_fp32_sampled():
    # the comparison path of the ragged batch: the same plan in float32
    # (radix 16 / 32 on the FP32 matrix cores), default per-phase launches
    shapes = ragged_shapes(1024, seed=52)
    say("ragged 1024 f32")
    Ns = [b ** n for b, n in shapes]
    offs = np.cumsum([0] + Ns[:-1])
    total = int(sum(Ns))
    rng = np.random.default_rng(53)
    xt = torch.from_numpy(rng.standard_normal(total, dtype=np.float32)).cuda()
    Ws = [haar_unitary(r, 54 + i, complex_=False).astype(np.float32) for i, r in enumerate((2, 4, 16, 32))]
    Wt = torch.cat([torch.from_numpy(w).reshape(-1) for w in Ws]).cuda()
    ridx = {2: 0, 4: 1, 16: 2, 32: 3}
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, torch.float32)
    y = plan.forward(Wt, xt)
    torch.cuda.synchronize()
    sample = list(range(0, 1024, 41))
    for b in (2, 4, 16, 32):  # the largest instance of every radix
        sample.append(max((t for t in range(1024) if shapes[t][0] == b), key=lambda t: Ns[t]))
    for t in sample:
        b, n = shapes[t]
        o, N = int(offs[t]), Ns[t]
        ref = O.staged(Ws[ridx[b]].astype(np.float64), host64(xt[o:o + N]), n)
        e = rel_err(host64(y[o:o + N]), ref)
        assert e < TOL[torch.float32], (t, b, n, e)
