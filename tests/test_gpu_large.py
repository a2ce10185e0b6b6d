"""Transforms with more than 2^31 elements in one launch (64-bit offsets on
every path).  The input is a Kronecker power u^{⊗n} (per instance), so by the
mixed-product property of the Kronecker product (Def. 2.4) the output is
(W u)^{⊗n}: every element has the closed form y_p = Π_j (W u)[p_j], checked
on sampled indices (the first, the last, around 2^31, and random ones)."""
import numpy as np
import pytest
import torch

from gpu_util import say
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import haar_unitary

pytestmark = pytest.mark.gpu


def _kron_power(u: torch.Tensor, n: int) -> torch.Tensor:
    v = u.clone()
    for _ in range(n - 1):
        v = torch.outer(v, u).reshape(-1)
    return v


def _digits(p: np.ndarray, b: int, n: int) -> np.ndarray:
    d = np.empty((p.size, n), dtype=np.int64)
    q = p.copy()
    for j in range(n):
        d[:, j] = q % b
        q //= b
    return d


def _sample_indices(N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    edge = [0, 1, N - 1, N - 2]
    edge += [v for v in (2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1) if v < N]
    return np.unique(np.concatenate([np.array(edge, dtype=np.int64), rng.integers(0, N, 4000)]))


def _need(bytes_: int):
    free, _ = torch.cuda.mem_get_info()
    if free < bytes_:
        pytest.skip(f"needs {bytes_ / 2**30:.0f} GiB of free device memory")


def test_f32_radix2_2pow31_elements():
    b, n = 2, 31
    N = b ** n
    _need(3 * N * 4)
    say(f"f32 b={b} n={n}: N = {N}")
    W64 = haar_unitary(b, 101, complex_=False)
    u64 = np.array([0.8, -0.6])
    W = torch.from_numpy(W64).to(torch.float32).cuda()
    x = _kron_power(torch.from_numpy(u64).to(torch.float32).cuda(), n).reshape(1, N)
    plan = G.Plan(b, n, 1, torch.float32)
    y = plan.forward(W, x)
    torch.cuda.synchronize()
    wu = W.double().cpu().numpy() @ u64.astype(np.float32).astype(np.float64)
    p = _sample_indices(N, 7)
    expect = np.prod(wu[_digits(p, b, n)], axis=1)
    got = y.reshape(-1)[torch.from_numpy(p).cuda()].double().cpu().numpy()
    scale = np.abs(wu).max() ** n
    assert np.max(np.abs(got - expect)) < 1e-5 * scale


def test_c64_radix8_two_instances_beyond_2pow31():
    b, n, batch = 8, 10, 2
    N = b ** n
    _need(3 * batch * N * 8)
    say(f"c64 b={b} n={n} batch={batch}: {batch * N} elements")
    W64 = haar_unitary(b, 102)
    W = torch.from_numpy(W64.astype(np.complex64)).cuda()
    rng = np.random.default_rng(103)
    us = []
    x = torch.empty(batch, N, dtype=torch.complex64, device="cuda")
    for i in range(batch):
        u = rng.standard_normal(b) + 1j * rng.standard_normal(b)
        u /= np.linalg.norm(u)
        us.append(u.astype(np.complex64).astype(np.complex128))
        x[i] = _kron_power(torch.from_numpy(u.astype(np.complex64)).cuda(), n)
    plan = G.Plan(b, n, batch, torch.complex64)
    y = plan.forward(W, x)
    xi = plan.inverse(W, y)
    torch.cuda.synchronize()
    W64s = W.cpu().numpy().astype(np.complex128)
    p = _sample_indices(N, 9)
    idx = torch.from_numpy(p).cuda()
    for i in range(batch):
        wu = W64s @ us[i]
        expect = np.prod(wu[_digits(p, b, n)], axis=1)
        got = y[i][idx].cpu().numpy().astype(np.complex128)
        scale = np.abs(wu).max() ** n
        assert np.max(np.abs(got - expect)) < 1e-5 * scale, i
        # inverse of forward recovers the Kronecker input (W unitary)
        back = xi[i][idx].cpu().numpy().astype(np.complex128)
        ref = np.prod(us[i][_digits(p, b, n)], axis=1)
        assert np.max(np.abs(back - ref)) < 1e-5 * np.abs(us[i]).max() ** n, i
