"""GPU parity of forward and inverse against the FP64 oracle, element by
element, over radices, digit counts, batch sizes, dtypes and edge cases
(sizes span several tiles and more than one digit group, ragged column
blocks for odd radices, n = 0 and n = 1)."""
import numpy as np
import pytest
import torch

from gpu_util import COMPLEX, TOL, host64, make_inputs, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import gaussian

pytestmark = pytest.mark.gpu

FLOAT_DTYPES = [torch.float64, torch.float32, torch.complex64, torch.complex128, torch.bfloat16, torch.float16]

# (b, n): small, multi-tile single group, and multi-group shapes
SHAPES = [(2, 1), (2, 5), (2, 12), (2, 17), (3, 1), (3, 7), (3, 11), (4, 3), (4, 7), (4, 9),
          (5, 4), (5, 7), (6, 3), (6, 6), (7, 3), (7, 6), (8, 2), (8, 4), (8, 6),
          (9, 3), (11, 3), (16, 3), (32, 2), (16, 4)]


def _skip_big(b, n, batch, dtype):
    return (b ** n) * batch > (1 << 20) and dtype in (torch.complex128,)


@pytest.mark.parametrize("dtype", FLOAT_DTYPES, ids=str)
@pytest.mark.parametrize("b,n", SHAPES)
def test_forward_matches_oracle(b, n, dtype):
    batch = 3
    if _skip_big(b, n, batch, dtype):
        pytest.skip("size")
    say(f"forward b={b} n={n} batch={batch} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=1000 + 17 * b + n)
    plan = G.Plan(b, n, batch, dtype)
    y = plan.forward(W, x)
    torch.cuda.synchronize()
    ref = O.staged(W64, x64, n)
    err = rel_err(host64(y), ref)
    assert err < TOL[dtype], (b, n, dtype, err, plan.describe())


# odd and non-power-of-two radices: scalar tiles (16-byte vectors do not
# fit b^k elements) take their addresses from a walk -- contiguous tiles and
# row tiles (at most 256 columns, so a thread keeps its column; shapes whose
# rows the planner would make wider are among these), with a partial last
# column block, through the single-tile load and the prefetching persistent
# loop (more tiles than the resident grid)
@pytest.mark.parametrize("b,n,batch,dtype", [
    (3, 9, 3, torch.float64), (3, 12, 8, torch.float32), (6, 6, 5, torch.float32), (6, 6, 64, torch.float32),
    (7, 5, 16, torch.complex64), (7, 5, 64, torch.float32), (6, 5, 16, torch.float64), (5, 8, 8, torch.float32),
    (3, 11, 16, torch.bfloat16), (3, 12, 24, torch.float32), (7, 5, 512, torch.float32)], ids=str)
def test_scalar_tile_walks(b, n, batch, dtype):
    say(f"scalar walk b={b} n={n} batch={batch} dtype={dtype}")
    plan = G.Plan(b, n, batch, dtype)
    groups = plan.describe()["groups"]
    assert any(g["mode"] in (1, 3) for g in groups), groups  # a scalar tile mode is exercised
    assert all(g["C"] <= 256 for g in groups if g["mode"] == 3), groups
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=5000 + 31 * b + n)
    y = plan.forward(W, x)
    xi = plan.inverse(W, x)
    torch.cuda.synchronize()
    assert rel_err(host64(y), O.staged(W64, x64, n)) < TOL[dtype], (b, n, batch, dtype, plan.describe())
    assert rel_err(host64(xi), O.adjoint(W64, x64, n)) < TOL[dtype], (b, n, batch, dtype)


# complex radix 8: every (digits, tile) variant of the matrix-core pass with
# per-lane addresses (1-4 digits, 2048 / 4096 element tiles, contiguous and
# strided groups) and the general kernel (8192 element tiles)
@pytest.mark.parametrize("n,batch", [(1, 512), (2, 64), (3, 4), (3, 8), (4, 2), (5, 3), (6, 8), (7, 1), (8, 1)])
def test_c64_radix8_tiles_forward_inverse(n, batch):
    b, dtype = 8, torch.complex64
    say(f"forward/inverse c64 b=8 n={n} batch={batch}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=3000 + n)
    plan = G.Plan(b, n, batch, dtype)
    y = plan.forward(W, x)
    xi = plan.inverse(W, x)
    torch.cuda.synchronize()
    assert rel_err(host64(y), O.staged(W64, x64, n)) < TOL[dtype]
    assert rel_err(host64(xi), O.adjoint(W64, x64, n)) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.float64, torch.bfloat16], ids=str)
@pytest.mark.parametrize("b,n", [(2, 14), (3, 9), (4, 8), (5, 5), (8, 5), (16, 3)])
def test_inverse_matches_oracle_and_roundtrip(b, n, dtype):
    batch = 2
    say(f"inverse b={b} n={n} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=2000 + 13 * b + n)
    plan = G.Plan(b, n, batch, dtype)
    xi = plan.inverse(W, x)
    torch.cuda.synchronize()
    assert rel_err(host64(xi), O.adjoint(W64, x64, n)) < TOL[dtype]
    # forward then inverse recovers x (W unitary)
    y = plan.forward(W, x)
    back = plan.inverse(W, y)
    torch.cuda.synchronize()
    assert rel_err(host64(back), x64) < 3 * TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.bfloat16], ids=str)
@pytest.mark.parametrize("b,n", [(2, 16), (3, 10), (4, 8), (8, 5)])
def test_in_place(b, n, dtype):
    say(f"in-place b={b} n={n} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, 2, dtype, seed=3000 + b + n)
    plan = G.Plan(b, n, 2, dtype)
    plan.forward(W, x, y=x)
    torch.cuda.synchronize()
    assert rel_err(host64(x), O.staged(W64, x64, n)) < TOL[dtype]


@pytest.mark.parametrize("dtype", FLOAT_DTYPES + [torch.int32], ids=str)
def test_n_zero_is_identity(dtype):
    say(f"n=0 dtype={dtype}")
    x = torch.arange(5, dtype=torch.float64).to(dtype).cuda().reshape(5, 1)
    W = torch.eye(3, dtype=G.W_DTYPE[dtype]).cuda()
    plan = G.Plan(3, 0, 5, dtype)
    y = plan.forward(W, x)
    torch.cuda.synchronize()
    assert torch.equal(y.cpu(), x.cpu())


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.float64, torch.complex128, torch.bfloat16,
                                   torch.int32], ids=str)
def test_signed_permutation_w_is_exact(dtype):
    # products with 0 and +-1 and sums with exact zeros are exact in every
    # dtype; complex data is compared in both components
    b, n, batch = 4, 7, 2
    say(f"signed permutation dtype={dtype}")
    perm = np.array([2, 0, 3, 1])
    sign = np.array([1, -1, -1, 1])
    Wn = np.zeros((4, 4))
    Wn[np.arange(4), perm] = sign
    rng = np.random.default_rng(7)
    if dtype == torch.int32:
        xn = rng.integers(-1000, 1000, size=(batch, b ** n))
    elif dtype in COMPLEX:
        xn = rng.standard_normal((batch, b ** n)) + 1j * rng.standard_normal((batch, b ** n))
    else:
        xn = rng.standard_normal((batch, b ** n))
    xt = torch.from_numpy(xn).to(dtype).cuda()
    Wt = torch.from_numpy(Wn).to(G.W_DTYPE[dtype]).cuda()
    y = G.Plan(b, n, batch, dtype).forward(Wt, xt)
    torch.cuda.synchronize()
    wide = torch.complex128 if dtype in COMPLEX else torch.float64
    x64 = xt.cpu().to(wide).numpy()
    ref = O.staged(Wn, x64, n)
    got = y.cpu().to(wide).numpy()
    if dtype in COMPLEX:
        assert np.array_equal(got.real, ref.real) and np.array_equal(got.imag, ref.imag)
        assert np.count_nonzero(ref.imag) > 0
    else:
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("which", ["hadamard", "orthogonal"])
def test_single_fp64_vector_b2_n10_against_dense(which):
    # one f64 vector, N = 2^10, x ~ N(0,1) (seed 11); W the normalised 2 x 2
    # Hadamard matrix or a 2 x 2 orthogonal matrix from QR of a Gaussian
    # (seed 12); checked against the dense 1024 x 1024 Kronecker matvec
    # (Def. 2.4) at 1e-12, and the Hadamard case also against the Sylvester
    # matrix (the Hadamard reduction of §2.6)
    from paper_2507_02420_amd.inputs import gaussian, hadamard2, haar_unitary
    b, n = 2, 10
    say(f"single f64 vector b=2 n=10 W={which}")
    Wn = hadamard2(True) if which == "hadamard" else haar_unitary(2, 12, complex_=False)
    xn = gaussian(b ** n, seed=11)
    xt = torch.from_numpy(xn).cuda().reshape(1, -1)
    Wt = torch.from_numpy(Wn).cuda()
    plan = G.Plan(b, n, 1, torch.float64)
    y = plan.forward(Wt, xt)
    back = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    got = host64(y)[0]
    ref = O.dense(Wn, xn, n)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
    if which == "hadamard":
        syl = O.sylvester_hadamard(n) / 2 ** (n / 2)
        assert np.linalg.norm(got - syl @ xn) / np.linalg.norm(xn) < 1e-12
    assert np.linalg.norm(host64(back)[0] - xn) / np.linalg.norm(xn) < 1e-12


def test_dft_base_matrix_is_fftn_on_gpu():
    # W = DFT_3: the transform is the 13-dimensional DFT of the 3 x ... x 3 array
    from paper_2507_02420_amd.inputs import dft_matrix
    b, n, batch = 3, 13, 2
    say("dft3 n=13")
    x, W, x64, W64 = make_inputs(b, n, batch, torch.complex64, seed=31, W=dft_matrix(3))
    y = G.Plan(b, n, batch, torch.complex64).forward(W, x)
    torch.cuda.synchronize()
    ref = np.fft.fftn(x64.reshape([batch] + [b] * n), axes=tuple(range(1, n + 1)), norm="ortho").reshape(batch, -1)
    assert rel_err(host64(y), ref) < 1e-5


def test_determinism_bitwise():
    b, n, batch = 4, 9, 3
    x, W, _, _ = make_inputs(b, n, batch, torch.complex64, seed=41)
    plan = G.Plan(b, n, batch, torch.complex64)
    y1 = plan.forward(W, x).clone()
    y2 = plan.forward(W, x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.float32, torch.float64], ids=str)
def test_mixed_radix_matches_kron(dtype):
    radices = [2, 3, 4, 5, 3]     # W_0 acts on the most significant digit
    Ns = int(np.prod(radices))
    batch = 3
    say(f"mixed radix {radices} dtype={dtype}")
    cplx = dtype in COMPLEX
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary
    Ws = [haar_unitary(r, 50 + i, complex_=cplx) for i, r in enumerate(radices)]
    x = gaussian((batch, Ns), seed=60, complex_=cplx)
    wdt = G.W_DTYPE[dtype]
    Wt = torch.cat([torch.from_numpy(w).to(wdt).reshape(-1) for w in Ws]).cuda()
    xt = torch.from_numpy(x).to(dtype).cuda()
    plan = G.Plan.mixed(radices, batch, dtype)
    y = plan.forward(Wt, xt)
    xi = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    Ws64 = [torch.from_numpy(w).to(wdt).to(torch.complex128).numpy() for w in Ws]
    x64 = host64(xt)
    ref = O.staged_mixed(Ws64, x64)
    assert rel_err(host64(y), ref) < TOL[dtype]
    assert rel_err(host64(xi), x64) < 3 * TOL[dtype]


# the runtime-radix kernel over many tiles and two digit groups (one strided,
# with a partial last column block): radices up to 16 in place, a radix above
# 16 out of place in the same group, contiguous tiles of several instances
@pytest.mark.parametrize("radices,batch,dtype", [
    ([8, 3, 4, 5, 2, 7], 64, torch.complex64), ([17, 3, 20, 2, 5], 5, torch.complex64),
    ([16, 9, 13, 6], 4, torch.float32), ([12, 11, 10, 15, 14], 2, torch.float64),
    ([7, 2, 5, 3, 8, 4], 10, torch.complex128), ([3, 5, 7, 9, 11], 6, torch.bfloat16)], ids=str)
def test_mixed_radix_tiles(radices, batch, dtype):
    Ns = int(np.prod(radices))
    say(f"mixed radix tiles {radices} batch={batch} dtype={dtype}")
    cplx = dtype in COMPLEX
    from paper_2507_02420_amd.inputs import haar_unitary
    Ws = [haar_unitary(r, 70 + i, complex_=cplx) for i, r in enumerate(radices)]
    x = gaussian((batch, Ns), seed=80 + len(radices), complex_=cplx)
    wdt = G.W_DTYPE[dtype]
    Wt = torch.cat([torch.from_numpy(w).to(wdt).reshape(-1) for w in Ws]).cuda()
    xt = torch.from_numpy(x).to(dtype).cuda()
    plan = G.Plan.mixed(radices, batch, dtype)
    groups = plan.describe()["groups"]
    assert len(groups) >= 2 and any(g["S"] > 1 for g in groups), groups
    assert sum(g["tiles"] for g in groups) > 2 * len(groups), groups
    y = plan.forward(Wt, xt)
    xi = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    Ws64 = [torch.from_numpy(w).to(wdt).to(torch.complex128).numpy() for w in Ws]
    x64 = host64(xt)
    assert rel_err(host64(y), O.staged_mixed(Ws64, x64)) < TOL[dtype], (radices, dtype, groups)
    assert rel_err(host64(xi), x64) < 3 * TOL[dtype], (radices, dtype)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16], ids=str)
@pytest.mark.parametrize("b,n,batch", [(16, 1, 5), (16, 2, 3), (16, 3, 2), (16, 5, 1), (32, 1, 7), (32, 2, 3),
                                       (32, 3, 1), (32, 4, 1)])
def test_mfma_radix_16_32(b, n, batch, dtype):
    # matrix-core path: 16-bit operands, W split in two 16-bit parts, FP32
    # accumulation; error against FP64 on the stored inputs
    say(f"mfma b={b} n={n} batch={batch} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=7000 + b + n)
    plan = G.Plan(b, n, batch, dtype)
    assert all(g["kind"] == "mfma" for g in plan.describe()["groups"])
    y = plan.forward(W, x)
    xi = plan.inverse(W, y)
    torch.cuda.synchronize()
    ref = O.staged(W64, x64, n)
    err = rel_err(host64(y), ref)
    say(f"  rel err {err:.3e}")
    assert err < 1e-2
    assert rel_err(host64(xi), x64) < 2e-2


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32], ids=str)
@pytest.mark.parametrize("b,n,batch", [(16, 4, 600), (32, 3, 1100)])
def test_mfma_many_tiles_sampled(b, n, batch, dtype):
    # more tiles than the device holds work-groups at once: the 16-bit pass
    # loops over tiles with the next one prefetched; rows checked against
    # the oracle on a sample that includes the first and the last tile
    say(f"mfma many tiles b={b} n={n} batch={batch} dtype={dtype}")
    N = b ** n
    x, W, _, W64 = make_inputs(b, 1, 1, dtype, seed=7100 + b)  # W only
    x = torch.from_numpy(gaussian((batch, N), seed=7200 + b)).to(dtype).cuda()
    plan = G.Plan(b, n, batch, dtype)
    assert plan.describe()["groups"][0]["tiles"] > 2048
    y = plan.forward(W, x)
    xi = plan.inverse(W, y)
    torch.cuda.synchronize()
    rows = sorted({0, 1, batch // 3, batch // 2, batch - 2, batch - 1})
    x64 = host64(x[rows])
    err = rel_err(host64(y[rows]), O.staged(W64, x64, n))
    say(f"  rel err {err:.3e}")
    assert err < TOL[dtype]
    assert rel_err(host64(xi[rows]), x64) < 3 * TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32], ids=str)
@pytest.mark.parametrize("b,n,batch", [(32, 3, 2), (16, 3, 3)])
def test_mfma_small_tiles_scalar_rows(b, n, batch, dtype):
    # tiles of 128 LDS bytes (tuning override): strided groups get rows of a
    # few elements, moved element by element instead of as 16-byte vectors
    say(f"mfma small tiles b={b} n={n} batch={batch} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=7300 + b + n)
    G.set_tuning(b, dtype, 128, 0, 0, n=n)
    try:
        plan = G.Plan(b, n, batch, dtype)
    finally:
        G.set_tuning(b, dtype, 0, 0, 0, n=n)
        G.load_tuning()          # the table's entry for (b, n), if any
    groups = plan.describe()["groups"]
    assert all(g["kind"] == "mfma" for g in groups)
    assert any(g["mode"] in (1, 3) for g in groups), groups  # a scalar mode
    y = plan.forward(W, x)
    xi = plan.inverse(W, y)
    torch.cuda.synchronize()
    assert rel_err(host64(y), O.staged(W64, x64, n)) < TOL[dtype]
    assert rel_err(host64(xi), x64) < 3 * TOL[dtype]


def test_strided_or_conjugate_views_are_refused():
    b, n = 4, 3
    x, W, _, _ = make_inputs(b, n, 2, torch.complex64, seed=5)
    plan = G.Plan(b, n, 2, torch.complex64)
    with pytest.raises(ValueError):
        plan.forward(W.t(), x)
    with pytest.raises(ValueError):
        plan.forward(W.conj(), x)
    with pytest.raises(ValueError):
        plan.forward(W, x.t().contiguous().t())      # column-major (2, N)


# radix 2 with at most ten digits in the group that starts at digit 0: the
# wavefront form (digits 0-3 in registers, 4..k-1 across lanes by DPP /
# ds_bpermute, no LDS); batches whose element count is not a multiple of
# the 1024 elements one wave covers, forward and inverse
@pytest.mark.parametrize("dtype", FLOAT_DTYPES, ids=str)
@pytest.mark.parametrize("n,batch", [(5, 3), (6, 1), (7, 5), (8, 2), (9, 3), (10, 1), (10, 6)])
def test_radix2_wavefront_digits(n, batch, dtype):
    say(f"radix-2 wavefront n={n} batch={batch} dtype={dtype}")
    x, W, x64, W64 = make_inputs(2, n, batch, dtype, seed=1700 + n + batch)
    plan = G.Plan(2, n, batch, dtype)
    y = plan.forward(W, x)
    xr = plan.inverse(W, y)
    torch.cuda.synchronize()
    ref = O.staged(W64, x64, n)
    assert rel_err(host64(y), ref) < TOL[dtype]
    assert rel_err(host64(xr), O.adjoint(W64, ref, n)) < TOL[dtype]
