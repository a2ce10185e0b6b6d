"""GPU backward (gx = G^H gy, gW = sum of per-fibre outer products) against the
FP64 oracle gradient (itself pinned to finite differences and torch autograd
on the CPU), plus torch.autograd.gradcheck through GTTFunction."""
import numpy as np
import pytest
import torch

from gpu_util import COMPLEX, TOL, host64, make_inputs, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import gaussian

pytestmark = pytest.mark.gpu


def _grad_case(b, n, batch, dtype, seed, use_saved=True):
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=seed)
    cplx = dtype in COMPLEX
    g = gaussian((batch, b ** n), seed=seed + 7, complex_=cplx)
    gt = torch.from_numpy(g).to(dtype).cuda()
    g64 = host64(gt)
    plan = G.Plan(b, n, batch, dtype)
    saved = None
    if use_saved:
        _, _, sv = plan.workspace_size()
        saved = torch.empty(max(sv, 16), dtype=torch.uint8, device="cuda") if sv else None
        plan.forward(W, x, saved=saved)
    gx, gW = plan.backward(W, x, gt, saved=saved)
    torch.cuda.synchronize()
    rgx, rgW = O.grad(W64, x64, g64, n)
    return host64(gx), host64(gW), rgx, rgW


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.complex64, torch.complex128], ids=str)
@pytest.mark.parametrize("b,n,batch", [(2, 3, 2), (2, 14, 2), (3, 5, 3), (3, 9, 2), (4, 4, 3), (4, 8, 2),
                                       (5, 4, 2), (6, 3, 2), (7, 3, 2), (8, 3, 2), (8, 5, 2), (11, 2, 3),
                                       (16, 2, 2), (16, 3, 1), (32, 2, 2), (32, 3, 1), (21, 2, 2)])
def test_backward_matches_oracle(b, n, batch, dtype):
    # gW is summed in FP64 for every dtype and rounded once: the FP32 / c64
    # bound holds for gW as for gx
    say(f"backward b={b} n={n} batch={batch} dtype={dtype}")
    gx, gW, rgx, rgW = _grad_case(b, n, batch, dtype, seed=5000 + 31 * b + n)
    tol = TOL[dtype]
    assert rel_err(gx, rgx) < tol
    assert np.linalg.norm(gW - rgW) / np.linalg.norm(rgW) < tol


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16], ids=str)
@pytest.mark.parametrize("b,n,batch", [(16, 2, 3), (16, 3, 2), (32, 2, 3), (32, 3, 1), (2, 13, 2), (4, 5, 3)])
def test_backward_16bit_storage(b, n, batch, dtype):
    # 16-bit storage: gx is rounded to the storage type (1e-2 bound); gW is
    # float32 (W's dtype), summed in FP64 from the stored operands
    say(f"backward 16-bit b={b} n={n} batch={batch} dtype={dtype}")
    gx, gW, rgx, rgW = _grad_case(b, n, batch, dtype, seed=5200 + b + n)
    assert rel_err(gx, rgx) < 1e-2
    assert np.linalg.norm(gW - rgW) / np.linalg.norm(rgW) < 1e-2


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64], ids=str)
@pytest.mark.parametrize("b,n", [(4, 8), (8, 5), (2, 15)])
def test_backward_without_saved_recomputes(b, n, dtype):
    say(f"backward (no saved) b={b} n={n} dtype={dtype}")
    gx, gW, rgx, rgW = _grad_case(b, n, 2, dtype, seed=6000 + b + n, use_saved=False)
    assert rel_err(gx, rgx) < TOL[dtype]
    assert np.linalg.norm(gW - rgW) / np.linalg.norm(rgW) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64], ids=str)
@pytest.mark.parametrize("use_saved", [True, False])
def test_backward_boundary_slots_of_odd_length(dtype, use_saved):
    # 3^7 = 2187 elements (not a multiple of 16 bytes) in four digit groups
    # (tuning override): the activations between groups sit in slots of the
    # saved / workspace buffer whose stride is rounded up to 256 bytes
    b, n = 3, 7
    say(f"backward odd-length slots dtype={dtype} saved={use_saved}")
    G.set_tuning(b, dtype, 0, 0, 2, n=n)
    try:
        gx, gW, rgx, rgW = _grad_case(b, n, 1, dtype, seed=6100, use_saved=use_saved)
        assert len(G.Plan(b, n, 1, dtype).describe()["groups"]) == 4
    finally:
        G.set_tuning(b, dtype, 0, 0, 0, n=n)
        G.load_tuning()
    assert rel_err(gx, rgx) < TOL[dtype]
    assert np.linalg.norm(gW - rgW) / np.linalg.norm(rgW) < TOL[dtype]


def test_backward_c128_b8_n3_tight():
    # the finite-difference case of the oracle pins, on the GPU in FP64
    say("backward c128 b=8 n=3")
    gx, gW, rgx, rgW = _grad_case(8, 3, 1, torch.complex128, seed=44)
    assert rel_err(gx, rgx) < 1e-12
    assert np.linalg.norm(gW - rgW) / np.linalg.norm(rgW) < 1e-12


def test_backward_bf16_within_budget():
    say("backward bf16 b=4 n=7")
    gx, gW, rgx, rgW = _grad_case(4, 7, 2, torch.bfloat16, seed=77)
    assert rel_err(gx, rgx) < 1e-2
    assert np.linalg.norm(gW - rgW) / np.linalg.norm(rgW) < 1e-2


def test_backward_only_gw_and_only_gx_and_inplace():
    b, n, batch, dtype = 4, 8, 2, torch.complex64
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=91)
    g = torch.from_numpy(gaussian((batch, b ** n), seed=92, complex_=True)).to(dtype).cuda()
    plan = G.Plan(b, n, batch, dtype)
    rgx, rgW = O.grad(W64, x64, host64(g), n)
    _, gW = plan.backward(W, x, g, want_gx=False)
    gx, _ = plan.backward(W, x, g, want_gW=False)
    g2 = g.clone()
    gx2, gW2 = plan.backward(W, x, g2, gx=g2)     # gx aliases gy
    torch.cuda.synchronize()
    assert rel_err(host64(gx), rgx) < 1e-5
    assert np.linalg.norm(host64(gW) - rgW) / np.linalg.norm(rgW) < 1e-5
    assert torch.equal(gx2, gx)
    assert torch.equal(gW2, gW)


@pytest.mark.parametrize("b,n,batch,dtype", [(4, 6, 4, torch.float32), (8, 3, 2, torch.complex64),
                                             (8, 4, 2, torch.complex64), (2, 10, 2, torch.float64)], ids=str)
def test_backward_gw_only_single_group(b, n, batch, dtype):
    # one digit group and no gx: the first group's cotangent is not stored;
    # x and gy must come back untouched
    say(f"backward gW only b={b} n={n} batch={batch} dtype={dtype}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=97 + b + n)
    g = torch.from_numpy(gaussian((batch, b ** n), seed=98, complex_=dtype.is_complex)).to(dtype).cuda()
    plan = G.Plan(b, n, batch, dtype)
    assert len(plan.describe()["groups"]) == 1
    x0, g0 = x.clone(), g.clone()
    _, gW = plan.backward(W, x, g, want_gx=False)
    torch.cuda.synchronize()
    assert torch.equal(x, x0) and torch.equal(g, g0)
    _, rgW = O.grad(W64, x64, host64(g), n)
    assert np.linalg.norm(host64(gW) - rgW) / np.linalg.norm(rgW) < TOL[dtype]


# complex radix-8 shapes covering every (digits, tile) variant of the
# matrix-core backward with per-lane addresses: 1-4 digits, 2048 / 4096
# element tiles, contiguous and strided (C = 8, 32, 256) groups
@pytest.mark.parametrize("n,batch", [(1, 512), (2, 64), (3, 4), (3, 8), (4, 2), (5, 2), (6, 8), (7, 1)])
@pytest.mark.parametrize("want_gx", [True, False])
def test_backward_c64_radix8_tiles(n, batch, want_gx):
    b, dtype = 8, torch.complex64
    say(f"backward c64 b=8 n={n} batch={batch} want_gx={want_gx}")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=700 + n)
    g = torch.from_numpy(gaussian((batch, b ** n), seed=800 + n, complex_=True)).to(dtype).cuda()
    plan = G.Plan(b, n, batch, dtype)
    gx, gW = plan.backward(W, x, g, want_gx=want_gx)
    torch.cuda.synchronize()
    rgx, rgW = O.grad(W64, x64, host64(g), n)
    if want_gx:
        assert rel_err(host64(gx), rgx) < TOL[dtype]
    assert np.linalg.norm(host64(gW) - rgW) / np.linalg.norm(rgW) < TOL[dtype]


def test_backward_deterministic():
    b, n, batch, dtype = 8, 6, 8, torch.complex64
    x, W, _, _ = make_inputs(b, n, batch, dtype, seed=93)
    g = torch.from_numpy(gaussian((batch, b ** n), seed=94, complex_=True)).to(dtype).cuda()
    plan = G.Plan(b, n, batch, dtype)
    a = plan.backward(W, x, g)
    c = plan.backward(W, x, g)
    torch.cuda.synchronize()
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1])


def test_full_size_differentiation_workload():
    # 256 x c64, b=8, n=6 (N = 262144): the launch configuration of the
    # benchmark.  y and gx on sampled instances against the oracle; gW (one
    # sum over all 256 instances, ~5e8 outer-product terms) against the
    # oracle gradient of the whole batch, computed in chunks of instances
    # (gW is a sum over instances).
    b, n, batch, dtype = 8, 6, 256, torch.complex64
    say("full-size differentiation 256 x 8^6 c64")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=41)
    g = gaussian((batch, b ** n), seed=43, complex_=True).astype(np.complex64)
    plan = G.Plan(b, n, batch, dtype)
    _, _, sv = plan.workspace_size()
    saved = torch.empty(sv, dtype=torch.uint8, device="cuda")
    y = plan.forward(W, x, saved=saved)
    gt = torch.from_numpy(g).cuda()
    gx, gW = plan.backward(W, x, gt, saved=saved)
    torch.cuda.synchronize()
    for i in (3, 128, 250):
        assert rel_err(host64(y[i]), O.staged(W64, x64[i], n)) < 1e-5
        assert rel_err(host64(gx[i]), O.adjoint(W64, host64(gt[i]), n)) < 1e-5
    rgW = np.zeros((b, b), dtype=np.complex128)
    g64 = g.astype(np.complex128)
    for c0 in range(0, batch, 16):
        _, part = O.grad(W64, x64[c0:c0 + 16], g64[c0:c0 + 16], n)
        rgW += part
    err = np.linalg.norm(host64(gW) - rgW) / np.linalg.norm(rgW)
    say(f"  gW rel err over 256 instances {err:.3e}")
    assert err < 1e-5


def test_full_size_complex_radix4_backward():
    # 64 x c64, b=4, n=10 (the complex64 radix-4 workload; matrix-core
    # gradient sums): the cotangent is nonzero on 8 instances spread over
    # the batch, so gW is the oracle's sum over those 8, gx matches the
    # oracle there and is exactly zero elsewhere
    b, n, batch, dtype = 4, 10, 64, torch.complex64
    say("full-size backward 64 x 4^10 c64")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=61)
    live = [0, 9, 17, 30, 31, 44, 58, 63]
    g = np.zeros((batch, b ** n), dtype=np.complex64)
    g[live] = gaussian((len(live), b ** n), seed=63, complex_=True).astype(np.complex64)
    plan = G.Plan(b, n, batch, dtype)
    gt = torch.from_numpy(g).cuda()
    gx, gW = plan.backward(W, x, gt)
    torch.cuda.synchronize()
    gx64 = host64(gx)
    dead = [i for i in range(batch) if i not in live]
    assert not np.any(gx64[dead]), "gx of zero cotangents"
    rgx, rgW = O.grad(W64, x64[live], g[live].astype(np.complex128), n)
    for j, i in enumerate(live):
        assert rel_err(gx64[i], rgx[j]) < 1e-5, i
    err = rel_err(host64(gW), rgW)
    say(f"  gW rel err {err:.3e}")
    assert err < 1e-5


def test_full_size_float32_radix3_backward():
    # 16 x f32, b=3, n=13 (the odd-radix workload: register-block backward
    # with element-wise tiles and the scalar address walk): cotangent on 4
    # spread instances; gW against the oracle's sum over them, gx against the
    # oracle there and exactly zero elsewhere
    b, n, batch, dtype = 3, 13, 16, torch.float32
    say("full-size backward 16 x 3^13 f32")
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=71)
    live = [0, 6, 11, 15]
    g = np.zeros((batch, b ** n), dtype=np.float32)
    g[live] = gaussian((len(live), b ** n), seed=73).astype(np.float32)
    plan = G.Plan(b, n, batch, dtype)
    gx, gW = plan.backward(W, x, torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    gx64 = host64(gx)
    assert not np.any(gx64[[i for i in range(batch) if i not in live]]), "gx of zero cotangents"
    rgx, rgW = O.grad(W64, x64[live], g[live].astype(np.float64), n)
    for j, i in enumerate(live):
        assert rel_err(gx64[i], rgx[j]) < 1e-5, i
    err = rel_err(host64(gW), rgW)
    say(f"  gW rel err {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("dtype", [torch.complex64, torch.float32, torch.float64, torch.complex128], ids=str)
@pytest.mark.parametrize("radices,batch", [([2, 3, 4, 5], 3), ([3, 8, 2, 7, 4], 2), ([16, 2, 9], 2),
                                           ([32, 4], 3), ([5, 5, 5, 5, 5, 5, 5], 2), ([2] * 14 + [3], 1),
                                           ([8, 3, 4, 5, 2, 7], 8)])
def test_mixed_radix_backward(radices, batch, dtype):
    # distinct factors W_0 kron ... kron W_{m-1}: gx and every factor's
    # gradient against the oracle (gW comes back in the W table's layout)
    say(f"mixed backward {radices} batch={batch} dtype={dtype}")
    cplx = dtype in COMPLEX
    from paper_2507_02420_amd.inputs import haar_unitary
    Ws = [haar_unitary(r, 150 + i, complex_=cplx) for i, r in enumerate(radices)]
    N = int(np.prod(radices))
    wdt = G.W_DTYPE[dtype]
    Wt = torch.cat([torch.from_numpy(w).to(wdt).reshape(-1) for w in Ws]).cuda()
    xt = torch.from_numpy(gaussian((batch, N), seed=160, complex_=cplx)).to(dtype).cuda()
    gt = torch.from_numpy(gaussian((batch, N), seed=161, complex_=cplx)).to(dtype).cuda()
    plan = G.Plan.mixed(radices, batch, dtype)
    _, _, sv = plan.workspace_size()
    saved = torch.empty(max(sv, 16), dtype=torch.uint8, device="cuda")
    plan.forward(Wt, xt, saved=saved)
    gx, gW = plan.backward(Wt, xt, gt, saved=saved)
    gx2, gW2 = plan.backward(Wt, xt, gt)          # activations recomputed
    torch.cuda.synchronize()
    Ws64 = [torch.from_numpy(w).to(wdt).to(torch.complex128).numpy() for w in Ws]
    rgx, rgWs = O.grad_mixed(Ws64, host64(xt), host64(gt))
    if not cplx:
        rgx = rgx.real
    tol = TOL[dtype]
    assert rel_err(host64(gx), rgx) < tol
    got = host64(gW)
    pos = 0
    for r, rg in zip(radices, rgWs):
        blk = got[pos:pos + r * r].reshape(r, r)
        rg = rg if cplx else rg.real
        assert np.linalg.norm(blk - rg) / np.linalg.norm(rg) < tol, (r, pos)
        pos += r * r
    assert torch.equal(gx2, gx) and torch.equal(gW2, gW)


def test_autograd_function_gradcheck():
    b, n = 3, 3
    x = torch.randn(2, b ** n, dtype=torch.complex128, device="cuda", requires_grad=True)
    from paper_2507_02420_amd.inputs import haar_unitary
    W = torch.from_numpy(haar_unitary(b, 5)).cuda().requires_grad_(True)
    f = lambda x_, W_: G.GTTFunction.apply(x_, W_, b, n)
    assert torch.autograd.gradcheck(f, (x, W), eps=1e-6, atol=1e-7)


def test_autograd_function_matches_oracle_c64():
    b, n, batch = 8, 4, 3
    x, W, x64, W64 = make_inputs(b, n, batch, torch.complex64, seed=99)
    x.requires_grad_(True)
    W.requires_grad_(True)
    g = torch.from_numpy(gaussian((batch, b ** n), seed=98, complex_=True)).to(torch.complex64).cuda()
    y = G.gtt(x, W, b, n)
    L = torch.real(torch.sum(torch.conj(g) * y))
    L.backward()
    torch.cuda.synchronize()
    rgx, rgW = O.grad(W64, x64, host64(g), n)
    assert rel_err(host64(x.grad), rgx) < 1e-5
    assert np.linalg.norm(host64(W.grad) - rgW) / np.linalg.norm(rgW) < 1e-5


def test_backward_every_workgroup_size():
    # the register-block backward runs 256-, 512- or 1024-thread work-groups,
    # whichever keeps the most waves resident for the tile's LDS; tuned LDS
    # budgets per work-group steer the choice through all three sizes
    # (labels of the timed launches carry the size), each checked against the
    # oracle; a budget too small for any schedule falls back to the built-in
    # ones
    seen = set()
    shapes = [(3, 9, 2, torch.float32), (4, 8, 2, torch.float32), (4, 6, 3, torch.complex64)]
    try:
        for b, n, batch, dtype in shapes:
            for lds in (20480, 81920, 163840):
                G.set_tuning(b, dtype, 0, 0, n=n, bwd_lds_bytes=lds)
                say(f"backward work-group size b={b} n={n} dtype={dtype} lds={lds}")
                x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=5900 + b + n)
                g = gaussian((batch, b ** n), seed=5901 + b, complex_=dtype in COMPLEX)
                gt = torch.from_numpy(g).to(dtype).cuda()
                plan = G.Plan(b, n, batch, dtype)
                plan.timing(True)
                gx, gW = plan.backward(W, x, gt)
                torch.cuda.synchronize()
                names = list(plan.timing_read())
                plan.timing(False)
                seen |= {int(nm.split("wg=")[1]) for nm in names if "wg=" in nm}
                rgx, rgW = O.grad(W64, x64, host64(gt), n)
                assert rel_err(host64(gx), rgx) < TOL[dtype]
                assert np.linalg.norm(host64(gW) - rgW) / np.linalg.norm(rgW) < TOL[dtype]
    finally:
        for b, n, _, dtype in shapes:
            G.set_tuning(b, dtype, 0, 0, n=n)  # all zeros: the entry is removed
        G.load_tuning()
    say(f"work-group sizes seen: {sorted(seen)}")
    assert {256, 512, 1024} <= seen, seen
