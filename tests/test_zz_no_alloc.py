"""gtt_backward_noalloc against gtt_backward through the C ABI: the same
gradients bit for bit (same kernels, same fixed-order sums) and within the
oracle's bounds, on two calls in a row, the second on a smaller input; and
the scratch-size limit reported before any GPU work."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import TOL, host64, make_inputs, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import gaussian

pytestmark = pytest.mark.gpu


def _noalloc(plan, W, x, gy, saved=None, gx=None, gW=None):
    st = G.lib().gtt_backward_noalloc(plan.handle, G._ptr(W), G._ptr(x), G._ptr(saved), G._ptr(gy), G._ptr(gx),
                                      G._ptr(gW), G._stream())
    return st


def _case(b, n, batch, dtype, seed, use_saved, want_gx):
    x, W, x64, W64 = make_inputs(b, n, batch, dtype, seed=seed)
    cplx = dtype.is_complex
    gy = torch.from_numpy(gaussian((batch, b ** n), seed=seed + 1, complex_=cplx)).to(dtype).cuda()
    plan = G.Plan(b, n, batch, dtype)
    saved = None
    if use_saved:
        _, _, sv = plan.workspace_size()
        saved = torch.empty(max(sv, 16), dtype=torch.uint8, device="cuda")
        plan.forward(W, x, saved=saved)
    ref_gx, ref_gW = plan.backward(W, x, gy, saved=saved, want_gx=want_gx)
    gx = torch.full_like(gy, float("nan")) if want_gx else None
    gW = torch.full_like(W, float("nan"))
    assert _noalloc(plan, W, x, gy, saved=saved, gx=gx, gW=gW) == 0
    torch.cuda.synchronize()
    if want_gx:
        assert torch.equal(gx, ref_gx)
    assert torch.equal(gW, ref_gW)
    rgx, rgW = O.grad(W64, x64, host64(gy), n)
    if want_gx:
        assert rel_err(host64(gx), rgx) < TOL[dtype]
    assert np.linalg.norm(host64(gW) - rgW) / np.linalg.norm(rgW) < TOL[dtype]


def test_noalloc_backward_matches_backward_two_calls():
    # first call: complex radix 8 on the matrix cores, two digit groups,
    # activations from `saved`; second call, smaller: float32 radix 4 on
    # the general kernel, activations recomputed in the scratch, gW only
    say("noalloc backward: c64 b=8 n=6 batch=8, then f32 b=4 n=7 batch=2")
    _case(8, 6, 8, torch.complex64, seed=3100, use_saved=True, want_gx=True)
    _case(4, 7, 2, torch.float32, seed=3200, use_saved=False, want_gx=False)


def test_noalloc_backward_reports_the_scratch_limit():
    # 256 x 8^6 complex64 without `saved`: the recomputed activations alone
    # exceed the scratch; refused before any GPU work
    plan = G.Plan(8, 6, 256, torch.complex64)
    a = ctypes.c_void_p(0x10000)
    st = G.lib().gtt_backward_noalloc(plan.handle, a, a, None, a, a, a, None)
    assert st == 5
