"""Ragged batches: instances of different radix and length in one buffer,
run as one persistent launch (grid barrier between digit groups), as one
launch per phase, or per instance; every instance checked against the FP64
oracle.  Also graph capture and replay of the persistent launch and of the
per-phase launches."""
import numpy as np
import pytest
import torch

from gpu_util import COMPLEX, TOL, host64, rel_err, say
from oracle import gtt_oracle as O
from paper_2507_02420_amd import gtt as G
from paper_2507_02420_amd.inputs import gaussian, haar_unitary, ragged_shapes

pytestmark = pytest.mark.gpu

MODES = {"phases": 0, "persistent": G.FLAG_PERSISTENT, "per_instance": G.FLAG_PER_INSTANCE}


def _ragged_inputs(shapes, dtype, seed, x_off=None, w_idx=None):
    cplx = dtype in COMPLEX
    Ns = [b ** n for b, n in shapes]
    if x_off is None:
        offs = np.cumsum([0] + Ns[:-1]).tolist()
        total = int(sum(Ns))
    else:
        offs = list(x_off)
        total = int(max(o + N for o, N in zip(offs, Ns)))
    total = (total + 7) // 8 * 8
    x = gaussian(total, seed=seed, complex_=cplx)
    if w_idx is None:
        radices = sorted(set(b for b, _ in shapes))
        Ws = [haar_unitary(r, seed + 1 + i, complex_=cplx) for i, r in enumerate(radices)]
        widx = [radices.index(b) for b, _ in shapes]
    else:
        nw = max(w_idx) + 1
        rad_of = {}
        for (b, _), w in zip(shapes, w_idx):
            rad_of[w] = b
        Ws = [haar_unitary(rad_of[w], seed + 50 + w, complex_=cplx) for w in range(nw)]
        widx = list(w_idx)
    wdt = G.W_DTYPE[dtype]
    Wt = torch.cat([torch.from_numpy(w).to(wdt).reshape(-1) for w in Ws]).cuda()
    xt = torch.from_numpy(x).to(dtype).cuda()
    W64 = [torch.from_numpy(w).to(wdt).to(torch.complex128 if cplx else torch.float64).numpy() for w in Ws]
    return xt, Wt, W64, widx, offs


SMALL = [(2, 11), (4, 3), (16, 2), (32, 2), (3, 4), (2, 0), (8, 3), (16, 3), (4, 7), (2, 15), (32, 1), (7, 2),
         (16, 4), (2, 1), (4, 5), (5, 3), (32, 3), (2, 17), (3, 1), (6, 3)]


# odd and mixed-parity radices large enough for a strided second digit group
# (element-wise row tiles, at most 256 columns wide)
ODD = [(7, 5), (6, 6), (3, 10), (5, 7), (3, 9), (2, 12), (7, 4)]


# radices without a specialised kernel: in place up to 16, out of place
# above (17, 20, 21), beside small ones; two digit groups where an
# instance exceeds one tile; both launch modes
GENERIC = [(17, 3), (9, 4), (20, 3), (12, 3), (2, 5), (21, 1), (11, 3)]


@pytest.mark.parametrize("mode", list(MODES), ids=str)
@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64], ids=str)
def test_ragged_runtime_radix_items(mode, dtype):
    say(f"ragged runtime radices {mode} {dtype}")
    xt, Wt, W64, widx, offs = _ragged_inputs(GENERIC, dtype, seed=950)
    plan = G.Plan([b for b, _ in GENERIC], [n for _, n in GENERIC], 1, dtype, flags=MODES[mode])
    y = plan.forward(Wt, xt)
    xi = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    x64, y64, xi64 = host64(xt), host64(y), host64(xi)
    for t, ((b, n), o) in enumerate(zip(GENERIC, offs)):
        N = b ** n
        assert rel_err(y64[o:o + N], O.staged(W64[widx[t]], x64[o:o + N], n)) < TOL[dtype], (t, b, n)
        assert rel_err(xi64[o:o + N], O.adjoint(W64[widx[t]], y64[o:o + N], n)) < TOL[dtype], (t, b, n)


@pytest.mark.parametrize("mode", list(MODES), ids=str)
@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.float64], ids=str)
def test_ragged_odd_radix_strided_groups(mode, dtype):
    say(f"ragged odd radices {mode} {dtype}")
    xt, Wt, W64, widx, offs = _ragged_inputs(ODD, dtype, seed=900)
    plan = G.Plan([b for b, _ in ODD], [n for _, n in ODD], 1, dtype, flags=MODES[mode])
    y = plan.forward(Wt, xt)
    xi = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    x64, y64, xi64 = host64(xt), host64(y), host64(xi)
    for t, ((b, n), o) in enumerate(zip(ODD, offs)):
        N = b ** n
        assert rel_err(y64[o:o + N], O.staged(W64[widx[t]], x64[o:o + N], n)) < TOL[dtype], (t, b, n)
        assert rel_err(xi64[o:o + N], O.adjoint(W64[widx[t]], y64[o:o + N], n)) < TOL[dtype], (t, b, n)


@pytest.mark.parametrize("mode", list(MODES), ids=str)
@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.complex64], ids=str)
def test_ragged_forward_inverse(mode, dtype):
    say(f"ragged {mode} {dtype}")
    shapes = SMALL
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=800)
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype, flags=MODES[mode])
    y = plan.forward(Wt, xt)
    xi = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    x64, y64, xi64 = host64(xt), host64(y), host64(xi)
    tol = TOL[dtype]
    for t, ((b, n), o) in enumerate(zip(shapes, offs)):
        N = b ** n
        ref = O.staged(W64[widx[t]], x64[o:o + N], n)
        e = rel_err(y64[o:o + N], ref)
        assert e < tol, (t, b, n, e)
        assert rel_err(xi64[o:o + N], x64[o:o + N]) < 3 * tol, (t, b, n)


def test_ragged_offsets_and_shared_w():
    # explicit offsets with gaps; two instances of radix 4 use different W
    shapes = [(4, 5), (2, 9), (4, 3), (16, 2), (2, 4)]
    x_off = [0, 1024 + 8, 1024 + 8 + 512 + 16, 2048, 4096]
    w_idx = [0, 1, 2, 3, 1]
    dtype = torch.complex64
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=900, x_off=x_off, w_idx=w_idx)
    for flags in (0, G.FLAG_PERSISTENT):
        plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype, flags=flags, x_off=x_off,
                      w_idx=w_idx)
        y = torch.zeros_like(xt)
        plan.forward(Wt, xt, y)
        torch.cuda.synchronize()
        x64, y64 = host64(xt), host64(y)
        for t, ((b, n), o) in enumerate(zip(shapes, offs)):
            N = b ** n
            assert rel_err(y64[o:o + N], O.staged(W64[widx[t]], x64[o:o + N], n)) < 1e-5


def test_ragged_backward_per_w():
    shapes = [(2, 10), (4, 4), (2, 6), (8, 3), (4, 6), (3, 5)]
    dtype = torch.complex64
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=1000)
    g = torch.from_numpy(gaussian(xt.numel(), seed=1001, complex_=True)).to(dtype).cuda()
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype)
    _, _, sv = plan.workspace_size()
    saved = torch.empty(sv, dtype=torch.uint8, device="cuda") if sv else None
    plan.forward(Wt, xt, saved=saved)
    gx, gW = plan.backward(Wt, xt, g, saved=saved)
    torch.cuda.synchronize()
    x64, g64, gx64, gW64 = host64(xt), host64(g), host64(gx), host64(gW)
    ref_gW = [np.zeros_like(w) for w in W64]
    for t, ((b, n), o) in enumerate(zip(shapes, offs)):
        N = b ** n
        rgx, rgW = O.grad(W64[widx[t]], x64[o:o + N], g64[o:o + N], n)
        assert rel_err(gx64[o:o + N], rgx) < 1e-5
        ref_gW[widx[t]] += rgW
    pos = 0
    for w in ref_gW:
        got = gW64[pos:pos + w.size].reshape(w.shape)
        assert np.linalg.norm(got - w) / np.linalg.norm(w) < 1e-5
        pos += w.size


@pytest.mark.parametrize("mode", ["phases", "persistent"])
def test_ragged_full_shape_list_bf16_every_shape(mode):
    # the 1024-instance shape list (b in {2,4,16,32}, N in [2^10, 2^20],
    # 268,417,024 elements) in bf16, per-phase launches (the default, as
    # benchmarked) and one persistent launch, checked against the FP64 oracle
    # on the stored bf16 values: the first instance of each of the 23
    # distinct (b, n) shapes, the last instance of the largest shape of each
    # radix, and every 61st instance; max / median error per radix reported
    shapes = ragged_shapes(1024, seed=52)
    say(f"ragged 1024 bf16 {mode}")
    Ns = [b ** n for b, n in shapes]
    offs = np.cumsum([0] + Ns[:-1])
    total = int(sum(Ns))
    rng = np.random.default_rng(53)
    xt = torch.from_numpy(rng.standard_normal(total, dtype=np.float32)).cuda().to(torch.bfloat16)
    Ws = [haar_unitary(r, 54 + i, complex_=False).astype(np.float32) for i, r in enumerate((2, 4, 16, 32))]
    Wt = torch.cat([torch.from_numpy(w).reshape(-1) for w in Ws]).cuda()
    ridx = {2: 0, 4: 1, 16: 2, 32: 3}
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, torch.bfloat16, flags=MODES[mode])
    y = plan.forward(Wt, xt)
    torch.cuda.synchronize()
    plan.check()
    first = {}
    for t, s_ in enumerate(shapes):
        first.setdefault(s_, t)
    assert len(first) == 23
    last_largest = [max((t for t in range(1024) if shapes[t][0] == b), key=lambda t: (Ns[t], t))
                    for b in (2, 4, 16, 32)]
    pick = sorted(set(first.values()) | set(last_largest) | set(range(0, 1024, 61)))
    errs = {}
    for t in pick:
        b, n = shapes[t]
        o, N = int(offs[t]), Ns[t]
        x64 = xt[o:o + N].float().cpu().double().numpy()
        ref = O.staged(Ws[ridx[b]].astype(np.float64), x64, n)
        e = rel_err(y[o:o + N].float().cpu().double().numpy(), ref)
        errs.setdefault(b, []).append(e)
        assert e < 1e-2, (t, b, n, e)
    say("  rel err vs FP64 oracle per radix (max / median): " +
        ", ".join(f"b={b}: {max(v):.2e} / {float(np.median(v)):.2e} ({len(v)})" for b, v in sorted(errs.items())))


def test_ragged_first_call_is_captured_in_a_graph():
    # the work list is uploaded by the plan, so the plan's very first call
    # can be recorded into a graph (no allocation, no synchronous copy)
    shapes = [(2, 12), (16, 3), (4, 7), (3, 8), (32, 2), (2, 5)]
    dtype = torch.bfloat16
    say("ragged first call under graph capture")
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=1150)
    for flags in (0, G.FLAG_PERSISTENT):
        plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype, flags=flags)
        y = torch.zeros_like(xt)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.forward(Wt, xt, y)
        for rep in range(2):
            y.zero_()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            plan.check()
            x64, y64 = host64(xt), host64(y)
            for t, ((b, n), o) in enumerate(zip(shapes, offs)):
                N = b ** n
                assert rel_err(y64[o:o + N], O.staged(W64[widx[t]], x64[o:o + N], n)) < 1e-2, (flags, rep, t)


def test_ragged_persistent_barrier_failure_is_reported():
    # the bounded wait of the grid barrier, made to give up at once from the
    # host (a limit of 0 polls): every work-group leaves the kernel at its
    # next barrier, and gtt_plan_check reports the failure once; with the
    # default limit the same plan runs correctly again
    shapes = SMALL
    dtype = torch.float32
    say("ragged persistent barrier failure")
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=1200)
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype, flags=G.FLAG_PERSISTENT)
    plan.forward(Wt, xt)
    plan.check()                               # clean
    plan.barrier_limit(0)
    plan.forward(Wt, xt)
    with pytest.raises(G.GTTError) as e:
        plan.check()
    assert e.value.status == G.ERR_TIMEOUT
    plan.check()                               # the record was cleared
    plan.barrier_limit(1 << 24)
    y = plan.forward(Wt, xt)
    plan.check()
    x64, y64 = host64(xt), host64(y)
    for t, ((b, n), o) in enumerate(zip(shapes, offs)):
        N = b ** n
        assert rel_err(y64[o:o + N], O.staged(W64[widx[t]], x64[o:o + N], n)) < TOL[dtype], t


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.complex64], ids=str)
def test_ragged_backward_with_radix_16_and_32(dtype):
    shapes = [(32, 2), (16, 3), (2, 10), (4, 5), (32, 3), (16, 2), (2, 0), (3, 4)]
    say(f"ragged backward with radix 16 / 32 {dtype}")
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=1300)
    cplx = dtype in COMPLEX
    g = torch.from_numpy(gaussian(xt.numel(), seed=1301, complex_=cplx)).to(dtype).cuda()
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype)
    gx, gW = plan.backward(Wt, xt, g)
    torch.cuda.synchronize()
    x64, g64, gx64, gW64 = host64(xt), host64(g), host64(gx), host64(gW)
    tol = 1e-2 if dtype == torch.bfloat16 else TOL[dtype]
    ref_gW = [np.zeros_like(w) for w in W64]
    for t, ((b, n), o) in enumerate(zip(shapes, offs)):
        N = b ** n
        rgx, rgW = O.grad(W64[widx[t]], x64[o:o + N], g64[o:o + N], n)
        assert rel_err(gx64[o:o + N], rgx) < tol, (t, b, n)
        ref_gW[widx[t]] += rgW
    pos = 0
    for w in ref_gW:
        got = gW64[pos:pos + w.size].reshape(w.shape)
        assert np.linalg.norm(got - w) / np.linalg.norm(w) < tol
        pos += w.size


@pytest.mark.parametrize("mode", ["persistent", "phases"])
def test_ragged_graph_replay(mode):
    # per-phase mode: one launch per phase and radix class, several classes
    # per phase (2, 3, 4 on the VALU, 16 on the matrix cores), all captured
    shapes = SMALL if mode == "persistent" else [(2, 12), (16, 3), (4, 7), (3, 8), (2, 5), (16, 4), (4, 3)]
    dtype = torch.bfloat16
    say(f"ragged graph replay, {mode}")
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=1100)
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype, flags=MODES[mode])
    y_eager = torch.zeros_like(xt)           # the buffer tail past the last instance stays 0
    plan.forward(Wt, xt, y_eager)
    torch.cuda.synchronize()
    y = torch.empty_like(xt)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(Wt, xt, y)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.forward(Wt, xt, y)
    for rep in range(3):
        y.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), rep
        # eager work between replays
        _ = plan.forward(Wt, xt)
        torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32], ids=str)
def test_ragged_matrix_core_items_loop_and_w_changes(dtype):
    # more matrix-core items per phase (18 instances x 64 or 128 tiles) than
    # one resident grid holds, so work-groups run several items; W drawn per
    # instance from two of each radix, so consecutive items of a work-group
    # both keep and change W (the class kernels reload W's fragments only
    # when it changes)
    shapes = [(16, 5)] * 18 + [(32, 4)] * 18
    rng = np.random.default_rng(951)
    w_idx = rng.integers(0, 2, 18).tolist() + (2 + rng.integers(0, 2, 18)).tolist()
    say(f"ragged matrix-core loop {dtype}")
    xt, Wt, W64, widx, offs = _ragged_inputs(shapes, dtype, seed=950, w_idx=w_idx)
    plan = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype, w_idx=w_idx)
    y = plan.forward(Wt, xt)
    xi = plan.inverse(Wt, y)
    torch.cuda.synchronize()
    x64, y64, xi64 = host64(xt), host64(y), host64(xi)
    tol = TOL[dtype]
    for t, ((b, n), o) in enumerate(zip(shapes, offs)):
        N = b ** n
        e = rel_err(y64[o:o + N], O.staged(W64[widx[t]], x64[o:o + N], n))
        assert e < tol, (t, b, n, e)
        assert rel_err(xi64[o:o + N], x64[o:o + N]) < 3 * tol
