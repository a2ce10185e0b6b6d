"""Benchmark of the fast generalized tensor transform on one MI355X.

Headline: forward + backward (dL/dx and dL/dW) of 256 complex64 vectors,
b = 8, n = 6 (N = 262,144; 67,108,864 elements), W a random 8 x 8 unitary,
loss L = Re <g, y>.  One step = gtt_forward (keeping the activations between
digit groups) + gtt_backward, inputs resident in HBM.  value = elements per
second of that step.

The JSON line also carries:
  roofline     -- the kernel with the largest share of a step (found in a
                  few steps with every launch timed, just before the timed
                  region): its algorithmic HBM bytes and matrix-core flops per
                  launch over its HIP-event duration inside the timed region
                  (where only its launches carry events), against the 8 TB/s
                  HBM peak and the 157.3 TFLOP/s FP32 MFMA peak; "bound" is
                  the resource whose time at peak is the larger (the roofline
                  that binds), and both views are kept;
  directions   -- forward and backward HBM rates (algorithmic bytes of all
                  their launches over their summed durations, from those
                  fully timed steps);
  cpu_baseline -- the FP64 oracle (numpy, one core) on a bounded sample of the
                  same workload, and the GPU error against it on that sample;
  workloads    -- the other configurations (single FP64 vector, complex64
                  round trip, odd radix, int32 Hadamard, ragged bf16 batch vs
                  the plain FP32 path), a few timed calls each.
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTT fwd+bwd elements/s and % of HBM roofline vs plain FP32 at stated error"
HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, FP32
# without packed instructions (disabled on this target) and FP64 alike
VALU_PEAK_TFLOPS = 78.6


def kernel_flops(name: str, elems: int) -> float:
    """Algorithmic flops of one launch named by the library's timing
    ("pass c64 b=8 cmfma s0=0 k=4", "bwd c64 ..."): per element and digit,
    one complex b-term dot product (8 b real flops) for a pass; the adjoint
    pass plus the gradient sums (16 b) for a backward launch.  Only the
    complex radix-8 launches are priced (0 otherwise)."""
    parts = dict(p.split("=", 1) for p in name.split() if "=" in p)
    if "c64" not in name or "cmfma" not in name or "k" not in parts or "b" not in parts:
        return 0.0
    b, k = int(parts["b"]), int(parts["k"])
    per = 16 * b if name.startswith("bwd") else 8 * b
    return float(per) * k * elems


def _sync():
    import torch
    torch.cuda.synchronize()


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_calls(fn, iters, flush=None):
    """Median milliseconds of fn() over iters calls, timed with HIP events on
    the current stream (the stream every call is enqueued on)."""
    ts = []
    for _ in range(iters):
        if flush is not None:
            flush()
            # let the flush drain first: an event recorded behind a running
            # kernel can take its timestamp before that kernel ends
            _sync()
        s, e = _events()
        s.record()
        fn()
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e))
    ts.sort()
    return ts[len(ts) // 2], ts


def dominant(timing: dict):
    name = max(timing, key=lambda k: timing[k]["total_ms"])
    t = timing[name]
    achieved = t["bytes_per_launch"] / (t["avg_ms"] * 1e-3) / 1e9
    return name, t, achieved


# C/C++ tokens that matter for stripping comments: string and character
# literals (kept whole, so a "//" inside one is not a comment), comments
_CXX_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/', re.S)


def _code_only(src: str) -> str:
    """C++ source without comments and with runs of blank space collapsed."""
    body = _CXX_TOKENS.sub(lambda m: " " if m.group(0)[0] == "/" else m.group(0), src)
    return " ".join(body.split())


def kernel_source_digest() -> str:
    """SHA-256 over the code of libgtt.so's HIP/C++ sources (sorted by name;
    comments and layout do not count: a counter table stays valid across a
    comment edit, and goes stale with any change to the code)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2507_02420_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(f.encode())
            h.update(_code_only(open(os.path.join(d, f), encoding="utf-8").read()).encode())
    return h.hexdigest()


def load_traffic(kernel_name: str, workload: str):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy-kernel factor) -- only when it was taken on
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_source_digest():
        return None
    ent = d.get("kernels", {}).get(kernel_name)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


# ---------------------------------------------------------------------------
# headline workload
# ---------------------------------------------------------------------------
def headline(steps, warmup):
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary

    b, n, batch = 8, 6, 256
    N = b ** n
    E = N * batch
    dev = torch.device("cuda:0")
    # seeded inputs: x (seed 41), W (seed 42), g (seed 43), generated per
    # instance block to bound host memory
    x = torch.empty(batch, N, dtype=torch.complex64, device=dev)
    g = torch.empty(batch, N, dtype=torch.complex64, device=dev)
    for i0 in range(0, batch, 32):
        x[i0:i0 + 32] = torch.from_numpy(gaussian((32, N), seed=41 * 1000 + i0, complex_=True).astype(np.complex64))
        g[i0:i0 + 32] = torch.from_numpy(gaussian((32, N), seed=43 * 1000 + i0, complex_=True).astype(np.complex64))
    W = torch.from_numpy(haar_unitary(b, 42).astype(np.complex64)).to(dev)
    plan = G.Plan(b, n, batch, torch.complex64)
    _, bwd_ws, sv = plan.workspace_size()
    saved = torch.empty(sv, dtype=torch.uint8, device=dev)
    y = torch.empty_like(x)
    gx = torch.empty_like(x)
    gW = torch.empty_like(W)

    def step():
        plan.forward(W, x, y, saved=saved)
        plan.backward(W, x, g, saved=saved, gx=gx, gW=gW)

    for _ in range(warmup):
        step()
    _sync()
    # per-kernel breakdown, before the timed region: every launch bracketed
    # by HIP events (the directions' rates and the dominant kernel's name)
    nb = max(1, min(steps, 10))
    plan.timing(True)
    for _ in range(nb):
        step()
    _sync()
    breakdown = plan.timing_read()
    dom_name = max(breakdown, key=lambda k: breakdown[k]["total_ms"])
    # the timed region: events only around the dominant kernel's launches
    # (events around every launch cost about 2 % of a step)
    plan.timing_filter(dom_name)
    _sync()
    marks = [_events()[0] for _ in range(steps + 1)]
    t0 = time.perf_counter()
    marks[0].record()
    for i in range(steps):
        step()
        marks[i + 1].record()
    _sync()
    wall = time.perf_counter() - t0
    plan.timing(False)
    plan.timing_filter(None)
    per_step = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))
    ms = marks[0].elapsed_time(marks[-1]) / steps
    timing = plan.timing_read()
    name, t, achieved = dominant(timing)
    q = lambda f: per_step[min(steps - 1, int(f * steps))]
    out = {
        "E": E, "ms_per_step": ms, "wall_s": wall, "timing": timing, "breakdown": breakdown, "breakdown_steps": nb,
        "plan": plan.describe(),
        "step_ms_p10_p50_p90": [q(0.1), q(0.5), q(0.9)],
        "dominant": name, "achieved_GBs": achieved, "bytes_per_launch": t["bytes_per_launch"],
        "tensors": (x, g, W, y, gx, gW),
    }
    return out


def copy_ceiling_gbs(nbytes=1 << 30, iters=5):
    """Device-to-device copy of a 1 GiB buffer: the practical HBM ceiling."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    ms, _ = time_calls(lambda: b.copy_(a), iters)
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def size_matched_copy(x, y, iters=10, flush=None):
    """A device copy of x into y (the same bytes a digit-group launch reads
    and writes, the same cache flushing): the practical ceiling at this size;
    returns {"GBs": ..., "bytes": ...}."""
    y.copy_(x)
    ms, _ = time_calls(lambda: y.copy_(x), iters, flush=flush)
    nb = 2 * x.numel() * x.element_size()
    return {"GBs": nb / (ms * 1e-3) / 1e9, "bytes": nb}


def _with_copy(e, cp):
    e["size_matched_copy_GBs"] = cp["GBs"]
    e["dominant_frac_of_copy"] = e["achieved_GBs"] / cp["GBs"]
    return e


def cpu_baseline_headline(tensors, budget_s=30.0):
    """FP64 oracle (numpy, single core) on the headline workload: forward +
    gradient of whole instances, timed, until every instance is done or about
    budget_s of CPU work; also the GPU error on those instances (y and gx per
    instance; gW, a sum over instances, when all of them were done)."""
    from oracle import gtt_oracle as O
    x, g, W, y, gx, gW = tensors
    b, n = 8, 6
    W64 = W.cpu().to(__import__("torch").complex128).numpy()
    try:
        prev = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(prev)})
    except (AttributeError, OSError):
        prev = None
    done = 0
    errs_y, errs_gx = [], []
    rgW = np.zeros((b, b), dtype=np.complex128)
    elapsed = 0.0
    # instances in a fixed scattered order until about budget_s of CPU work
    for i in [(37 * j) % 256 for j in range(256)]:
        xi = x[i].cpu().numpy().astype(np.complex128)
        gi = g[i].cpu().numpy().astype(np.complex128)
        ts = time.perf_counter()
        yi = O.staged(W64, xi, n)
        gxi, gWi = O.grad(W64, xi, gi, n)
        elapsed += time.perf_counter() - ts
        rgW += gWi
        done += 1
        errs_y.append(float(np.linalg.norm(y[i].cpu().numpy() - yi) / np.linalg.norm(yi)))
        errs_gx.append(float(np.linalg.norm(gx[i].cpu().numpy() - gxi) / np.linalg.norm(gxi)))
        if elapsed > budget_s:
            break
    cores = 1
    if prev is not None:
        os.sched_setaffinity(0, prev)
    elems = done * b ** n
    out = {
        "value": elems / elapsed, "unit": "elements/s", "cores": cores, "kind": "oracle",
        "sample": f"{done} of 256 instances (N=262144 c64 upcast to complex128): numpy staged forward + "
                  f"stage-wise gradient, {elapsed:.2f} s on one pinned host core",
        "gpu_rel_err_y_max": max(errs_y), "gpu_rel_err_gx_max": max(errs_gx),
        "cpu_model": _cpu_model(), "cores_available": len(prev) if prev else os.cpu_count(),
    }
    if done == 256:
        gw = gW.cpu().numpy().astype(np.complex128)
        out["gpu_rel_err_gW_all_256"] = float(np.linalg.norm(gw - rgW) / np.linalg.norm(rgW))
    return out


def oracle_rate(fn, elems: int) -> dict:
    """Elements/s of one oracle call on one pinned host core."""
    try:
        prev = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(prev)})
    except (AttributeError, OSError):
        prev = None
    t0 = time.perf_counter()
    out = fn()
    dt = time.perf_counter() - t0
    if prev is not None:
        os.sched_setaffinity(0, prev)
    return {"elements_per_s": elems / dt, "seconds": dt, "cores": 1, "kind": "oracle", "result": out}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# secondary workloads (GPU-only checks: round trips, bit exactness, the plain
# FP32 path as reference for the bf16 ragged batch)
# ---------------------------------------------------------------------------
def _gpu():
    import torch
    return torch.device("cuda:0")


def _flusher():
    import torch
    scratch = torch.empty(1 << 28, dtype=torch.float32, device=_gpu())  # 1 GiB
    return lambda: scratch.zero_()  # evicts the 256 MB Infinity Cache


def _timed_plan(p, fn, iters, flush=None):
    """Median ms of fn() without instrumentation, and the plan's per-kernel
    timing (HIP events around every launch) over as many further calls."""
    fn()
    _sync()
    ms, _ = time_calls(fn, iters, flush=flush)
    p.timing(True)
    time_calls(fn, iters, flush=flush)
    tm = p.timing_read()
    p.timing(False)
    return ms, tm


def _dominant_entry(tm, E, flops_per_elem_digit=None):
    """The kernel with the largest share: its HBM rate and fraction; with
    flops_per_elem_digit (the algorithmic vector-ALU flops of one digit pass
    per element: 2b real, 8b complex, twice that for a backward digit), also
    its ALU view against the vector peak and which roofline binds it (the
    larger time at peak), with the fraction of that roofline."""
    nm_, t_, ach = dominant(tm)
    e = {"dominant": nm_, "dominant_avg_ms": t_["avg_ms"], "dominant_bytes_per_launch": t_["bytes_per_launch"],
         "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS}
    if flops_per_elem_digit:
        import re
        k = int(re.search(r"k=(\d+)", nm_).group(1))
        flops = float(E) * k * flops_per_elem_digit
        t = t_["avg_ms"] * 1e-3
        alu = flops / t / 1e12
        t_hbm = t_["bytes_per_launch"] / (HBM_PEAK_GBS * 1e9)
        t_alu = flops / (VALU_PEAK_TFLOPS * 1e12)
        e.update({"alu_flops_per_launch": flops, "alu_TFLOPs": alu, "alu_frac": alu / VALU_PEAK_TFLOPS,
                  "bound": "alu" if t_alu > t_hbm else "hbm", "binding_frac": max(t_alu, t_hbm) / t})
    return e


def _backward_entry(p, W, x, iters=10, seed=7, alu=True):
    """Forward keeping the activations between digit groups, then the
    backward (gx and gW) of the same plan, timed alone: elements/s and HBM
    rate of the algorithmic bytes (read gy and x, write gx: 3 E s)."""
    import torch
    from paper_2507_02420_amd.inputs import gaussian
    g = torch.from_numpy(gaussian(tuple(x.shape), seed=seed, complex_=x.is_complex()).astype(
        np.complex64 if x.is_complex() else np.float32)).to(x.device).to(x.dtype)
    _, _, sv = p.workspace_size()
    saved = torch.empty(max(sv, 16), dtype=torch.uint8, device=x.device)
    y = torch.empty_like(x)
    p.forward(W, x, y, saved=saved)
    gx = torch.empty_like(x)
    gW = torch.empty_like(W)
    ms, tm = _timed_plan(p, lambda: p.backward(W, x, g, saved=saved, gx=gx, gW=gW), iters)
    E = x.numel()
    alg = 3.0 * E * x.element_size()
    bw = {k: v for k, v in tm.items() if k.startswith("bwd")}
    return {"ms": ms, "elements_per_s": E / (ms * 1e-3), "algorithmic_bytes": alg,
            "algorithmic_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "round_trips": len(p.describe()["bwd_groups"]),
            **_dominant_entry(bw, E, (16 if x.is_complex() else 4) * p.describe()["b"] if alu else None),
            "kernels": tm}


def wl_c1(iters=50, cpu=True):
    """Single FP64 vector, b=2, n=10: normalised Hadamard and a random 2x2
    orthogonal W; latency-bound (one wave: digits 0-3 in registers, 4-9
    across lanes)."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import gaussian, hadamard2, haar_unitary
    res = {}
    xn = gaussian(1024, seed=11)
    x = torch.from_numpy(xn).to(_gpu())
    p = G.Plan(2, 10, 1, torch.float64)
    for nm, Wn in (("hadamard", hadamard2(True)), ("orthogonal", haar_unitary(2, 12, complex_=False))):
        Wt = torch.from_numpy(Wn).to(_gpu())
        y = torch.empty_like(x)
        ms, _ = time_calls(lambda: p.forward(Wt, x, y), iters)
        # the kernel alone (HIP events around its launch, inside the library):
        # a call is mostly host-side launch latency at this size
        p.timing(True)
        for _ in range(iters):
            p.forward(Wt, x, y)
        _sync()
        tm = p.timing_read()
        p.timing(False)
        kern = {k: v["avg_ms"] * 1e3 for k, v in tm.items()}
        e = {"us_per_call": ms * 1e3, "elements_per_s": 1024 / (ms * 1e-3), "kernel_us": kern}
        if cpu:
            from oracle import gtt_oracle as O
            r = oracle_rate(lambda: O.dense(Wn, xn, 10), 1024)
            ref = r.pop("result")
            r["form"] = "dense 1024 x 1024 Kronecker matvec"
            e["cpu_oracle"] = r
            e["rel_err_vs_dense"] = float(np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref))
        res[f"f64_b2_n10_{nm}"] = e
    return res


def wl_c2(iters=10, cpu=True):
    """64 x complex64, b=4, n=10: forward then inverse."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary
    b, n, batch = 4, 10, 64
    xn = gaussian((batch, b ** n), seed=21, complex_=True).astype(np.complex64)
    x = torch.from_numpy(xn).to(_gpu())
    W = torch.from_numpy(haar_unitary(4, 22).astype(np.complex64)).to(_gpu())
    p = G.Plan(b, n, batch, torch.complex64)
    y = torch.empty_like(x)
    xr = torch.empty_like(x)
    ms, tm = _timed_plan(p, lambda: (p.forward(W, x, y), p.inverse(W, y, xr)), iters)
    E = batch * b ** n
    err = float((torch.linalg.vector_norm(xr - x) / torch.linalg.vector_norm(x)).item())
    e = {"ms": ms, "elements_per_s": E / (ms * 1e-3), "roundtrip_rel_err": err, **_dominant_entry(tm, E, 8 * b),
         "kernels": tm, "backward": _backward_entry(p, W, x)}
    _with_copy(e, size_matched_copy(x, xr))
    if cpu:
        from oracle import gtt_oracle as O
        W64 = W.cpu().to(torch.complex128).numpy()
        x0 = xn[0].astype(np.complex128)
        r = oracle_rate(lambda: O.staged(W64, x0, n), b ** n)
        ref = r.pop("result")
        r["sample"] = "instance 0 (N=1048576), numpy staged forward"
        e["cpu_oracle"] = r
        e["rel_err_fwd_instance0_vs_oracle"] = float(np.linalg.norm(y[0].cpu().numpy() - ref) / np.linalg.norm(ref))
    return e


def wl_c3a(iters=10, cpu=True):
    """16 x float32, b=3, n=13 (odd strides), MALL flushed."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import haar_unitary, uniform
    b, n, batch = 3, 13, 16
    xn = uniform((batch, b ** n), seed=31).astype(np.float32)
    x = torch.from_numpy(xn).to(_gpu())
    W = torch.from_numpy(haar_unitary(3, 32, complex_=False).astype(np.float32)).to(_gpu())
    p = G.Plan(b, n, batch, torch.float32)
    y = torch.empty_like(x)
    ms, tm = _timed_plan(p, lambda: p.forward(W, x, y), iters, flush=_flusher())
    xr = p.inverse(W, y)
    err = float((torch.linalg.vector_norm(xr - x) / torch.linalg.vector_norm(x)).item())
    E = batch * b ** n
    e = {"ms": ms, "elements_per_s": E / (ms * 1e-3), "roundtrip_rel_err": err, **_dominant_entry(tm, E, 2 * b),
         "kernels": tm, "backward": _backward_entry(p, W, x)}
    _with_copy(e, size_matched_copy(x, xr, flush=_flusher()))
    if cpu:
        from oracle import gtt_oracle as O
        W64 = W.cpu().double().numpy()
        x0 = xn[0].astype(np.float64)
        r = oracle_rate(lambda: O.staged(W64, x0, n), b ** n)
        ref = r.pop("result")
        r["sample"] = "instance 0 (N=1594323), numpy staged forward"
        e["cpu_oracle"] = r
        e["rel_err_fwd_instance0_vs_oracle"] = float(np.linalg.norm(y[0].cpu().double().numpy() - ref) /
                                                     np.linalg.norm(ref))
    return e


def wl_c3b(iters=10, cpu=True):
    """16 x int32, b=2, n=20, unnormalised Hadamard, MALL flushed; bit-exact."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import hadamard2, int_uniform
    b, n, batch = 2, 20, 16
    xn = int_uniform((batch, b ** n), seed=33, lo=-100, hi=100)
    xi = torch.from_numpy(xn).to(torch.int32).to(_gpu())
    H = torch.from_numpy(hadamard2(False)).to(torch.int32).to(_gpu())
    p = G.Plan(b, n, batch, torch.int32)
    y = torch.empty_like(xi)
    ms, tm = _timed_plan(p, lambda: p.forward(H, xi, y), iters, flush=_flusher())
    back = p.inverse(H, y)
    exact = bool(torch.equal(back, xi * (1 << n)))
    E = batch * b ** n
    e = {"ms": ms, "elements_per_s": E / (ms * 1e-3), "inverse_of_forward_is_2^n_x_exactly": exact,
         **_dominant_entry(tm, E), "kernels": tm}
    _with_copy(e, size_matched_copy(xi, back, flush=_flusher()))
    if cpu:
        from oracle import gtt_oracle as O
        r = oracle_rate(lambda: O.staged_int32(hadamard2(False).astype(np.int64), xn[0], n), b ** n)
        ref = r.pop("result")
        r["sample"] = "instance 0 (N=1048576), exact integer staged forward"
        e["cpu_oracle"] = r
        e["fwd_instance0_bit_exact_vs_oracle"] = bool(np.array_equal(y[0].cpu().numpy(), ref))
    return e


def wl_c5(iters=5, cpu=True):
    """Ragged bf16 batch: 1024 instances, b in {2,4,16,32}, N in [2^10, 2^20],
    against the plain FP32 path (the same plan with f32 storage)."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import haar_unitary, ragged_shapes
    shapes = ragged_shapes(1024, seed=52)
    bs = [s_[0] for s_ in shapes]
    ns = [s_[1] for s_ in shapes]
    Ns = [b_ ** n_ for b_, n_ in shapes]
    Ntot = sum(Ns)
    rng = np.random.default_rng(53)
    x32 = torch.from_numpy(rng.standard_normal(Ntot, dtype=np.float32)).to(_gpu())
    xb = x32.to(torch.bfloat16)
    xf = xb.to(torch.float32)     # the same values, plain FP32 storage
    del x32
    Ws = [haar_unitary(r, 54 + i, complex_=False).astype(np.float32) for i, r in enumerate((2, 4, 16, 32))]
    Wt = torch.cat([torch.from_numpy(w).reshape(-1) for w in Ws]).to(_gpu())
    pb = G.Plan(bs, ns, 1, torch.bfloat16)
    pf = G.Plan(bs, ns, 1, torch.float32)
    yb = torch.empty_like(xb)
    yf = torch.empty_like(xf)
    msb, tmb = _timed_plan(pb, lambda: pb.forward(Wt, xb, yb), iters)
    msf, _ = _timed_plan(pf, lambda: pf.forward(Wt, xf, yf), iters)
    # the same batch as ONE persistent launch (grid barriers between phases)
    pp = G.Plan(bs, ns, 1, torch.bfloat16, flags=G.FLAG_PERSISTENT)
    yp = torch.empty_like(xb)
    pp.forward(Wt, xb, yp)
    msp, _ = time_calls(lambda: pp.forward(Wt, xb, yp), iters)
    pp.check()
    # the default per-phase launches captured in a HIP graph: one launch
    # for the caller (the work list was uploaded by the plan)
    yg = torch.empty_like(xb)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pb.forward(Wt, xb, yg)
    yg.zero_()
    msg, _ = time_calls(graph.replay, iters)
    _sync()
    same = bool(torch.equal(yp, yb)) and bool(torch.equal(yg, yb))
    # HBM: algorithmic bytes (read x, write y once: 2 E s) and the bytes the
    # launches move (every digit-group phase reads and writes its instances)
    alg = 2.0 * Ntot * 2
    moved = sum(v["bytes_per_launch"] * v["launches"] for v in tmb.values()) / iters
    ms_launches = sum(v["total_ms"] for v in tmb.values()) / iters
    per_class = {}
    for k, v in tmb.items():
        cls = k.split(" ", 3)[-1]
        c = per_class.setdefault(cls, {"ms": 0.0, "bytes": 0.0})
        c["ms"] += v["total_ms"] / iters
        c["bytes"] += v["bytes_per_launch"] * v["launches"] / iters
    for c in per_class.values():
        c["GBs"] = c["bytes"] / (c["ms"] * 1e-3) / 1e9
        c["frac"] = c["GBs"] / HBM_PEAK_GBS
    e = {"elements": Ntot, "ms_bf16": msb, "elements_per_s_bf16": Ntot / (msb * 1e-3),
         "ms_bf16_persistent_launch": msp, "ms_bf16_graph_replay": msg,
         "persistent_and_graph_equal_phases": same,
         "ms_plain_fp32": msf, "elements_per_s_plain_fp32": Ntot / (msf * 1e-3), "speedup_vs_plain_fp32": msf / msb,
         "hbm": {"algorithmic_bytes": alg, "algorithmic_frac": alg / (msb * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "moved_bytes": moved, "round_trips": moved / alg,
                 "achieved_frac": moved / (msb * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "achieved_frac_launches_only": moved / (ms_launches * 1e-3) / 1e9 / HBM_PEAK_GBS},
         "classes": per_class}
    # per-instance error of the bf16 path against the FP64 oracle on the
    # stored bf16 values: the first instance of every distinct (b, n) shape
    # and the last instance of each radix's largest shape
    from oracle import gtt_oracle as O
    offs = np.cumsum([0] + Ns)
    first = {}
    for t, s_ in enumerate(shapes):
        first.setdefault(s_, t)
    last_largest = [max((t for t in range(1024) if shapes[t][0] == b), key=lambda t: (Ns[t], t)) for b in (2, 4, 16, 32)]
    pick = sorted(set(first.values()) | set(last_largest))
    ridx = {2: 0, 4: 1, 16: 2, 32: 3}
    errs, errs32 = {}, {}
    t_or, n_or = 0.0, 0
    for t in pick:
        b_, n_ = shapes[t]
        a, c = int(offs[t]), int(offs[t + 1])
        xv = xb[a:c].float().cpu().double().numpy()
        ts = time.perf_counter()
        ref = O.staged(Ws[ridx[b_]].astype(np.float64), xv, n_)
        t_or += time.perf_counter() - ts
        n_or += c - a
        errs.setdefault(b_, []).append(float(np.linalg.norm(yb[a:c].float().cpu().double().numpy() - ref) /
                                             np.linalg.norm(ref)))
        errs32.setdefault(b_, []).append(float(np.linalg.norm(yf[a:c].cpu().double().numpy() - ref) /
                                               np.linalg.norm(ref)))
    e["rel_err_vs_fp64_oracle"] = {f"b={b_}": {"max": max(v), "median": float(np.median(v)), "instances": len(v)}
                                   for b_, v in sorted(errs.items())}
    e["plain_fp32_rel_err_vs_fp64_oracle"] = {f"b={b_}": {"max": max(v), "median": float(np.median(v))}
                                              for b_, v in sorted(errs32.items())}
    e["instances_checked"] = len(pick)
    if cpu:
        e["cpu_oracle"] = {"elements_per_s": n_or / t_or, "seconds": t_or, "cores": 1, "kind": "oracle",
                           "sample": f"{len(pick)} instances ({n_or} elements): one of every distinct (b, n) "
                                     "shape and each radix's largest, numpy staged forward (FP64)"}
    return e


def wl_mixed(iters=10, cpu=True):
    """Distinct factors W_0 kron ... kron W_5 (remark on distinct tensor
    factors after Def. 2.4), radices 8, 3, 4, 5, 2, 7 (N = 6720), 4096 x
    complex64: forward then inverse, and the backward (gx and every
    factor's gradient)."""
    import re as _re
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary
    radices, batch = [8, 3, 4, 5, 2, 7], 4096
    N = int(np.prod(radices))
    xn = gaussian((batch, N), seed=81, complex_=True).astype(np.complex64)
    x = torch.from_numpy(xn).to(_gpu())
    Ws = [haar_unitary(r, 82 + i).astype(np.complex64) for i, r in enumerate(radices)]
    W = torch.cat([torch.from_numpy(w).reshape(-1) for w in Ws]).to(_gpu())
    p = G.Plan.mixed(radices, batch, torch.complex64)
    y = torch.empty_like(x)
    xr = torch.empty_like(x)
    ms, tm = _timed_plan(p, lambda: (p.forward(W, x, y), p.inverse(W, y, xr)), iters)
    E = batch * N
    err = float((torch.linalg.vector_norm(xr - x) / torch.linalg.vector_norm(x)).item())
    e = {"radices": radices, "ms": ms, "elements_per_s": E / (ms * 1e-3), "roundtrip_rel_err": err,
         **_dominant_entry(tm, E), "kernels": tm}
    # ALU view of the dominant group: 8 b_j real flops per element and digit
    # j of the group (digit j has the radix of factor m-1-j)
    m_ = _re.search(r"s0=(\d+) k=(\d+)", e["dominant"])
    if m_:
        s0, k = int(m_.group(1)), int(m_.group(2))
        rd = radices[::-1]
        flops = 8.0 * E * sum(rd[s0:s0 + k])
        e["alu_flops_per_launch"] = flops
        e["alu_frac"] = flops / (e["dominant_avg_ms"] * 1e-3) / 1e12 / VALU_PEAK_TFLOPS
    e["backward"] = _backward_entry(p, W, x, alu=False)
    _with_copy(e, size_matched_copy(x, xr))
    if cpu:
        from oracle import gtt_oracle as O
        Ws64 = [w.astype(np.complex128) for w in Ws]
        x0 = xn[:4].astype(np.complex128)
        r = oracle_rate(lambda: O.staged_mixed(Ws64, x0), 4 * N)
        ref = r.pop("result")
        r["sample"] = "instances 0-3 (4 x 6720), numpy staged forward with distinct factors"
        e["cpu_oracle"] = r
        e["rel_err_fwd_instances0_3_vs_oracle"] = float(np.linalg.norm(y[:4].cpu().numpy() - ref) /
                                                        np.linalg.norm(ref))
    return e


def wl_filter(iters=10, cpu=True):
    """Natural-order filter (classical form of Alg. 3): 64 x complex64,
    b=4, n=10, cutoff N/2 -- forward, the coefficients split at the cut-off
    (mask fused into the inverse's tile loads), both parts back."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary
    b, n, batch = 4, 10, 64
    N = b ** n
    xn = gaussian((batch, N), seed=91, complex_=True).astype(np.complex64)
    x = torch.from_numpy(xn).to(_gpu())
    W = torch.from_numpy(haar_unitary(4, 92).astype(np.complex64)).to(_gpu())
    p = G.Plan(b, n, batch, torch.complex64)
    out = {}
    ms, tm = _timed_plan(p, lambda: out.update(zip(("lo", "hi"), p.filter(W, x, N // 2))), iters)
    E = batch * N
    lo, hi = out["lo"], out["hi"]
    split_err = float((torch.linalg.vector_norm(lo + hi - x) / torch.linalg.vector_norm(x)).item())
    e = {"cutoff": N // 2, "ms": ms, "elements_per_s": E / (ms * 1e-3), "low_plus_high_vs_x_rel_err": split_err,
         **_dominant_entry(tm, E, 8 * b), "kernels": tm}
    if cpu:
        from oracle import gtt_oracle as O
        W64 = W.cpu().to(torch.complex128).numpy()
        x0 = xn[0].astype(np.complex128)
        r = oracle_rate(lambda: O.natural_filter(W64, x0, n, N // 2), N)
        rlo, rhi = r.pop("result")
        r["sample"] = "instance 0 (N=1048576), numpy forward, split, two inverses"
        e["cpu_oracle"] = r
        e["rel_err_low_instance0_vs_oracle"] = float(np.linalg.norm(lo[0].cpu().numpy() - rlo) / np.linalg.norm(rlo))
        e["rel_err_high_instance0_vs_oracle"] = float(np.linalg.norm(hi[0].cpu().numpy() - rhi) / np.linalg.norm(rhi))
    return e


def wl_compress(iters=10, cpu=True):
    """State transmission (§4.1.1): 16 x float32, b=2, n=20, the k = N/64
    coefficients of largest magnitude per instance (radix select, ascending
    indices) and the reconstruction from them."""
    import torch
    from paper_2507_02420_amd import gtt as G
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary
    b, n, batch = 2, 20, 16
    N = b ** n
    k = N // 64
    xn = gaussian((batch, N), seed=101).astype(np.float32)
    x = torch.from_numpy(xn).to(_gpu())
    W = torch.from_numpy(haar_unitary(2, 102, complex_=False).astype(np.float32)).to(_gpu())
    p = G.Plan(b, n, batch, torch.float32)
    out = {}
    ms, tm = _timed_plan(p, lambda: out.update(zip(("idx", "val", "recon"), p.compress(W, x, k))), iters)
    E = batch * N
    e = {"k": k, "ms": ms, "elements_per_s": E / (ms * 1e-3), **_dominant_entry(tm, E), "kernels": tm}
    if cpu:
        from oracle import gtt_oracle as O
        W64 = W.cpu().to(torch.float64).numpy()
        x0 = xn[0].astype(np.float64)
        r = oracle_rate(lambda: O.topk_compress(W64, x0, n, k), N)
        ridx, rval, rrec = r.pop("result")
        r["sample"] = "instance 0 (N=1048576), numpy forward, top-k, inverse"
        e["cpu_oracle"] = r
        e["instance0_indices_equal_oracle"] = bool(np.array_equal(out["idx"][0].cpu().numpy(), ridx))
        e["rel_err_recon_instance0_vs_oracle"] = float(np.linalg.norm(out["recon"][0].cpu().numpy() - rrec) /
                                                       np.linalg.norm(rrec))
    return e


def wl_wtune(steps=10, cpu=True):
    """Gradient-based tuning of W (§4.2): 256 x complex64, b=8, n=4, k=64
    kept coefficients; one step = top-k selection + backward (gW only) +
    Cayley retraction, with the host reading the kept energy each step."""
    import torch
    from paper_2507_02420_amd import wtune
    from paper_2507_02420_amd.inputs import gaussian, haar_unitary
    b, n, batch, k = 8, 4, 256, 64
    N = b ** n
    xn = gaussian((batch, N), seed=111, complex_=True).astype(np.complex64)
    x = torch.from_numpy(xn).to(_gpu())
    W0 = torch.from_numpy(haar_unitary(8, 112).astype(np.complex64)).to(_gpu())
    wtune.tune(x, W0, b, n, k, steps=2, backtrack=False)  # warm-up (plan, kernels)
    _sync()
    t0 = time.perf_counter()
    res = wtune.tune(x, W0, b, n, k, steps=steps, backtrack=False)
    _sync()
    dt = (time.perf_counter() - t0) / steps
    E = batch * N
    e = {"k": k, "steps": steps, "ms_per_step": dt * 1e3, "elements_per_s": E / dt,
         "kept_fraction_first_last": [res.kept_fraction[0], res.kept_fraction[-1]]}
    if cpu:
        from oracle import gtt_oracle as O
        W64 = W0.cpu().to(torch.complex128).numpy()
        x0 = xn[0].astype(np.complex128)

        def one():
            idx, val, _ = O.topk_compress(W64, x0, n, k)
            g = np.zeros(N, dtype=np.complex128)
            g[idx] = 2 * val
            return O.grad(W64, x0, g, n)
        r = oracle_rate(one, N)
        r.pop("result")
        r["sample"] = "instance 0 (N=4096): numpy forward, top-k and gradient (one step's transform work)"
        e["cpu_oracle"] = r
    return e


WL_NAMES = {"c1": "f64_b2_n10", "c2": "c64_b4_n10_x64_fwd_inv", "c3a": "f32_b3_n13_x16_fwd",
            "c3b": "i32_hadamard_b2_n20_x16_fwd", "c5": "ragged_bf16_1024",
            "mixed": "c64_mixed_8_3_4_5_2_7_x4096_fwd_inv", "filter": "c64_b4_n10_x64_filter",
            "compress": "f32_b2_n20_x16_topk_n64", "wtune": "c64_b8_n4_x256_wtune_k64"}

WORKLOADS = {"c1": wl_c1, "c2": wl_c2, "c3a": wl_c3a, "c3b": wl_c3b, "c5": wl_c5,
             "mixed": wl_mixed, "filter": wl_filter, "compress": wl_compress, "wtune": wl_wtune}


def secondary(cpu=True, only=None):
    res = {}
    for k, fn in WORKLOADS.items():
        if only and k not in only:
            continue
        print(f"bench: workload {k}", file=sys.stderr, flush=True)
        r = fn(cpu=cpu)
        if k == "c1":
            res.update(r)
        else:
            res[WL_NAMES[k]] = r
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", default="",
                    help="comma-separated secondary workloads to run alone (c1,c2,c3a,c3b,c5), no headline "
                         "(for profiling); prints their JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.only:
        only = [w.strip() for w in args.only.split(",") if w.strip()]
        bad = [w for w in only if w not in WORKLOADS]
        if bad:
            print(f"unknown workloads {bad}; known: {sorted(WORKLOADS)}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps(secondary(cpu=not args.no_cpu, only=only)), flush=True)
        return
    print("bench: headline fwd+bwd 256 x 8^6 c64", file=sys.stderr, flush=True)
    h = headline(args.steps, args.warmup)
    E = h["E"]
    value = E / (h["ms_per_step"] * 1e-3)
    traffic = load_traffic(h["dominant"], "c64_b8_n6_x256")
    t_dom = h["timing"][h["dominant"]]
    flops = kernel_flops(h["dominant"], E)
    achieved_tf = flops / (t_dom["avg_ms"] * 1e-3) / 1e12
    hbm_view = {"achieved": h["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": h["achieved_GBs"] / HBM_PEAK_GBS}
    mfma_view = {"achieved": achieved_tf, "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": achieved_tf / MFMA_F32_PEAK_TFLOPS, "algorithmic_flops_per_launch": flops}
    # the binding roofline: the larger of the two times at peak
    t_hbm = h["bytes_per_launch"] / (HBM_PEAK_GBS * 1e9)
    t_mfma = flops / (MFMA_F32_PEAK_TFLOPS * 1e12)
    bound, view = ("mfma", mfma_view) if t_mfma > t_hbm else ("hbm", hbm_view)
    roof = {"bound": bound, "achieved": view["achieved"], "peak": view["peak"], "unit": view["unit"],
            "frac": view["frac"], "traffic": traffic,
            "kernel": h["dominant"], "algorithmic_bytes_per_launch": h["bytes_per_launch"],
            "hbm_view": hbm_view, "mfma_view": mfma_view,
            "round_trips_measured_over_algorithmic": (traffic / h["bytes_per_launch"]) if traffic else None,
            "copy_ceiling_GBs": copy_ceiling_gbs()}
    # directions: kernel times of the breakdown steps (every launch timed)
    directions = {}
    for d, pref in (("forward", "pass"), ("backward", "bwd")):
        ks = [v for k, v in h["breakdown"].items() if k.startswith(pref) or (d == "backward" and k.startswith("reduce"))]
        by = sum(v["bytes_per_launch"] * v["launches"] for v in ks)
        ms_ = sum(v["total_ms"] for v in ks)
        directions[d] = {"ms": ms_ / h["breakdown_steps"], "GBs": by / (ms_ * 1e-3) / 1e9,
                         "frac_of_hbm_peak": by / (ms_ * 1e-3) / 1e9 / HBM_PEAK_GBS}
    cpu = None
    if not args.no_cpu:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline_headline(h["tensors"])
    extra = None
    if not args.no_extra:
        extra = secondary(cpu=not args.no_cpu)
    line = {
        "metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_step"], "step_ms_p10_p50_p90": h["step_ms_p10_p50_p90"],
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "fwd+bwd: 256 x complex64, b=8, n=6 (N=262144), W 8x8 unitary, L=Re<g,y>",
                   "b": 8, "n": 6, "batch": 256, "elements": E, "parallelism": "single GPU"},
        "roofline": roof, "directions": directions, "cpu_baseline": cpu,
        "kernels": {k: {kk: round(vv, 6) if isinstance(vv, float) else vv for kk, vv in v.items()}
                    for k, v in h["breakdown"].items()},
        "kernels_note": ("per-kernel HIP-event times of separate steps before the timed region; "
                         "in the timed region only the dominant kernel carries events"),
        "workloads": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
