"""CPU checks of the C ABI: the library loads, exports every declared symbol,
passes its host self-test, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest
import torch

from conftest import ROOT

torch = pytest.importorskip("torch")
from paper_2507_02420_amd import gtt as G  # noqa: E402


def header_symbols():
    with open(os.path.join(ROOT, "include", "gtt.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:gtt_status|const char\*)\s+(gtt_\w+)\s*\(", src, re.M)))


def test_exports_match_header():
    L = G.lib()
    syms = header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(G.EXPORTS) == syms


def test_selftest():
    assert G.selftest() == 0


def test_status_strings():
    L = G.lib()
    for code, name in G.STATUS_NAMES.items():
        assert L.gtt_status_string(code).decode() == name


def _plan(count, b, n, batch=1, dtype=G.F32, flags=0, x_off=None, w_idx=None):
    L = G.lib()
    h = ctypes.c_void_p()
    arr = lambda t, v: None if v is None else (t * len(v))(*v)
    st = L.gtt_plan(ctypes.byref(h), count, arr(ctypes.c_int32, b), arr(ctypes.c_int32, n), batch,
                    arr(ctypes.c_int64, x_off), arr(ctypes.c_int32, w_idx), dtype, flags)
    return st, h


def test_plan_validation():
    L = G.lib()
    assert _plan(1, [1], [3])[0] == 2          # b < 2
    assert _plan(1, [2], [-1])[0] == 2         # n < 0
    assert _plan(1, [2], [80])[0] == 2         # b^n overflows
    assert _plan(1, [2], [4], batch=0)[0] == 2
    assert _plan(1, [2], [4], dtype=9)[0] == 3
    assert _plan(1, [2], [4], flags=0x100)[0] == 1
    assert _plan(0, [2], [4])[0] == 1
    assert _plan(2, [2, 4], [4, 2], batch=2)[0] == 2
    assert _plan(2, [2, 4], [4, 2], w_idx=[0, 0])[0] == 1   # W index used with two radices
    assert _plan(2, [2, 4], [4, 2], w_idx=[0, 2])[0] == 1   # W index 1 unused
    h = ctypes.c_void_p()
    assert L.gtt_plan(None, 1, (ctypes.c_int32 * 1)(2), (ctypes.c_int32 * 1)(3), 1, None, None, 1, 0) == 1
    st, h = _plan(1, [3], [0])
    assert st == 0
    assert L.gtt_plan_destroy(h) == 0
    assert L.gtt_plan_destroy(None) == 0


def test_call_validation_before_any_hip_call():
    L = G.lib()
    st, h = _plan(1, [2], [10])
    assert st == 0
    a, m = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x10004)
    S = ctypes.c_void_p()
    assert L.gtt_forward(h, a, a, None, None, None, 0, S) == 1
    assert L.gtt_forward(None, a, a, a, None, None, 0, S) == 1
    assert L.gtt_forward(h, a, m, a, None, None, 0, S) == 4
    assert L.gtt_forward(h, a, a, m, None, None, 0, S) == 4
    assert L.gtt_inverse(h, m, a, a, None, 0, S) == 4
    assert L.gtt_backward(h, a, a, None, a, None, None, None, 0, S) == 1
    assert L.gtt_backward(h, a, a, m, a, a, a, None, 0, S) == 4
    assert L.gtt_filter(h, a, a, -1, a, None, None, 0, S) == 1
    L.gtt_plan_destroy(h)
    st, h = _plan(1, [2], [10], dtype=G.I32)
    assert L.gtt_backward(h, a, a, None, a, a, a, None, 0, S) == 6
    L.gtt_plan_destroy(h)


def test_tuning_validation():
    L = G.lib()
    assert L.gtt_set_tuning(1, 0, G.F32, 0, 0, 0, 0) == 1
    assert L.gtt_set_tuning(2, 0, G.F32, 200 * 1024, 0, 0, 0) == 1
    assert L.gtt_set_tuning(2, 0, G.F32, 0, 0, -1, 0) == 1
    assert L.gtt_set_tuning(2, -1, G.F32, 0, 0, 0, 0) == 1
    assert L.gtt_set_tuning(2, 0, G.F32, 0, 0, 0, 200 * 1024) == 1


def test_tuning_changes_split_and_not_results():
    G.set_tuning(8, torch.complex64, 0, 0, 3, n=6)
    try:
        ks = [g["k"] for g in G.Plan(8, 6, 256, torch.complex64).describe()["groups"]]
    finally:
        G.set_tuning(8, torch.complex64, 0, 0, 0, n=6)
        G.load_tuning()
    assert ks == [3, 3]
    ks = [g["k"] for g in G.Plan(8, 6, 256, torch.complex64).describe()["groups"]]
    assert ks == [4, 2]


def _describe(b, n, batch, dtype):
    p = G.Plan(b, n, batch, dtype)
    return p.describe()


@pytest.mark.parametrize("b,n,batch,dtype,R", [
    (2, 10, 1, torch.float64, 1),          # single FP64 vector, N = 1024
    (4, 10, 64, torch.complex64, 2),       # 64 x 4^10 complex64
    (3, 13, 16, torch.float32, 2),         # 16 x 3^13 float32
    (2, 20, 16, torch.int32, 2),           # 16 x 2^20 int32
    (8, 6, 256, torch.complex64, 2),       # 256 x 8^6 complex64
])
def test_plan_groups_for_workloads(b, n, batch, dtype, R):
    d = _describe(b, n, batch, dtype)
    gs = d["groups"]
    assert len(gs) == R
    assert sum(g["k"] for g in gs) == n
    assert gs[0]["S"] == 1 and gs[0]["C"] == 1
    for g in gs:
        assert g["lds_bytes"] <= 160 * 1024
        assert g["tiles"] * g["tile_elems"] >= (b ** n) * batch
        if g["S"] > 1:
            # strided groups read rows of at least 64 contiguous bytes
            assert g["C"] * {torch.float64: 8, torch.complex64: 8, torch.float32: 4,
                             torch.int32: 4}[dtype] >= 64


def test_mixed_plan_and_describe():
    p = G.Plan.mixed([2, 3, 4, 5], batch=3, dtype=torch.complex64)
    d = p.describe()
    assert d["kind"] == "mixed"
    assert sum(g["k"] for g in d["groups"]) == 4


def test_binding_refuses_host_tensors():
    import pytest
    with pytest.raises(ValueError):
        G._ptr(torch.zeros(4))


def test_planner_layouts_match_compiled_specializations():
    # the radix-8 kernels have compile-time-offset instantiations for the
    # layouts of the 256 x 8^6 complex64 workload (cmfma_c64.hip: FwdLay4,
    # FwdLay2, BwdLay4, BwdLay2); the planner must keep producing them, or
    # that workload silently falls back to run-time offsets
    d = G.Plan(8, 6, 256, torch.complex64).describe()
    fwd = [(g["k"], g["fast_ni"], g["C"], g["pad_shift"], g["fmap"]) for g in d["groups"]]
    bwd = [(g["k"], g["fast_ni"], g["C"], g["pad_shift"], g["fmap"], g["pmap"]) for g in d["bwd_groups"]]
    assert fwd == [(4, 2, 1, 0x1f0a05, 0x1e001b00270017), (2, 2, 64, 0x1f0a05, 0x1e001b)]
    assert bwd == [(4, 2, 1, 0x1f0805, 0x81b031b01870887, 0x7878), (2, 2, 64, 0x1f0905, 0x31d081b, 0)]


def _wave_positions(mask, j):
    # tile-position bits (logC = 0, three bits per digit) that carry the wave
    # index under fibre-bit mask `mask` of digit j
    return {b if b < 3 * j else b + 3 for b in range(8) if not mask >> b & 1}


def test_paired_backward_layout_keeps_each_pair_inside_a_wave():
    # four-digit backward on 4096-element tiles: the fused phases of digits 1
    # and 0, and the recomputing passes of digits 1 and 2, run without a
    # barrier in between; that is sound when both phases of a pair give every
    # wave the same positions, i.e. the same four wave position bits, none in
    # the pair's digits
    g = G.Plan(8, 6, 256, torch.complex64).describe()["bwd_groups"][0]
    assert (g["k"], g["fast_ni"], g["C"]) == (4, 2, 1)
    fm, pm = g["fmap"], g["pmap"]
    w0 = _wave_positions(fm & 0xff, 0)
    w1 = _wave_positions((fm >> 16) & 0xff, 1)
    assert w0 == w1 and len(w0) == 4 and w0 <= set(range(6, 12))
    p1 = _wave_positions(pm & 0xff, 1)
    p2 = _wave_positions((pm >> 8) & 0xff, 2)
    assert p1 == p2 and len(p1) == 4 and p1 <= {0, 1, 2, 9, 10, 11}
    # the loop-step bit (fibre bit 8) is not a wave bit: it is position 11
    # for digits 0..2
    assert 11 not in w0 and 11 not in p1


def test_fp32_intermediate_plan_sizes_and_limits():
    L = G.lib()
    F = G.FLAG_FP32_INTERMEDIATE
    b, n, batch = 4, 8, 3
    E = batch * b ** n
    buf = (E * 4 + 255) // 256 * 256
    for dt in (torch.bfloat16, torch.float16):
        p, q = G.Plan(b, n, batch, dt, flags=F), G.Plan(b, n, batch, torch.float32)
        (f, bw, sv), (f0, bw0, sv0) = p.workspace_size(), q.workspace_size()
        # float32 operand copies ahead of the float32 plan's workspace;
        # saved activations are float32
        assert (f, bw, sv) == (f0 + buf, bw0 + 2 * buf, sv0)
        d = p.describe()
        assert d["fp32_intermediate"] is True and d["dtype"] == G.TORCH_TO_GTT[dt]
        assert [g["k"] for g in d["groups"]] == [g["k"] for g in q.describe()["groups"]]
    # filter and compress refuse such plans before any HIP call
    hp = G.Plan(b, n, batch, torch.bfloat16, flags=F)
    buf16 = ctypes.c_void_p(256)
    assert L.gtt_filter(hp.handle, buf16, buf16, 3, buf16, buf16, buf16, 1 << 30, None) == 6
    assert L.gtt_compress(hp.handle, buf16, buf16, 3, buf16, buf16, buf16, buf16, 1 << 30, None) == 6
    # too small a workspace is refused before any HIP call
    assert L.gtt_forward(hp.handle, buf16, buf16, buf16, None, buf16, 16, None) == 5
    assert L.gtt_forward(hp.handle, buf16, buf16, buf16, None, None, 0, None) == 5
    assert L.gtt_backward(hp.handle, buf16, buf16, None, buf16, buf16, buf16, buf16, 16, None) == 5
    # ragged and mixed-radix plans: unsupported
    assert _plan(2, [2, 4], [4, 2], dtype=G.BF16, flags=F)[0] == 6
    h = ctypes.c_void_p()
    assert L.gtt_plan_mixed(ctypes.byref(h), 2, (ctypes.c_int32 * 2)(2, 3), 1, G.BF16, F) == 6
    # the flag alone on float32 / int32 plans changes nothing
    assert (G.Plan(b, n, batch, torch.float32, flags=F).workspace_size()
            == G.Plan(b, n, batch, torch.float32).workspace_size())
    assert "fp32_intermediate" not in G.Plan(b, n, batch, torch.int32, flags=F).describe()


def _phys(x, pad):
    return x + sum(x >> ((pad >> (8 * i)) & 31) for i in range(3))


def _mfma_bank_cost(B, k, logC, pad, tileE, lds16):
    # worst bank degree per half-wave (32 banks) of the LDS accesses of a
    # matrix-core pass, in 32-bit words: an FP32 tile holds element x in
    # word _phys(x), a 16-bit tile in word _phys(x >> 1).  Tile transfers move
    # four words a thread; per digit, element 4q+v of the fibre of lane
    # (q, i): four accesses, or two word accesses for a contiguous digit of
    # a 16-bit tile.  Lanes on one word do not conflict.  A sample of the tile.
    def degree(addrs):
        tot = 0
        for h in (addrs[:32], addrs[32:]):
            per = {}
            for a in set(h):
                per.setdefault(a & 31, set()).add(a)
            tot += max(len(v) for v in per.values())
        return tot
    word = (lambda x: _phys(x >> 1, pad)) if lds16 else (lambda x: _phys(x, pad))
    vec = 8 if lds16 else 4
    cost = 0
    for w0 in range(0, tileE // vec - 63, 256):
        for e in range(4):
            cost += degree([_phys(4 * (w0 + l) + e, pad) for l in range(64)])
    F = tileE // B
    for j in range(k):
        bj = B ** j
        step = bj << logC
        vs = (0, 2) if lds16 and step == 1 else (0, 1, 2, 3)
        for grp in range(0, (F + 15) // 16, 4):
            for h in range(B // 16):
                for v in vs:
                    addrs = []
                    for lane in range(64):
                        q, lo = lane >> 4, lane & 15
                        f = (grp * 16 + lo) % F
                        c, f1 = f & ((1 << logC) - 1), f >> logC
                        lam0 = (((f1 // bj) * bj * B + f1 % bj) << logC) | c
                        addrs.append(word(lam0 + (16 * h + 4 * q + v) * step))
                    cost += degree(addrs)
    return cost


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16, torch.float32], ids=str)
@pytest.mark.parametrize("b,n,batch", [(16, 4, 4096), (32, 3, 64), (16, 5, 4)])
def test_matrix_core_lds_padding(b, n, batch, dtype):
    nopad = 31 | (31 << 8) | (31 << 16)
    lds16 = dtype != torch.float32   # 16-bit storage keeps a 16-bit tile; pads count words
    # the built-in tile budgets (the tuning table may choose others)
    for g in G.Plan(b, n, batch, dtype, flags=G.FLAG_NO_TUNE).describe()["groups"]:
        assert g["kind"] == "mfma"
        pad, tileE = g["pad_shift"], g["tile_elems"]
        units = (tileE + 1) // 2 if lds16 else tileE
        shifts = [(pad >> (8 * i)) & 31 for i in range(3)]
        # a 16-byte vector (four words) never straddles a pad; growth <= 1/8
        assert all((1 << s_) >= 4 for s_ in shifts)
        assert _phys(units, pad) - units <= units // 8
        assert g["lds_bytes"] == (_phys(units, pad) + 1) * 4
        # 16-bit tiles hold twice the elements of FP32 ones in the same LDS
        assert tileE * (2 if lds16 else 4) in (32768, 65536) or tileE < 8192
        logC = g["C"].bit_length() - 1
        chosen = _mfma_bank_cost(b, g["k"], logC, pad, tileE, lds16)
        plain = _mfma_bank_cost(b, g["k"], logC, nopad, tileE, lds16)
        assert chosen <= plain
        if g["C"] > 1:  # strided tiles: the unpadded layout conflicts
            assert chosen < plain


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.complex64], ids=str)
def test_ragged_packed_instances_off_16_byte_boundary(dtype):
    # packed back to back, the instances after one of 3 elements start off
    # a 16-byte boundary and must move their tiles element by element
    shapes = [(3, 1), (2, 5), (16, 3), (4, 2)]
    p = G.Plan([b for b, _ in shapes], [n for _, n in shapes], 1, dtype)
    assert p.describe()["scalar_instances"] == 3
    aligned = [(2, 5), (16, 3), (4, 2)]
    p = G.Plan([b for b, _ in aligned], [n for _, n in aligned], 1, dtype)
    assert p.describe()["scalar_instances"] == 0


# element sizes of the storage dtypes (vector-mode tiles move 16 bytes a lane)
_ES = {torch.float64: 8, torch.float32: 4, torch.complex64: 8, torch.complex128: 16, torch.int32: 4}


@pytest.mark.parametrize("dtype", list(_ES))
def test_vector_tile_address_walk(dtype):
    """The VALU pass kernels of power-of-two radices take the addresses of a
    vector-mode tile as a walk: lane tid's m-th 16-byte vector at global
    element g0 + m * gstep and at LDS element l0 + m * lstep, when the pads'
    periods divide 256 vectors and row tiles hold one hi block with rows of at
    most 256 vectors.  This re-derives both address maps from the plan's
    geometry and checks that, wherever that condition holds, the walk equals
    the per-vector formulas (row decomposition, lds_phys)."""
    KT = 256
    V = 16 // _ES[dtype]
    lv = V.bit_length() - 1

    def lds_phys(x, ps):
        return x + sum(x >> ((ps >> (8 * k)) & 31) for k in range(3))

    def per_vector(g, t, i):
        tileE = g["tile_elems"]
        if g["mode"] == 0:
            return t * tileE + i * V
        lcv = g["logC"] - lv
        hb, l = divmod(t, g["L"])
        r, cc = i >> lcv, i & ((1 << lcv) - 1)
        p, gg = divmod(r, g["G"]) if g["P"] != 1 else (0, r)
        return (hb * g["P"] + p) * (g["G"] * g["S"]) + gg * g["S"] + (l << g["logC"]) + cc * V

    walked = 0
    for b in (2, 4, 8):
        for n in range(4, 15):
            for batch in (1, 5):
                if b ** n * batch > 2 ** 20:
                    continue
                for g in G.Plan(b, n, batch, dtype).describe()["groups"]:
                    if g["mode"] not in (0, 2):
                        continue
                    g["logC"] = g["C"].bit_length() - 1
                    shifts = [(g["pad_shift"] >> (8 * k)) & 31 for k in range(3)]
                    ok = all(s == 31 or s <= 8 + lv for s in shifts) and (
                        g["mode"] == 0 or (g["P"] == 1 and lv <= g["logC"] <= 8 + lv))
                    if not ok:
                        continue
                    walked += 1
                    lcv = g["logC"] - lv
                    nvec = g["tile_elems"] // V
                    for t in sorted({0, g["tiles"] // 2, g["tiles"] - 1}):
                        hb, l = divmod(t, g["L"])
                        for tid in range(0, KT, 7):
                            if g["mode"] == 0:
                                g0, gs = t * g["tile_elems"] + tid * V, KT * V
                            else:
                                g0 = (hb * g["G"] * g["S"] + (l << g["logC"]) + (tid >> lcv) * g["S"]
                                      + (tid & ((1 << lcv) - 1)) * V)
                                gs = (KT >> lcv) * g["S"]
                            l0, ls = lds_phys(tid * V, g["pad_shift"]), lds_phys(KT * V, g["pad_shift"])
                            for m, i in enumerate(range(tid, nvec, KT)):
                                assert g0 + m * gs == per_vector(g, t, i)
                                assert l0 + m * ls == lds_phys(i * V, g["pad_shift"])
    assert walked > 0


@pytest.mark.parametrize("dtype", [torch.float32, torch.complex64, torch.int32])
def test_last_stage_direct_store_covers_tile(dtype):
    """Power-of-two-radix VALU pass kernels store the group's last
    super-stage straight to global memory (contiguous tiles, and row tiles
    of one hi block).  Re-derive each lane's fibre and its 32-bit element
    offsets from the plan's geometry: every tile element is written exactly
    once, at the address of the tile-to-memory map, within 2^31 bytes."""
    es = _ES[dtype]
    checked = 0
    for b, rd in ((2, 4), (4, 2), (8, 1)):
        for n in range(1, 13):
            for batch in (1, 3):
                if b ** n * batch > 2 ** 18:
                    continue
                for g in G.Plan(b, n, batch, dtype).describe()["groups"]:
                    k, logc = g["k"], g["C"].bit_length() - 1
                    if g["kind"] != "valu" or k == 0 or not (g["mode"] == 0 or (g["mode"] == 2 and g["P"] == 1)):
                        continue
                    checked += 1
                    j = rd * ((k - 1) // rd)
                    nb, bj, bjr, cm = b ** (k - j), b ** j, b ** k, (1 << logc) - 1
                    tile_e, step, row = g["tile_elems"], bj << logc, g["mode"] == 2
                    for t in sorted({0, g["tiles"] - 1}):
                        hb, l = divmod(t, g["L"])
                        gt0 = hb * g["G"] * g["S"] + (l << logc) if row else t * tile_e
                        seen = set()
                        for f in range(tile_e // nb):
                            q, glo = divmod(f >> logc, bj)
                            lam0 = ((q * bjr + glo) << logc) | (f & cm)
                            o0 = (lam0 >> logc) * g["S"] + (lam0 & cm) if row else lam0
                            om = bj * g["S"] if row else step
                            for m in range(nb):
                                lam = lam0 + m * step
                                want = (gt0 + (lam >> logc) * g["S"] + (lam & cm)) if row else gt0 + lam
                                assert gt0 + o0 + m * om == want
                                assert (o0 + m * om) * es < 2 ** 31
                                seen.add(lam)
                        assert seen == set(range(tile_e))
    assert checked > 0


def test_check_and_barrier_limit_without_a_gpu_call():
    # uniform plans have no barrier: check is a no-op, the limit is refused;
    # a ragged plan created without a visible device defers its upload, and
    # checking it needs no HIP call either
    L = G.lib()
    st, h = _plan(1, [4], [5])
    assert st == 0
    assert L.gtt_plan_check(h, None) == 0
    assert L.gtt_plan_barrier_limit(h, 10) == 1
    assert L.gtt_plan_check(None, None) == 1
    L.gtt_plan_destroy(h)
    if not torch.cuda.is_available():
        st, h = _plan(3, [2, 4, 16], [10, 5, 3], flags=G.FLAG_PERSISTENT)
        assert st == 0
        assert L.gtt_plan_barrier_limit(h, 0) == 0
        assert L.gtt_plan_check(h, None) == 0
        L.gtt_plan_destroy(h)
    assert L.gtt_status_string(9).decode() == "GTT_ERR_TIMEOUT"


def test_backward_refuses_radix_above_32_before_any_hip_call():
    L = G.lib()
    a = ctypes.c_void_p(0x10000)
    for b, dt in ((33, G.F32), (64, G.C64)):
        st, h = _plan(1, [b], [2], dtype=dt)
        assert st == 0
        assert L.gtt_backward(h, a, a, None, a, a, a, a, 1 << 20, None) == 6
        L.gtt_plan_destroy(h)
    # radix 32 has a backward (rejected here only for the missing workspace)
    st, h = _plan(1, [32], [2], dtype=G.BF16)
    assert L.gtt_backward(h, a, a, None, a, a, a, None, 0, None) == 5
    L.gtt_plan_destroy(h)


def test_noalloc_backward_checks_before_any_hip_call():
    L = G.lib()
    a, m = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x10004)
    st, h = _plan(1, [8], [6], batch=256, dtype=G.C64)
    assert st == 0
    assert L.gtt_backward_noalloc(None, a, a, None, a, a, a, None) == 1
    assert L.gtt_backward_noalloc(h, a, a, None, a, None, None, None) == 1    # neither gx nor gW
    assert L.gtt_backward_noalloc(h, a, m, None, a, a, a, None) == 4
    # 256 x 8^6 complex64 without saved activations: more than the scratch
    assert L.gtt_backward_noalloc(h, a, a, None, a, a, a, None) == 5
    L.gtt_plan_destroy(h)
    st, h = _plan(1, [2], [5], dtype=G.I32)
    assert L.gtt_backward_noalloc(h, a, a, None, a, a, a, None) == 6
    L.gtt_plan_destroy(h)


def test_tuning_per_digit_count_and_backward_budget():
    # an entry for (b, n) takes precedence over the radix-wide entry (n = 0);
    # the backward's LDS budget per work-group sets its checkpoint slots
    G.set_tuning(8, torch.complex64, 0, 0, 3)
    G.set_tuning(8, torch.complex64, 0, 0, 2, n=5)
    try:
        k6 = [g["k"] for g in G.Plan(8, 6, 4, torch.complex64).describe()["groups"]]
        k5 = [g["k"] for g in G.Plan(8, 5, 4, torch.complex64).describe()["groups"]]
    finally:
        G.set_tuning(8, torch.complex64, 0, 0, 0, n=5)
        G.set_tuning(8, torch.complex64, 0, 0, 0)
        G.load_tuning()
    assert k6 == [3, 3] and max(k5) <= 2 and sum(k5) == 5
    base = G.Plan(4, 5, 3, torch.float32).describe()["bwd_groups"][0]
    G.set_tuning(4, torch.float32, 0, 0, 0, n=5, bwd_lds_bytes=16 * 1024)
    try:
        g = G.Plan(4, 5, 3, torch.float32).describe()["bwd_groups"][0]
    finally:
        G.set_tuning(4, torch.float32, 0, 0, 0, n=5)
        G.load_tuning()
    units = -(-base["k"] // base["bwd_rd"])
    assert base["bwd_slots"] == units + 1
    assert g["bwd_ok"] and 3 <= g["bwd_slots"] < units + 1 and g["bwd_fwd_passes"] > base["bwd_fwd_passes"]


def test_plan_destruction_is_deferred_during_graph_capture(monkeypatch):
    # a plan collected while the current stream captures a graph is freed
    # only after the capture (hipFree would invalidate it); the capture state
    # is simulated on the host
    monkeypatch.setattr(G, "_capturing", lambda: True)
    p = G.Plan(2, 4, 1, torch.float32)
    h = p.handle
    del p
    assert h in G._DEFERRED
    monkeypatch.setattr(G, "_capturing", lambda: False)
    q = G.Plan(2, 4, 1, torch.float32)  # a new plan frees the deferred ones first
    assert not G._DEFERRED
    del q


@pytest.mark.parametrize("radices,batch,dtype", [
    ([8, 3, 4, 5, 2, 7], 4096, torch.complex64), ([17, 3, 20, 2, 5], 5, torch.complex64),
    ([16, 9, 13, 6], 4, torch.float32), ([7, 2, 5, 3, 8, 4], 10, torch.complex128),
    ([33, 40], 3, torch.float64), ([11, 11, 11, 11], 256, torch.bfloat16)], ids=str)
def test_runtime_radix_lds_contract(radices, batch, dtype):
    # the runtime-radix pass stages every digit's W (rounded up to 16 entries)
    # and works in place on one unpadded tile when every radix of the group
    # is at most 16; a larger radix runs out of place into a second buffer.
    # The kernel places that buffer one element past the tile, so the plan's
    # LDS is (W + (tile + 1) per buffer) compute elements.
    plan = G.Plan.mixed(radices, batch, dtype)
    rad = radices[::-1]  # digit d is factor m-1-d
    csize = {torch.complex64: 8, torch.complex128: 16, torch.float32: 4, torch.float64: 8, torch.bfloat16: 4}[dtype]
    no_pad = 31 | (31 << 8) | (31 << 16)
    groups = plan.describe()["groups"]
    assert sum(g["k"] for g in groups) == len(radices)
    for g in groups:
        assert g["kind"] == "generic" and g["pad_shift"] == no_pad, g
        digits = rad[g["s0"]:g["s0"] + g["k"]]
        w = sum(r * r for r in digits)
        nbuf = 1 if max(digits) <= 16 else 2
        assert g["lds_bytes"] == (((w + 15) // 16) * 16 + nbuf * (g["tile_elems"] + 1)) * csize, (g, digits)
        assert g["lds_bytes"] <= 160 * 1024
