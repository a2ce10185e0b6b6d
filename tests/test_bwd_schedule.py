"""CPU checks of the backward's checkpoint schedules and tile plans.

The general backward kernel executes, per tile, a list of operations that the
host planned: forward passes that rebuild activations in LDS slots, gradient
sweeps and adjoint passes.  Here every schedule of many plans is replayed
symbolically: each slot carries the set of digits applied to the group input,
the cotangent the set of digits whose adjoint has been applied.  Digit s's
gradient sweep must see a_s (digits 0..s-1 applied) and the cotangent at its
output (adjoints of digits s+1..k-1 applied), the group input must never be
overwritten, and every digit must be swept and reversed exactly once.
"""
import pytest
import torch

from paper_2507_02420_amd import gtt as G

FWD, GW, ADJ = 0, 1, 2


def decode(op):
    return op & 3, (op >> 2) & 63, (op >> 8) & 15, (op >> 12) & 15


def replay(k, nslots, ops):
    """Symbolic execution; returns the number of forward passes."""
    slot = {0: frozenset()}
    ct = frozenset()
    swept, reversed_ = [], []
    fwd = 0
    for op in ops:
        kind, j, src, dst = decode(op)
        assert 0 <= j < k
        if kind == FWD:
            assert dst >= 2 and dst < nslots, "forward pass into the input or cotangent slot"
            assert slot.get(src) == frozenset(range(j)), ("forward pass on a slot that is not a_j", j, src)
            slot[dst] = frozenset(range(j + 1))
            fwd += 1
        elif kind == GW:
            assert src < nslots
            assert slot.get(src) == frozenset(range(j)), ("gradient sweep without a_j", j)
            assert ct == frozenset(range(j + 1, k)), ("gradient sweep on the wrong cotangent", j)
            swept.append(j)
        else:
            assert kind == ADJ
            assert swept and swept[-1] == j, "adjoint pass before its gradient sweep"
            assert ct == frozenset(range(j + 1, k))
            ct = ct | {j}
            reversed_.append(j)
    assert swept == list(range(k - 1, -1, -1))
    assert reversed_ == swept
    assert ct == frozenset(range(k))
    return fwd


def closed_form_passes(k, free):
    """Fewest forward passes for small cases with a known closed form: one
    free slot recomputes every activation from the input (k(k-1)/2); k-1 free
    slots compute each activation once (k-1)."""
    if free == 1:
        return k * (k - 1) // 2
    if free >= k - 1:
        return max(k - 1, 0)
    return None


PLANS = [(b, n, batch, dt) for dt in (torch.float32, torch.bfloat16, torch.complex64, torch.float64,
                                      torch.complex128)
         for (b, n, batch) in [(2, 5, 3), (2, 13, 2), (2, 20, 16), (3, 7, 2), (3, 13, 16), (4, 5, 3), (4, 9, 2),
                               (4, 10, 64), (5, 6, 2), (6, 5, 2), (7, 4, 2), (8, 5, 2), (8, 6, 4), (11, 3, 2),
                               (16, 3, 2), (16, 4, 1), (32, 2, 2), (32, 3, 2)]]


@pytest.mark.parametrize("b,n,batch,dtype", PLANS, ids=str)
def test_backward_schedules_replay(b, n, batch, dtype):
    d = G.Plan(b, n, batch, dtype).describe()
    assert len(d["bwd_groups"]) == len(d["groups"])
    for g, f in zip(d["bwd_groups"], d["groups"]):
        assert (g["s0"], g["k"]) == (f["s0"], f["k"])
        if g["kind"] == "cmfma":
            continue
        assert g["bwd_ok"], g
        # the register-block kernel schedules blocks of bwd_rd digits
        k = -(-g["k"] // g["bwd_rd"]) if g["bwd_rd"] else g["k"]
        slots = g["bwd_slots"]
        assert 2 <= slots <= 16 and (slots >= 3 or k == 1)
        fwd = replay(k, slots, g["bwd_schedule"])
        assert fwd == g["bwd_fwd_passes"]
        cf = closed_form_passes(k, slots - 2)
        if cf is not None:
            assert fwd == cf, (k, slots, fwd, cf)
        # never worse than recomputing from the group input (one free slot)
        assert fwd <= k * (k - 1) // 2


def test_five_digit_group_is_linear():
    # a 5-digit group of float32 and bf16 data: every activation (at the
    # start of a register block of 2 digits) computed once; at most 2k - 1
    # LDS passes a tile (here 2 forward and 3 gradient / adjoint passes)
    for dtype in (torch.float32, torch.bfloat16):
        d = G.Plan(4, 5, 3, dtype).describe()
        (g,) = d["bwd_groups"]
        units = -(-g["k"] // g["bwd_rd"]) if g["bwd_rd"] else g["k"]
        assert g["k"] == 5 and g["bwd_slots"] == units + 1
        ops = [decode(o) for o in g["bwd_schedule"]]
        fwd = sum(1 for o in ops if o[0] == FWD)
        adj = sum(1 for o in ops if o[0] == ADJ)
        assert fwd == units - 1 and adj == units
        assert fwd + adj <= 2 * 5 - 1


def test_mixed_radix_plans_have_backward_schedules():
    for radices in ([2, 3, 4, 5], [3, 8, 2, 7, 4], [16, 2, 9], [32, 4], [5, 5, 5, 5, 5, 5, 5]):
        p = G.Plan.mixed(radices, 3, torch.complex64)
        d = p.describe()
        assert len(d["bwd_groups"]) == len(d["groups"])
        for g in d["bwd_groups"]:
            assert g["bwd_ok"] and g["bwd_rd"] == 0
            replay(g["k"], g["bwd_slots"], g["bwd_schedule"])


def test_radix_above_32_has_no_backward():
    d = G.Plan(33, 2, 1, torch.float32).describe()
    assert not all(g["bwd_ok"] for g in d["bwd_groups"])


def _phys(x, ps):
    return x + (x >> (ps & 31)) + (x >> ((ps >> 8) & 31)) + (x >> ((ps >> 16) & 31))


@pytest.mark.parametrize("b,n,batch,dtype", [(2, 13, 2, torch.float32), (2, 20, 16, torch.float32),
                                             (4, 10, 64, torch.float32), (4, 10, 64, torch.complex64),
                                             (3, 13, 16, torch.float32), (5, 6, 2, torch.float64),
                                             (4, 8, 2, torch.bfloat16), (2, 12, 3, torch.complex128)], ids=str)
def test_radix_backward_lds_offsets_are_additive(b, n, batch, dtype):
    # the register-block backward addresses position m of a block (its
    # digits j0 .. j0+r-1) as phys(lam0) + phys(m * step); check it against
    # phys(lam0 + m * step) for every block of every planned tile
    d = G.Plan(b, n, batch, dtype).describe()
    for g in d["bwd_groups"]:
        rd = g["bwd_rd"]
        if g["kind"] == "cmfma" or rd == 0:
            continue
        ps, logC = g["pad_shift"], (g["C"]).bit_length() - 1
        rows = g["P"] * g["G"]
        for j0 in range(0, g["k"], rd):
            r = min(rd, g["k"] - j0)
            nb = b ** r
            bj, bjr = b ** j0, b ** (j0 + r)
            step = bj << logC
            off = [_phys(m * step, ps) for m in range(nb)]
            for f in range((rows << logC) // nb):
                c, f1 = f & ((1 << logC) - 1), f >> logC
                Q = f1 // bj
                lam0 = ((Q * bjr + (f1 - Q * bj)) << logC) | c
                base = _phys(lam0, ps)
                for m in range(nb):
                    assert base + off[m] == _phys(lam0 + m * step, ps), (j0, f, m)


def test_tuned_backward_budget_too_small_falls_back():
    # a tuned LDS budget per backward work-group that holds no schedule
    # (fewer than three tiles) must not leave a group without a backward
    try:
        for b, n, batch, dtype in [(3, 9, 2, torch.float32), (4, 6, 3, torch.complex64)]:
            G.set_tuning(b, dtype, 0, 0, n=n, bwd_lds_bytes=20480)
            d = G.Plan(b, n, batch, dtype).describe()
            assert all(g["bwd_ok"] for g in d["bwd_groups"]), d["bwd_groups"]
            G.set_tuning(b, dtype, 0, 0, n=n)
    finally:
        G.set_tuning(3, torch.float32, 0, 0, n=9)
        G.set_tuning(4, torch.complex64, 0, 0, n=6)
        G.load_tuning()
