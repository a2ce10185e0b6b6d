// Host side of backward (checkpoint schedules, launch sequence, gW
// reduction) and of the natural-order filter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gtt_bwd.hpp"
#include "gtt_launch.hpp"
#include "gtt_plan.hpp"

namespace gtt {

void fill_pass_args(PassArgs* a, const Group& g, const std::vector<int>& rad, const std::vector<int64_t>& wofs,
                    int64_t N);

static DT to_dt(gtt_dtype d) { return static_cast<DT>((int)d); }
static const char* kDtName[] = {"f64", "f32", "c128", "c64", "bf16", "f16", "i32"};

size_t acc_size(gtt_dtype d) { return (d == GTT_C64 || d == GTT_C128) ? 16 : 8; }

size_t bwd_overhead_bytes(int wloc, gtt_dtype dt) {
    const size_t cs = compute_size(dt), as = acc_size(dt);
    return bwd_align16((size_t)wloc * as) + (size_t)kThreads * as + 2 * bwd_align16((size_t)wloc * cs);
}

// LDS bytes of the backward kernel for a group
size_t bwd_lds_bytes(const Group& g, gtt_dtype dt) {
    const size_t cs = compute_size(dt);
    const int64_t tileP = lds_tile_elems_host(g.tileE, g.pad_shift);
    if (g.kind == kKindCMfma)
        return std::max<size_t>((size_t)((g.k >= 3 ? 4 : 3) * tileP + 1) * cs, 16 * 256 * sizeof(double));
    return bwd_overhead_bytes(g.bwd_wloc, dt) + (size_t)g.bwd_slots * (size_t)tileP * cs;
}

// ---------------------------------------------------------------------------
// Checkpoint schedules.  The digits of a group are reversed from k-1 down to
// 0; digit s needs the activation a_s (digits 0..s-1 applied to the group
// input a_0).  cost[n][s] is the fewest forward passes that reverse a chain
// of n digits whose first activation is held, with s free slots: advance m
// digits into a free slot, reverse the upper n-m digits from there with one
// slot fewer, then free the slot and reverse the lower m digits.
// ---------------------------------------------------------------------------
namespace {
constexpr int kInf = 1 << 28;
struct ChainTable {
    int cost[kMaxDigits + 1][kMaxBwdSlots + 1];
    int split[kMaxDigits + 1][kMaxBwdSlots + 1];
    ChainTable() {
        for (int s = 0; s <= kMaxBwdSlots; ++s) {
            cost[0][s] = 0;
            cost[1][s] = 0;
            split[0][s] = split[1][s] = 0;
        }
        for (int n = 2; n <= kMaxDigits; ++n) {
            cost[n][0] = kInf;
            split[n][0] = 0;
            for (int s = 1; s <= kMaxBwdSlots; ++s) {
                int best = kInf, arg = 1;
                for (int m = 1; m < n; ++m) {
                    const int c = m + cost[n - m][s - 1] + cost[m][s];
                    if (c < best) {
                        best = c;
                        arg = m;
                    }
                }
                cost[n][s] = best;
                split[n][s] = arg;
            }
        }
    }
};
const ChainTable& chain_table() {
    static const ChainTable t;
    return t;
}

void gen_chain(std::vector<uint16_t>* ops, int base, int lo, int n, std::vector<int>* free_slots) {
    if (n <= 0) return;
    if (n == 1) {
        ops->push_back(bwd_op(kOpGw, lo, base, 0));
        ops->push_back(bwd_op(kOpAdj, lo, 1, 1));
        return;
    }
    const int s = std::min<int>((int)free_slots->size(), kMaxBwdSlots);
    const int m = chain_table().split[n][s];
    const int t = free_slots->back();
    free_slots->pop_back();
    ops->push_back(bwd_op(kOpFwd, lo, base, t));
    for (int i = 1; i < m; ++i) ops->push_back(bwd_op(kOpFwd, lo + i, t, t));
    gen_chain(ops, t, lo + m, n - m, free_slots);
    free_slots->push_back(t);
    gen_chain(ops, base, lo, m, free_slots);
}
}  // namespace

int bwd_fwd_passes(int k, int free_slots) {
    if (k < 1) return 0;
    if (k > kMaxDigits || free_slots < 1) return k <= 1 ? 0 : kInf;
    return chain_table().cost[k][std::min(free_slots, kMaxBwdSlots)];
}

std::vector<uint16_t> bwd_schedule(int k, int nslots) {
    std::vector<uint16_t> ops;
    std::vector<int> free_slots;
    for (int i = nslots - 1; i >= 2; --i) free_slots.push_back(i);
    gen_chain(&ops, 0, 0, k, &free_slots);
    return ops;
}

// work-groups of one backward launch (fixed per plan: determinism of gW);
// the matrix-core kernel is one 1024-thread work-group per compute unit
static unsigned bwd_grid(const Group& g) {
    if (g.kind == kKindCMfma) {
        // 1024-thread work-groups: at most two per compute unit (32 waves),
        // fewer when their LDS does not fit twice
        const size_t lds = bwd_lds_bytes(g, GTT_C64);
        const int per_cu = lds * 2 <= 160 * 1024 ? 2 : 1;
        return (unsigned)std::min<int64_t>(g.ntiles, 256 * per_cu);
    }
    return (unsigned)std::min<int64_t>(g.ntiles, 2048);
}

size_t bwd_partials_elems(const std::vector<Group>& bg, int wslot) {
    size_t e = 0;
    for (const Group& g : bg) e += (size_t)bwd_grid(g) * (size_t)wslot;
    return e;
}

// Backward of one instance set (a uniform or mixed-radix batch, or one
// ragged instance): digit groups in reverse order; every launch writes its
// work-groups' partial vectors (wslot entries each) at `partials`.
// shared_w: every digit uses the one matrix at W (uniform); else digit d
// uses the matrix at wofs[d] (mixed radix).
static gtt_status bwd_run(gtt_plan_s* tp, gtt_dtype dt, const std::vector<Group>& bg, const std::vector<int>& rad,
                          const std::vector<int64_t>& wofs, int64_t N, size_t slot, int wslot, bool shared_w,
                          const void* W, const void* x, const char* saved, const void* gy, void* gx, char* cbuf,
                          char* partials, hipStream_t s) {
    const size_t es = storage_size(dt), as = acc_size(dt);
    const int R = (int)bg.size();
    const void* c_out = gy;
    char* part = partials;
    for (int g = R - 1; g >= 0; --g) {
        const Group& G = bg[g];
        PassArgs pa;
        fill_pass_args(&pa, G, rad, wofs, N);
        pa.W = W;
        pa.in = (g == 0) ? x : (const void*)(saved + (size_t)(g - 1) * slot * es);
        // the first group's cotangent is gx itself; with gx null it is not
        // stored at all (no buffer is reserved for it)
        void* c_in = (g == 0) ? gx : (void*)cbuf;
        pa.out = c_in;
        const unsigned grid = bwd_grid(G);
        int threads = 0;  // work-group size of a general-kernel launch
        std::string nm;   // timing label (the general kernels' labels carry the work-group size)
        const bool timed = tp && tp->timing.enabled;
        if (G.kind == kKindCMfma) {
            CBwdArgs ca;
            std::memset(&ca, 0, sizeof ca);
            ca.p = pa;
            ca.c_out = c_out;
            ca.partials = part;
            const int ni = G.fast_ni;
            const size_t lds = bwd_lds_bytes(G, dt);
            if (timed) {
                char buf[96];
                std::snprintf(buf, sizeof buf, "bwd %s b=%d cmfma s0=%d k=%d", kDtName[(int)dt], rad[G.s0], G.s0, G.k);
                nm = buf;
            }
            timing_begin(tp, s, nm);
            const hipError_t e = ni ? launch_cbwd8_fast(G.k, ni, ca, grid, lds, s) : launch_cbwd8(ca, grid, lds, s);
            if (e != hipSuccess) return GTT_ERR_HIP;
        } else {
            if (!G.bwd_ok) return GTT_ERR_UNSUPPORTED;
            BwdArgs ba;
            std::memset(&ba, 0, sizeof ba);
            ba.p = pa;
            ba.c_out = c_out;
            ba.partials = part;
            ba.nslots = G.bwd_slots;
            ba.wloc = G.bwd_wloc;
            ba.wslot = wslot;
            if ((int)G.bwd_ops.size() > kMaxBwdOps) return GTT_ERR_INTERNAL;
            ba.nops = (int)G.bwd_ops.size();
            std::copy(G.bwd_ops.begin(), G.bwd_ops.end(), ba.ops);
            if (shared_w) {
                ba.nf = 1;
                ba.f_goff[0] = 0;
                ba.f_b[0] = rad[G.s0];
                ba.f_loff[0] = 0;
                for (int j = 0; j < G.k; ++j) ba.lofs[j] = 0;
            } else {
                ba.nf = G.k;
                int lo = 0;
                for (int j = 0; j < G.k; ++j) {
                    ba.f_goff[j] = (int32_t)wofs[G.s0 + j];
                    ba.f_b[j] = rad[G.s0 + j];
                    ba.f_loff[j] = lo;
                    ba.lofs[j] = lo;
                    lo += rad[G.s0 + j] * rad[G.s0 + j];
                }
            }
            // the register-block kernel when the plan chose it (one W for
            // every digit; its schedule counts blocks); the matrix-core
            // kernel for radix-16 / 32 groups on the matrix cores (one W)
            int radix = (shared_w && G.bwd_rd > 0) ? rad[G.s0] : 0;
            if (shared_w && G.kind == kKindMfma) radix = rad[G.s0];
            if (!shared_w && G.bwd_rd > 0) return GTT_ERR_INTERNAL;
            const size_t lds = bwd_lds_bytes(G, dt);
            threads = launch_bwd_threads(to_dt(dt), radix, lds);
            if (timed) {
                char buf[96];
                std::snprintf(buf, sizeof buf, "bwd %s b=%d s0=%d k=%d wg=%d", kDtName[(int)dt], rad[G.s0], G.s0, G.k,
                              threads);
                nm = buf;
            }
            timing_begin(tp, s, nm);
            if (launch_bwd(to_dt(dt), ba, G.bwd_maxb, radix, grid, threads, lds, s) != hipSuccess)
                return GTT_ERR_HIP;
        }
        if (timed) timing_end(tp, s, nm, 3.0 * (double)G.elems * (double)es);
        part += (size_t)grid * wslot * as;
        c_out = c_in;
    }
    return GTT_OK;
}

static bool groups_have_bwd(const std::vector<Group>& bg) {
    for (const Group& g : bg)
        if (g.kind != kKindCMfma && !g.bwd_ok) return false;
    return true;
}

bool plan_has_backward(const gtt_plan_s* p) {
    if (p->dtype == GTT_I32) return false;
    if (p->kind == PlanKind::Ragged) {
        for (const Instance& t : p->inst)
            if (!groups_have_bwd(t.bwd_groups)) return false;
        return true;
    }
    return groups_have_bwd(p->bwd_groups);
}

size_t backward_ws_need(const gtt_plan_s* p, bool have_saved, bool cb_in_gx) {
    const size_t es = p->esize;
    size_t need = bwd_partial_bytes(p);
    if (p->kind != PlanKind::Ragged) {
        const int R = (int)p->groups.size();
        if (R > 1 && !have_saved) need += (size_t)(R - 1) * (size_t)p->slot * es;
        if (R > 1 && !cb_in_gx) need += (size_t)p->total_elems * es;
    } else {
        int maxR = 0;
        for (const Instance& t : p->inst) maxR = std::max(maxR, (int)t.groups.size());
        if (maxR > 1 && !have_saved) need += (size_t)(maxR - 1) * (size_t)p->slot * es;
        if (!cb_in_gx) need += (size_t)p->slot * es;
    }
    return need;
}

gtt_status backward_impl(gtt_plan_s* p, const void* W, const void* x, const void* saved, const void* gy, void* gx,
                         void* gW, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t es = p->esize, cs = p->csize, as = acc_size(p->dtype);
    const DT dt = to_dt(p->dtype);
    if (!plan_has_backward(p)) return GTT_ERR_UNSUPPORTED;
    const size_t part_bytes = bwd_partial_bytes(p);
    char* wsb = static_cast<char*>(ws);
    if (ws_bytes < part_bytes || (part_bytes && !ws)) return GTT_ERR_WORKSPACE;
    char* partials = wsb;
    char* extra = wsb + part_bytes;
    size_t extra_bytes = ws_bytes - part_bytes;
    // rad / wofs: radix and W offset per digit; elems: elements of the
    // buffers; slot: stride of the boundary slots
    auto run_set = [&](const std::vector<Group>& fg, const std::vector<Group>& bg, const std::vector<int>& rad,
                       const std::vector<int64_t>& wofs, int wslot, bool shared_w, int64_t N, size_t elems,
                       size_t slot, const void* w, const char* xin, const char* sv_in, const char* gyin, char* gxout,
                       char* part, char* sv_tmp, char* cb) -> gtt_status {
        const int R = (int)fg.size();
        if (R == 0) {  // n == 0: gx = gy, gW = 0 (no factor of W)
            if (gxout && gxout != gyin && hipMemcpyAsync(gxout, gyin, elems * es, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return GTT_ERR_HIP;
            return GTT_OK;
        }
        const char* svp = sv_in;
        if (R > 1 && !svp) {
            // recompute the activations at the group boundaries
            const void* cur = xin;
            for (int g = 0; g + 1 < R; ++g) {
                char* dst = sv_tmp + (size_t)g * slot * es;
                gtt_status st = launch_group_rw(p, p->dtype, fg[g], rad, wofs, N, w, false, cur, dst, s);
                if (st != GTT_OK) return st;
                cur = dst;
            }
            svp = sv_tmp;
        }
        return bwd_run(p, p->dtype, bg, rad, wofs, N, slot, wslot, shared_w, w, xin, svp, gyin, gxout, cb, part, s);
    };
    if (p->kind != PlanKind::Ragged) {
        // uniform batch or mixed radix: one instance set
        const size_t E = (size_t)p->total_elems, SL = (size_t)p->slot;
        const int R = (int)p->groups.size();
        const bool shared_w = p->kind == PlanKind::Uniform;
        const int wslot = (int)p->w_elems;
        // cotangent buffer between groups: gx when given and not aliasing gy,
        // else workspace
        size_t need = 0;
        if (R > 1 && !saved) need += (size_t)(R - 1) * SL * es;
        const bool cb_in_gx = gx && gx != gy;
        if (R > 1 && !cb_in_gx) need += E * es;
        if (extra_bytes < need) return GTT_ERR_WORKSPACE;
        char* sv_tmp = extra;
        char* cb = cb_in_gx ? static_cast<char*>(gx) : extra + ((R > 1 && !saved) ? (size_t)(R - 1) * SL * es : 0);
        gtt_status st = run_set(p->groups, p->bwd_groups, p->rad, p->wofs, wslot, shared_w, p->N, E, SL, W,
                                (const char*)x, (const char*)saved, (const char*)gy, (char*)gx, partials, sv_tmp, cb);
        if (st != GTT_OK) return st;
        if (gW) {
            const int64_t nparts = (int64_t)(bwd_partials_elems(p->bwd_groups, wslot) / (size_t)wslot);
            if (R == 0) {
                if (launch_zero(gW, (size_t)wslot * cs, s) != hipSuccess) return GTT_ERR_HIP;
            } else {
                const std::string rnm = std::string("reduce ") + kDtName[(int)p->dtype];
                timing_begin(p, s, rnm);
                if (launch_reduce(dt, partials, nparts, wslot, gW, s) != hipSuccess) return GTT_ERR_HIP;
                timing_end(p, s, rnm, (double)nparts * wslot * as);
            }
        }
        return GTT_OK;
    }
    // ragged: instances one by one; partial vectors laid out grouped by W
    // index; boundary slots of stride E (total elements rounded up to 256
    // bytes)
    const size_t E = (size_t)p->slot;
    int maxR = 0;
    for (const Instance& t : p->inst) maxR = std::max(maxR, (int)t.groups.size());
    size_t need = 0;
    if (maxR > 1 && !saved) need += (size_t)(maxR - 1) * E * es;
    const bool cb_in_gx = gx && gx != gy;
    if (!cb_in_gx) need += E * es;
    if (extra_bytes < need) return GTT_ERR_WORKSPACE;
    char* sv_tmp = extra;
    char* cb_base = cb_in_gx ? static_cast<char*>(gx) : extra + ((maxR > 1 && !saved) ? (size_t)(maxR - 1) * E * es : 0);
    const int nw = (int)p->w_b.size();
    // region of W entry w: its instances' partials, then the reduction's
    // first-stage vectors
    std::vector<size_t> wpart(nw, 0), wstart(nw + 1, 0);
    for (const Instance& t : p->inst) wpart[t.w] += bwd_partials_elems(t.bwd_groups, t.b * t.b) * as;
    for (int w = 0; w < nw; ++w)
        wstart[w + 1] = wstart[w] + wpart[w] + kReduceBlocks * (size_t)p->w_b[w] * p->w_b[w] * as;
    std::vector<size_t> wcur(wstart.begin(), wstart.end() - 1);
    for (const Instance& t : p->inst) {
        const char* xin = static_cast<const char*>(x) + t.off * es;
        const char* gyin = static_cast<const char*>(gy) + t.off * es;
        char* gxout = gx ? static_cast<char*>(gx) + t.off * es : nullptr;
        const char* svin = saved ? static_cast<const char*>(saved) + t.off * es : nullptr;
        const char* w = static_cast<const char*>(W) + p->w_off[t.w] * cs;
        char* part = partials + wcur[t.w];
        wcur[t.w] += bwd_partials_elems(t.bwd_groups, t.b * t.b) * as;
        const std::vector<int> rad(std::max(t.n, 1), t.b);
        const std::vector<int64_t> wofs(std::max(t.n, 1), 0);
        // saved activations of a ragged plan: group boundary g of instance t
        // at element g * E + off (the workspace copy: the same layout)
        gtt_status st = run_set(t.groups, t.bwd_groups, rad, wofs, t.b * t.b, true, t.N, 1, E, w, xin, svin, gyin,
                                gxout, part, sv_tmp + t.off * es, cb_base + t.off * es);
        if (st != GTT_OK) return st;
    }
    if (gW) {
        for (int w = 0; w < nw; ++w) {
            const int bb = p->w_b[w] * p->w_b[w];
            char* out = static_cast<char*>(gW) + p->w_off[w] * cs;
            const int64_t nparts = (int64_t)(wpart[w] / as / bb);
            if (nparts == 0) {
                if (launch_zero(out, (size_t)bb * cs, s) != hipSuccess) return GTT_ERR_HIP;
            } else if (launch_reduce(dt, partials + wstart[w], nparts, bb, out, s) != hipSuccess) {
                return GTT_ERR_HIP;
            }
        }
    }
    return GTT_OK;
}

}  // namespace gtt
