// Host side of backward and of the natural-order filter.
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

// LDS bytes of the backward kernel for a tile geometry
size_t bwd_lds_bytes(const Group& g, size_t csize, int b) {
    const int64_t tileP = lds_tile_elems_host(g.tileE, g.pad_shift);
    if (g.kind == kKindCMfma)
        return std::max<size_t>((size_t)((g.k >= 3 ? 4 : 3) * tileP + 1) * csize, 16 * 256 * sizeof(double));
    const int maxb = b <= 8 ? 8 : 16;
    return (size_t)(3 * maxb * maxb + kThreads + 3 * tileP) * csize;
}

// work-groups of one backward launch (fixed per plan: determinism of gW);
// the matrix-core kernel is one 1024-thread work-group per compute unit
static unsigned bwd_grid(const Group& g) {
    if (g.kind == kKindCMfma) {
        // 1024-thread work-groups: at most two per compute unit (32 waves),
        // fewer when their LDS does not fit twice
        const size_t lds = bwd_lds_bytes(g, 8, 8);
        const int per_cu = lds * 2 <= 160 * 1024 ? 2 : 1;
        return (unsigned)std::min<int64_t>(g.ntiles, 256 * per_cu);
    }
    return (unsigned)std::min<int64_t>(g.ntiles, 2048);
}

size_t bwd_partials_elems(const std::vector<Group>& bg, int b) {
    size_t e = 0;
    for (const Group& g : bg) e += (size_t)bwd_grid(g) * b * b;
    return e;
}

// partial vectors of the reduction's first stage (after the bwd partials)
static constexpr size_t kReduceScratchVectors = 64;

// backward of one instance set (uniform batch, or one ragged instance)
static gtt_status bwd_run(gtt_plan_s* tp, gtt_dtype dt, const std::vector<Group>& fg, const std::vector<Group>& bg, int b,
                          int64_t N, size_t elems, const void* W, const void* x, const char* saved, const void* gy,
                          void* gx, char* cbuf, char* partials, hipStream_t s) {
    const size_t es = storage_size(dt), cs = compute_size(dt);
    const int R = (int)bg.size();
    std::vector<int> rad(64, b);
    std::vector<int64_t> wofs(64, 0);
    const void* c_out = gy;
    char* part = partials;
    for (int g = R - 1; g >= 0; --g) {
        const Group& G = bg[g];
        BwdArgs ba;
        std::memset(&ba, 0, sizeof ba);
        fill_pass_args(&ba.p, G, rad, wofs, N);
        ba.p.W = W;
        ba.p.in = (g == 0) ? x : (const void*)(saved + (size_t)(g - 1) * elems * es);
        // the first group's cotangent is gx itself; with gx null it is not
        // stored at all (no buffer is reserved for it)
        void* c_in = (g == 0) ? gx : (void*)cbuf;
        ba.p.out = c_in;
        ba.c_out = c_out;
        ba.partials = part;
        ba.b = b;
        const unsigned grid = bwd_grid(G);
        timing_begin(tp, s);
        if (G.kind == kKindCMfma) {
            CBwdArgs ca;
            std::memset(&ca, 0, sizeof ca);
            ca.p = ba.p;
            ca.c_out = ba.c_out;
            ca.partials = ba.partials;
            const int ni = G.fast_ni;
            const size_t lds = bwd_lds_bytes(G, cs, b);
            const hipError_t e = ni ? launch_cbwd8_fast(G.k, ni, ca, grid, lds, s) : launch_cbwd8(ca, grid, lds, s);
            if (e != hipSuccess) return GTT_ERR_HIP;
        } else if (launch_bwd(to_dt(dt), ba, grid, bwd_lds_bytes(G, cs, b), s) != hipSuccess) {
            return GTT_ERR_HIP;
        }
        if (tp && tp->timing.enabled) {
            char nm[96];
            std::snprintf(nm, sizeof nm, "bwd %s b=%d%s s0=%d k=%d", kDtName[(int)dt], b,
                          G.kind == kKindCMfma ? " cmfma" : "", G.s0, G.k);
            timing_end(tp, s, nm, 3.0 * (double)G.elems * (double)es);
        }
        part += (size_t)grid * b * b * cs;
        c_out = c_in;
    }
    (void)fg;
    return GTT_OK;
}

gtt_status backward_impl(gtt_plan_s* p, const void* W, const void* x, const void* saved, const void* gy, void* gx,
                         void* gW, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t es = p->esize, cs = p->csize;
    const DT dt = to_dt(p->dtype);
    const size_t part_bytes = bwd_partial_bytes(p);
    char* wsb = static_cast<char*>(ws);
    if (ws_bytes < part_bytes || (part_bytes && !ws)) return GTT_ERR_WORKSPACE;
    char* partials = wsb;
    char* extra = wsb + part_bytes;
    size_t extra_bytes = ws_bytes - part_bytes;
    // elems: elements of the buffers; slot: stride of the boundary slots
    auto uniform_like = [&](const std::vector<Group>& fg, const std::vector<Group>& bg, int b, int64_t N,
                            size_t elems, size_t slot, const char* xin, const char* sv_in, const char* gyin,
                            char* gxout, char* part, char* sv_tmp, char* cb) -> gtt_status {
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
                gtt_status st = launch_group_inst(p, p->dtype, fg[g], b, N, W, false, cur, dst, s);
                if (st != GTT_OK) return st;
                cur = dst;
            }
            svp = sv_tmp;
        }
        return bwd_run(p, p->dtype, fg, bg, b, N, slot, W, xin, svp, gyin, gxout, cb, part, s);
    };
    if (p->kind == PlanKind::Uniform) {
        const size_t E = (size_t)p->total_elems, SL = (size_t)p->slot;
        const int R = (int)p->groups.size();
        // cotangent buffer between groups: gx when given and not aliasing gy,
        // else workspace
        char* cb = nullptr;
        size_t need = 0;
        if (R > 1 && !saved) need += (size_t)(R - 1) * SL * es;
        const bool cb_in_gx = gx && gx != gy;
        if (R > 1 && !cb_in_gx) need += E * es;
        if (extra_bytes < need) return GTT_ERR_WORKSPACE;
        char* sv_tmp = extra;
        cb = cb_in_gx ? static_cast<char*>(gx) : extra + ((R > 1 && !saved) ? (size_t)(R - 1) * SL * es : 0);
        gtt_status st = uniform_like(p->groups, p->bwd_groups, p->b, p->N, E, SL, (const char*)x, (const char*)saved,
                                     (const char*)gy, (char*)gx, partials, sv_tmp, cb);
        if (st != GTT_OK) return st;
        if (gW) {
            const int64_t nparts = (int64_t)(bwd_partials_elems(p->bwd_groups, p->b) / ((size_t)p->b * p->b));
            if (R == 0) {
                if (hipMemsetAsync(gW, 0, (size_t)p->b * p->b * cs, s) != hipSuccess) return GTT_ERR_HIP;
            } else {
                timing_begin(p, s);
                if (launch_reduce(dt, partials, nparts, p->b * p->b, gW, s) != hipSuccess) return GTT_ERR_HIP;
                timing_end(p, s, std::string("reduce ") + kDtName[(int)p->dtype], (double)nparts * p->b * p->b * cs);
            }
        }
        return GTT_OK;
    }
    // ragged: instances one by one; partial sums laid out grouped by W index;
    // boundary slots of stride E (total elements rounded up to 256 bytes)
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
    for (const Instance& t : p->inst) wpart[t.w] += bwd_partials_elems(t.bwd_groups, t.b) * cs;
    for (int w = 0; w < nw; ++w)
        wstart[w + 1] = wstart[w] + wpart[w] + kReduceScratchVectors * (size_t)p->w_b[w] * p->w_b[w] * cs;
    std::vector<size_t> wcur(wstart.begin(), wstart.end() - 1);
    for (const Instance& t : p->inst) {
        const char* xin = static_cast<const char*>(x) + t.off * es;
        const char* gyin = static_cast<const char*>(gy) + t.off * es;
        char* gxout = gx ? static_cast<char*>(gx) + t.off * es : nullptr;
        const char* svin = saved ? static_cast<const char*>(saved) + t.off * es : nullptr;
        // per-instance views into the boundary buffers (stride E elements)
        const char* w = static_cast<const char*>(W) + p->w_off[t.w] * cs;
        char* part = partials + wcur[t.w];
        wcur[t.w] += bwd_partials_elems(t.bwd_groups, t.b) * cs;
        const int R = (int)t.groups.size();
        if (R == 0) {
            if (gxout && gxout != gyin && hipMemcpyAsync(gxout, gyin, es, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return GTT_ERR_HIP;
            continue;
        }
        // saved activations of a ragged plan: group boundary g of instance t at
        // element g * E + off
        const char* svp = svin;
        if (R > 1 && !svp) {
            const void* cur = xin;
            for (int g = 0; g + 1 < R; ++g) {
                char* dst = sv_tmp + ((size_t)g * E + t.off) * es;
                gtt_status st = launch_group_inst(p, p->dtype, t.groups[g], t.b, t.N, w, false, cur, dst, s);
                if (st != GTT_OK) return st;
                cur = dst;
            }
            svp = sv_tmp + t.off * es;
        }
        gtt_status st = bwd_run(p, p->dtype, t.groups, t.bwd_groups, t.b, t.N, E, w, xin, svp, gyin, gxout,
                                cb_base + t.off * es, part, s);
        if (st != GTT_OK) return st;
    }
    if (gW) {
        for (int w = 0; w < nw; ++w) {
            const int bb = p->w_b[w] * p->w_b[w];
            char* out = static_cast<char*>(gW) + p->w_off[w] * cs;
            const int64_t nparts = (int64_t)(wpart[w] / cs / bb);
            if (nparts == 0) {
                if (hipMemsetAsync(out, 0, (size_t)bb * cs, s) != hipSuccess) return GTT_ERR_HIP;
            } else if (launch_reduce(dt, partials + wstart[w], nparts, bb, out, s) != hipSuccess) {
                return GTT_ERR_HIP;
            }
        }
    }
    return GTT_OK;
}


}  // namespace gtt
