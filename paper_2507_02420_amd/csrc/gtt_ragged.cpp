// Ragged batches (instances of different radix and length in one buffer),
// workspace sizing and plan descriptions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <cstdio>
#include <map>
#include <string>

#include "gtt_launch.hpp"
#include "gtt_plan.hpp"
#include "gtt_ragged.hpp"

namespace gtt {

void fill_pass_args(PassArgs* a, const Group& g, const std::vector<int>& rad, const std::vector<int64_t>& wofs,
                    int64_t N);

// Device work list of a ragged plan: built on the host and uploaded at plan
// time to the device current then (when no device is visible at plan time,
// on the first call instead).
struct RaggedState {
    std::vector<RaggedDesc> desc;
    std::vector<RaggedItem> items;
    std::vector<int64_t> phase_start;
    // per-phase launches: runs of items of one class (item range, LDS of the
    // largest tile in the run, algorithmic bytes)
    struct Seg {
        int phase, cls;
        int64_t start, end;
        size_t lds;
        double bytes;
    };
    std::vector<Seg> segs;
    size_t lds_max = 0;
    bool uploaded = false;
    RaggedDesc* d_desc = nullptr;
    RaggedItem* d_items = nullptr;
    unsigned* d_bar = nullptr;
    int grid_persistent = 0;
    int cus = 0;
    int device = -1;                   // device holding the work list
    uint32_t spin_limit = 1u << 24;    // polls of a grid-barrier wait
};

static void build_worklist(gtt_plan_s* p) {
    RaggedState* rs = new RaggedState();
    p->rs = rs;
    int maxR = 1;
    for (const Instance& t : p->inst) maxR = std::max(maxR, (int)t.groups.size());
    const int64_t E = p->slot;  // stride of the boundary slots in `saved`
    struct Tmp {
        int phase, cls;
        int64_t cost;
        RaggedItem it;
        size_t lds;
        double bytes;
    };
    std::vector<Tmp> tmp;
    for (const Instance& t : p->inst) {
        // n == 0 (N = 1, the identity): a one-element tile with no digit
        std::vector<Group> idg;
        if (t.groups.empty()) {
            Group g0;
            g0.k = 0;
            g0.G = 1;
            g0.S = 1;
            g0.C = 1;
            g0.P = 1;
            g0.L = 1;
            g0.ntiles = 1;
            g0.tileE = 1;
            g0.elems = 1;
            g0.mode = kContigScalar;
            g0.pad_shift = kNoPad;
            g0.kind = kKindValu;
            g0.lds_bytes = 16 * p->csize;
            idg.push_back(g0);
        }
        const std::vector<Group>& groups = t.groups.empty() ? idg : t.groups;
        const int R = (int)groups.size();
        std::vector<int> rad(std::max(t.n, 1), t.b);
        std::vector<int64_t> wofs(std::max(t.n, 1), 0);
        for (int g = 0; g < R; ++g) {
            const Group& G = groups[g];
            RaggedDesc d;
            std::memset(&d, 0, sizeof d);
            fill_pass_args(&d.a, G, rad, wofs, t.N);
            d.b = t.groups.empty() ? 2 : t.b;  // identity tiles take the radix-2 path (no digit)
            d.kind = G.kind;
            d.w_off = p->w_off[t.w];
            d.in_sel = (g == 0) ? 0 : 2;
            d.in_off = t.off;
            d.in_off_saved = (int64_t)(g - 1) * E + t.off;
            d.out_sel = (g == R - 1) ? 1 : 2;
            d.out_off = t.off;
            d.mid_off_saved = (int64_t)g * E + t.off;
            const int di = (int)rs->desc.size();
            rs->desc.push_back(d);
            const size_t extra = 64 * p->csize;
            rs->lds_max = std::max(rs->lds_max, G.lds_bytes + extra);
            // cost estimate of one tile: elements x digits x radix work
            const int64_t work = (G.kind == kKindMfma) ? 8 : t.b;
            const int64_t cost = G.tileE * G.k * work;
            const int cls = ragged_class(d.kind, d.b);
            const double bytes = 2.0 * (double)G.tileE * (double)p->esize;
            for (int64_t i = 0; i < G.ntiles; ++i)
                tmp.push_back(Tmp{g, cls, cost, RaggedItem{di, 0, i}, G.lds_bytes + extra, bytes});
        }
    }
    // phase-major, then by item class (one specialised launch per run of a
    // class); within a run the costliest tiles first, so that the round-robin
    // assignment ends with the cheap ones (longest-processing-time order)
    std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) {
        if (a.phase != b.phase) return a.phase < b.phase;
        if (a.cls != b.cls) return a.cls < b.cls;
        return a.cost > b.cost;
    });
    rs->phase_start.assign(maxR + 1, 0);
    for (const Tmp& t : tmp) rs->phase_start[t.phase + 1]++;
    for (int ph = 0; ph < maxR; ++ph) rs->phase_start[ph + 1] += rs->phase_start[ph];
    for (size_t i = 0; i < tmp.size(); ++i) {
        const Tmp& t = tmp[i];
        rs->items.push_back(t.it);
        if (rs->segs.empty() || rs->segs.back().phase != t.phase || rs->segs.back().cls != t.cls)
            rs->segs.push_back(RaggedState::Seg{t.phase, t.cls, (int64_t)i, (int64_t)i, 0, 0.0});
        RaggedState::Seg& sg = rs->segs.back();
        sg.end = (int64_t)i + 1;
        sg.lds = std::max(sg.lds, t.lds);
        sg.bytes += t.bytes;
    }
}

static gtt_status upload_worklist(gtt_plan_s* p) {
    RaggedState* rs = p->rs;
    if (rs->uploaded) return GTT_OK;
    const DT dt = static_cast<DT>((int)p->dtype);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GTT_ERR_HIP;
    if (hipMalloc(&rs->d_desc, rs->desc.size() * sizeof(RaggedDesc)) != hipSuccess) return GTT_ERR_HIP;
    if (hipMalloc(&rs->d_items, std::max<size_t>(1, rs->items.size()) * sizeof(RaggedItem)) != hipSuccess)
        return GTT_ERR_HIP;
    if (hipMalloc(&rs->d_bar, 4 * sizeof(unsigned)) != hipSuccess) return GTT_ERR_HIP;
    if (hipMemcpy(rs->d_desc, rs->desc.data(), rs->desc.size() * sizeof(RaggedDesc), hipMemcpyHostToDevice) !=
        hipSuccess)
        return GTT_ERR_HIP;
    if (!rs->items.empty() &&
        hipMemcpy(rs->d_items, rs->items.data(), rs->items.size() * sizeof(RaggedItem), hipMemcpyHostToDevice) !=
            hipSuccess)
        return GTT_ERR_HIP;
    if (hipMemset(rs->d_bar, 0, 4 * sizeof(unsigned)) != hipSuccess) return GTT_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GTT_ERR_HIP;
    rs->cus = prop.multiProcessorCount;
    int per_cu = 0;
    if (ragged_occupancy(dt, rs->lds_max, &per_cu) != hipSuccess || per_cu < 1) return GTT_ERR_HIP;
    rs->grid_persistent = per_cu * rs->cus;
    rs->device = dev;
    rs->uploaded = true;
    return GTT_OK;
}

// a device is visible to this process (no HIP context is created on a
// machine without one)
static bool device_present() {
    int n = 0;
    return hipGetDeviceCount(&n) == hipSuccess && n > 0;
}

gtt_status plan_ragged(gtt_plan_s* p, int32_t count, const int32_t* b, const int32_t* n, const int64_t* x_off,
                       const int32_t* w_idx) {
    p->kind = PlanKind::Ragged;
    p->batch = 1;
    p->inst.resize(count);
    // W table
    std::vector<int> widx(count);
    if (w_idx) {
        int wmax = -1;
        for (int t = 0; t < count; ++t) {
            if (w_idx[t] < 0) return GTT_ERR_INVALID_VALUE;
            wmax = std::max(wmax, w_idx[t]);
        }
        p->w_b.assign(wmax + 1, 0);
        for (int t = 0; t < count; ++t) {
            int& wb = p->w_b[w_idx[t]];
            if (wb != 0 && wb != b[t]) return GTT_ERR_INVALID_VALUE;
            wb = b[t];
            widx[t] = w_idx[t];
        }
        for (int wb : p->w_b)
            if (wb == 0) return GTT_ERR_INVALID_VALUE;
    } else {
        std::map<int, int> m;
        for (int t = 0; t < count; ++t) m[b[t]] = 0;
        int i = 0;
        for (auto& kv : m) {
            kv.second = i++;
            p->w_b.push_back(kv.first);
        }
        for (int t = 0; t < count; ++t) widx[t] = m[b[t]];
    }
    int64_t acc = 0;
    for (int wb : p->w_b) {
        p->w_off.push_back(acc);
        acc += (int64_t)wb * wb;
    }
    p->w_elems = acc;
    int64_t off = 0, end = 0;
    for (int t = 0; t < count; ++t) {
        Instance& in = p->inst[t];
        in.b = b[t];
        in.n = n[t];
        int64_t N = 1;
        for (int i = 0; i < n[t]; ++i) N *= b[t];
        in.N = N;
        if (x_off) {
            if (x_off[t] < 0) return GTT_ERR_INVALID_VALUE;
            // every instance must start on a 16-byte boundary
            if ((x_off[t] * (int64_t)p->esize) % 16) return GTT_ERR_ALIGNMENT;
            in.off = x_off[t];
        } else {
            in.off = off;
        }
        off = in.off + N;
        end = std::max(end, in.off + N);
        in.w = widx[t];
        std::vector<int> rad(n[t], b[t]);
        gtt_status st = plan_groups(rad, 1, p->dtype, p->flags, true, &in.groups, &in.bwd_groups, true);
        if (st != GTT_OK) return st;
        // packed instances may start off a 16-byte boundary (a previous
        // instance of a length that is not a multiple of 16 bytes): their
        // tiles move element by element
        if ((in.off * (int64_t)p->esize) % 16) {
            for (std::vector<Group>* gs : {&in.groups, &in.bwd_groups})
                for (Group& g : *gs) {
                    if (g.mode == kContigVec) g.mode = kContigScalar;
                    if (g.mode == kRowVec) g.mode = kRowScalar;
                }
            ++p->ragged_scalar_instances;
        }
    }
    p->total_elems = end;
    p->slot = slot_elems(end, p->esize);
    int maxR = 0;
    for (const Instance& t : p->inst) maxR = std::max(maxR, (int)t.groups.size());
    if (maxR > kMaxPhases) return GTT_ERR_UNSUPPORTED;
    build_worklist(p);
    // the work list goes to the device now, so that forward / inverse
    // allocate nothing and can be captured from the first call
    if (device_present()) return upload_worklist(p);
    return GTT_OK;
}

gtt_status ragged_check(gtt_plan_s* p, hipStream_t s) {
    RaggedState* rs = p->rs;
    if (!rs || !rs->uploaded) return GTT_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return GTT_ERR_HIP;
    unsigned w[4] = {0, 0, 0, 0};
    if (hipMemcpy(w, rs->d_bar, sizeof w, hipMemcpyDeviceToHost) != hipSuccess) return GTT_ERR_HIP;
    if (w[2] == 0 && w[3] == 0) return GTT_OK;
    // clear the failure words (the arrival and generation words are reset
    // before every persistent launch)
    const unsigned z[2] = {0, 0};
    if (hipMemcpy(rs->d_bar + 2, z, sizeof z, hipMemcpyHostToDevice) != hipSuccess) return GTT_ERR_HIP;
    return GTT_ERR_TIMEOUT;
}

gtt_status ragged_set_spin_limit(gtt_plan_s* p, uint32_t polls) {
    if (!p->rs) return GTT_ERR_INVALID_VALUE;
    p->rs->spin_limit = polls;
    return GTT_OK;
}

void destroy_ragged(gtt_plan_s* p) {
    timing_release(p);
    if (p->rs) {
        if (p->rs->d_desc) (void)hipFree(p->rs->d_desc);
        if (p->rs->d_items) (void)hipFree(p->rs->d_items);
        if (p->rs->d_bar) (void)hipFree(p->rs->d_bar);
    }
    delete p->rs;
    p->rs = nullptr;
}


static gtt_status ragged_per_instance(gtt_plan_s* p, const void* W, const void* in, void* out, bool adjoint,
                                      char* saved, hipStream_t s);

// One persistent launch for all digit groups (GTT_FLAG_PERSISTENT), or one
// launch per phase; GTT_FLAG_PER_INSTANCE selects one launch per digit group
// per instance (the plain path).
gtt_status ragged_apply(gtt_plan_s* p, const void* W, const void* in, void* out, bool adjoint, char* saved,
                        hipStream_t s) {
    if (p->flags & GTT_FLAG_PER_INSTANCE) return ragged_per_instance(p, W, in, out, adjoint, saved, s);
    gtt_status st = upload_worklist(p);
    if (st != GTT_OK) return st;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return GTT_ERR_HIP;
    if (dev != p->rs->device) return GTT_ERR_INVALID_VALUE;  // the work list lives on another device
    RaggedState* rs = p->rs;
    const DT dt = static_cast<DT>((int)p->dtype);
    RaggedArgs a;
    std::memset(&a, 0, sizeof a);
    a.desc = rs->d_desc;
    a.items = rs->d_items;
    a.nphases = (int)rs->phase_start.size() - 1;
    for (int i = 0; i <= a.nphases; ++i) a.phase_start[i] = rs->phase_start[i];
    a.adjoint = adjoint ? 1 : 0;
    a.x = in;
    a.y = out;
    a.saved = adjoint ? nullptr : saved;
    a.W = W;
    a.bar = rs->d_bar;
    a.spin_limit = rs->spin_limit;
    static const char* dn[] = {"f64", "f32", "c128", "c64", "bf16", "f16", "i32"};
    if (p->flags & GTT_FLAG_PERSISTENT) {
        int64_t most = 0;
        for (int i = 0; i < a.nphases; ++i) most = std::max(most, rs->phase_start[i + 1] - rs->phase_start[i]);
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rs->grid_persistent, most));
        a.persistent = 1;
        if (launch_barrier_reset(rs->d_bar, s) != hipSuccess) return GTT_ERR_HIP;
        const std::string nm = std::string("ragged persistent ") + dn[(int)p->dtype];
        timing_begin(p, s, nm);
        if (launch_ragged(dt, a, grid, rs->lds_max, s) != hipSuccess) return GTT_ERR_HIP;
        timing_end(p, s, nm, 2.0 * (double)p->total_elems * (double)p->esize * (double)a.nphases);
        return GTT_OK;
    }
    // one launch per run of one item class in a phase, in order on the
    // caller's stream.  (The runs of a phase touch disjoint instances, but
    // the matrix-core runs fill the device with resident work-groups, and
    // concurrent runs on helper streams measured slower.)
    a.persistent = 0;
    a.phase = 0;
    for (const RaggedState::Seg& sg : rs->segs) {
        a.phase_start[0] = sg.start;
        a.phase_start[1] = sg.end;
        const unsigned grid = (unsigned)std::min<int64_t>(sg.end - sg.start, (int64_t)0x7fffffff);
        std::string nm;
        if (p->timing.enabled)
            nm = std::string("ragged phase ") + std::to_string(sg.phase) + " " + dn[(int)p->dtype] +
                 (sg.cls == kClsGeneric ? " generic" : (sg.cls >= 16 ? " mfma b=" : " b=") + std::to_string(sg.cls));
        timing_begin(p, s, nm);
        if (launch_ragged_cls(dt, sg.cls, a, grid, sg.lds, s) != hipSuccess) return GTT_ERR_HIP;
        timing_end(p, s, nm, sg.bytes);
    }
    return GTT_OK;
}

// Per-instance launches (one launch per digit group per instance).
static gtt_status ragged_per_instance(gtt_plan_s* p, const void* W, const void* in, void* out, bool adjoint,
                                      char* saved, hipStream_t s) {
    const size_t es = p->esize, cs = p->csize;
    for (const Instance& t : p->inst) {
        const char* src = static_cast<const char*>(in) + t.off * es;
        char* dst = static_cast<char*>(out) + t.off * es;
        const char* w = static_cast<const char*>(W) + p->w_off[t.w] * cs;
        if (t.groups.empty()) {
            if (src != dst && hipMemcpyAsync(dst, src, es, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return GTT_ERR_HIP;
            continue;
        }
        const void* cur = src;
        for (size_t i = 0; i < t.groups.size(); ++i) {
            void* nxt = dst;
            if (saved && i + 1 < t.groups.size())
                nxt = saved + ((int64_t)i * p->slot + t.off) * es;
            gtt_status st = launch_group_inst(p, p->dtype, t.groups[i], t.b, t.N, w, adjoint, cur, nxt, s);
            if (st != GTT_OK) return st;
            cur = nxt;
        }
    }
    return GTT_OK;
}

static int max_groups(const gtt_plan_s* p) {
    if (p->kind != PlanKind::Ragged) return (int)p->groups.size();
    int r = 0;
    for (const Instance& t : p->inst) r = std::max(r, (int)t.groups.size());
    return r;
}

size_t bwd_partial_bytes(const gtt_plan_s* p) {
    // per-work-group partial vectors (accumulation dtype), plus the
    // reduction's first-stage vectors after the partials of each W
    const size_t as = acc_size(p->dtype);
    size_t partial = 0;
    if (p->kind == PlanKind::Ragged) {
        for (const Instance& t : p->inst) partial += bwd_partials_elems(t.bwd_groups, t.b * t.b) * as;
        for (int wb : p->w_b) partial += (size_t)kReduceBlocks * wb * wb * as;
    } else {
        const int wslot = (int)p->w_elems;
        partial += bwd_partials_elems(p->bwd_groups, wslot) * as;
        partial += (size_t)kReduceBlocks * wslot * as;
    }
    return (partial + 255) & ~(size_t)255;
}

void workspace_sizes(const gtt_plan_s* p, size_t* fwd, size_t* bwd, size_t* saved) {
    const int R = max_groups(p);
    *fwd = 0;
    *saved = (R > 1) ? (size_t)(R - 1) * (size_t)p->slot * p->esize : 0;
    // backward: per-tile partial sums of the weight gradient (compute dtype,
    // b*b per tile and group) plus room to recompute the saved activations
    const size_t partial = bwd_partial_bytes(p);
    // + a cotangent buffer between digit groups (used when gx is NULL or
    // aliases gy)
    const size_t cbuf = (R > 1 || p->kind == PlanKind::Ragged) ? (size_t)p->slot * p->esize : 0;
    *bwd = partial + *saved + cbuf;
}

static hipEvent_t pool_get(Timing& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static thread_local hipEvent_t t_open = nullptr;

void timing_begin(gtt_plan_s* p, hipStream_t s, const std::string& name) {
    t_open = nullptr;
    if (!p || !p->timing.enabled) return;
    const std::string& f = p->timing.filter;
    if (!f.empty() && name.compare(0, f.size(), f) != 0) return;
    t_open = pool_get(p->timing);
    if (t_open) (void)hipEventRecord(t_open, s);
}

void timing_end(gtt_plan_s* p, hipStream_t s, const std::string& name, double bytes) {
    if (!p || !p->timing.enabled || !t_open) return;
    hipEvent_t e = pool_get(p->timing);
    if (!e) return;
    (void)hipEventRecord(e, s);
    p->timing.pending.push_back(TimedLaunch{name, t_open, e, bytes});
    t_open = nullptr;
}

void timing_release(gtt_plan_s* p) {
    for (auto& tl : p->timing.pending) {
        (void)hipEventDestroy(tl.start);
        (void)hipEventDestroy(tl.stop);
    }
    for (auto e : p->timing.pool) (void)hipEventDestroy(e);
    p->timing.pending.clear();
    p->timing.pool.clear();
}

std::string timing_read(gtt_plan_s* p) {
    struct Agg {
        int n = 0;
        double ms = 0, bytes = 0;
    };
    std::map<std::string, Agg> agg;
    for (auto& tl : p->timing.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(tl.stop) == hipSuccess && hipEventElapsedTime(&ms, tl.start, tl.stop) == hipSuccess) {
            Agg& a = agg[tl.name];
            a.n += 1;
            a.ms += ms;
            a.bytes += tl.bytes;
        }
        p->timing.pool.push_back(tl.start);
        p->timing.pool.push_back(tl.stop);
    }
    p->timing.pending.clear();
    std::string s = "{";
    bool first = true;
    for (auto& kv : agg) {
        char b[512];
        std::snprintf(b, sizeof b, "%s\"%s\":{\"launches\":%d,\"total_ms\":%.6f,\"avg_ms\":%.6f,\"bytes_per_launch\":%.1f}",
                      first ? "" : ",", kv.first.c_str(), kv.second.n, kv.second.ms, kv.second.ms / kv.second.n,
                      kv.second.bytes / kv.second.n);
        s += b;
        first = false;
    }
    s += "}";
    return s;
}

std::string describe_plan(const gtt_plan_s* p) {
    auto grp = [](const Group& g) {
        char b[512];
        std::snprintf(b, sizeof b,
                      "{\"s0\":%d,\"k\":%d,\"S\":%lld,\"G\":%lld,\"C\":%d,\"P\":%d,\"L\":%lld,\"tiles\":%lld,"
                      "\"tile_elems\":%lld,\"mode\":%d,\"pad_shift\":%d,\"kind\":\"%s\",\"lds_bytes\":%zu,"
                      "\"fast_ni\":%d,\"fmap\":%llu,\"pmap\":%u,\"fast_conflicts\":%d,\"bwd_slots\":%d,"
                      "\"bwd_ops\":%d,\"bwd_fwd_passes\":%d,\"bwd_ok\":%s,\"bwd_rd\":%d,\"bwd_schedule\":[",
                      g.s0, g.k, (long long)g.S, (long long)g.G, g.C, g.P, (long long)g.L, (long long)g.ntiles,
                      (long long)g.tileE, g.mode, g.pad_shift, g.kind == 0 ? "valu" : g.kind == 1 ? "generic" : g.kind == 2 ? "mfma" : "cmfma",
                      g.lds_bytes, g.fast_ni, (unsigned long long)g.fmap, g.pmap, g.fast_conflicts, g.bwd_slots,
                      (int)g.bwd_ops.size(),
                      g.bwd_slots ? bwd_fwd_passes(g.bwd_rd > 0 ? (g.k + g.bwd_rd - 1) / g.bwd_rd : g.k, g.bwd_slots - 2)
                                  : 0,
                      g.bwd_ok ? "true" : "false", g.bwd_rd);
        std::string r(b);
        for (size_t i = 0; i < g.bwd_ops.size(); ++i) r += (i ? "," : "") + std::to_string((int)g.bwd_ops[i]);
        return r + "]}";
    };
    std::string s = "{";
    char head[256];
    const char* kind = p->kind == PlanKind::Uniform ? "uniform" : p->kind == PlanKind::Mixed ? "mixed" : "ragged";
    std::snprintf(head, sizeof head, "\"kind\":\"%s\",\"dtype\":%d,\"b\":%d,\"n\":%d,\"N\":%lld,\"batch\":%lld,",
                  kind, (int)p->dtype, p->b, p->n, (long long)p->N, (long long)p->batch);
    s += head;
    if (p->kind != PlanKind::Ragged) {
        // with a float32 inner plan, its digit groups are the ones that run
        const gtt_plan_s* q = p->inner ? p->inner : p;
        s += p->inner ? "\"fp32_intermediate\":true,\"groups\":[" : "\"groups\":[";
        for (size_t i = 0; i < q->groups.size(); ++i) {
            if (i) s += ",";
            s += grp(q->groups[i]);
        }
        s += "],\"bwd_groups\":[";
        for (size_t i = 0; i < q->bwd_groups.size(); ++i) {
            if (i) s += ",";
            s += grp(q->bwd_groups[i]);
        }
        s += "]";
    } else {
        char b[192];
        std::snprintf(b, sizeof b, "\"instances\":%zu,\"w_table\":%zu,\"max_groups\":%d,\"scalar_instances\":%d",
                      p->inst.size(), p->w_b.size(), max_groups(p), p->ragged_scalar_instances);
        s += b;
    }
    s += "}";
    return s;
}

}  // namespace gtt
