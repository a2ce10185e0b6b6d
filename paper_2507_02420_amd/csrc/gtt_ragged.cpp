// Ragged batches (instances of different radix and length in one buffer),
// workspace sizing and plan descriptions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>

#include "gtt_launch.hpp"
#include "gtt_plan.hpp"

namespace gtt {

struct RaggedState {
    int dummy = 0;
};

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
        gtt_status st = plan_groups(rad, 1, p->dtype, p->flags, true, &in.groups);
        if (st != GTT_OK) return st;
    }
    p->total_elems = end;
    return GTT_OK;
}

void destroy_ragged(gtt_plan_s* p) {
    delete p->rs;
    p->rs = nullptr;
}

gtt_status launch_group_inst(gtt_dtype dt, const Group& g, int b, int64_t N, const void* W, bool adjoint,
                             const void* in, void* out, hipStream_t s);

// Per-instance launches (one launch per digit group per instance).
gtt_status ragged_apply(gtt_plan_s* p, const void* W, const void* in, void* out, bool adjoint, char* saved,
                        hipStream_t s) {
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
                nxt = saved + ((int64_t)i * p->total_elems + t.off) * es;
            gtt_status st = launch_group_inst(p->dtype, t.groups[i], t.b, t.N, w, adjoint, cur, nxt, s);
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

void workspace_sizes(const gtt_plan_s* p, size_t* fwd, size_t* bwd, size_t* saved) {
    const int R = max_groups(p);
    const size_t E = (size_t)p->total_elems;
    *fwd = 0;
    *saved = (R > 1) ? (size_t)(R - 1) * E * p->esize : 0;
    // backward: per-tile partial sums of the weight gradient (compute dtype,
    // b*b per tile and group) plus room to recompute the saved activations
    size_t partial = 0;
    auto add_groups = [&](const std::vector<Group>& gs, int b) {
        for (const Group& g : gs) partial += (size_t)g.ntiles * b * b * p->csize;
    };
    if (p->kind == PlanKind::Ragged) {
        for (const Instance& t : p->inst) add_groups(t.groups, t.b);
        partial += 256;
    } else {
        add_groups(p->groups, p->b);
    }
    partial = (partial + 255) & ~(size_t)255;
    *bwd = partial + *saved;
}

std::string describe_plan(const gtt_plan_s* p) {
    auto grp = [](const Group& g) {
        char b[320];
        std::snprintf(b, sizeof b,
                      "{\"s0\":%d,\"k\":%d,\"S\":%lld,\"G\":%lld,\"C\":%d,\"P\":%d,\"L\":%lld,\"tiles\":%lld,"
                      "\"tile_elems\":%lld,\"mode\":%d,\"pad_shift\":%d,\"generic\":%s,\"lds_bytes\":%zu}",
                      g.s0, g.k, (long long)g.S, (long long)g.G, g.C, g.P, (long long)g.L, (long long)g.ntiles,
                      (long long)g.tileE, g.mode, g.pad_shift, g.generic ? "true" : "false", g.lds_bytes);
        return std::string(b);
    };
    std::string s = "{";
    char head[256];
    const char* kind = p->kind == PlanKind::Uniform ? "uniform" : p->kind == PlanKind::Mixed ? "mixed" : "ragged";
    std::snprintf(head, sizeof head, "\"kind\":\"%s\",\"dtype\":%d,\"b\":%d,\"n\":%d,\"N\":%lld,\"batch\":%lld,",
                  kind, (int)p->dtype, p->b, p->n, (long long)p->N, (long long)p->batch);
    s += head;
    if (p->kind != PlanKind::Ragged) {
        s += "\"groups\":[";
        for (size_t i = 0; i < p->groups.size(); ++i) {
            if (i) s += ",";
            s += grp(p->groups[i]);
        }
        s += "]";
    } else {
        char b[128];
        std::snprintf(b, sizeof b, "\"instances\":%zu,\"w_table\":%zu,\"max_groups\":%d", p->inst.size(),
                      p->w_b.size(), max_groups(p));
        s += b;
    }
    s += "}";
    return s;
}

}  // namespace gtt
