// Host side of libgtt.so: argument checking, planning (digit groups and tile
// shapes) and kernel launch sequences for the C ABI declared in gtt.h.
#include "gtt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gtt_args.hpp"
#include "gtt_launch.hpp"
#include "gtt_plan.hpp"

using namespace gtt;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
namespace gtt {

FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1);
    return f;
}

uint32_t host_fdiv(uint32_t n, const FastDiv& f) {
    const uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
    return (hi + n) >> f.s;
}

size_t storage_size(gtt_dtype d) {
    switch (d) {
        case GTT_F64: return 8;
        case GTT_F32: return 4;
        case GTT_C128: return 16;
        case GTT_C64: return 8;
        case GTT_BF16: return 2;
        case GTT_F16: return 2;
        case GTT_I32: return 4;
    }
    return 0;
}

size_t compute_size(gtt_dtype d) {
    switch (d) {
        case GTT_F64: return 8;
        case GTT_F32: return 4;
        case GTT_C128: return 16;
        case GTT_C64: return 8;
        case GTT_BF16: return 4;
        case GTT_F16: return 4;
        case GTT_I32: return 4;
    }
    return 0;
}

size_t f32_buf_bytes(const gtt_plan_s* p) {
    return (((size_t)p->total_elems * sizeof(float)) + 255) & ~(size_t)255;
}

static bool valid_dtype(int d) { return d >= GTT_F64 && d <= GTT_I32; }

static int ilog2_floor(uint64_t v) {
    int r = -1;
    while (v) { v >>= 1; ++r; }
    return r;
}

// tuning table: (b, n, dtype) -> overrides; n == 0 applies to every n of
// that radix without an entry of its own
struct TuneEntry {
    int b;
    int n;
    int dtype;
    int lds_budget;
    int min_row_bytes;
    int max_group_digits;
    int bwd_lds;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

struct Tuning {
    int budget = 0, minrow = 0, maxk = 0, bwd_lds = 0;
};

static Tuning tuning_for(int b, int n, gtt_dtype dt, uint32_t flags) {
    Tuning t;
    if (flags & GTT_FLAG_NO_TUNE) return t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneEntry* any = nullptr;
    const TuneEntry* exact = nullptr;
    for (const auto& e : g_tune)
        if (e.b == b && e.dtype == (int)dt) {
            if (e.n == n) exact = &e;
            if (e.n == 0) any = &e;
        }
    const TuneEntry* e = exact ? exact : any;
    if (e) {
        t.budget = e->lds_budget;
        t.minrow = e->min_row_bytes;
        t.maxk = e->max_group_digits;
        t.bwd_lds = e->bwd_lds;
    }
    return t;
}

// ---------------------------------------------------------------------------
// Planner: split the digits (radix list, least significant first) into groups
// of consecutive digits and choose the tile of every group.
// ---------------------------------------------------------------------------
static int64_t prod_range(const std::vector<int>& rad, int a, int b) {
    int64_t p = 1;
    for (int i = a; i < b; ++i) p *= rad[i];
    return p;
}

static uint64_t pow2_floor(uint64_t v) { return v ? (uint64_t(1) << ilog2_floor(v)) : 0; }

// Try to split the n digits into exactly R groups; group 0 contiguous, the
// others strided with C columns.  Returns false if infeasible.
static bool try_split(const std::vector<int>& rad, int R, int64_t T, int64_t Gmax, int64_t cmin_elems,
                      std::vector<int>* ks, int maxk) {
    const int n = (int)rad.size();
    if (maxk <= 0) maxk = 64;
    // group 0: as many digits as fit
    int k0 = 0;
    int64_t g = 1;
    while (k0 < n && k0 < maxk && g * rad[k0] <= std::min(T, Gmax)) g *= rad[k0++];
    if (k0 == 0) return false;
    if (R == 1) {
        if (k0 < n) return false;
        ks->assign(1, n);
        return true;
    }
    if (k0 >= n) return false;  // R=1 would do
    // strided groups: greedily from the low side, each as many digits as fit
    // with at least cmin columns; then require that all digits are covered.
    std::vector<int> out{k0};
    int s = k0;
    for (int r = 1; r < R && s < n; ++r) {
        int k = 0;
        int64_t G = 1;
        while (s + k < n && k < maxk && G * rad[s + k] * cmin_elems <= T && G * rad[s + k] <= Gmax)
            G *= rad[s + k++];
        if (k == 0) return false;
        out.push_back(k);
        s += k;
    }
    if (s < n || (int)out.size() != R) return false;
    // balance the strided groups: move digits from earlier strided groups to
    // later ones while it does not shrink the minimum column count
    *ks = out;
    return true;
}

static void fill_group(Group* gr, const std::vector<int>& rad, int s0, int k, int64_t total_elems,
                       int64_t T, size_t esize, size_t csize, int kind, int64_t row_elems_target) {
    gr->s0 = s0;
    gr->k = k;
    gr->elems = total_elems;
    gr->S = prod_range(rad, 0, s0);
    gr->G = prod_range(rad, s0, s0 + k);
    const int64_t GS = gr->G * gr->S;
    const int64_t hi_total = total_elems / GS;  // hi blocks over the whole buffer
    if (gr->S == 1) {
        gr->C = 1;
        // P: hi blocks per tile (a divisor of hi_total), tile <= T
        int64_t P = std::max<int64_t>(1, T / gr->G);
        P = std::min(P, hi_total);
        while (P > 1 && hi_total % P) --P;
        gr->P = (int)P;
        gr->L = 1;
    } else {
        int64_t C = (int64_t)pow2_floor((uint64_t)std::max<int64_t>(1, T / gr->G));
        // never wider than the row itself
        C = std::min<int64_t>(C, (int64_t)pow2_floor((uint64_t)gr->S));
        gr->C = (int)C;
        gr->P = 1;
        gr->L = (gr->S + C - 1) / C;
        (void)row_elems_target;
    }
    gr->logC = ilog2_floor((uint64_t)gr->C);
    gr->ntiles = (hi_total / gr->P) * gr->L;
    const int64_t tileE = (int64_t)gr->P * gr->G * gr->C;
    gr->tileE = tileE;
    const size_t V = 16 / esize;
    if (gr->C == gr->S || gr->S == 1) {
        gr->mode = ((tileE * (int64_t)esize) % 16 == 0) ? kContigVec : kContigScalar;
    } else if ((gr->C * esize) % 16 == 0 && (gr->S * (int64_t)esize) % 16 == 0 && gr->S % gr->C == 0) {
        gr->mode = kRowVec;
    } else {
        gr->mode = kRowScalar;
        // element-wise rows: at most one work-group's threads wide, so a
        // thread keeps its column over the tile (the kernels' address walk)
        if (gr->C > kThreads) {
            gr->C = kThreads;
            gr->logC = ilog2_floor((uint64_t)gr->C);
            gr->L = (gr->S + gr->C - 1) / gr->C;
            gr->ntiles = (hi_total / gr->P) * gr->L;
            gr->tileE = (int64_t)gr->P * gr->G * gr->C;
        }
    }
    (void)V;
    gr->kind = kind;
    // LDS padding (see lds_phys): for a power-of-two radix, pads one digit
    // apart starting at the register block (contiguous tiles) or at the row
    // (strided tiles), so digit strides become odd bank strides; odd radices
    // need none; radix 6 gets the register-block level only
    int pad = kNoPad;
    if (gr->kind != kKindGeneric) {
        const int b = rad[s0];
        const int lv = ilog2_floor(16 / esize);  // vector runs must not straddle a pad
        int p1 = -1, step = 0;
        if ((b & (b - 1)) == 0) {
            const int nb = (b == 2 || b == 4) ? 16 : b;  // register block size
            p1 = (gr->C == 1) ? ilog2_floor((uint64_t)nb) : gr->logC;
            step = ilog2_floor((uint64_t)b);
            if (step < 2) step = 2;
        } else if (b == 6) {
            p1 = (gr->C == 1) ? 4 : gr->logC;
            step = 0;
        }
        if (p1 >= 0) {
            if (p1 < 2) p1 = 2;
            if (gr->mode == kContigVec || gr->mode == kRowVec) p1 = std::max(p1, lv);
            int p2 = step ? std::min(31, p1 + step) : 31;
            int p3 = step ? std::min(31, p1 + 2 * step) : 31;
            // the extra levels only where the tile has that many digits
            const int64_t span = gr->tileE;
            if (p2 < 31 && (int64_t(1) << p2) >= span) p2 = 31;
            if (p3 < 31 && (int64_t(1) << p3) >= span) p3 = 31;
            pad = p1 | (p2 << 8) | (p3 << 16);
        }
    }
    // matrix-core passes: padding from the bank-conflict search over the
    // tile transfers and the digit passes' fragment loads
    // (a 16-bit tile, csize 2: pads count 32-bit words, a 16-byte vector is
    // four of them)
    const bool lds16 = gr->kind == kKindMfma && csize == 2;
    if (gr->kind == kKindMfma && gr->tileE % 64 == 0)
        pad = lds16 ? mfma_pad(rad[s0], k, gr->logC, gr->tileE, 2, 8, true)
                    : mfma_pad(rad[s0], k, gr->logC, gr->tileE, ilog2_floor(16 / esize), (int)(16 / esize), false);
    gr->pad_shift = pad;
    if (gr->kind == kKindGeneric) {
        // radices <= 16 run in place on one tile buffer; a larger radix needs
        // a second buffer.  Unpadded (the kernel is bound by its VALU work,
        // and the pad's address arithmetic cost more than the bank conflicts
        // it removed)
        int64_t wtot = 0;
        int maxr = 0;
        for (int j = 0; j < k; ++j) {
            wtot += (int64_t)rad[s0 + j] * rad[s0 + j];
            maxr = std::max(maxr, rad[s0 + j]);
        }
        const bool inplace = maxr <= kGenericInplaceMax;
        gr->pad_shift = kNoPad;
        const int64_t phys = lds_tile_elems_host(gr->tileE, gr->pad_shift);
        gr->wtotal = (int)wtot;
        gr->lds_bytes = (size_t)(((wtot + 15) & ~15LL) + (inplace ? 1 : 2) * phys) * csize;
    } else {
        const int64_t phys =
            lds16 ? 2 * lds_tile_elems_host((gr->tileE + 1) / 2, pad) : lds_tile_elems_host(gr->tileE, pad);
        gr->wtotal = 0;
        gr->lds_bytes = (size_t)phys * csize;
    }
}

// Complex radix-8 matrix-core groups of up to four digits on tiles of 2048
// or 4096 elements run the kernels with per-lane LDS addresses, on the
// padding and fibre-to-lane maps chosen for them (bwd: with the gradient
// sums' accesses).
static void make_fast(Group* g, size_t csize, bool bwd) {
    g->fast_ni = 0;
    g->fmap = 0;
    g->pmap = 0;
    if (g->kind != kKindCMfma || g->k < 1 || g->k > 4) return;
    if (g->mode != kContigVec && g->mode != kRowVec) return;
    const int ni = g->tileE == 2048 ? 1 : g->tileE == 4096 ? 2 : 0;
    if (!ni) return;
    const FastMap m = fast_map(g->k, ni, g->logC, bwd);
    g->fast_ni = ni;
    g->fmap = m.map;
    g->pmap = m.pmap;
    g->fast_conflicts = m.conflicts;
    g->pad_shift = m.pad;
    g->lds_bytes = (size_t)lds_tile_elems_host(g->tileE, m.pad) * csize;
}

// Tile and checkpoint schedule of a backward group on the general kernel.
// Candidate tiles hold G * 2^i elements (at most 40 KiB, or one group's
// positions) and a work-group holds as many of them as fit its LDS budget
// (40, 64, 80, 120 or 160 KiB), at most k + 1 (then every activation of the
// group is computed once).  A work-group is four waves, one per SIMD, so the
// budget sets the waves per SIMD (160 KiB / budget, at most four) that hide
// the latency of LDS and global accesses.  Preference: HBM rows of at least
// 32 bytes for strided groups (where any tile allows), then the smallest
// estimated time per element, LDS passes (forward passes of the schedule
// plus a gradient sweep and an adjoint pass per digit) over
// (waves / 4)^0.75, then the larger tile.
static void plan_bwd_general(Group* out, const std::vector<int>& rad, int s0, int k, int64_t total, gtt_dtype dt,
                             int kind, int64_t cmin, bool shared_w, int bwd_lds) {
    const size_t es = storage_size(dt), cs = compute_size(dt);
    int maxb = 0;
    int64_t wloc = 0, G = 1;
    for (int j = 0; j < k; ++j) {
        maxb = std::max(maxb, rad[s0 + j]);
        wloc += (int64_t)rad[s0 + j] * rad[s0 + j];
        G *= rad[s0 + j];
    }
    if (shared_w) wloc = (int64_t)rad[s0] * rad[s0];
    const bool radix_ok = maxb <= 32 && wloc <= 4096 && k <= kMaxDigits;
    // one W for every digit and a radix with a register-block kernel: the
    // schedule runs over blocks of rd digits (one LDS round trip a block)
    const int rd0 = shared_w ? bwd_block_digits(static_cast<DT>((int)dt), rad[s0]) : 0;
    const bool pow2 = (rad[s0] & (rad[s0] - 1)) == 0;
    const size_t over = radix_ok ? bwd_overhead_bytes((int)wloc, dt) : 0;
    const int64_t Tmax = std::max<int64_t>(G, (int64_t)(40 * 1024) / (int64_t)cs);
    // strided tiles: rows of at least this many bytes are preferred before
    // the schedule's cost.  Power-of-two radices move 16-byte vectors and
    // want the forward's row width (whole 128-byte lines: 32-byte rows cost
    // 17-28 % on the complex64 radix-4 and float32 radix-2 / 4 strided
    // groups); odd radices move 4-byte elements, where the smaller tiles'
    // occupancy measured better than wider rows (float32 radix 3: 10 %).
    const int64_t row_cap = pow2 ? std::max<int64_t>(32, cmin * (int64_t)es) : 32;
    bool found = false;
    Group best;
    int best_passes = 0, best_slots = 0, best_rd = 0, best_units = 0;
    int64_t best_row = 0;
    const std::vector<size_t> default_caps = {(size_t)40 * 1024, (size_t)64 * 1024, (size_t)80 * 1024,
                                              (size_t)120 * 1024, (size_t)160 * 1024};
    double best_cost = 0.0;
    auto search = [&](const std::vector<size_t>& caps) {
        for (size_t cap : caps) {
            for (int64_t T = G; T <= Tmax && radix_ok; T *= 2) {
                Group c;
                fill_group(&c, rad, s0, k, total, T, es, cs, kind, cmin);
                const size_t tb = (size_t)lds_tile_elems_host(c.tileE, c.pad_shift) * cs;
                if (over + 3 * tb > cap) break;  // tiles only grow with T
                // the register-block kernel addresses a block as one padded
                // base plus fixed offsets: a power-of-two radix, or an
                // unpadded tile
                const int rd = (rd0 > 0 && (pow2 || c.pad_shift == kNoPad)) ? rd0 : 0;
                const int units = rd > 0 ? (k + rd - 1) / rd : k;
                const int slots =
                    (int)std::min<size_t>((cap - over) / tb, (size_t)std::min(units + 1, kMaxBwdSlots));
                const int passes = bwd_fwd_passes(units, slots - 2) + 2 * units;
                const size_t lds = over + (size_t)slots * tb;
                const int waves = (int)std::min<size_t>(4, (160 * 1024) / lds);
                const double cost = (double)passes / std::pow((double)waves / 4.0, 0.75);
                const int64_t row = std::min<int64_t>(c.S == 1 ? INT64_MAX : (int64_t)c.C * (int64_t)es, row_cap);
                bool better = !found;
                if (!better) {
                    if (row != best_row) better = row > best_row;
                    else if (cost != best_cost) better = cost < best_cost;
                    else better = c.tileE > best.tileE;
                }
                if (better) {
                    found = true;
                    best = c;
                    best_rd = rd;
                    best_units = units;
                    best_passes = passes;
                    best_slots = slots;
                    best_row = row;
                    best_cost = cost;
                }
            }
        }
    };
    // tuned: one LDS budget per work-group; a budget that holds no schedule
    // (fewer than three tiles) falls back to the built-in budgets
    if (bwd_lds > 0) search({(size_t)bwd_lds});
    if (!found) search(default_caps);
    if (!found) {
        // no backward for this group: keep the forward geometry for the
        // plan's description
        fill_group(out, rad, s0, k, total, Tmax, es, cs, kind, cmin);
        out->bwd_ok = false;
        out->bwd_maxb = maxb;
        return;
    }
    *out = best;
    out->bwd_ok = true;
    out->bwd_slots = best_slots;
    out->bwd_maxb = maxb;
    out->bwd_wloc = (int)wloc;
    out->bwd_rd = best_rd;
    out->bwd_ops = bwd_schedule(best_units, best_slots);
}

// Plan the digit groups for one radix list.
gtt_status plan_groups(const std::vector<int>& rad, int64_t batch, gtt_dtype dt, uint32_t flags,
                       bool uniform, std::vector<Group>* groups, std::vector<Group>* bwd_groups, bool ragged) {
    groups->clear();
    if (bwd_groups) bwd_groups->clear();
    const int n = (int)rad.size();
    if (n == 0) return GTT_OK;
    const size_t es = storage_size(dt), cs = compute_size(dt);
    const int b0 = rad[0];
    // specialised kernels: radix <= 8 on the VALU (complex double: <= 5,
    // larger W would not fit in registers); radix 16 / 32 with 16-bit or
    // FP32 storage on the matrix cores; everything else on the runtime-radix
    // kernel
    int kind = kKindGeneric;
    // (the one-launch ragged kernel carries the VALU code for radix <= 5 only)
    if (uniform && (b0 <= 5 || (b0 <= 8 && dt != GTT_C128 && !ragged))) kind = kKindValu;
    if (uniform && (b0 == 16 || b0 == 32) && (dt == GTT_BF16 || dt == GTT_F16 || dt == GTT_F32)) kind = kKindMfma;
    if (uniform && b0 == 8 && dt == GTT_C64 && !ragged) kind = kKindCMfma;
    const bool small_b = kind != kKindGeneric;
    // the bf16 / f16 matrix-core pass keeps its tile in the storage type
    const size_t cs_fwd = (kind == kKindMfma && es == 2) ? es : cs;
    const Tuning tu = tuning_for(uniform ? b0 : 0, n, dt, flags);
    const int tb = tu.budget, tr = tu.minrow, tk = tu.maxk;
    std::vector<int64_t> budgets;
    if (tb > 0) {
        budgets.push_back(tb);
    } else {
        budgets = {32768, 65536};
    }
    const int64_t min_row_bytes = tr > 0 ? tr : 128;
    int64_t N = 1;
    int maxrad = 0;
    for (int r : rad) {
        N *= r;
        maxrad = std::max(maxrad, r);
    }
    const int64_t total = N * batch;
    for (int64_t relax_row = min_row_bytes; relax_row >= (int64_t)es; relax_row /= 2) {
        for (int R = 1; R <= n; ++R) {
            for (int64_t bud : budgets) {
                int64_t T = bud / (int64_t)cs_fwd;
                // the runtime-radix kernel double-buffers for radices above 16
                if (!small_b && maxrad > kGenericInplaceMax) T /= 2;
                const int64_t cmin = std::max<int64_t>(1, relax_row / (int64_t)es);
                std::vector<int> ks;
                // a group's positions must fit three times in LDS for backward
                const int64_t Gmax = (int64_t)(40 * 1024) / (int64_t)cs;
                if (!try_split(rad, R, T, Gmax, cmin, &ks, tk)) continue;
                int s = 0;
                for (int k : ks) {
                    Group g;
                    fill_group(&g, rad, s, k, total, T, es, cs_fwd, kind, cmin);
                    groups->push_back(g);
                    s += k;
                }
                for (Group& g : *groups) make_fast(&g, cs, false);
                if (bwd_groups) {
                    // backward: same digit groups.  Complex radix 8 takes the
                    // matrix-core backward (up to 4 digits on vector tiles of
                    // at most 8192 elements); every other group the general
                    // backward, on tiles chosen for its checkpoint schedule
                    bwd_groups->clear();
                    for (const Group& fg : *groups) {
                        Group g;
                        if (kind == kKindCMfma) {
                            const int64_t Tb = (int64_t)(40 * 1024) / (int64_t)cs;
                            fill_group(&g, rad, fg.s0, fg.k, total, Tb, es, cs, kind, cmin);
                            if (g.k <= 4 && g.tileE <= 8192 && (g.mode == kContigVec || g.mode == kRowVec)) {
                                make_fast(&g, cs, true);
                                bwd_groups->push_back(g);
                                continue;
                            }
                        }
                        plan_bwd_general(&g, rad, fg.s0, fg.k, total, dt, kind == kKindCMfma ? kKindValu : kind,
                                         cmin, uniform, tu.bwd_lds);
                        bwd_groups->push_back(g);
                    }
                }
                return GTT_OK;
            }
        }
    }
    return GTT_ERR_UNSUPPORTED;  // a single digit does not fit in LDS
}

}  // namespace gtt

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
static DT to_dt(gtt_dtype d) { return static_cast<DT>((int)d); }

namespace gtt {
void fill_pass_args(PassArgs* a, const Group& g, const std::vector<int>& rad, const std::vector<int64_t>& wofs,
                      int64_t N) {
    std::memset(a, 0, sizeof(*a));
    a->k = g.k;
    a->G = (int32_t)g.G;
    a->P = g.P;
    a->logC = g.logC;
    a->mode = g.mode;
    a->pad_shift = g.pad_shift;
    a->cut = -1;
    a->S = g.S;
    a->L = g.L;
    a->ntiles = g.ntiles;
    a->N = N;
    a->divG = make_fastdiv((uint32_t)g.G);
    a->divL = make_fastdiv(g.L < (int64_t(1) << 31) ? (uint32_t)g.L : 1u);
    int64_t pv = 1;
    for (int j = 0; j <= g.k; ++j) {
        a->bpow[j] = (int32_t)pv;
        a->divb[j] = make_fastdiv((uint32_t)pv);
        if (j < g.k) {
            const int r = rad[g.s0 + j];
            a->rad[j] = r;
            a->divrad[j] = make_fastdiv((uint32_t)r);
            a->wofs[j] = (int32_t)wofs[g.s0 + j];
            pv *= r;
        }
    }
    a->wtotal = g.wtotal;
    a->fmap = g.fmap;
    a->pmap = g.pmap;
}
}  // namespace gtt

static const char* dt_name(gtt_dtype d) {
    static const char* n[] = {"f64", "f32", "c128", "c64", "bf16", "f16", "i32"};
    return n[(int)d];
}

static gtt_status launch_group(gtt_plan_s* tp, gtt_dtype dt, const Group& g, const std::vector<int>& rad,
                               const std::vector<int64_t>& wofs, int64_t N, const void* W, bool adjoint,
                               const void* in, void* out, hipStream_t s, int64_t cut = -1, bool keep_high = false) {
    PassArgs a;
    fill_pass_args(&a, g, rad, wofs, N);
    a.cut = cut;
    a.cut_keep_high = keep_high ? 1 : 0;
    a.in = in;
    a.out = out;
    a.W = W;
    a.adjoint = adjoint ? 1 : 0;
    // one work-group per tile
    const int64_t gmax = (int64_t)0x7fffffff;
    unsigned grid = (unsigned)std::min<int64_t>(g.ntiles, gmax);
    // complex radix-8 tiles of 2048 / 4096 elements: the matrix-core pass
    // with per-lane addresses, two 1024-thread work-groups per compute unit
    // looping over tiles with a register prefetch
    const int fast_ni = cut < 0 ? g.fast_ni : 0;
    std::string nm;
    if (tp && tp->timing.enabled) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "pass %s b=%d%s s0=%d k=%d%s", dt_name(dt), rad[g.s0],
                      g.kind == kKindGeneric ? " generic" : g.kind == kKindMfma ? " mfma"
                                                   : g.kind == kKindCMfma ? " cmfma" : "",
                      g.s0, g.k, adjoint ? " adjoint" : "");
        nm = buf;
    }
    timing_begin(tp, s, nm);
    hipError_t e;
    if (fast_ni) {
        grid = (unsigned)std::min<int64_t>(g.ntiles, 2 * 256);
        e = launch_cpass8_fast(g.k, fast_ni, a, grid, g.lds_bytes, s);
    } else {
        e = launch_pass(to_dt(dt), rad[g.s0], g.kind, a, grid, g.lds_bytes, s);
    }
    if (tp && tp->timing.enabled) timing_end(tp, s, nm, 2.0 * (double)g.elems * (double)storage_size(dt));
    return e == hipSuccess ? GTT_OK : GTT_ERR_HIP;
}

namespace gtt {
gtt_status launch_group_rw(gtt_plan_s* tp, gtt_dtype dt, const Group& g, const std::vector<int>& rad,
                           const std::vector<int64_t>& wofs, int64_t N, const void* W, bool adjoint, const void* in,
                           void* out, hipStream_t s) {
    return launch_group(tp, dt, g, rad, wofs, N, W, adjoint, in, out, s);
}
gtt_status launch_group_inst(gtt_plan_s* tp, gtt_dtype dt, const Group& g, int b, int64_t N, const void* W,
                             bool adjoint, const void* in, void* out, hipStream_t s) {
    std::vector<int> rad(g.s0 + g.k, b);
    std::vector<int64_t> wofs(g.s0 + g.k, 0);
    return launch_group(tp, dt, g, rad, wofs, N, W, adjoint, in, out, s);
}
}  // namespace gtt

// Run a sequence of digit groups over one buffer set: group 0 reads `in`;
// group i < R-1 writes `mid[i]` (or `out` when mid is null); the last writes out.
static gtt_status run_groups(gtt_plan_s* tp, gtt_dtype dt, const std::vector<Group>& groups, const std::vector<int>& rad,
                             const std::vector<int64_t>& wofs, int64_t N, const void* W, bool adjoint,
                             const void* in, void* out, char* saved, size_t elems, hipStream_t s,
                             int64_t cut = -1, bool keep_high = false) {
    const size_t es = storage_size(dt);
    if (groups.empty()) {
        if (in != out)
            if (hipMemcpyAsync(out, in, elems * es, hipMemcpyDeviceToDevice, s) != hipSuccess) return GTT_ERR_HIP;
        return GTT_OK;
    }
    const void* src = in;
    for (size_t i = 0; i < groups.size(); ++i) {
        void* dst = out;
        if (i + 1 < groups.size() && saved) dst = saved + i * (size_t)tp->slot * es;
        gtt_status st = launch_group(tp, dt, groups[i], rad, wofs, N, W, adjoint, src, dst, s, i == 0 ? cut : -1,
                                     keep_high);
        if (st != GTT_OK) return st;
        src = dst;
    }
    return GTT_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* gtt_status_string(gtt_status s) {
    switch (s) {
        case GTT_OK: return "GTT_OK";
        case GTT_ERR_INVALID_VALUE: return "GTT_ERR_INVALID_VALUE";
        case GTT_ERR_SHAPE: return "GTT_ERR_SHAPE";
        case GTT_ERR_DTYPE: return "GTT_ERR_DTYPE";
        case GTT_ERR_ALIGNMENT: return "GTT_ERR_ALIGNMENT";
        case GTT_ERR_WORKSPACE: return "GTT_ERR_WORKSPACE";
        case GTT_ERR_UNSUPPORTED: return "GTT_ERR_UNSUPPORTED";
        case GTT_ERR_HIP: return "GTT_ERR_HIP";
        case GTT_ERR_INTERNAL: return "GTT_ERR_INTERNAL";
        case GTT_ERR_TIMEOUT: return "GTT_ERR_TIMEOUT";
    }
    return "GTT_ERR_UNKNOWN";
}

static bool pow_fits(int64_t b, int64_t n, int64_t* out) {
    int64_t v = 1;
    for (int64_t i = 0; i < n; ++i) {
        if (v > (int64_t)(INT64_MAX / b)) return false;
        v *= b;
    }
    *out = v;
    return true;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// ---------------------------------------------------------------------------
// GTT_FLAG_FP32_INTERMEDIATE (16-bit storage): convert the operands to
// float32 in the workspace, run the float32 plan there (in place), convert
// the results back (round to nearest even).
// ---------------------------------------------------------------------------

static gtt_status f32_apply(gtt_plan_s* p, const void* W, const void* in, void* out, void* saved, void* ws,
                            size_t ws_bytes, bool adjoint, hipStream_t s) {
    size_t fi = 0, bi = 0, si = 0;
    workspace_sizes(p->inner, &fi, &bi, &si);
    const size_t buf = f32_buf_bytes(p);
    if (!ws || ws_bytes < buf + fi) return GTT_ERR_WORKSPACE;
    char* xf = static_cast<char*>(ws);
    const DT dt = to_dt(p->dtype);
    const int64_t E = p->total_elems;
    if (launch_convert(dt, DT::F32, in, xf, E, s) != hipSuccess) return GTT_ERR_HIP;
    gtt_status st = adjoint ? gtt_inverse(p->inner, W, xf, xf, fi ? xf + buf : nullptr, fi, s)
                            : gtt_forward(p->inner, W, xf, xf, saved, fi ? xf + buf : nullptr, fi, s);
    if (st != GTT_OK) return st;
    return launch_convert(DT::F32, dt, xf, out, E, s) == hipSuccess ? GTT_OK : GTT_ERR_HIP;
}

static gtt_status f32_backward(gtt_plan_s* p, const void* W, const void* x, const void* saved, const void* gy,
                               void* gx, void* gW, void* ws, size_t ws_bytes, hipStream_t s) {
    // the inner plan checks the rest of the workspace against its own needs
    const size_t buf = f32_buf_bytes(p);
    if (!ws || ws_bytes < 2 * buf) return GTT_ERR_WORKSPACE;
    char* xf = static_cast<char*>(ws);
    char* gf = xf + buf;
    const DT dt = to_dt(p->dtype);
    const int64_t E = p->total_elems;
    if (launch_convert(dt, DT::F32, x, xf, E, s) != hipSuccess) return GTT_ERR_HIP;
    if (launch_convert(dt, DT::F32, gy, gf, E, s) != hipSuccess) return GTT_ERR_HIP;
    gtt_status st = gtt_backward(p->inner, W, xf, saved, gf, gx ? gf : nullptr, gW, gf + buf,
                                 ws_bytes - 2 * buf, s);
    if (st != GTT_OK || !gx) return st;
    return launch_convert(DT::F32, dt, gf, gx, E, s) == hipSuccess ? GTT_OK : GTT_ERR_HIP;
}

gtt_status gtt_plan(gtt_plan_t* out, int32_t count, const int32_t* b, const int32_t* n, int64_t batch,
                    const int64_t* x_off, const int32_t* w_idx, gtt_dtype dtype, uint32_t flags) {
    if (!out) return GTT_ERR_INVALID_VALUE;
    *out = nullptr;
    if (count < 1 || !b || !n) return GTT_ERR_INVALID_VALUE;
    if (!valid_dtype((int)dtype)) return GTT_ERR_DTYPE;
    if (flags & ~(GTT_FLAG_FP32_INTERMEDIATE | GTT_FLAG_NO_TUNE | GTT_FLAG_PERSISTENT | GTT_FLAG_PER_INSTANCE))
        return GTT_ERR_INVALID_VALUE;
    if ((flags & GTT_FLAG_FP32_INTERMEDIATE) && count != 1) return GTT_ERR_UNSUPPORTED;
    if (batch < 1) return GTT_ERR_SHAPE;
    if (count == 1 && (x_off || w_idx)) return GTT_ERR_INVALID_VALUE;
    if (count > 1 && batch != 1) return GTT_ERR_SHAPE;
    for (int32_t t = 0; t < count; ++t) {
        if (b[t] < 2 || n[t] < 0) return GTT_ERR_SHAPE;
        int64_t N;
        if (!pow_fits(b[t], n[t], &N)) return GTT_ERR_SHAPE;
        if (N > ((int64_t)1 << 40)) return GTT_ERR_SHAPE;
        if (count == 1 && N > INT64_MAX / batch) return GTT_ERR_SHAPE;
    }
    gtt_plan_s* p = new (std::nothrow) gtt_plan_s();
    if (!p) return GTT_ERR_INTERNAL;
    p->dtype = dtype;
    p->flags = flags;
    p->esize = storage_size(dtype);
    p->csize = compute_size(dtype);
    gtt_status st = GTT_OK;
    if (count == 1) {
        p->kind = PlanKind::Uniform;
        p->b = b[0];
        p->n = n[0];
        pow_fits(b[0], n[0], &p->N);
        p->batch = batch;
        p->rad.assign(n[0], b[0]);
        p->wofs.assign(n[0], 0);
        st = plan_groups(p->rad, batch, dtype, flags, true, &p->groups, &p->bwd_groups);
        p->total_elems = p->N * batch;
        p->slot = slot_elems(p->total_elems, p->esize);
        p->w_elems = (int64_t)b[0] * b[0];
        // float32 between digit groups: only the 16-bit storage types keep
        // less (the other dtypes already compute and store in >= 32 bits)
        if (st == GTT_OK && (flags & GTT_FLAG_FP32_INTERMEDIATE) && (dtype == GTT_BF16 || dtype == GTT_F16))
            st = gtt_plan(&p->inner, 1, b, n, batch, nullptr, nullptr, GTT_F32, flags & ~GTT_FLAG_FP32_INTERMEDIATE);
    } else {
        st = plan_ragged(p, count, b, n, x_off, w_idx);
    }
    if (st != GTT_OK) {
        delete p;
        return st;
    }
    *out = p;
    return GTT_OK;
}

gtt_status gtt_plan_mixed(gtt_plan_t* out, int32_t m, const int32_t* radices, int64_t batch, gtt_dtype dtype,
                          uint32_t flags) {
    if (!out) return GTT_ERR_INVALID_VALUE;
    *out = nullptr;
    if (m < 0 || (m > 0 && !radices)) return GTT_ERR_INVALID_VALUE;
    if (!valid_dtype((int)dtype)) return GTT_ERR_DTYPE;
    if (flags & ~(GTT_FLAG_NO_TUNE)) return (flags & GTT_FLAG_FP32_INTERMEDIATE) ? GTT_ERR_UNSUPPORTED
                                                                                 : GTT_ERR_INVALID_VALUE;
    if (batch < 1) return GTT_ERR_SHAPE;
    int64_t N = 1;
    for (int k = 0; k < m; ++k) {
        if (radices[k] < 2 || radices[k] > 64) return radices[k] < 2 ? GTT_ERR_SHAPE : GTT_ERR_UNSUPPORTED;
        if (N > ((int64_t)1 << 40) / radices[k]) return GTT_ERR_SHAPE;
        N *= radices[k];
    }
    if (N > INT64_MAX / batch) return GTT_ERR_SHAPE;
    gtt_plan_s* p = new (std::nothrow) gtt_plan_s();
    if (!p) return GTT_ERR_INTERNAL;
    p->kind = PlanKind::Mixed;
    p->dtype = dtype;
    p->flags = flags;
    p->esize = storage_size(dtype);
    p->csize = compute_size(dtype);
    p->N = N;
    p->batch = batch;
    p->n = m;
    p->total_elems = N * batch;
    p->slot = slot_elems(p->total_elems, p->esize);
    // digit d (least significant first) is factor m-1-d
    p->rad.resize(m);
    p->wofs.resize(m);
    std::vector<int64_t> fofs(m);
    int64_t acc = 0;
    for (int k = 0; k < m; ++k) {
        fofs[k] = acc;
        acc += (int64_t)radices[k] * radices[k];
    }
    p->w_elems = acc;
    for (int d = 0; d < m; ++d) {
        p->rad[d] = radices[m - 1 - d];
        p->wofs[d] = fofs[m - 1 - d];
    }
    gtt_status st = plan_groups(p->rad, batch, dtype, flags, false, &p->groups, &p->bwd_groups);
    if (st != GTT_OK) {
        delete p;
        return st;
    }
    *out = p;
    return GTT_OK;
}

gtt_status gtt_plan_destroy(gtt_plan_t p) {
    if (!p) return GTT_OK;
    if (p->inner) gtt_plan_destroy(p->inner);
    destroy_ragged(p);
    delete p;
    return GTT_OK;
}

gtt_status gtt_plan_check(gtt_plan_t p, void* stream) {
    if (!p) return GTT_ERR_INVALID_VALUE;
    if (p->kind != PlanKind::Ragged) return GTT_OK;
    return ragged_check(p, static_cast<hipStream_t>(stream));
}

gtt_status gtt_plan_barrier_limit(gtt_plan_t p, uint32_t polls) {
    if (!p || p->kind != PlanKind::Ragged) return GTT_ERR_INVALID_VALUE;
    return ragged_set_spin_limit(p, polls);
}

gtt_status gtt_workspace_size(gtt_plan_t p, size_t* fwd, size_t* bwd, size_t* saved) {
    if (!p) return GTT_ERR_INVALID_VALUE;
    size_t f = 0, bw = 0, sv = 0;
    if (p->inner) {
        // float32 copies of the operands ahead of the inner plan's workspace
        workspace_sizes(p->inner, &f, &bw, &sv);
        const size_t buf = f32_buf_bytes(p);
        f += buf;
        bw += 2 * buf;
    } else {
        workspace_sizes(p, &f, &bw, &sv);
    }
    if (fwd) *fwd = f;
    if (bwd) *bwd = bw;
    if (saved) *saved = sv;
    return GTT_OK;
}

gtt_status gtt_forward(gtt_plan_t p, const void* W, const void* x, void* y, void* saved, void* ws,
                       size_t ws_bytes, void* stream) {
    if (!p || !W || !x || !y) return GTT_ERR_INVALID_VALUE;
    if (!aligned16(x) || !aligned16(y) || !aligned16(W) || (saved && !aligned16(saved)) ||
        (ws && !aligned16(ws)))
        return GTT_ERR_ALIGNMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->inner) return f32_apply(p, W, x, y, saved, ws, ws_bytes, false, s);
    if (p->kind == PlanKind::Ragged) return ragged_apply(p, W, x, y, false, (char*)saved, s);
    return run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, false, x, y, (char*)saved,
                      (size_t)p->total_elems, s);
}

gtt_status gtt_inverse(gtt_plan_t p, const void* W, const void* y, void* x, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!p || !W || !x || !y) return GTT_ERR_INVALID_VALUE;
    if (!aligned16(x) || !aligned16(y) || !aligned16(W) || (ws && !aligned16(ws))) return GTT_ERR_ALIGNMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->inner) return f32_apply(p, W, y, x, nullptr, ws, ws_bytes, true, s);
    if (p->kind == PlanKind::Ragged) return ragged_apply(p, W, y, x, true, nullptr, s);
    // the adjoint applies W^H per digit; digit passes commute, so the group
    // order of the forward plan is reused as is
    return run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, true, y, x, nullptr,
                      (size_t)p->total_elems, s);
}

gtt_status gtt_plan_describe(gtt_plan_t p, char* buf, size_t len) {
    if (!p || !buf || len == 0) return GTT_ERR_INVALID_VALUE;
    std::string s = describe_plan(p);
    std::snprintf(buf, len, "%s", s.c_str());
    return GTT_OK;
}

gtt_status gtt_plan_timing(gtt_plan_t p, int32_t enable) {
    if (!p) return GTT_ERR_INVALID_VALUE;
    p->timing.enabled = enable != 0;
    if (p->inner) p->inner->timing.enabled = enable != 0;
    return GTT_OK;
}

gtt_status gtt_plan_timing_filter(gtt_plan_t p, const char* prefix) {
    if (!p) return GTT_ERR_INVALID_VALUE;
    p->timing.filter = prefix ? prefix : "";
    if (p->inner) p->inner->timing.filter = p->timing.filter;
    return GTT_OK;
}

gtt_status gtt_plan_timing_read(gtt_plan_t p, char* buf, size_t len) {
    if (!p || !buf || len == 0) return GTT_ERR_INVALID_VALUE;
    std::string s = timing_read(p);
    if (p->inner) {
        // one JSON object: the conversions, then the float32 launches
        const std::string in = timing_read(p->inner);
        if (in.size() > 2) s = (s.size() > 2 ? s.substr(0, s.size() - 1) + "," : std::string("{")) + in.substr(1);
    }
    std::snprintf(buf, len, "%s", s.c_str());
    return GTT_OK;
}

gtt_status gtt_set_tuning(int32_t b, int32_t n, gtt_dtype dtype, int32_t lds_budget_bytes, int32_t min_row_bytes,
                          int32_t max_group_digits, int32_t bwd_lds_bytes) {
    if (b < 2 || n < 0 || !valid_dtype((int)dtype)) return GTT_ERR_INVALID_VALUE;
    if (lds_budget_bytes < 0 || lds_budget_bytes > 160 * 1024 || min_row_bytes < 0 || max_group_digits < 0 ||
        bwd_lds_bytes < 0 || bwd_lds_bytes > 160 * 1024)
        return GTT_ERR_INVALID_VALUE;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    // all zeros: remove the entry (so that it no longer shadows the radix-wide one)
    const bool clear = !lds_budget_bytes && !min_row_bytes && !max_group_digits && !bwd_lds_bytes;
    for (size_t i = 0; i < g_tune.size(); ++i) {
        TuneEntry& e = g_tune[i];
        if (e.b == b && e.n == n && e.dtype == (int)dtype) {
            if (clear) {
                g_tune.erase(g_tune.begin() + (long)i);
                return GTT_OK;
            }
            e.lds_budget = lds_budget_bytes;
            e.min_row_bytes = min_row_bytes;
            e.max_group_digits = max_group_digits;
            e.bwd_lds = bwd_lds_bytes;
            return GTT_OK;
        }
    }
    if (clear) return GTT_OK;
    g_tune.push_back(
        TuneEntry{b, n, (int)dtype, lds_budget_bytes, min_row_bytes, max_group_digits, bwd_lds_bytes});
    return GTT_OK;
}

gtt_status gtt_selftest(void) {
    // fast division by invariant integers: exhaustive over a range of n for
    // every divisor used by the planner (place values up to 2^24 and radices)
    std::vector<uint32_t> ds;
    for (uint32_t d = 1; d <= 64; ++d) ds.push_back(d);
    for (uint32_t b = 2; b <= 8; ++b)
        for (uint64_t v = b; v < (1u << 24); v *= b) ds.push_back((uint32_t)v);
    for (uint32_t d : ds) {
        FastDiv f = make_fastdiv(d);
        for (uint32_t n = 0; n < 70000; ++n)
            if (host_fdiv(n, f) != n / d) return GTT_ERR_INTERNAL;
        for (uint32_t n = 0x7fffffffu; n > 0x7fffffffu - 70000u; --n)
            if (host_fdiv(n, f) != n / d) return GTT_ERR_INTERNAL;
        for (uint64_t n = 1; n < 0x80000000ull; n = n * 3 + 1)
            if (host_fdiv((uint32_t)n, f) != (uint32_t)n / d) return GTT_ERR_INTERNAL;
    }
    // planner invariants: groups cover the digits exactly, tiles fit and
    // partition the buffer
    const gtt_dtype dts[] = {GTT_F64, GTT_F32, GTT_C128, GTT_C64, GTT_BF16, GTT_F16, GTT_I32};
    for (gtt_dtype dt : dts)
        for (int b = 2; b <= 33; ++b)
            for (int n = 1; n <= 20; ++n) {
                int64_t N;
                if (!pow_fits(b, n, &N) || N > (1 << 22)) break;
                std::vector<int> rad(n, b);
                std::vector<Group> gs;
                std::vector<Group> bgs;
                if (plan_groups(rad, 3, dt, GTT_FLAG_NO_TUNE, true, &gs, &bgs) != GTT_OK) return GTT_ERR_INTERNAL;
                if (bgs.size() != gs.size()) return GTT_ERR_INTERNAL;
                for (size_t i = 0; i < gs.size(); ++i)
                    if (bgs[i].s0 != gs[i].s0 || bgs[i].k != gs[i].k ||
                        (bgs[i].bwd_ok && bwd_lds_bytes(bgs[i], dt) > 160 * 1024) || (b <= 32 && !bgs[i].bwd_ok))
                        return GTT_ERR_INTERNAL;
                int s = 0;
                for (const Group& g : gs) {
                    if (g.s0 != s || g.k < 1) return GTT_ERR_INTERNAL;
                    s += g.k;
                    if (g.lds_bytes > 160 * 1024) return GTT_ERR_INTERNAL;
                    if ((int64_t)g.P * g.G * g.C != g.tileE) return GTT_ERR_INTERNAL;
                    // tiles x tile elements cover the buffer (column blocks may overhang)
                    if (g.ntiles * g.tileE < N * 3) return GTT_ERR_INTERNAL;
                    if (g.C > g.S && g.S != 1) return GTT_ERR_INTERNAL;
                    if (g.S == 1 && g.C != 1) return GTT_ERR_INTERNAL;
                }
                if (s != n) return GTT_ERR_INTERNAL;
            }
    return GTT_OK;
}

}  // extern "C"

extern "C" {

gtt_status gtt_backward(gtt_plan_t p, const void* W, const void* x, const void* saved, const void* gy, void* gx,
                        void* gW, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !W || !x || !gy || (!gx && !gW)) return GTT_ERR_INVALID_VALUE;
    if (!aligned16(W) || !aligned16(x) || !aligned16(gy) || (gx && !aligned16(gx)) || (gW && !aligned16(gW)) ||
        (saved && !aligned16(saved)) || (ws && !aligned16(ws)))
        return GTT_ERR_ALIGNMENT;
    if (p->dtype == GTT_I32) return GTT_ERR_UNSUPPORTED;
    if (p->inner) return f32_backward(p, W, x, saved, gy, gx, gW, ws, ws_bytes, static_cast<hipStream_t>(stream));
    return backward_impl(p, W, x, saved, gy, gx, gW, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

gtt_status gtt_filter(gtt_plan_t p, const void* W, const void* x, int64_t cutoff, void* low, void* high, void* ws,
                      size_t ws_bytes, void* stream) {
    if (!p || !W || !x || (!low && !high)) return GTT_ERR_INVALID_VALUE;
    if (!aligned16(W) || !aligned16(x) || (low && !aligned16(low)) || (high && !aligned16(high)) ||
        (ws && !aligned16(ws)))
        return GTT_ERR_ALIGNMENT;
    if (p->kind != PlanKind::Uniform || p->dtype == GTT_I32 || p->inner) return GTT_ERR_UNSUPPORTED;
    if (cutoff < 0) return GTT_ERR_INVALID_VALUE;
    return filter_impl(p, W, x, cutoff, low, high, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace gtt {
// Natural-order filter (§4.3, Alg. 3 classical analogue): coefficients into
// the workspace, then two inverse transforms whose first digit group masks
// the coefficients by natural index as it loads them.
gtt_status filter_impl(gtt_plan_s* p, const void* W, const void* x, int64_t cutoff, void* low, void* high, void* ws,
                       size_t ws_bytes, hipStream_t s) {
    const size_t E = (size_t)p->total_elems;
    size_t f = 0, bw = 0, sv = 0;
    workspace_sizes(p, &f, &bw, &sv);
    if (ws_bytes < f + E * p->esize || !ws) return GTT_ERR_WORKSPACE;
    if (p->groups.empty()) return GTT_ERR_UNSUPPORTED;  // n == 0: nothing to filter
    char* coef = static_cast<char*>(ws) + f;
    const int64_t cut = std::min<int64_t>(cutoff, p->N);
    gtt_status st = run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, false, x, coef, nullptr, E, s);
    if (st != GTT_OK) return st;
    if (low) {
        st = run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, true, coef, low, nullptr, E, s, cut, false);
        if (st != GTT_OK) return st;
    }
    if (high) {
        st = run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, true, coef, high, nullptr, E, s, cut, true);
        if (st != GTT_OK) return st;
    }
    return GTT_OK;
}
}  // namespace gtt

extern "C" gtt_status gtt_compress_workspace_size(gtt_plan_t p, size_t* bytes) {
    if (!p || !bytes) return GTT_ERR_INVALID_VALUE;
    if (p->kind != PlanKind::Uniform || p->inner) return GTT_ERR_UNSUPPORTED;
    size_t f = 0, bw = 0, sv = 0;
    workspace_sizes(p, &f, &bw, &sv);
    const size_t E = (size_t)p->total_elems;
    *bytes = f + ((E * p->esize + 255) & ~(size_t)255) + topk_meta_bytes(p->N, p->batch);
    return GTT_OK;
}

extern "C" gtt_status gtt_compress(gtt_plan_t p, const void* W, const void* x, int64_t k, int64_t* idx, void* val,
                                   void* recon, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !W || !x || !idx || !val) return GTT_ERR_INVALID_VALUE;
    if (!aligned16(W) || !aligned16(x) || !aligned16(idx) || !aligned16(val) || (recon && !aligned16(recon)) ||
        (ws && !aligned16(ws)))
        return GTT_ERR_ALIGNMENT;
    if (p->kind != PlanKind::Uniform || p->inner) return GTT_ERR_UNSUPPORTED;
    if (k < 1 || k > p->N) return GTT_ERR_INVALID_VALUE;
    size_t need = 0;
    gtt_compress_workspace_size(p, &need);
    if (!ws || ws_bytes < need) return GTT_ERR_WORKSPACE;
    size_t f = 0, bw = 0, sv = 0;
    workspace_sizes(p, &f, &bw, &sv);
    const size_t E = (size_t)p->total_elems;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* coef = static_cast<char*>(ws) + f;
    char* meta = coef + ((E * p->esize + 255) & ~(size_t)255);
    gtt_status st = run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, false, x, coef, nullptr, E, s);
    if (st != GTT_OK) return st;
    const std::string tnm = std::string("topk ") + dt_name(p->dtype);
    timing_begin(p, s, tnm);
    if (launch_topk(to_dt(p->dtype), coef, p->N, p->batch, k, idx, val, recon, meta, s) != hipSuccess)
        return GTT_ERR_HIP;
    timing_end(p, s, tnm, (double)E * (double)p->esize * 5.0);
    if (recon)
        return run_groups(p, p->dtype, p->groups, p->rad, p->wofs, p->N, W, true, recon, recon, nullptr, E, s);
    return GTT_OK;
}
