// LDS layout of the radix-8 matrix-core kernels with per-lane addresses:
// padding shifts and, per digit, the fibre-to-lane map, chosen so that the
// kernels' LDS accesses avoid bank conflicts.
//
// Bank model (measured on gfx950 with ds_read_b32/b64/b128 patterns):
// 64-bit accesses are served 32 lanes per cycle over 64 four-byte banks, so
// the 32 complex64 elements of a half-wave conflict exactly when two
// distinct elements agree modulo 32; 32-bit accesses are served 32 lanes
// per cycle over 32 banks; equal addresses are broadcast.
//
// Tile positions are bit strings (logC column bits, three bits per digit,
// row bits); the padding phys(x) = x + sum_p (x >> p) is additive over
// disjoint bits, which is what lets the kernels split addresses into lane
// and loop parts.  Per digit j the low eight bits of a fibre index carry
// the lane and wave: the four bits in mask_j take the lane's 16-value index,
// the other four the wave.  In the gradient sums, lane group k (0..3) sets
// fibre bits kb0_j (k & 1) and kb1_j (k >> 1); the remaining two mask bits
// are the loop over the four MFMAs of a block.
//
// Paired phases (backward, four digits, 4096-element contiguous tiles): two
// consecutive phases on digits x and y need no work-group barrier when every
// wave owns the same positions in both, i.e. when the four tile-position
// bits that carry the wave index lie outside digits x and y and are the same
// set for both digits' maps; a wave then reads back only what it wrote
// itself.  The adjoint phases of digits 1 and 0 are paired this way (wave
// bits in digits 2 and 3), and so are the recomputing forward passes of
// digits 1 and 2 (wave bits in digits 0 and 3), which get pass-only maps of
// their own (PassArgs::pmap).  (Pairing the phases of digits 3 and 2 too,
// wave bits in digits 0 and 1, leaves no conflict-free maps for digits 0
// and 3 and measured slower.)
#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gtt_plan.hpp"

namespace gtt {

namespace {

struct Pads {
    int p[3];
    int n;
    uint32_t phys(uint32_t x) const {
        uint32_t r = x;
        for (int i = 0; i < n; ++i) r += x >> p[i];
        return r;
    }
    int packed() const {
        int q[3] = {31, 31, 31};
        for (int i = 0; i < n; ++i) q[i] = p[i];
        return q[0] | (q[1] << 8) | (q[2] << 16);
    }
};

uint32_t dep3(uint32_t v, uint32_t h) { return ((v >> h) << (h + 3)) | (v & ((1u << h) - 1u)); }

uint32_t pdep8(uint32_t v, uint32_t mask) {
    uint32_t r = 0;
    for (int b = 0; b < 8; ++b)
        if (mask >> b & 1u) {
            r |= (v & 1u) << b;
            v >>= 1;
        }
    return r;
}

// largest number of distinct elements sharing a residue modulo `mod`
int conflict(const uint32_t* e, int n, uint32_t mod = 32) {
    int worst = 0;
    for (int i = 0; i < n; ++i) {
        bool dup = false;
        for (int k = 0; k < i; ++k) dup |= e[k] == e[i];
        if (dup) continue;
        int c = 0;
        for (int k = 0; k <= i; ++k) {
            bool first = true;
            for (int m = 0; m < k; ++m) first &= e[m] != e[k];
            if (first && (e[k] & (mod - 1u)) == (e[i] & (mod - 1u))) ++c;
        }
        if (c > worst) worst = c;
    }
    return worst;
}

// passes: half-waves (q in {0,1} or {2,3}) of the loads at elements 2q and
// 2q+1 of the 16 fibres of a block
int stage_cost(const Pads& pd, uint32_t h, uint32_t mask) {
    int tot = 0;
    for (int qh = 0; qh < 2; ++qh)
        for (int which = 0; which < 2; ++which) {
            uint32_t e[32];
            int n = 0;
            for (int q = 2 * qh; q < 2 * qh + 2; ++q)
                for (uint32_t x = 0; x < 16; ++x)
                    e[n++] = pd.phys(dep3(pdep8(x, mask), h) | ((uint32_t)(2 * q + which) << h));
            tot += conflict(e, n) - 1;
        }
    return tot;
}

// gradient sums: per MFMA, lane groups k = 0, 1 (and 2, 3) read one
// 32-bit component of the 8 elements of fibres with bits kb0, kb1 set from k;
// 32-bit accesses are served 32 lanes per cycle over 32 banks, so the 16
// elements of a half-wave must differ modulo 16
int gw_cost(const Pads& pd, uint32_t h, uint32_t mask, int kb0, int kb1) {
    int ob[2], no = 0;
    for (int b = 0; b < 8; ++b)
        if ((mask >> b & 1u) && b != kb0 && b != kb1) ob[no++] = b;
    int tot = 0;
    for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t base = ((u & 1u) << ob[0]) | ((u >> 1) << ob[1]);
        for (uint32_t kh = 0; kh < 2; ++kh) {
            uint32_t e[16];
            int n = 0;
            for (uint32_t kl = 0; kl < 2; ++kl) {
                const uint32_t f = base | (kl << kb0) | (kh << kb1);
                for (uint32_t el = 0; el < 8; ++el) e[n++] = pd.phys(dep3(f, h) | (el << h));
            }
            tot += conflict(e, n, 16) - 1;
        }
    }
    return tot;
}

// tile load / store: a half-wave holds 64 consecutive elements, two per
// lane, and accesses the even ones, then the odd ones
int io_cost(const Pads& pd, uint32_t tileE) {
    int tot = 0;
    for (uint32_t s = 0; s < tileE; s += 64)
        for (uint32_t odd = 0; odd < 2; ++odd) {
            uint32_t e[32];
            for (uint32_t l = 0; l < 32; ++l) e[l] = pd.phys(s + 2 * l + odd);
            tot += conflict(e, 32) - 1;
        }
    return tot;
}

struct Best {
    int cost = 1 << 30;
    FastMap m;
};

// fibre-index mask (8 bits) of digit j whose wave bits are the tile-position
// bits in S (logC = 0: fibre bit b is position bit b below digit j, b + 3
// above it); 0 when some bit of S is not a fibre bit below 8
uint32_t mask_for_wave_bits(uint32_t S, int j) {
    uint32_t wave = 0;
    for (int b = 0; b < 8; ++b) {
        const int p = b < 3 * j ? b : b + 3;
        if (S >> p & 1u) wave |= 1u << b;
    }
    if (__builtin_popcount(wave) != 4 || (uint32_t)__builtin_popcount(S) != 4u) return 0;
    return ~wave & 0xffu;
}

// least conflict cost of a fused (pass + gradient) map of digit j with the
// given mask, and its code (mask | kb0 << 8 | kb1 << 11)
int fused_cost(const Pads& pd, int j, uint32_t mask, uint64_t* code) {
    const uint32_t h = 3u * (uint32_t)j;
    const int sc = stage_cost(pd, h, mask);
    int best = 1 << 30;
    for (int kb0 = 0; kb0 < 8 && best > 0; ++kb0)
        for (int kb1 = 0; kb1 < 8 && best > 0; ++kb1) {
            if (kb0 == kb1 || !(mask >> kb0 & 1u) || !(mask >> kb1 & 1u)) continue;
            const int c = sc + gw_cost(pd, h, mask, kb0, kb1);
            if (c < best) {
                best = c;
                *code = mask | ((uint64_t)kb0 << 8) | ((uint64_t)kb1 << 11);
            }
        }
    return best;
}

// the paired layout of the four-digit backward on 4096-element tiles
FastMap search_paired() {
    const uint32_t tileE = 4096u;
    Best best;
    for (int n = 0; n <= 3; ++n) {
        int p[3];
        for (p[0] = 4; p[0] <= 12; ++p[0])
            for (p[1] = (n > 1 ? p[0] + 1 : 13); p[1] <= (n > 1 ? 12 : 13); ++p[1])
                for (p[2] = (n > 2 ? p[1] + 1 : 13); p[2] <= (n > 2 ? 12 : 13); ++p[2]) {
                    Pads pd{{p[0], p[1], p[2]}, n};
                    if (n == 0 && p[0] != 4) continue;
                    uint32_t extra = 0;
                    for (int i = 0; i < n; ++i) extra += tileE >> pd.p[i];
                    if (extra > tileE / 8) continue;  // LDS budget of the four backward tiles
                    int total = io_cost(pd, tileE);
                    if (total >= best.cost) continue;
                    FastMap m;
                    m.pad = pd.packed();
                    // digits 0 and 1 (adjoint pair): wave bits among positions 6..10
                    int bc = 1 << 30;
                    uint64_t c01 = 0;
                    for (uint32_t S = 0; S < 4096u; ++S) {
                        if ((S & ~0x7c0u) || __builtin_popcount(S) != 4) continue;
                        uint64_t k0 = 0, k1 = 0;
                        const int c = fused_cost(pd, 0, mask_for_wave_bits(S, 0), &k0) +
                                      fused_cost(pd, 1, mask_for_wave_bits(S, 1), &k1);
                        if (c < bc) {
                            bc = c;
                            c01 = k0 | (k1 << 16);
                        }
                    }
                    total += bc;
                    // digits 2 and 3: free
                    uint64_t c23 = 0;
                    for (int j = 2; j < 4; ++j) {
                        int bj = 1 << 30;
                        uint64_t cj = 0;
                        for (uint32_t mask = 0; mask < 256 && bj > 0; ++mask) {
                            if (__builtin_popcount(mask) != 4) continue;
                            uint64_t k = 0;
                            const int c = fused_cost(pd, j, mask, &k);
                            if (c < bj) {
                                bj = c;
                                cj = k;
                            }
                        }
                        total += bj;
                        c23 |= cj << (16 * (j - 2));
                    }
                    // pass maps of digits 1 and 2 (recompute pair): wave bits
                    // among positions 0..2, 9, 10
                    int bp = 1 << 30;
                    uint32_t pm = 0;
                    for (uint32_t S = 0; S < 4096u; ++S) {
                        if ((S & ~0x607u) || __builtin_popcount(S) != 4) continue;
                        const uint32_t m1 = mask_for_wave_bits(S, 1), m2 = mask_for_wave_bits(S, 2);
                        const int c = stage_cost(pd, 3u, m1) + stage_cost(pd, 6u, m2);
                        if (c < bp) {
                            bp = c;
                            pm = m1 | (m2 << 8);
                        }
                    }
                    total += bp;
                    m.map = c01 | (c23 << 32);
                    m.pmap = pm;
                    if (total < best.cost) {
                        best.cost = total;
                        best.m = m;
                    }
                }
    }
    best.m.conflicts = best.cost;
    return best.m;
}

FastMap search(int K, int NI, int logC, bool gw) {
    if (gw && K == 4 && NI == 2 && logC == 0) return search_paired();
    const uint32_t tileE = 2048u * (uint32_t)NI;
    // candidate paddings, fewest extra elements first
    std::vector<std::pair<uint32_t, Pads>> cands;
    for (int n = 0; n <= 3; ++n) {
        int p[3];
        for (p[0] = 4; p[0] <= 12; ++p[0])
            for (p[1] = (n > 1 ? p[0] + 1 : 13); p[1] <= (n > 1 ? 12 : 13); ++p[1])
                for (p[2] = (n > 2 ? p[1] + 1 : 13); p[2] <= (n > 2 ? 12 : 13); ++p[2]) {
                    Pads pd{{p[0], p[1], p[2]}, n};
                    if (n == 0 && p[0] != 4) continue;
                    uint32_t extra = 0;
                    for (int i = 0; i < n; ++i) extra += tileE >> pd.p[i];
                    if (extra > tileE / 8) continue;  // LDS budget of the four backward tiles
                    cands.push_back({extra, pd});
                }
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const std::pair<uint32_t, Pads>& a, const std::pair<uint32_t, Pads>& b) {
                         return a.first < b.first;
                     });
    Best best;
    for (const auto& c : cands) {
        const Pads& pd = c.second;
        int total = io_cost(pd, tileE);
        FastMap m;
        m.pad = pd.packed();
        m.map = 0;
        for (int j = 0; j < K && total < best.cost; ++j) {
            const uint32_t h = (uint32_t)logC + 3u * (uint32_t)j;
            int bj = 1 << 30;
            uint64_t code = 0;
            for (uint32_t mask = 0; mask < 256 && bj > 0; ++mask) {
                if (__builtin_popcount(mask) != 4) continue;
                const int sc = stage_cost(pd, h, mask);
                if (sc >= bj) continue;
                if (!gw) {
                    bj = sc;
                    code = mask;
                    continue;
                }
                for (int kb0 = 0; kb0 < 8 && bj > 0; ++kb0)
                    for (int kb1 = 0; kb1 < 8 && bj > 0; ++kb1) {
                        if (kb0 == kb1 || !(mask >> kb0 & 1u) || !(mask >> kb1 & 1u)) continue;
                        const int cst = sc + gw_cost(pd, h, mask, kb0, kb1);
                        if (cst < bj) {
                            bj = cst;
                            code = mask | ((uint64_t)kb0 << 8) | ((uint64_t)kb1 << 11);
                        }
                    }
            }
            total += bj;
            m.map |= code << (16 * j);
        }
        if (total < best.cost) {
            best.cost = total;
            best.m = m;
            if (total == 0) break;
        }
    }
    best.m.conflicts = best.cost;
    return best.m;
}

}  // namespace

// ---------------------------------------------------------------------------
// LDS padding of the matrix-core passes (radix 16 / 32).  FP32 tile (f32
// storage): element x at word lds_phys(x); 16-bit tile (bf16 / f16): element
// x in word lds_phys(x >> 1), the pads counting words.  The tile transfers
// move a 16-byte vector per thread as 32-bit accesses, so the lanes of one
// access sit four words apart; a digit pass reads and writes element
// 16 h + 4 q + v of the fibre of lane (q, i), 16 fibres by four q: four
// 32-bit accesses (FP32), two word accesses (16-bit, contiguous digit) or
// four 16-bit accesses (16-bit, strided digit; two lanes in one word do not
// conflict).  Each access costs its half-waves' worst bank degree (32
// banks); the search takes the pad triple (each level one element or word)
// with the least total cost over a sample of the tile, LDS growth at most
// 1/8.
// ---------------------------------------------------------------------------
namespace {

int conflict32(const uint32_t* e) {
    uint32_t v[32];
    for (int i = 0; i < 32; ++i) v[i] = e[i];
    std::sort(v, v + 32);
    int cnt[32] = {0};
    int worst = 0;
    for (int i = 0; i < 32; ++i) {
        if (i && v[i] == v[i - 1]) continue;  // equal addresses broadcast
        const int c = ++cnt[v[i] & 31u];
        if (c > worst) worst = c;
    }
    return worst;
}

int mfma_cost(const Pads& pd, int B, int k, int logC, uint32_t tileE, uint32_t vec, bool lds16) {
    int tot = 0;
    uint32_t e[32];
    const uint32_t nvec = tileE / vec;
    const uint32_t nw = lds16 ? vec / 2 : vec;  // words per vector
    for (uint32_t w0 = 0; w0 + 64 <= nvec; w0 += 256)
        for (uint32_t el = 0; el < nw; ++el)
            for (uint32_t half = 0; half < 2; ++half) {
                for (uint32_t l = 0; l < 32; ++l) e[l] = pd.phys(nw * (w0 + 32u * half + l) + el);
                tot += 2 * conflict32(e);  // load and store
            }
    const uint32_t F = tileE / (uint32_t)B;
    const uint32_t Cm = (1u << logC) - 1u;
    uint32_t bj = 1;
    for (int j = 0; j < k; ++j, bj *= (uint32_t)B) {
        const uint32_t bj1 = bj * (uint32_t)B, step = bj << logC;
        const bool pairs = lds16 && step == 1;
        for (uint32_t grp = 0; grp < (F + 15) / 16; grp += 4)
            for (int h = 0; h < B / 16; ++h)
                for (uint32_t v = 0; v < 4; v += pairs ? 2 : 1)
                    for (uint32_t half = 0; half < 2; ++half) {
                        for (uint32_t l = 0; l < 32; ++l) {
                            const uint32_t lane = 32u * half + l, q = lane >> 4, lo = lane & 15u;
                            const uint32_t f = (grp * 16u + lo) % F;
                            const uint32_t c = f & Cm, f1 = f >> logC;
                            const uint32_t Q = f1 / bj, glo = f1 % bj;
                            const uint32_t lam0 = ((Q * bj1 + glo) << logC) | c;
                            const uint32_t x = lam0 + (16u * h + 4u * q + v) * step;
                            e[l] = lds16 ? pd.phys(x >> 1) : pd.phys(x);
                        }
                        tot += 2 * conflict32(e);
                    }
    }
    return tot;
}

int mfma_search(int B, int k, int logC, uint32_t tileE, int min_shift, uint32_t vec, bool lds16) {
    Pads best{{31, 31, 31}, 0};
    const uint32_t units = lds16 ? (tileE + 1) / 2 : tileE;  // padded elements or words
    int best_cost = mfma_cost(best, B, k, logC, tileE, vec, lds16);
    uint32_t best_extra = 0;
    std::vector<int> sh;
    for (int p = min_shift; p <= 13; ++p) sh.push_back(p);
    for (size_t a = 0; a < sh.size(); ++a)
        for (size_t b = a; b <= sh.size(); ++b)
            for (size_t c = b; c <= sh.size(); ++c) {
                Pads pd{{sh[a], b < sh.size() ? sh[b] : 31, c < sh.size() ? sh[c] : 31}, 0};
                pd.n = 1 + (b < sh.size()) + (c < sh.size());
                if (b == sh.size() && c < sh.size()) continue;
                const uint32_t extra = pd.phys(units) - units;
                if (extra > units / 8) continue;
                const int cst = mfma_cost(pd, B, k, logC, tileE, vec, lds16);
                if (cst < best_cost || (cst == best_cost && extra < best_extra)) {
                    best = pd;
                    best_cost = cst;
                    best_extra = extra;
                }
            }
    return best.packed();
}

}  // namespace

int mfma_pad(int B, int k, int logC, int64_t tileE, int min_shift, int vec, bool lds16) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int64_t, int, int, bool>, int> cache;
    const auto key = std::make_tuple(B, k, logC, tileE, min_shift, vec, lds16);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int pad = mfma_search(B, k, logC, (uint32_t)tileE, min_shift, (uint32_t)vec, lds16);
    cache[key] = pad;
    return pad;
}

FastMap fast_map(int K, int NI, int logC, bool gw) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, bool>, FastMap> cache;
    const auto key = std::make_tuple(K, NI, logC, gw);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const FastMap m = search(K, NI, logC, gw);
    cache[key] = m;
    return m;
}

}  // namespace gtt
