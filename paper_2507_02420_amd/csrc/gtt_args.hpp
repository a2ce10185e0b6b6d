// Launch descriptors shared by the host planner and the device kernels.
//
// A "digit group" is a run of k consecutive base-b digits s0 .. s0+k-1 of the
// element index.  Seen through one group, an instance is a 3-D array
//     [hi][g][lo],   g < G = b^k (the group's digits),  lo < S = b^s0,
// and the group pass applies W along each of the k digits of g (the fast
// algorithm of §3 performs one such digit per recursion level; a group pass
// performs k of them on a tile held on chip).  A tile is
//     P consecutive hi blocks x G group positions x C consecutive lo columns.
#pragma once

#include <stdint.h>

namespace gtt {

constexpr int kMaxDigits = 32;
constexpr int kThreads = 256;  // work-group size of every pass kernel
// first-stage vectors of the gW reduction (room for them follows the
// partial vectors in the workspace)
constexpr int kReduceBlocks = 64;
// general backward: schedule operations and LDS tiles of a work-group
constexpr int kMaxBwdOps = 192;
constexpr int kMaxBwdSlots = 16;

// q = floor(n / d) for 0 <= n < 2^31 via one multiply-high (Granlund and
// Montgomery's division by invariant integers): m = floor(2^32 (2^s - d) / d) + 1,
// s = ceil(log2 d); q = (umulhi(n, m) + n) >> s.
struct FastDiv {
    uint32_t d, m, s;
};

enum LoadMode : int32_t {
    kContigVec = 0,   // the tile is one contiguous run; 16-byte vector accesses
    kContigScalar = 1,// the tile is one contiguous run; element accesses
    kRowVec = 2,      // P*G rows of C contiguous elements; 16-byte accesses
    kRowScalar = 3,   // rows of C elements, last column block may be partial
};

struct PassArgs {
    const void* in;
    void* out;
    const void* W;      // b x b base matrix, compute dtype, row-major
    int32_t adjoint;    // 1: apply W^H (conjugate transpose) instead of W
    int32_t k;          // digits in this group
    int32_t G;          // b^k
    int32_t P;          // hi blocks per tile
    int32_t logC;       // C = 2^logC columns per tile
    int32_t mode;       // LoadMode
    int32_t pad_shift;  // LDS: one pad element after every 2^pad_shift elements
    int32_t cut_keep_high;  // with cut >= 0: keep natural indices >= cut instead of < cut
    int64_t cut;        // >= 0: zero the loaded elements by natural index (filter)
    int64_t S;          // place value of the group's lowest digit, b^s0
    int64_t L;          // column blocks per hi block, ceil(S / C)
    int64_t ntiles;     // tiles in this launch
    int64_t N;          // elements per instance (masking by natural index)
    FastDiv divG;       // division by G (row -> hi block within the tile)
    FastDiv divL;       // division by L (tile -> hi block), valid when L < 2^31
    FastDiv divb[kMaxDigits + 1];  // division by b^j, j = 0..k
    int32_t bpow[kMaxDigits + 1];  // b^j, j = 0..k (fits: G <= 2^24); for a
                                   // mixed-radix group, the place value of
                                   // group digit j inside g
    // mixed-radix / generic-radix groups only (the runtime-radix kernel):
    int32_t rad[kMaxDigits];       // radix of group digit j
    int32_t wofs[kMaxDigits];      // element offset of digit j's matrix in W
    FastDiv divrad[kMaxDigits];    // division by rad[j]
    int32_t wtotal;                // elements of W to stage in LDS
    // radix-8 matrix-core kernels with per-lane addresses: per digit j,
    // bits 16j..16j+7 = fibre-bit mask of the lane index, then the two
    // gradient lane-group bits (3 bits each)
    uint64_t fmap;
    // paired four-digit backward layouts: fibre-bit masks of the recomputing
    // passes of digits 1 (bits 0..7) and 2 (bits 8..15); 0 otherwise
    uint32_t pmap;
};

// backward of one group, complex64 radix 8 on the matrix cores
struct CBwdArgs {
    PassArgs p;          // tile geometry; p.in = a_in, p.out = c_in, p.W = W
    const void* c_out;   // cotangent at the group's output
    void* partials;      // [gridDim.x][64] complex double
};

}  // namespace gtt
