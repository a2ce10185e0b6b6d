// Plan object behind gtt_plan_t.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "gtt.h"
#include "gtt_args.hpp"

namespace gtt {

constexpr int kNoPad = 31 | (31 << 8) | (31 << 16);

// host mirror of the device LDS size of a padded tile
inline int64_t lds_tile_elems_host(int64_t tileE, int ps) {
    return tileE + (tileE >> (ps & 31)) + (tileE >> ((ps >> 8) & 31)) + (tileE >> ((ps >> 16) & 31)) + 1;
}

struct Group {
    int s0 = 0;         // lowest digit of the group
    int k = 0;          // digits in the group
    int64_t S = 1;      // place value of digit s0
    int64_t G = 1;      // product of the group's radices
    int C = 1, logC = 0;
    int P = 1;
    int64_t L = 1;      // column blocks per hi block
    int64_t ntiles = 0;
    int64_t tileE = 0;
    int mode = 0;
    int pad_shift = kNoPad;  // packed LDS pad shifts (see lds_phys)
    int kind = 0;       // kKindValu / kKindGeneric / kKindMfma
    int wtotal = 0;
    size_t lds_bytes = 0;
    int64_t elems = 0;  // elements covered by one launch of this group
    int fast_ni = 0;     // > 0: radix-8 matrix-core kernel with per-lane addresses, tile 2048 * fast_ni
    uint64_t fmap = 0;   // its fibre-to-lane maps (PassArgs::fmap)
    uint32_t pmap = 0;   // pass-only maps of a paired backward layout (PassArgs::pmap)
    int fast_conflicts = 0;  // residual LDS bank conflicts of that layout (model)
    // backward groups on the general kernel (every kind but the complex
    // radix-8 matrix-core one): LDS tiles per work-group, the checkpoint
    // schedule run on them, the largest radix and the staged matrix entries
    int bwd_slots = 0;
    int bwd_rd = 0;      // > 0: register-block kernel, schedule over blocks of bwd_rd digits
    int bwd_maxb = 0;
    int bwd_wloc = 0;
    bool bwd_ok = true;  // false: no backward kernel covers the group
    std::vector<uint16_t> bwd_ops;
};

// LDS layout of the per-lane-address radix-8 kernels for K digits, tiles of
// 2048 * NI elements, 2^logC columns; gw: the backward's gradient sums too
struct FastMap {
    int pad = kNoPad;   // packed pad shifts
    uint64_t map = 0;   // PassArgs::fmap
    uint32_t pmap = 0;  // PassArgs::pmap (paired layouts; 0: none)
    int conflicts = 0;  // residual bank conflicts of the layout (0: none)
};
FastMap fast_map(int K, int NI, int logC, bool gw);
// LDS padding (packed shifts) of a matrix-core pass: radix B, k digits,
// 2^logC columns, tileE elements, no shift below min_shift, vec elements per
// 16-byte tile transfer; lds16: a 16-bit tile whose pads count 32-bit words
// (else an FP32 tile, pads in elements)
int mfma_pad(int B, int k, int logC, int64_t tileE, int min_shift, int vec, bool lds16);

enum class PlanKind { Uniform, Ragged, Mixed };

struct Instance {
    int b = 2, n = 0;
    int64_t N = 1;
    int64_t off = 0;   // element offset in the data buffers
    int w = 0;         // W table index
    std::vector<Group> groups;
    std::vector<Group> bwd_groups;
};

struct RaggedState;  // device work list (persistent launch)

// Optional per-launch HIP-event timing (instrumentation; see gtt_plan_timing)
struct TimedLaunch {
    std::string name;
    hipEvent_t start, stop;
    double bytes;  // algorithmic bytes moved by this launch
};
struct Timing {
    bool enabled = false;
    std::string filter;  // time only launches whose name starts with it (empty: all)
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
};

}  // namespace gtt

struct gtt_plan_s {
    gtt::PlanKind kind = gtt::PlanKind::Uniform;
    gtt_dtype dtype = GTT_F32;
    uint32_t flags = 0;
    size_t esize = 4, csize = 4;
    // uniform / mixed
    int b = 2, n = 0;
    int64_t N = 1, batch = 1;
    int64_t total_elems = 0;  // elements in a data buffer
    int64_t slot = 0;         // element stride of the boundary slots in saved / workspace buffers
                              // (total_elems rounded up to 256 bytes: every slot 16-byte aligned)
    int64_t w_elems = 0;      // elements of W (or of the W table)
    std::vector<int> rad;     // radix per digit, least significant first
    std::vector<int64_t> wofs;// W offset per digit (elements)
    std::vector<gtt::Group> groups;
    std::vector<gtt::Group> bwd_groups;  // backward tiles (same digit groups)
    // ragged
    std::vector<gtt::Instance> inst;
    std::vector<int> w_b;         // radix of W table entry
    std::vector<int64_t> w_off;   // element offset of W table entry
    gtt::RaggedState* rs = nullptr;
    int ragged_scalar_instances = 0;  // instances off a 16-byte boundary (element-wise tile I/O)
    gtt::Timing timing;
    // GTT_FLAG_FP32_INTERMEDIATE on a 16-bit storage dtype: the same
    // transform planned in float32; calls convert at the boundaries and run it
    gtt_plan_s* inner = nullptr;
};

namespace gtt {

inline int64_t slot_elems(int64_t total, size_t esize) {
    const int64_t bytes = (total * (int64_t)esize + 255) & ~(int64_t)255;
    return bytes / (int64_t)esize;
}

FastDiv make_fastdiv(uint32_t d);
uint32_t host_fdiv(uint32_t n, const FastDiv& f);
size_t storage_size(gtt_dtype d);
size_t compute_size(gtt_dtype d);
gtt_status plan_groups(const std::vector<int>& rad, int64_t batch, gtt_dtype dt, uint32_t flags, bool uniform,
                       std::vector<Group>* groups, std::vector<Group>* bwd_groups, bool ragged = false);
// accumulation dtype of the weight gradient: FP64, complex FP64 for complex data
size_t acc_size(gtt_dtype d);
size_t bwd_lds_bytes(const Group& g, gtt_dtype dt);
// LDS bytes of the general backward besides its tiles
size_t bwd_overhead_bytes(int wloc, gtt_dtype dt);
// forward passes of the optimal checkpoint schedule (k digits, `free_slots`
// activation slots besides the group input and the cotangent)
int bwd_fwd_passes(int k, int free_slots);
// the schedule itself (operations as in gtt_bwd.hpp)
std::vector<uint16_t> bwd_schedule(int k, int nslots);
// partial-vector entries of every backward launch of a group list (wslot
// entries per work-group)
size_t bwd_partials_elems(const std::vector<Group>& bg, int wslot);

gtt_status plan_ragged(gtt_plan_s* p, int32_t count, const int32_t* b, const int32_t* n, const int64_t* x_off,
                       const int32_t* w_idx);
void destroy_ragged(gtt_plan_s* p);
// waits for `s`, then reports and clears a grid-barrier failure of the
// plan's persistent launches (GTT_ERR_TIMEOUT)
gtt_status ragged_check(gtt_plan_s* p, hipStream_t s);
gtt_status ragged_set_spin_limit(gtt_plan_s* p, uint32_t polls);
gtt_status ragged_apply(gtt_plan_s* p, const void* W, const void* in, void* out, bool adjoint, char* saved,
                        hipStream_t s);
void workspace_sizes(const gtt_plan_s* p, size_t* fwd, size_t* bwd, size_t* saved);
size_t bwd_partial_bytes(const gtt_plan_s* p);
// every digit group of the plan has a backward kernel (floating dtypes,
// radices <= 32, LDS)
bool plan_has_backward(const gtt_plan_s* p);
// workspace bytes one gtt_backward call needs (saved passed or not; the
// cotangent between digit groups kept in gx or not)
size_t backward_ws_need(const gtt_plan_s* p, bool have_saved, bool cb_in_gx);
// bytes of one float32 copy of a buffer (GTT_FLAG_FP32_INTERMEDIATE plans)
size_t f32_buf_bytes(const gtt_plan_s* p);
std::string describe_plan(const gtt_plan_s* p);
// bracket a launch with events when timing is enabled (no-ops otherwise)
void timing_begin(gtt_plan_s* p, hipStream_t s, const std::string& name);
void timing_end(gtt_plan_s* p, hipStream_t s, const std::string& name, double bytes);
void timing_release(gtt_plan_s* p);
std::string timing_read(gtt_plan_s* p);
gtt_status launch_group_rw(gtt_plan_s* tp, gtt_dtype dt, const Group& g, const std::vector<int>& rad,
                           const std::vector<int64_t>& wofs, int64_t N, const void* W, bool adjoint, const void* in,
                           void* out, hipStream_t s);
gtt_status launch_group_inst(gtt_plan_s* tp, gtt_dtype dt, const Group& g, int b, int64_t N, const void* W,
                             bool adjoint, const void* in, void* out, hipStream_t s);
gtt_status backward_impl(gtt_plan_s* p, const void* W, const void* x, const void* saved, const void* gy, void* gx,
                         void* gW, void* ws, size_t ws_bytes, hipStream_t s);
gtt_status filter_impl(gtt_plan_s* p, const void* W, const void* x, int64_t cutoff, void* low, void* high,
                       void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace gtt
