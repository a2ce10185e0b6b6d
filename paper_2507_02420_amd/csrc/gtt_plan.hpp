// Plan object behind gtt_plan_t.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "gtt.h"
#include "gtt_args.hpp"

namespace gtt {

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
    int pad_shift = 31;
    bool generic = false;
    int wtotal = 0;
    size_t lds_bytes = 0;
};

enum class PlanKind { Uniform, Ragged, Mixed };

struct Instance {
    int b = 2, n = 0;
    int64_t N = 1;
    int64_t off = 0;   // element offset in the data buffers
    int w = 0;         // W table index
    std::vector<Group> groups;
};

struct RaggedState;  // device work list (persistent launch)

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
    int64_t w_elems = 0;      // elements of W (or of the W table)
    std::vector<int> rad;     // radix per digit, least significant first
    std::vector<int64_t> wofs;// W offset per digit (elements)
    std::vector<gtt::Group> groups;
    // ragged
    std::vector<gtt::Instance> inst;
    std::vector<int> w_b;         // radix of W table entry
    std::vector<int64_t> w_off;   // element offset of W table entry
    gtt::RaggedState* rs = nullptr;
};

namespace gtt {

FastDiv make_fastdiv(uint32_t d);
uint32_t host_fdiv(uint32_t n, const FastDiv& f);
size_t storage_size(gtt_dtype d);
size_t compute_size(gtt_dtype d);
gtt_status plan_groups(const std::vector<int>& rad, int64_t batch, gtt_dtype dt, uint32_t flags, bool uniform,
                       std::vector<Group>* groups);

gtt_status plan_ragged(gtt_plan_s* p, int32_t count, const int32_t* b, const int32_t* n, const int64_t* x_off,
                       const int32_t* w_idx);
void destroy_ragged(gtt_plan_s* p);
gtt_status ragged_apply(gtt_plan_s* p, const void* W, const void* in, void* out, bool adjoint, char* saved,
                        hipStream_t s);
void workspace_sizes(const gtt_plan_s* p, size_t* fwd, size_t* bwd, size_t* saved);
std::string describe_plan(const gtt_plan_s* p);
gtt_status backward_impl(gtt_plan_s* p, const void* W, const void* x, const void* saved, const void* gy, void* gx,
                         void* gW, void* ws, size_t ws_bytes, hipStream_t s);
gtt_status filter_impl(gtt_plan_s* p, const void* W, const void* x, int64_t cutoff, void* low, void* high,
                       void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace gtt
