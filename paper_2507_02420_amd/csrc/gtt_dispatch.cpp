// Dtype dispatch to the per-dtype kernel translation units.
#include "gtt_launch.hpp"

namespace gtt {

hipError_t launch_pass_f64(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_f32(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_c128(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_c64(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_bf16(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_f16(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);
hipError_t launch_pass_i32(int, bool, const PassArgs&, unsigned, size_t, hipStream_t);

hipError_t launch_pass(DT dt, int b, bool generic, const PassArgs& a, unsigned grid, size_t lds, hipStream_t s) {
    switch (dt) {
        case DT::F64: return launch_pass_f64(b, generic, a, grid, lds, s);
        case DT::F32: return launch_pass_f32(b, generic, a, grid, lds, s);
        case DT::C128: return launch_pass_c128(b, generic, a, grid, lds, s);
        case DT::C64: return launch_pass_c64(b, generic, a, grid, lds, s);
        case DT::BF16: return launch_pass_bf16(b, generic, a, grid, lds, s);
        case DT::F16: return launch_pass_f16(b, generic, a, grid, lds, s);
        case DT::I32: return launch_pass_i32(b, generic, a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gtt
