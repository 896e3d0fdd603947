// In-place fused passes of the 3D 7-point star in FP64 ((1,8,4), k = 1..3) and
// with 16-bit storage ((1,16,4), k = 1..6).
#include "inst_stream.hpp"
namespace {
const stn::InplaceRegs<double, 3, 1, false, 1, 8, 4, 1, 2, 3> reg64;
const stn::InplaceRegs<::stn::bf16_t, 3, 1, false, 1, 16, 4, 1, 2, 3, 4, 5, 6> regbf;
const stn::InplaceRegs<_Float16, 3, 1, false, 1, 16, 4, 1, 2, 3, 4, 5, 6> regh;
}  // namespace
