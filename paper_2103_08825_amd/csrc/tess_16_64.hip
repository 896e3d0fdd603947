// Tessellated 3D sweeps of the 7-point star with 16-bit storage ((1,16,4),
// k = 1..6) and in FP64 ((1,8,4), k = 1..3).
#include "inst_stream.hpp"
namespace {
const stn::TessRegs<::stn::bf16_t, 1, false, 1, 16, 4, 4, 1, 2, 3, 4, 5, 6> reg_bf16;
const stn::TessRegs<_Float16, 1, false, 1, 16, 4, 4, 1, 2, 3, 4, 5, 6> reg_f16;
const stn::TessRegs<double, 1, false, 1, 8, 4, 4, 1, 2, 3> reg_f64;
}  // namespace
