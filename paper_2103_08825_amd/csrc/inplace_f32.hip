// In-place fused passes, FP32: 3D 7-point star ((1,16,4), k = 1..6), 27-point
// box ((1,16,4), k = 1..3), 13-point order-2 star ((1,8,4), k = 1..2); 2D
// 5-point star and 9-point box ((4,4), k = 1..8).
#include "inst_stream.hpp"
namespace {
const stn::InplaceRegs<float, 3, 1, false, 1, 16, 4, 1, 2, 3, 4, 5, 6> reg7;
const stn::InplaceRegs<float, 3, 1, true, 1, 16, 4, 1, 2, 3> reg27;
const stn::InplaceRegs<float, 3, 2, false, 1, 8, 4, 1, 2> reg13;
const stn::InplaceRegs<float, 2, 1, false, 4, 4, 1, 1, 2, 3, 4, 5, 6, 7, 8> reg2s;
const stn::InplaceRegs<float, 2, 1, true, 4, 4, 1, 1, 2, 3, 4, 5, 6, 7, 8> reg2b;
}  // namespace
