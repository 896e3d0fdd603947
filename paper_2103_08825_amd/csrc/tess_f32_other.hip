// Tessellated 3D sweeps, FP32: the 27-point box ((1,16,4) stage-A tile, k = 1..3,
// 8-row stage-B frames) and the 13-point order-2 star ((1,8,4), k = 1..2, 16-row
// frames).
#include "inst_stream.hpp"
namespace {
const stn::TessRegs<float, 1, true, 1, 16, 4, 2, 1, 2, 3> reg27;
const stn::TessRegs<float, 2, false, 1, 8, 4, 4, 1, 2> reg13;
}  // namespace
