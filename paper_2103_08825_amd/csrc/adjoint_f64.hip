// Fused adjoint passes in FP64: 3D 7-point star on the (1,8,4) tile; 2D
// 5-point star on the (1,4) tile.
#include "inst_stream.hpp"
namespace {
const stn::AdjointRegs<double, 3, 1, false, 1, 8, 4, 1, 2> reg7;
const stn::AdjointRegs<double, 2, 1, false, 1, 4, 1, 1, 2> reg2s;
}  // namespace
