// Fused adjoint passes (mirrored steps with the coefficient gradient folded
// in), FP32: 3D 7-point star on the (1,8,4) tile; 27-point box and 13-point
// order-2 star on the (1,4,8) tile (one wave per SIMD: their 27 and 13 gradient
// sums do not fit the 256 registers an 8-wave tile leaves each lane); 2D 5-point
// star and 9-point box on the (1,4) tile.
#include "inst_stream.hpp"
namespace {
const stn::AdjointRegs<float, 3, 1, false, 1, 8, 4, 1, 2, 3, 4> reg7;
const stn::AdjointRegs<float, 3, 1, true, 1, 4, 8, 1, 2> reg27;
const stn::AdjointRegs<float, 3, 2, false, 1, 4, 8, 1, 2> reg13;
const stn::AdjointRegs<float, 2, 1, false, 1, 4, 1, 1, 2, 3, 4> reg2s;
const stn::AdjointRegs<float, 2, 1, true, 1, 4, 1, 1, 2, 3, 4> reg2b;
}  // namespace
// Level-storing forward passes (the adjoint's segment recompute): 3D 7-point
// star on the (1,4,8) tile, 2D 5-point star on the (1,4) tile, k = 2..4.
namespace {
const stn::LevelsRegs<float, 3, 1, false, 1, 4, 8, 2, 3, 4> lreg7;
const stn::LevelsRegs<float, 2, 1, false, 1, 4, 1, 2, 3, 4> lreg2;
}  // namespace
