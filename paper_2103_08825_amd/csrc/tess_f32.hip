// Tessellated 3D sweeps (two stages per pass), FP32: the 7-point star with the
// (1,16,4) stage-A tile, k = 1..6; stage B on 16-row frames.
#include "inst_stream.hpp"
namespace {
const stn::TessRegs<float, 1, false, 1, 16, 4, 4, 1, 2, 3, 4, 5, 6> reg;
}  // namespace
