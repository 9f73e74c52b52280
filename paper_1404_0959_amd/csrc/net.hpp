// net.hpp -- host entry points of the learned pressure-guess network kernels
// (net.hip) used by the step orchestration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>

#include "launch.hpp"

namespace pisoc {

constexpr int kNetWeights = 15120;   // 27 (2*16 + 16*16 + 16*16 + 16*1)

// Offset of layer l in the FP32 weight vector (layer-major, [co][ci][27]).
size_t net_weight_offset(int layer);
// Bytes of the packed BF16 MFMA operands of the four forward layers.
size_t net_packed_bytes();
// Pack FP32 weights into per-lane BF16 MFMA operands (device to device).
void net_pack_forward(hipStream_t s, const float* w32, void* wpk);
// Four layers on BF16 channel-last input x4 [cells][4]; y = yscale * output.
// a, b: BF16 [cells][16] scratch.  n must be a multiple of 16.
void net_forward(hipStream_t s, int n, int batch, const void* wpk, const uint16_t* x4, uint16_t* a,
                 uint16_t* b, float* y, float yscale);

}  // namespace pisoc
