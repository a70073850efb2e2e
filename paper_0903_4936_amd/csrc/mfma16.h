// Layout of v_mfma_f32_16x16x4f32 accumulators, shared by the block kernels
// and the operator's Gram epilogue.
#pragma once

#include <hip/hip_runtime.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));

// (i, j) of P held by accumulator register v of this lane: from D = A B with
// A[i][0] = i + 1, B[0][j] = 1 (gives i + 1) and A[i][0] = 1, B[0][j] = j + 1.
struct L8Layout {
  int i[4], j[4];
};

__device__ __forceinline__ L8Layout l8_layout() {
  const int lane = threadIdx.x & 63;
  const float code = lane < 16 ? (float)(lane + 1) : 0.f;
  const float one = lane < 16 ? 1.f : 0.f;
  const f32x4 z{0.f, 0.f, 0.f, 0.f};
  const f32x4 di = __builtin_amdgcn_mfma_f32_16x16x4f32(code, one, z, 0, 0, 0);
  const f32x4 dj = __builtin_amdgcn_mfma_f32_16x16x4f32(one, code, z, 0, 0, 0);
  L8Layout o;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // the codes are exact small integers; the mask keeps every LDS index in
    // range whatever the instruction returned
    o.i[v] = ((int)di[v] - 1) & 15;
    o.j[v] = ((int)dj[v] - 1) & 15;
  }
  return o;
}
