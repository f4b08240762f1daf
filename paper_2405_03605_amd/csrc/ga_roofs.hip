// Microbenchmarks for the two limits of the generation step on gfx950: HBM
// bandwidth for an in-place update of the population planes (what the
// per-generation streaming kernel must at least move), and the rate of the
// counter-based RNG block every child draws (Philox4x32-10) and of its two
// instruction kinds (32x32->64 multiply-add, three-input XOR), which bound the
// LDS-resident form. Measurement only: nothing here is part of a run.
#include "ga_device.hpp"

namespace ga {
namespace {

// Every word of `planes` planes of `words` u32 each read and written once
// (incremented), 16 bytes per access.
__global__ void inplace_kernel(uint4* base, size_t vec_per_plane, uint32_t planes) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < vec_per_plane; i += stride) {
    for (uint32_t p = 0; p < planes; ++p) {
      uint4 x = base[p * vec_per_plane + i];
      x.x += 1u;
      x.y += 1u;
      x.z += 1u;
      x.w += 1u;
      base[p * vec_per_plane + i] = x;
    }
  }
}

// `blocks` full Philox4x32-10 blocks per thread, counter (thread, j, 0, 3),
// their words XOR-folded into one output word per thread.
__global__ void philox_kernel(uint32_t* out, uint32_t blocks, uint32_t k0, uint32_t k1) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0u;
  for (uint32_t j = 0; j < blocks; ++j) {
    const Block b = philox10(id, j, 0u, 3u, k0, k1);
    acc ^= xor3(b.x, b.y, b.z) ^ b.w;
  }
  out[id] = acc;
}

// Eight independent dependency chains of `iters` steps each of one
// instruction kind: kind 0 a three-input XOR, kind 1 a 32x32->64
// multiply-add (one v_mad_u64_u32). The chains keep the SIMD's issue slots
// full at any latency.
template <int KIND>
__global__ void valu_kernel(uint32_t* out, uint32_t iters, uint32_t seed) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) a[c] = id * 8u + (uint32_t)c + seed;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (KIND == 0) {
        a[c] = xor3(a[c], a[(c + 1) & 7], seed + i);
      } else {
        const uint64_t p = (uint64_t)a[c] * kMulA + a[(c + 1) & 7];
        a[c] = (uint32_t)p ^ (uint32_t)(p >> 32);
      }
    }
  }
  uint32_t acc = 0u;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc ^= a[c];
  out[id] = acc;
}

}  // namespace

hipError_t launch_roof_inplace(void* base, size_t words_per_plane, uint32_t planes,
                               hipStream_t stream) {
  const size_t vec = words_per_plane / 4u;
  if (vec == 0 || planes == 0) return hipSuccess;
  size_t groups = (vec + 255u) / 256u;
  if (groups > 65536u) groups = 65536u;
  inplace_kernel<<<dim3((uint32_t)groups), dim3(256), 0, stream>>>(static_cast<uint4*>(base), vec,
                                                                    planes);
  return hipGetLastError();
}

hipError_t launch_roof_philox(uint32_t* out, uint32_t threads, uint32_t blocks,
                              hipStream_t stream) {
  if (threads == 0) return hipSuccess;
  philox_kernel<<<dim3((threads + 255u) / 256u), dim3(256), 0, stream>>>(out, blocks, 0x1234u,
                                                                         0x5678u);
  return hipGetLastError();
}

hipError_t launch_roof_valu(uint32_t* out, uint32_t threads, uint32_t iters, uint32_t kind,
                            hipStream_t stream) {
  if (threads == 0) return hipSuccess;
  const dim3 grid((threads + 255u) / 256u), block(256);
  if (kind == 0)
    valu_kernel<0><<<grid, block, 0, stream>>>(out, iters, 7u);
  else if (kind == 1)
    valu_kernel<1><<<grid, block, 0, stream>>>(out, iters, 7u);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace ga
