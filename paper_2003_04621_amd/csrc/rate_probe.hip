// rate_probe.hip -- issue rate of the VALU instructions the Metropolis word
// update is built from, on this GPU: sixteen independent dependency chains per
// lane, each instruction in inline assembly so that the compiler can neither
// fold nor reorder the chains.  Prints lane-operations per second for each
// instruction and its ratio to v_add_u32.  Measurement support for the
// roofline of the fused kernel; not part of the library.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "device.h"

namespace {

constexpr int kChains = 16;

template <int OP>
__global__ void __launch_bounds__(256) chains(uint32_t* out, uint32_t seed, int iters) {
  uint32_t a[kChains];
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kChains; ++j) a[j] = gid * 2654435761u + seed + (uint32_t)j;
  const uint32_t m = 0xD2511F53u ^ seed;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if (OP == 0) {
        asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a[j]) : "v"(m));
      } else if (OP == 1) {
        uint64_t r;
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(a[j]), "v"(m) : "vcc");
        a[j] = (uint32_t)r;
      } else if (OP == 2) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[j]) : "v"(m));
      } else if (OP == 3) {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[j]) : "v"(m));
      } else if (OP == 4) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(a[j]) : "v"(m));
      } else if (OP == 5) {
        asm volatile("v_mul_u32_u24_e32 %0, %0, %1" : "+v"(a[j]) : "v"(m));
      } else if (OP == 6) {  // one 64-bit multiply and one three-input xor, as in Philox
        uint64_t r;
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(a[j]), "v"(m) : "vcc");
        a[j] = (uint32_t)r;
        asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(a[j]) : "v"(m));
      }
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) x ^= a[j];
  out[gid] = x;
}

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

template <int OP>
double rate(uint32_t* d, int blocks, int iters) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, 0, d, 1u, 16);
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, 0, d, 1u, iters);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return (double)blocks * 256 * iters * kChains * (OP == 6 ? 2 : 1) / (ms * 1e-3);
}

// The sweep's inner loop without the rest of the word update: one
// Philox4x32-10 call per iteration (counter as the sweep forms it) and the 3D
// acceptance planes of its four words.  Its rate bounds the fused kernel from
// above for this instruction sequence.
__global__ void __launch_bounds__(256) philox_sites(uint32_t* out, uint32_t k0, uint32_t k1,
                                                    int iters) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t C1 = 0, C2 = 0;
  for (int i = iters - 1; i >= 0; --i) {
    const ptsg::Ctr4 r =
        ptsg::philox10(ptsg::Ctr4{(uint32_t)i, gid, 7u, 3u << 28}, k0, k1);
    ptsg::shift_in_k_pair(C1, C2, r.w, r.z, 0x80000000u, 0x40000000u, 0x20000000u);
    ptsg::shift_in_k_pair(C1, C2, r.y, r.x, 0x80000000u, 0x40000000u, 0x20000000u);
  }
  out[gid] = C1 ^ (3u * C2);
}

double philox_rate(uint32_t* d, int ncu, int waves_per_cu, int iters) {
  const int blocks = ncu * waves_per_cu / 4;
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(philox_sites, dim3(blocks), dim3(256), 0, 0, d, 1u, 2u, 16);
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(philox_sites, dim3(blocks), dim3(256), 0, 0, d, 1u, 2u, iters);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return (double)blocks * 256 * iters * 4 / (ms * 1e6);  // sites per ns
}

}  // namespace

int main() {
  const int blocks = 256 * 32, iters = 2048;  // 32 workgroups of 256 per CU
  uint32_t* d = nullptr;
  CHECK(hipMalloc(&d, sizeof(uint32_t) * (size_t)blocks * 256));
  int clk = 0;
  CHECK(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, 0));
  const char* names[] = {"v_add_u32", "v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32",
                         "v_bitop3_b32", "v_mul_u32_u24", "mad_u64+bitop3"};
  double r[7];
  r[0] = rate<0>(d, blocks, iters);
  r[1] = rate<1>(d, blocks, iters);
  r[2] = rate<2>(d, blocks, iters);
  r[3] = rate<3>(d, blocks, iters);
  r[4] = rate<4>(d, blocks, iters);
  r[5] = rate<5>(d, blocks, iters);
  r[6] = rate<6>(d, blocks, iters);
  std::printf("clock attribute: %d kHz\n", clk);
  for (int i = 0; i < 7; ++i)
    std::printf("%-16s %7.2f T lane-ops/s  %.3f of v_add_u32\n", names[i], r[i] / 1e12, r[i] / r[0]);
  int ncu = 0;
  CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
  for (int w : {8, 16, 24, 32})  // at most 32 wavefronts per CU: within the buffer
    std::printf("Philox4x32-10 + 3D compares, %2d wavefronts/CU: %6.0f sites/ns\n", w,
                philox_rate(d, ncu, w, 4096));
  CHECK(hipFree(d));
  return 0;
}
