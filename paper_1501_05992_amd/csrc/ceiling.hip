// ceiling.hip -- issue-rate probes for the two instructions the X-engines are
// built on, so that their roofline fractions can be quoted against measured
// ceilings as well as published peaks (the arithmetic-intensity argument of
// Sec. 3.4.2 bounds a kernel by the slower of memory and arithmetic):
//
//   dot4_probe: v_dot4_i32_i8, the vector-ALU engine's only multiply (one
//               instruction = 4 multiply-adds = 8 integer ops per lane);
//   mfma_probe: v_mfma_i32_32x32x32_i8, the int8 matrix-core engine's
//               instruction (32 * 32 * 32 * 2 = 65536 ops per wave).
//
// Each wave runs independent dependency chains of the one instruction on
// register operands: no memory traffic inside the loop, one store per lane at
// the end.  Each workgroup also records the shader-clock and the 100 MHz
// constant-clock counters around its loop, from which the host derives the
// shader clock under that load.  Built as its own library (libceiling.so);
// nothing in the correlator calls it.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kChains = 8;  // independent v_dot4 chains per lane

// clk: per workgroup {shader cycles, constant-clock ticks} of the loop.
__global__ __launch_bounds__(256) void dot4_probe(int* out, long long* clk, int iters, int seed) {
  int c[kChains];
  int a[kChains];
  const int b = seed * 0x01010101 + (int)blockIdx.x;
#pragma unroll
  for (int u = 0; u < kChains; ++u) {
    c[u] = (int)threadIdx.x + u;
    a[u] = (seed + u) * 0x03050709 ^ (int)threadIdx.x;
  }
  __syncthreads();
  const long long t0 = __builtin_amdgcn_s_memtime();
  const long long r0 = __builtin_amdgcn_s_memrealtime();
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < kChains; ++u) c[u] = __builtin_amdgcn_sdot4(a[u], b, c[u], false);
  }
  __syncthreads();
  const long long t1 = __builtin_amdgcn_s_memtime();
  const long long r1 = __builtin_amdgcn_s_memrealtime();
  int s = 0;
#pragma unroll
  for (int u = 0; u < kChains; ++u) s ^= c[u];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
}

constexpr int kAccs = 4;  // independent MFMA accumulators per wave

// seed 0: every operand byte 1 (quiet operands); otherwise hashed bytes
// (every bit toggling): the matrix cores' power, and so the clock under the
// power limit, depends on the operand data.
__global__ __launch_bounds__(256) void mfma_probe(int* out, long long* clk, int iters, int seed) {
  const int lane = (int)threadIdx.x;
  v4i a, b;
  for (int e = 0; e < 4; ++e) {
    a[e] = seed == 0 ? 0x01010101 : (seed + e) * 0x01030507 ^ lane;
    b[e] = seed == 0 ? 0x01010101 : (seed - e) * 0x07050301 + lane;
  }
  v16i acc[kAccs];
#pragma unroll
  for (int u = 0; u < kAccs; ++u)
    for (int e = 0; e < 16; ++e) acc[u][e] = u + e;
  __syncthreads();
  const long long t0 = __builtin_amdgcn_s_memtime();
  const long long r0 = __builtin_amdgcn_s_memrealtime();
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < kAccs; ++u) acc[u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[u], 0, 0, 0);
  }
  __syncthreads();
  const long long t1 = __builtin_amdgcn_s_memtime();
  const long long r1 = __builtin_amdgcn_s_memrealtime();
  int s = 0;
#pragma unroll
  for (int u = 0; u < kAccs; ++u)
    for (int e = 0; e < 16; ++e) s ^= acc[u][e];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
}

}  // namespace

extern "C" {

// Integer ops one launch performs (for the host's rate computation).
double ceiling_dot4_ops(int blocks, int iters) { return (double)blocks * 256 * iters * kChains * 8.0; }
double ceiling_mfma_ops(int blocks, int iters) { return (double)blocks * 4 * iters * kAccs * 65536.0; }

// Enqueue one probe launch of `blocks` workgroups of 256 threads.  out:
// device, blocks * 256 ints; clk: device, blocks * 2 long longs.  kind 0 =
// dot4, 1 = mfma.  Returns 0, or -1 on a bad argument / failed launch.
int ceiling_launch(int kind, int blocks, int iters, int seed, void* out, void* clk, void* stream) {
  if (blocks < 1 || iters < 1 || !out || !clk || (kind != 0 && kind != 1)) return -1;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (kind == 0)
    hipLaunchKernelGGL(dot4_probe, dim3(blocks), dim3(256), 0, s, static_cast<int*>(out),
                       static_cast<long long*>(clk), iters, seed);
  else
    hipLaunchKernelGGL(mfma_probe, dim3(blocks), dim3(256), 0, s, static_cast<int*>(out),
                       static_cast<long long*>(clk), iters, seed);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
