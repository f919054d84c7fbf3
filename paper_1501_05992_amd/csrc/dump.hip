// dump.hip -- accumulator fill, output reordering (Appendix C "GPU Output"),
// and the incoherent-beam mode (Sec. 3.4).

#include "corrx_internal.h"

namespace corrx {

__global__ void fill_zero(int4* acc4, int* acc, int64_t n4, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += stride)
    acc4[k] = make_int4(0, 0, 0, 0);
  for (int64_t k = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) acc[k] = 0;
}

int launch_zero(int* acc, int64_t n_words, hipStream_t s) {
  const bool al = (reinterpret_cast<uintptr_t>(acc) & 15) == 0;
  const int64_t n4 = al ? n_words / 4 : 0;
  const int64_t work = n4 > 0 ? n4 : n_words;
  const int grid = (int)((work + 255) / 256 < 8192 ? (work + 255) / 256 : 8192);
  hipLaunchKernelGGL(fill_zero, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, reinterpret_cast<int4*>(acc), acc,
                     n4, n_words);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

// Triangle index b -> (s1, s2) with b = s1(s1+1)/2 + s2, 0 <= s2 <= s1.
__device__ inline void tri_decode(int64_t b, int& s1, int& s2) {
  int r = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)(r + 1) * (r + 2) / 2 <= b) ++r;
  while ((int64_t)r * (r + 1) / 2 > b) --r;
  s1 = r;
  s2 = (int)(b - (int64_t)r * (r + 1) / 2);
}

template <typename T>
__device__ inline T conv(int v);
template <>
__device__ inline int conv<int>(int v) { return v; }
template <>
__device__ inline float conv<float>(int v) { return (float)v; }

template <typename T>
__global__ void dump_tri(const int2* acc, T* dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int2 v = acc[k];
    dst[2 * k] = conv<T>(v.x);
    dst[2 * k + 1] = conv<T>(v.y);
  }
}

// out element o = ((f * B(S) + bs) * 2 + p1) * 2 + p2, complex.
template <typename T>
__global__ void dump_station_pol(const int2* acc, T* dst, int n_inputs, int64_t n_station_bl, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nb = tri_index(n_inputs, 0);
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += stride) {
    const int p2 = (int)(o & 1), p1 = (int)((o >> 1) & 1);
    const int64_t rest = o >> 2;
    const int64_t f = rest / n_station_bl, bs = rest % n_station_bl;
    int s1, s2;
    tri_decode(bs, s1, s2);
    const int i = 2 * s1 + p1, j = 2 * s2 + p2;
    int2 v;
    if (i >= j) {
      v = acc[f * nb + tri_index(i, j)];
    } else {
      v = acc[f * nb + tri_index(j, i)];
      v.y = -v.y;
    }
    dst[2 * o] = conv<T>(v.x);
    dst[2 * o + 1] = conv<T>(v.y);
  }
}

int launch_dump(const int* acc, int n_inputs, int n_chan, int order, int dtype, void* dst, hipStream_t s) {
  const int2* a2 = reinterpret_cast<const int2*>(acc);
  int64_t n;
  if (order == CORRX_TRI_INPUT)
    n = (int64_t)n_chan * tri_index(n_inputs, 0);
  else
    n = (int64_t)n_chan * tri_index(n_inputs / 2, 0) * 4;
  const int grid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  const dim3 g(grid > 0 ? grid : 1), b(256);
  if (order == CORRX_TRI_INPUT) {
    if (dtype == CORRX_I32)
      hipLaunchKernelGGL(dump_tri<int>, g, b, 0, s, a2, reinterpret_cast<int*>(dst), n);
    else
      hipLaunchKernelGGL(dump_tri<float>, g, b, 0, s, a2, reinterpret_cast<float*>(dst), n);
  } else {
    const int64_t nsb = tri_index(n_inputs / 2, 0);
    if (dtype == CORRX_I32)
      hipLaunchKernelGGL(dump_station_pol<int>, g, b, 0, s, a2, reinterpret_cast<int*>(dst), n_inputs, nsb, n);
    else
      hipLaunchKernelGGL(dump_station_pol<float>, g, b, 0, s, a2, reinterpret_cast<float*>(dst), n_inputs, nsb,
                         n);
  }
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

// Incoherent beam: out[f][t] = sum_i |x_i(f,t)|^2.  One thread per (f, t)
// row; four samples per dword through the biased parts u = re + 8, w = im + 8:
//     re^2 + im^2 = u^2 + w^2 - 16 (u + w) + 128.
__global__ void beam_rows(Problem p, int* out, int64_t nrows) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool aligned = (p.n_inputs % 4 == 0) && ((reinterpret_cast<uintptr_t>(p.in) & 3) == 0);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += stride) {
    const int f = (int)(r / p.n_time), t = (int)(r % p.n_time);
    const uint8_t* row = p.in + row_offset(p, f, t);
    uint32_t sq = 0, lin = 0, cnt = 0;
    for (int i = 0; i < p.n_inputs; i += 4) {
      uint32_t x;
      uint32_t nvalid = (uint32_t)min(4, p.n_inputs - i);
      if (aligned && nvalid == 4) {
        x = *reinterpret_cast<const uint32_t*>(row + i);
      } else {
        x = 0;
        for (uint32_t b = 0; b < nvalid; ++b) x |= uint32_t(row[i + b]) << (8 * b);
      }
      const uint32_t y = mask_invalid(bias4(x));  // missing bytes and invalid samples become 0 + 0j
      const uint32_t u = bre4(y), w = bim4(y);
      sq = __builtin_amdgcn_udot4(u, u, sq, false);
      sq = __builtin_amdgcn_udot4(w, w, sq, false);
      lin = bytesum(u, lin);
      lin = bytesum(w, lin);
      cnt += 4;
    }
    out[r] = (int)(sq - 16u * lin + 128u * cnt);
  }
}

int launch_beam(const Problem& p, int* out, hipStream_t s) {
  const int64_t nrows = (int64_t)p.n_chan * p.n_time;
  const int grid = (int)((nrows + 255) / 256 < 16384 ? (nrows + 255) / 256 : 16384);
  hipLaunchKernelGGL(beam_rows, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, p, out, nrows);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

}  // namespace corrx
