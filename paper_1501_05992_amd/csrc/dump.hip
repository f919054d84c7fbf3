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
  int r = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
  while ((int64_t)(r + 1) * (r + 2) / 2 <= b) ++r;
  while ((int64_t)r * (r + 1) / 2 > b) --r;
  s1 = r;
  s2 = (int)(b - (int64_t)r * (r + 1) / 2);
}

template <typename T>
__device__ inline T conv(int v, float scale);
template <>
__device__ inline int conv<int>(int v, float) { return v; }
template <>
__device__ inline float conv<float>(int v, float scale) { return (float)v * scale; }

// Sum of fa adjacent channels g*fa .. g*fa+fa-1 of one accumulator element.
__device__ inline int2 chan_sum(const int2* acc, int64_t nb, int64_t g, int fa, int64_t b) {
  const int2* a = acc + g * fa * nb + b;
  int2 v = a[0];
  for (int q = 1; q < fa; ++q) {
    const int2 w = a[q * nb];
    v.x += w.x;
    v.y += w.y;
  }
  return v;
}

// Input order: dst[g][b][re, im] = sum over the fa channels of group g.
template <typename T>
__global__ void dump_tri(const int2* acc, T* dst, int64_t nb, int fa, float scale, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int64_t g = k / nb, b = k % nb;
    const int2 v = chan_sum(acc, nb, g, fa, b);
    dst[2 * k] = conv<T>(v.x, scale);
    dst[2 * k + 1] = conv<T>(v.y, scale);
  }
}

// Station/polarisation order (Appendix C "GPU Output"): one thread per
// (channel group g, station pair bs = s1(s1+1)/2 + s2), writing its four
// polarisation products (p1, p2) = (0,0), (0,1), (1,0), (1,1), complex; the
// inputs are i = 2 s1 + p1, j = 2 s2 + p2, and (s, s, 0, 1) is the conjugate
// of the stored (2s+1, 2s) element.
template <typename T>
__global__ void dump_station_pol(const int2* acc, T* dst, int n_inputs, int64_t n_station_bl, int fa, float scale,
                                 int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nb = tri_index(n_inputs, 0);
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += stride) {
    const int64_t g = o / n_station_bl, bs = o % n_station_bl;
    int s1, s2;
    tri_decode(bs, s1, s2);
    T* out = dst + 8 * o;
#pragma unroll
    for (int p1 = 0; p1 < 2; ++p1)
#pragma unroll
      for (int p2 = 0; p2 < 2; ++p2) {
        const int i = 2 * s1 + p1, j = 2 * s2 + p2;
        int2 v;
        if (i >= j) {
          v = chan_sum(acc, nb, g, fa, tri_index(i, j));
        } else {
          v = chan_sum(acc, nb, g, fa, tri_index(j, i));
          v.y = -v.y;
        }
        out[4 * p1 + 2 * p2] = conv<T>(v.x, scale);
        out[4 * p1 + 2 * p2 + 1] = conv<T>(v.y, scale);
      }
  }
}

int launch_dump(const int* acc, int n_inputs, int n_chan, int order, int dtype, int f_avg, float scale, void* dst,
                hipStream_t s) {
  const int2* a2 = reinterpret_cast<const int2*>(acc);
  const int64_t groups = n_chan / f_avg;
  const int64_t nb = tri_index(n_inputs, 0);
  const int64_t nsb = tri_index(n_inputs / 2, 0);
  const int64_t n = order == CORRX_TRI_INPUT ? groups * nb : groups * nsb;
  const int grid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  const dim3 g(grid > 0 ? grid : 1), b(256);
  if (order == CORRX_TRI_INPUT) {
    if (dtype == CORRX_I32)
      hipLaunchKernelGGL(dump_tri<int>, g, b, 0, s, a2, reinterpret_cast<int*>(dst), nb, f_avg, scale, n);
    else
      hipLaunchKernelGGL(dump_tri<float>, g, b, 0, s, a2, reinterpret_cast<float*>(dst), nb, f_avg, scale, n);
  } else {
    if (dtype == CORRX_I32)
      hipLaunchKernelGGL(dump_station_pol<int>, g, b, 0, s, a2, reinterpret_cast<int*>(dst), n_inputs, nsb, f_avg,
                         scale, n);
    else
      hipLaunchKernelGGL(dump_station_pol<float>, g, b, 0, s, a2, reinterpret_cast<float*>(dst), n_inputs, nsb,
                         f_avg, scale, n);
  }
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

// ---- PFB packet order (Appendix A, B, C) ---------------------------------------

// Packet position k (0..63) of a PFB's inputs holds PFB input 16 (k % 4) + k / 4;
// the inverse: input a sits at position 4 (a % 16) + a / 16.
__device__ inline int pfb_pos_of_input(int a) { return 4 * (a & 15) + (a >> 4); }

// Corner turn of lane payloads into the TFI input buffer.  One wave per
// (fibre n, coarse c, group s, time t): lanes 16b .. 16b+15 read PFB b's
// packet (256 bytes, 16 per lane: fine channel f2 = j / 4, positions
// 16 (j % 4) .. +15) and write the four rows (t, 128c + 16n + 4s + f2) at
// columns 64b ..  Packet order copies the 16 bytes; natural order transposes
// them as a 4 x 4 byte block, since positions 16u .. 16u+15 hold inputs
// 16r + 4u + q (r = position % 4, q = 0..3), i.e. byte r of each of the four
// dwords goes to dword 4r + u of the row segment.
__global__ void pfb_ingest(PfbLanes lanes, uint8_t* out, int n_pfb, int n_coarse, int n_time, int natural,
                           int64_t n_waves) {
  const int lane = threadIdx.x & 63;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int b = lane >> 4, j = lane & 15, f2 = j >> 2, u = j & 3;
  const int n_chan = 128 * n_coarse, width = 64 * n_pfb;
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < n_waves; w += wstride) {
    if (b >= n_pfb) continue;
    // w -> (n, c, s, t) with t fastest: consecutive waves stream each lane
    const int t = (int)(w % n_time);
    int64_t r = w / n_time;
    const int s = (int)(r % 4);
    r /= 4;
    const int c = (int)(r % n_coarse);
    const int n = (int)(r / n_coarse);
    const uint8_t* pkt = lanes.p[8 * b + n] + ((((int64_t)c * 4 + s) * n_time + t) << 8);
    const uint4 v = *reinterpret_cast<const uint4*>(pkt + 64 * f2 + 16 * u);
    const int f = 128 * c + 16 * n + 4 * s + f2;
    uint8_t* row = out + ((int64_t)t * n_chan + f) * width + 64 * b;
    if (!natural) {
      *reinterpret_cast<uint4*>(row + 16 * u) = v;
    } else {
      uint32_t e0, e1, e2, e3;
      transpose4x4(v.x, v.y, v.z, v.w, e0, e1, e2, e3);
      *reinterpret_cast<uint32_t*>(row + 4 * u) = e0;
      *reinterpret_cast<uint32_t*>(row + 16 + 4 * u) = e1;
      *reinterpret_cast<uint32_t*>(row + 32 + 4 * u) = e2;
      *reinterpret_cast<uint32_t*>(row + 48 + 4 * u) = e3;
    }
  }
}

int launch_pfb_ingest(const PfbLanes& lanes, uint8_t* out, int n_pfb, int n_coarse, int n_time, int natural,
                      hipStream_t s) {
  const int64_t n_waves = (int64_t)8 * n_coarse * 4 * n_time;
  const int64_t blocks = (n_waves + 3) / 4;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(pfb_ingest, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, lanes, out, n_pfb, n_coarse, n_time,
                     natural, n_waves);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

// Product remap, packet order -> natural order, one thread per output element:
// natural inputs i >= j sit at packet indices P(i), P(j); the product is
// V_pkt[P(i)][P(j)] when P(i) >= P(j), else the conjugate of V_pkt[P(j)][P(i)].
__global__ void pfb_remap(const int2* src, int2* dst, int n_inputs, int64_t nb, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int64_t f = k / nb, b = k % nb;
    int i, j;
    tri_decode(b, i, j);
    const int pi = (i & ~63) + pfb_pos_of_input(i & 63), pj = (j & ~63) + pfb_pos_of_input(j & 63);
    int2 v;
    if (pi >= pj) {
      v = src[f * nb + tri_index(pi, pj)];
    } else {
      v = src[f * nb + tri_index(pj, pi)];
      v.y = -v.y;
    }
    dst[k] = v;
  }
}

int launch_pfb_remap(const int* src, int* dst, int n_inputs, int n_chan, hipStream_t s) {
  const int64_t nb = tri_index(n_inputs, 0);
  const int64_t n = (int64_t)n_chan * nb;
  const int grid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  hipLaunchKernelGGL(pfb_remap, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, reinterpret_cast<const int2*>(src),
                     reinterpret_cast<int2*>(dst), n_inputs, nb, n);
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
