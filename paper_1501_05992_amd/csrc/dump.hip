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
    if (((reinterpret_cast<uintptr_t>(dst)) & 7) == 0) {
      using V2 = typename std::conditional<std::is_same<T, float>::value, float2, int2>::type;
      reinterpret_cast<V2*>(dst)[k] = V2{conv<T>(v.x, scale), conv<T>(v.y, scale)};
    } else {
      dst[2 * k] = conv<T>(v.x, scale);
      dst[2 * k + 1] = conv<T>(v.y, scale);
    }
  }
}

// Station/polarisation order (Appendix C "GPU Output"): one thread per
// (channel group g, station pair bs = s1(s1+1)/2 + s2), writing its four
// polarisation products (p1, p2) = (0,0), (0,1), (1,0), (1,1), complex; the
// inputs are i = 2 s1 + p1, j = 2 s2 + p2, and (s, s, 0, 1) is the conjugate
// of the stored (2s+1, 2s) element.
// VEC: dst is 16-byte aligned and each thread's 32 bytes go out as two
// 16-byte stores.
template <typename T, bool VEC>
__global__ void dump_station_pol(const int2* acc, T* dst, int n_inputs, int64_t n_station_bl, int fa, float scale,
                                 int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nb = tri_index(n_inputs, 0);
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += stride) {
    const int64_t g = o / n_station_bl, bs = o % n_station_bl;
    int s1, s2;
    tri_decode(bs, s1, s2);
    T val[8];
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
        val[4 * p1 + 2 * p2] = conv<T>(v.x, scale);
        val[4 * p1 + 2 * p2 + 1] = conv<T>(v.y, scale);
      }
    T* out = dst + 8 * o;
    if constexpr (VEC) {
      using V4 = typename std::conditional<std::is_same<T, float>::value, float4, int4>::type;
      reinterpret_cast<V4*>(out)[0] = V4{val[0], val[1], val[2], val[3]};
      reinterpret_cast<V4*>(out)[1] = V4{val[4], val[5], val[6], val[7]};
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) out[q] = val[q];
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
  } else if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    if (dtype == CORRX_I32)
      hipLaunchKernelGGL((dump_station_pol<int, true>), g, b, 0, s, a2, reinterpret_cast<int*>(dst), n_inputs, nsb,
                         f_avg, scale, n);
    else
      hipLaunchKernelGGL((dump_station_pol<float, true>), g, b, 0, s, a2, reinterpret_cast<float*>(dst), n_inputs,
                         nsb, f_avg, scale, n);
  } else {
    if (dtype == CORRX_I32)
      hipLaunchKernelGGL((dump_station_pol<int, false>), g, b, 0, s, a2, reinterpret_cast<int*>(dst), n_inputs,
                         nsb, f_avg, scale, n);
    else
      hipLaunchKernelGGL((dump_station_pol<float, false>), g, b, 0, s, a2, reinterpret_cast<float*>(dst),
                         n_inputs, nsb, f_avg, scale, n);
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
// dwords goes to dword 4r + u of the row segment; the dwords are regrouped
// through the wave's own 1 KB of LDS so that every lane stores 16 contiguous
// bytes.
__global__ __launch_bounds__(256) void pfb_ingest(PfbLanes lanes, uint8_t* out, int n_pfb, int n_coarse,
                                                  int n_time, int natural, int64_t n_waves) {
  __shared__ __attribute__((aligned(16))) uint32_t stage[4][256];  // per wave: 4 rows x 64 dwords
  uint32_t* ws = stage[threadIdx.x >> 6];
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
      uint32_t* seg = ws + 64 * f2 + 16 * b;  // row f2, PFB b: 16 dwords
      seg[u] = e0;
      seg[4 + u] = e1;
      seg[8 + u] = e2;
      seg[12 + u] = e3;
      // The LDS unit runs one wave's operations in order; keep the compiler
      // from moving the reads above the writes.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      *reinterpret_cast<uint4*>(row + 16 * u) = reinterpret_cast<const uint4*>(seg)[u];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// Product remap, packet order -> natural order: natural inputs i >= j sit at
// packet indices P(i), P(j); the product is V_pkt[P(i)][P(j)] when
// P(i) >= P(j), else the conjugate of V_pkt[P(j)][P(i)].  One thread per
// baseline decodes (i, j) once and moves it for kRemapChans channels
// (blockIdx.y picks the channel group).
constexpr int kRemapChans = 8;

__global__ void pfb_remap(const int2* src, int2* dst, int n_chan, int64_t nb) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int i, j;
  tri_decode(b, i, j);
  const int pi = (i & ~63) + pfb_pos_of_input(i & 63), pj = (j & ~63) + pfb_pos_of_input(j & 63);
  const bool direct = pi >= pj;
  const int64_t from = direct ? tri_index(pi, pj) : tri_index(pj, pi);
  for (int f0 = blockIdx.y * kRemapChans; f0 < n_chan; f0 += gridDim.y * kRemapChans) {
    const int f1 = min(n_chan, f0 + kRemapChans);
    for (int f = f0; f < f1; ++f) {
      int2 v = src[(int64_t)f * nb + from];
      if (!direct) v.y = -v.y;
      dst[(int64_t)f * nb + b] = v;
    }
  }
}

int launch_pfb_remap(const int* src, int* dst, int n_inputs, int n_chan, hipStream_t s) {
  const int64_t nb = tri_index(n_inputs, 0);
  const int64_t gx = (nb + 255) / 256;
  int64_t gy = (n_chan + kRemapChans - 1) / kRemapChans;
  if (gy > 65535) gy = 65535;
  if (gx > 0x7FFFFFFF) return CORRX_EINVAL;
  hipLaunchKernelGGL(pfb_remap, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s,
                     reinterpret_cast<const int2*>(src), reinterpret_cast<int2*>(dst), n_chan, nb);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

// Incoherent beam: out[f][t] = sum_i |x_i(f,t)|^2, four samples per dword
// through the biased parts u = re + 8, w = im + 8:
//     re^2 + im^2 = u^2 + w^2 - 16 (u + w) + 128.
// General path (any N and alignment): one thread per (f, t) row.
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

// Fast path (N a multiple of 16, 16-byte aligned input): 16 lanes per input
// row, each lane one 16-byte load per 256 bytes of the row, then a 16-lane
// reduction, so that one wave load covers four whole rows.  partial16 gives
// sum (u^2 + w^2 - 16 (u + w)) over the 16 samples of one load; the row adds
// 128 N.  Invalid samples are masked in a branch only such loads take.
__device__ inline int beam_partial16(uint4 v) {
  uint32_t y[4] = {bias4(v.x), bias4(v.y), bias4(v.z), bias4(v.w)};
  if (invalid_flags(y[0]) | invalid_flags(y[1]) | invalid_flags(y[2]) | invalid_flags(y[3])) {
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = mask_invalid(y[k]);
  }
  uint32_t sq = 0, lin = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t u = bre4(y[k]), w = bim4(y[k]);
    sq = __builtin_amdgcn_udot4(u, u, sq, false);
    sq = __builtin_amdgcn_udot4(w, w, sq, false);
    lin = bytesum(u + w, lin);  // u + w <= 30: no carry between bytes
  }
  return (int)(sq - 16u * lin);
}

__device__ inline int beam_reduce16(int part, int n_inputs) {
  part += __shfl_xor(part, 8, 16);
  part += __shfl_xor(part, 4, 16);
  part += __shfl_xor(part, 2, 16);
  part += __shfl_xor(part, 1, 16);
  return part + 128 * n_inputs;
}

// Rows r0, r0 + 16, .., r0 + 16 (R - 1) of this lane's group: all loads are
// issued before any arithmetic.  SMALL (N <= 256): one load per lane and
// row; otherwise a loop over the row's 256-byte pieces.
template <bool SMALL, int R, class RowPtr>
__device__ inline void beam_rows_batch(const RowPtr& row_of, int r0, int n_inputs, int l, int (&v)[R]) {
  if constexpr (SMALL) {
    uint4 x[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
      x[k] = 16 * l < n_inputs ? *reinterpret_cast<const uint4*>(row_of(r0 + 16 * k) + 16 * l) : uint4{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = beam_reduce16(16 * l < n_inputs ? beam_partial16(x[k]) : 0, n_inputs);
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint8_t* row = row_of(r0 + 16 * k);
      int part = 0;
      for (int i = 16 * l; i < n_inputs; i += 256) part += beam_partial16(*reinterpret_cast<const uint4*>(row + i));
      v[k] = beam_reduce16(part, n_inputs);
    }
  }
}

constexpr int kBeamTile = 64;
constexpr int kBeamBatch = 8;  // rows in flight per 16-lane group

// TFI: a block takes 64 channels x 64 times; row (t0 + j, f0 + a) for
// r = 64 j + a, so that neighbouring groups read neighbouring rows; the
// results go through LDS and leave as contiguous runs of out[f][t0 .. t0+63].
template <bool SMALL>
__global__ __launch_bounds__(256) void beam_tfi(Problem p, int* out, int nfb) {
  __shared__ int tile[kBeamTile][kBeamTile + 1];
  const int fb = blockIdx.x % nfb, tb = blockIdx.x / nfb;
  const int f0 = fb * kBeamTile, t0 = tb * kBeamTile;
  const int nf = min(kBeamTile, p.n_chan - f0), nt = min(kBeamTile, p.n_time - t0);
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  // rows outside the array (ragged tiles) read the tile's first row instead
  auto row_of = [&](int r) {
    const int a = r % kBeamTile, j = r / kBeamTile;
    const int64_t m = a < nf && j < nt ? (int64_t)(t0 + j) * p.n_chan + f0 + a : (int64_t)t0 * p.n_chan + f0;
    return p.in + m * p.n_inputs;
  };
  for (int r0 = g; r0 < kBeamTile * kBeamTile; r0 += 16 * kBeamBatch) {
    int v[kBeamBatch];
    beam_rows_batch<SMALL>(row_of, r0, p.n_inputs, l, v);
    if (l == 0) {
#pragma unroll
      for (int k = 0; k < kBeamBatch; ++k) {
        const int r = r0 + 16 * k;
        tile[r % kBeamTile][r / kBeamTile] = v[k];
      }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kBeamTile * kBeamTile; idx += 256) {
    const int a = idx / kBeamTile, j = idx % kBeamTile;
    if (a < nf && j < nt) out[(int64_t)(f0 + a) * p.n_time + t0 + j] = tile[a][j];
  }
}

// FTI: memory row m = f T + t is also the output index.  Rows past the end
// read the last row and are not stored.
template <bool SMALL>
__global__ __launch_bounds__(256) void beam_fti(Problem p, int* out, int64_t nrows) {
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  const int64_t step = (int64_t)gridDim.x * 16 * kBeamBatch;
  for (int64_t m0 = (int64_t)blockIdx.x * 16 * kBeamBatch; m0 < nrows; m0 += step) {
    auto row_of = [&](int r) { return p.in + min(m0 + r, nrows - 1) * p.n_inputs; };
    int v[kBeamBatch];
    beam_rows_batch<SMALL>(row_of, g, p.n_inputs, l, v);
    if (l == 0) {
#pragma unroll
      for (int k = 0; k < kBeamBatch; ++k)
        if (m0 + g + 16 * k < nrows) out[m0 + g + 16 * k] = v[k];
    }
  }
}

int launch_beam(const Problem& p, int* out, hipStream_t s) {
  const int64_t nrows = (int64_t)p.n_chan * p.n_time;
  if (nrows == 0) return CORRX_OK;
  const bool fast = p.n_inputs % 16 == 0 && (reinterpret_cast<uintptr_t>(p.in) & 15) == 0;
  const bool small = p.n_inputs <= 256;
  if (fast && p.layout == CORRX_LAYOUT_TFI) {
    const int64_t nfb = (p.n_chan + kBeamTile - 1) / kBeamTile, ntb = (p.n_time + kBeamTile - 1) / kBeamTile;
    if (nfb * ntb > 0x7FFFFFFF) return CORRX_EINVAL;
    if (small)
      hipLaunchKernelGGL(beam_tfi<true>, dim3((unsigned)(nfb * ntb)), dim3(256), 0, s, p, out, (int)nfb);
    else
      hipLaunchKernelGGL(beam_tfi<false>, dim3((unsigned)(nfb * ntb)), dim3(256), 0, s, p, out, (int)nfb);
  } else if (fast) {
    const int64_t blocks = (nrows + 16 * kBeamBatch - 1) / (16 * kBeamBatch);
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    if (small)
      hipLaunchKernelGGL(beam_fti<true>, dim3(grid), dim3(256), 0, s, p, out, nrows);
    else
      hipLaunchKernelGGL(beam_fti<false>, dim3(grid), dim3(256), 0, s, p, out, nrows);
  } else {
    const int grid = (int)((nrows + 255) / 256 < 16384 ? (nrows + 255) / 256 : 16384);
    hipLaunchKernelGGL(beam_rows, dim3(grid), dim3(256), 0, s, p, out, nrows);
  }
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

}  // namespace corrx
