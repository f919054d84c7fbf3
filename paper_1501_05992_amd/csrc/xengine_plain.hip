// xengine_plain.hip -- X-engine on the vector ALUs only (no matrix cores).
//
// The straightforward formulation of Sec. 3.4.2: every baseline (i, j) of the
// lower triangle accumulates Re and Im of x_i conj(x_j) directly,
//     Re += re_i re_j + im_i im_j,   Im += im_i re_j - re_i im_j,
// tiled over 64 x 64 baselines per workgroup (the m x n tiles of Sec. 3.4.2)
// and 4 x 4 baselines per thread, integrating in registers over the whole
// time range (the register-level integration of Sec. 3.4.2).  Two samples
// are handled per packed-int8 dot product (v_dot4_i32_i8):
//     P = (re(t), im(t), re(t+1), im(t+1)),  Q = (im(t), -re(t), im(t+1), -re(t+1))
//     Re += dot4(P_i, P_j),                   Im += dot4(Q_i, P_j).
// Diagonal tiles are computed in full and only their lower half is written.

#include "corrx_internal.h"

namespace corrx {

namespace {

constexpr int kTile = 64;        // baselines per tile side
constexpr int kPairs = 16;       // sample pairs per staged chunk (32 samples)
constexpr int kThreads = 256;    // 16 x 16 threads, 4 x 4 baselines each

__device__ inline void decode1(uint32_t b, int& re, int& im) {
  int hi = (int)(int8_t)(uint8_t)(b & 0xF0u) >> 4;
  int lo = (int)(int8_t)(uint8_t)(b << 4) >> 4;
  const bool bad = (hi == -8) | (lo == -8);
  re = bad ? 0 : hi;
  im = bad ? 0 : lo;
}

__device__ inline uint32_t pack4(int a, int b, int c, int d) {
  return (uint32_t)(a & 0xFF) | ((uint32_t)(b & 0xFF) << 8) | ((uint32_t)(c & 0xFF) << 16) |
         ((uint32_t)(d & 0xFF) << 24);
}

__device__ inline uint8_t load1(const Problem& p, int f, int t, int i, int t1) {
  if (t >= t1 || i >= p.n_inputs) return 0;
  return p.in[row_offset(p, f, t) + i];
}

}  // namespace

__global__ __launch_bounds__(kThreads) void xmac_plain(Problem p, int ntiles, int nsplit, int tsplit, int mode) {
  __shared__ uint32_t sP[kPairs][kTile];   // row block, P
  __shared__ uint32_t sQ[kPairs][kTile];   // row block, Q
  __shared__ uint32_t sC[kPairs][kTile];   // column block, P

  int u = blockIdx.x;
  const int sp = u % nsplit;
  u /= nsplit;
  const int tile = u % ntiles;
  const int f = u / ntiles;
  // tile -> (I, J), I >= J, row-major over the lower triangle of tiles
  int I = (int)((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while ((I + 1) * (I + 2) / 2 <= tile) ++I;
  while (I * (I + 1) / 2 > tile) --I;
  const int J = tile - I * (I + 1) / 2;
  const int i0 = I * kTile, j0 = J * kTile;
  const int t0 = sp * tsplit, t1 = min(p.n_time, t0 + tsplit);

  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  int re_acc[4][4], im_acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) re_acc[a][b] = im_acc[a][b] = 0;

  // staging role: 128 items (pair, octet) for the row block, 128 for the column block
  const bool rows = tid < 128;
  const int item = tid & 127;
  const int pr = item / 8, oc = item % 8;

  // Eight consecutive inputs of a row as one 8-byte load when the row segment
  // is whole and aligned; byte loads (bounds-checked) otherwise.
  const bool aligned8 = p.n_inputs % 8 == 0 && (reinterpret_cast<uintptr_t>(p.in) & 7) == 0;
  for (int tb = t0; tb < t1; tb += 2 * kPairs) {
    {
      const int base = rows ? i0 : j0;
      const int ta = tb + 2 * pr;
      uint2 w0 = uint2{0, 0}, w1 = uint2{0, 0};
      if (aligned8 && base + 8 * oc + 8 <= p.n_inputs && ta + 1 < t1) {
        const uint8_t* r = p.in + row_offset(p, f, ta) + base + 8 * oc;
        w0 = *reinterpret_cast<const uint2*>(r);
        w1 = *reinterpret_cast<const uint2*>(r + row_offset(p, f, ta + 1) - row_offset(p, f, ta));
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t b0 = load1(p, f, ta, base + 8 * oc + e, t1), b1 = load1(p, f, ta + 1, base + 8 * oc + e, t1);
          if (e < 4) {
            w0.x |= b0 << (8 * e);
            w1.x |= b1 << (8 * e);
          } else {
            w0.y |= b0 << (8 * (e - 4));
            w1.y |= b1 << (8 * (e - 4));
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int il = 8 * oc + e;
        int r0, m0, r1, m1;
        decode1(((e < 4 ? w0.x : w0.y) >> (8 * (e & 3))) & 0xFFu, r0, m0);
        decode1(((e < 4 ? w1.x : w1.y) >> (8 * (e & 3))) & 0xFFu, r1, m1);
        if (rows) {
          sP[pr][il] = pack4(r0, m0, r1, m1);
          sQ[pr][il] = pack4(m0, -r0, m1, -r1);
        } else {
          sC[pr][il] = pack4(r0, m0, r1, m1);
        }
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kPairs; ++k) {
      const uint4 pv = *reinterpret_cast<const uint4*>(&sP[k][4 * tr]);
      const uint4 qv = *reinterpret_cast<const uint4*>(&sQ[k][4 * tr]);
      const uint4 cv = *reinterpret_cast<const uint4*>(&sC[k][4 * tc]);
      const uint32_t P[4] = {pv.x, pv.y, pv.z, pv.w};
      const uint32_t Q[4] = {qv.x, qv.y, qv.z, qv.w};
      const uint32_t C[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          re_acc[a][b] = __builtin_amdgcn_sdot4((int)P[a], (int)C[b], re_acc[a][b], false);
          im_acc[a][b] = __builtin_amdgcn_sdot4((int)Q[a], (int)C[b], im_acc[a][b], false);
        }
    }
    __syncthreads();
  }

  const int64_t nb = tri_index(p.n_inputs, 0);
  int* out = p.acc + (int64_t)f * nb * 2;
  const int wmode = nsplit > 1 ? kWriteAtomic : mode;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + 4 * tr + a, j = j0 + 4 * tc + b;
      if (i >= p.n_inputs || j > i) continue;
      int* o = out + 2 * tri_index(i, j);
      if (wmode == kWriteAtomic) {
        atomicAdd(o, re_acc[a][b]);
        atomicAdd(o + 1, im_acc[a][b]);
      } else if (wmode == kWriteAdd) {
        o[0] += re_acc[a][b];
        o[1] += im_acc[a][b];
      } else {
        o[0] = re_acc[a][b];
        o[1] = im_acc[a][b];
      }
    }
}

int launch_plain(const Problem& p, int nsplit, int mode, hipStream_t s) {
  const int nbk = (p.n_inputs + kTile - 1) / kTile;
  const int ntiles = nbk * (nbk + 1) / 2;
  const int tsplit = (p.n_time + nsplit - 1) / nsplit;
  const int64_t grid = (int64_t)p.n_chan * ntiles * nsplit;
  if (grid > 0x7FFFFFFF) return CORRX_EINVAL;
  hipLaunchKernelGGL(xmac_plain, dim3((unsigned)grid), dim3(kThreads), 0, s, p, ntiles, nsplit, tsplit, mode);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

}  // namespace corrx
