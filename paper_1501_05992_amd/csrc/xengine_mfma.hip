// xengine_mfma.hip -- int8 MFMA X-engine for gfx950 (CDNA4).
//
// Operation (Ord et al. Sec. 2 eq. (3), Sec. 3.4.2, Appendix C): for every
// channel, V[i][j] = sum_t x_i(t) conj(x_j(t)) over the lower triangle i >= j.
//
// Formulation.  Write x = re + j*im with 4-bit parts and the biased parts
// u = re + 8, w = im + 8 (0..15).  For each sample form the two real K-pairs
//     A_i = (u_i, w_i)                   0..15
//     B_j = (u_j + w_j, w_j - u_j + 15)  0..30
// and the real product G_b = A B^T over K = 2T (one int8 GEMM, N x N).  With
// G[i][j] = Re V_ij - Im V_ij (the unbiased product), G[j][i] = Re V_ij + Im V_ij,
// so one full square yields both parts of every baseline with no triangle waste:
//     2 Re V_ij = G_b[i][j] + G_b[j][i] - e_i - e_j + 256 T
//     2 Im V_ij = G_b[j][i] - G_b[i][j] + g_i - g_j
// where, with Sy_k = sum_t (16 u_k + w_k) and Sw_k = sum_t w_k over the T
// processed samples, e_k = Sy_k + 30 Sw_k and g_k = Sy_k - 2 Sw_k.  Both
// identities are exact integer algebra; every sum stays inside int32 for
// T <= 2^20 samples per work unit.
//
// Kernel structure (one workgroup = one channel x one time range, the
// "diagonal unit" of NB inputs):
//   - global -> registers: each thread loads 16 time rows x 4 inputs as dwords
//     (lanes cover consecutive inputs of one row: coalesced), one chunk of TC
//     samples ahead of the chunk being multiplied;
//   - registers -> LDS: 4x4 byte transposes (time-major -> input-major), bias,
//     invalid-code masking (rare path), split into A-operand bytes
//     [u(t..t+3), w(t..t+3), u(t+4..t+7), w(t+4..t+7)] per 16-byte chunk, XOR
//     swizzled across rows to keep ds_write_b128 / ds_read_b128 conflict-free;
//   - LDS -> MFMA: each wave owns a WT x WT block of G_b in AGPR/VGPR
//     accumulators (v_mfma_i32_32x32x32_i8); row fragments are read as
//     A-operands, column fragments are read and converted to B-operands in
//     registers (3 ALU ops per 4 samples);
//   - epilogue: per-input sums reduced in LDS, mirror blocks exchanged through
//     LDS so that each lower-triangle element meets its transpose, then
//     acc += (Re, Im) (plain read-modify-write, or atomics for time splits).

#include "corrx_internal.h"

namespace corrx {

template <int NB, int TC>
struct Diag {
  static constexpr int WT = NB >= 128 ? 128 : NB;  // wave tile side
  static constexpr int WG = NB / WT;               // waves per side
  static constexpr int NW = WG * WG;               // waves per workgroup
  static constexpr int NT = 64 * NW;               // threads per workgroup
  static constexpr int TPW = WT / 32;              // 32x32 MFMA tiles per wave side
  static constexpr int ROWB = 2 * TC;              // staged bytes per input and chunk
  static constexpr int CHUNKS = ROWB / 16;         // 16-byte chunks per row
  static constexpr int KSTEPS = TC / 16;           // K=32 (16-sample) MFMA steps per chunk
  static constexpr int QUADS = NB / 4;
  static constexpr int SLABS = TC / 16;
  static constexpr int ITEMS = QUADS * SLABS;
  static constexpr int ITER = ITEMS / NT;          // unpack items per thread and chunk
  static constexpr int STAGE = NB * ROWB;          // bytes of one stage buffer
  static constexpr int XPITCH = WT + 1;
  static constexpr int XAREA = WT * XPITCH;        // int32 words of one exchange area
  static constexpr int NXAREA = WG == 2 ? 2 : 1;
  static constexpr int LDS = (2 * STAGE > NXAREA * XAREA * 4) ? 2 * STAGE : NXAREA * XAREA * 4;
  static_assert(ITER >= 1 && ITEMS % NT == 0, "unpack work must divide evenly");
  static_assert(NT == (NB >= 256 ? 256 : 64), "thread count must match the launch bounds");
  static_assert(CHUNKS == 8 || CHUNKS == 4, "swizzle assumes 4 or 8 chunks per row");
};

// Row-dependent XOR swizzle of 16-byte chunks: conflict-free for the unpack
// writes (rows 4l + c across lanes) and the fragment reads (rows r0 + m).
template <int CHUNKS>
__device__ inline int swz(int row) {
  return (row ^ (row >> 2)) & (CHUNKS - 1);
}

// Map the hardware workgroup id so that consecutive logical units land on the
// same XCD (ids are dealt round-robin over 8 XCDs): neighbouring channels then
// share an L2.
__device__ inline int xcd_remap(int b, int n) {
  if (n % 8) return b;
  return (b % 8) * (n / 8) + b / 8;
}

template <int NB, int TC>
struct DiagUnit {
  using D = Diag<NB, TC>;

  // Load chunk c of the unit into registers.
  //   ALIGNED (N % 4 == 0, 4-byte aligned buffer): raw buffer loads through a
  //   descriptor that starts at the chunk's first row and ends at the end of
  //   the channel's last valid row, so rows past the unit's time range read 0
  //   in hardware; quads past N use an out-of-range offset.  No branch and no
  //   select follows a load, so all 16 loads stay in flight.
  //   Otherwise: byte loads (slow path).
  template <bool ALIGNED>
  __device__ static void load_chunk(const Problem& p, int f, int t0, int t1, int c, int64_t stride,
                                    uint32_t (&ld)[D::ITER][16]) {
    const int tb = t0 + c * TC;
    if constexpr (ALIGNED) {
      const int rows = min(t1 - tb, TC);
      const uint32_t nrec = (uint32_t)((rows - 1) * stride + p.n_inputs);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t*>(p.in + row_offset(p, f, tb)), (short)0, (int)nrec, kBufferRsrcWord3);
#pragma unroll
      for (int k = 0; k < D::ITER; ++k) {
        const int item = threadIdx.x + k * D::NT;
        const int q = item % D::QUADS, s = item / D::QUADS;
        const uint32_t off0 = 4 * q < p.n_inputs ? (uint32_t)(16 * s * stride + 4 * q) : 0x80000000u;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          ld[k][r] = __builtin_amdgcn_raw_buffer_load_b32(rs, off0 + (uint32_t)(r * stride), 0, 0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < D::ITER; ++k) {
        const int item = threadIdx.x + k * D::NT;
        const int q = item % D::QUADS, s = item / D::QUADS;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int t = tb + 16 * s + r;
          uint32_t v = 0;
          if (t < t1) {
            const uint8_t* row = p.in + row_offset(p, f, t);
            for (int b = 0; b < 4; ++b)
              if (4 * q + b < p.n_inputs) v |= uint32_t(row[4 * q + b]) << (8 * b);
          }
          ld[k][r] = v;
        }
      }
    }
  }

  // Transpose, bias, mask and store one chunk into a stage buffer; accumulate
  // per-input byte sums.
  __device__ static void unpack_store(const uint32_t (&ld)[D::ITER][16], uint8_t* st,
                                      uint32_t (&sy)[D::ITER][4], uint32_t (&sw)[D::ITER][4]) {
#pragma unroll
    for (int k = 0; k < D::ITER; ++k) {
      const int item = threadIdx.x + k * D::NT;
      const int q = item % D::QUADS, s = item / D::QUADS;
      uint32_t y[4][4];  // [time quad][input c]
#pragma unroll
      for (int tq = 0; tq < 4; ++tq) {
        uint32_t e0, e1, e2, e3;
        transpose4x4(ld[k][4 * tq], ld[k][4 * tq + 1], ld[k][4 * tq + 2], ld[k][4 * tq + 3], e0, e1, e2, e3);
        y[tq][0] = bias4(e0);
        y[tq][1] = bias4(e1);
        y[tq][2] = bias4(e2);
        y[tq][3] = bias4(e3);
      }
      uint32_t bad = 0;
#pragma unroll
      for (int tq = 0; tq < 4; ++tq)
#pragma unroll
        for (int c = 0; c < 4; ++c) bad |= invalid_flags(y[tq][c]);
      if (bad) {
#pragma unroll
        for (int tq = 0; tq < 4; ++tq)
#pragma unroll
          for (int c = 0; c < 4; ++c) y[tq][c] = mask_invalid(y[tq][c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int row = 4 * q + c;
        uint32_t r8[4], i8[4];
#pragma unroll
        for (int tq = 0; tq < 4; ++tq) {
          r8[tq] = bre4(y[tq][c]);
          i8[tq] = bim4(y[tq][c]);
          sy[k][c] = bytesum(y[tq][c], sy[k][c]);
          sw[k][c] = bytesum(i8[tq], sw[k][c]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int chunk = 2 * s + h;
          v4i v;
          v.x = (int)r8[2 * h];
          v.y = (int)i8[2 * h];
          v.z = (int)r8[2 * h + 1];
          v.w = (int)i8[2 * h + 1];
          *reinterpret_cast<v4i*>(st + row * D::ROWB + ((chunk ^ swz<D::CHUNKS>(row)) << 4)) = v;
        }
      }
    }
  }

  __device__ static v4i read_frag(const uint8_t* st, int row, int chunk) {
    return *reinterpret_cast<const v4i*>(st + row * D::ROWB + ((chunk ^ swz<D::CHUNKS>(row)) << 4));
  }

  __device__ static v4i to_b(v4i a) {
    v4i b;
    b.x = (int)op_s((uint32_t)a.x, (uint32_t)a.y);
    b.y = (int)op_d((uint32_t)a.x, (uint32_t)a.y);
    b.z = (int)op_s((uint32_t)a.z, (uint32_t)a.w);
    b.w = (int)op_d((uint32_t)a.z, (uint32_t)a.w);
    return b;
  }

  // Row (within a 32x32 tile) held by accumulator register r of this lane.
  __device__ static int acc_row(int r, int lane) { return ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3); }

  __device__ static void store_block(int* xa, const v16i (&acc)[D::TPW][D::TPW], int lane) {
#pragma unroll
    for (int x = 0; x < D::TPW; ++x)
#pragma unroll
      for (int y = 0; y < D::TPW; ++y)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          xa[(32 * x + acc_row(r, lane)) * D::XPITCH + 32 * y + (lane & 31)] = acc[x][y][r];
  }

  // All threads: combine the block of G_b at rows ib.., columns jb.. (in `own`)
  // with its mirror block at rows jb.., columns ib.. (in `mir`; the same area
  // for a diagonal block) and add the lower triangle into the accumulator.
  __device__ static void combine(const Problem& p, int f, const int* own, const int* mir, int ib, int jb,
                                 const uint32_t* s_sy, const uint32_t* s_sw, uint32_t tproc, bool atomic) {
    const int64_t nb = tri_index(p.n_inputs, 0);
    int* out = p.acc + (int64_t)f * nb * 2;
    for (int idx = threadIdx.x; idx < D::WT * D::WT; idx += D::NT) {
      const int il = idx / D::WT, jl = idx % D::WT;
      const int i = ib + il, j = jb + jl;
      if (i < j || i >= p.n_inputs) continue;
      const uint32_t gij = (uint32_t)own[il * D::XPITCH + jl];
      const uint32_t gji = (uint32_t)mir[jl * D::XPITCH + il];
      const uint32_t syi = s_sy[i], swi = s_sw[i], syj = s_sy[j], swj = s_sw[j];
      const uint32_t ei = syi + 30u * swi, ej = syj + 30u * swj;
      const uint32_t gi = syi - 2u * swi, gj = syj - 2u * swj;
      const int re2 = (int)(gij + gji - ei - ej + 256u * tproc);
      const int im2 = (int)(gji - gij + gi - gj);
      int* o = out + 2 * tri_index(i, j);
      if (atomic) {
        atomicAdd(o, re2 >> 1);
        atomicAdd(o + 1, im2 >> 1);
      } else {
        int2 v = *reinterpret_cast<int2*>(o);
        v.x += re2 >> 1;
        v.y += im2 >> 1;
        *reinterpret_cast<int2*>(o) = v;
      }
    }
  }
};

template <int NB>
constexpr int diag_threads = NB >= 256 ? 256 : 64;

template <int NB, int TC, bool ALIGNED>
__global__ __launch_bounds__(diag_threads<NB>, 1) void xmac_diag_i8(Problem p, int nsplit, int tsplit) {
  using D = Diag<NB, TC>;
  using U = DiagUnit<NB, TC>;
  __shared__ __attribute__((aligned(16))) uint8_t lds[D::LDS];
  __shared__ uint32_t s_sy[NB], s_sw[NB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / D::WG, wc = wave % D::WG;
  const int u = xcd_remap(blockIdx.x, gridDim.x);
  const int f = u / nsplit, sp = u % nsplit;
  const int t0 = sp * tsplit;
  const int t1 = min(p.n_time, t0 + tsplit);
  const int nchunks = t1 > t0 ? (t1 - t0 + TC - 1) / TC : 0;
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;

  for (int k = tid; k < NB; k += D::NT) {
    s_sy[k] = 0;
    s_sw[k] = 0;
  }

  v16i acc[D::TPW][D::TPW];
#pragma unroll
  for (int x = 0; x < D::TPW; ++x)
#pragma unroll
    for (int y = 0; y < D::TPW; ++y) acc[x][y] = v16i{0};
  uint32_t sy[D::ITER][4], sw[D::ITER][4];
#pragma unroll
  for (int k = 0; k < D::ITER; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) sy[k][c] = sw[k][c] = 0;

  uint32_t ld[D::ITER][16];
  if (nchunks > 0) {
    U::template load_chunk<ALIGNED>(p, f, t0, t1, 0, stride, ld);
    U::unpack_store(ld, lds, sy, sw);
  }
  __syncthreads();

  for (int c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) U::template load_chunk<ALIGNED>(p, f, t0, t1, c + 1, stride, ld);
    const uint8_t* st = lds + (c & 1) * D::STAGE;
#pragma unroll
    for (int ks = 0; ks < D::KSTEPS; ++ks) {
      const int chunk = 2 * ks + (lane >> 5);
      v4i a[D::TPW], b[D::TPW];
#pragma unroll
      for (int x = 0; x < D::TPW; ++x) a[x] = U::read_frag(st, wr * D::WT + 32 * x + (lane & 31), chunk);
      if (wr == wc) {
#pragma unroll
        for (int y = 0; y < D::TPW; ++y) b[y] = U::to_b(a[y]);
      } else {
#pragma unroll
        for (int y = 0; y < D::TPW; ++y)
          b[y] = U::to_b(U::read_frag(st, wc * D::WT + 32 * y + (lane & 31), chunk));
      }
#pragma unroll
      for (int x = 0; x < D::TPW; ++x)
#pragma unroll
        for (int y = 0; y < D::TPW; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (more) U::unpack_store(ld, lds + ((c + 1) & 1) * D::STAGE, sy, sw);
    __syncthreads();
  }

  // Per-input sums of this unit.
#pragma unroll
  for (int k = 0; k < D::ITER; ++k) {
    const int q = (tid + k * D::NT) % D::QUADS;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      atomicAdd(&s_sy[4 * q + c], sy[k][c]);
      atomicAdd(&s_sw[4 * q + c], sw[k][c]);
    }
  }
  __syncthreads();

  const uint32_t tproc = (uint32_t)(nchunks * TC);
  const bool atomic = nsplit > 1;
  int* xa = reinterpret_cast<int*>(lds);
  int* xb = xa + (D::NXAREA - 1) * D::XAREA;
  if (D::WG == 1) {
    U::store_block(xa, acc, lane);
    __syncthreads();
    U::combine(p, f, xa, xa, 0, 0, s_sy, s_sw, tproc, atomic);
  } else {
    // Off-diagonal quadrant (1,0) against its mirror (0,1).
    if (wave == 1) U::store_block(xa, acc, lane);
    if (wave == 2) U::store_block(xb, acc, lane);
    __syncthreads();
    U::combine(p, f, xb, xa, D::WT, 0, s_sy, s_sw, tproc, atomic);
    __syncthreads();
    // Diagonal quadrants (0,0) and (1,1), each against itself.
    if (wave == 0) U::store_block(xa, acc, lane);
    if (wave == 3) U::store_block(xb, acc, lane);
    __syncthreads();
    U::combine(p, f, xa, xa, 0, 0, s_sy, s_sw, tproc, atomic);
    U::combine(p, f, xb, xb, D::WT, D::WT, s_sy, s_sw, tproc, atomic);
  }
}

template <int NB, int TC>
static int launch_diag(const Problem& p, int nsplit, hipStream_t s) {
  using D = Diag<NB, TC>;
  const int tsplit = (p.n_time + nsplit - 1) / nsplit;
  const int64_t grid = (int64_t)p.n_chan * nsplit;
  if (grid > 0x7FFFFFFF) return CORRX_EINVAL;
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;
  const bool aligned = (p.n_inputs % 4 == 0) && ((reinterpret_cast<uintptr_t>(p.in) & 3) == 0) &&
                       (int64_t)TC * stride + p.n_inputs < 0x7FFFFFFF;
  if (aligned)
    hipLaunchKernelGGL((xmac_diag_i8<NB, TC, true>), dim3((unsigned)grid), dim3(D::NT), 0, s, p, nsplit, tsplit);
  else
    hipLaunchKernelGGL((xmac_diag_i8<NB, TC, false>), dim3((unsigned)grid), dim3(D::NT), 0, s, p, nsplit, tsplit);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

int launch_mfma(const Problem& p, int engine, int nsplit, int tile_cfg, hipStream_t s) {
  if (engine != CORRX_ENGINE_MFMA_I8) return CORRX_EUNSUPPORTED;
  (void)tile_cfg;
  if (p.n_inputs <= 64) return launch_diag<64, 64>(p, nsplit, s);
  if (p.n_inputs <= 128) return launch_diag<128, 64>(p, nsplit, s);
  if (p.n_inputs <= 256) return launch_diag<256, 64>(p, nsplit, s);
  return CORRX_EUNSUPPORTED;
}

}  // namespace corrx
