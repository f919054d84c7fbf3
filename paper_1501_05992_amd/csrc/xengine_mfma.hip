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
// "diagonal unit" of NB inputs, 2 x WC waves, two waves per SIMD so that one
// wave's vector-ALU and LDS work overlaps the other's MFMAs):
//   - global -> registers: raw buffer loads of 8 time rows x 4 inputs per
//     thread (lanes cover consecutive inputs of one row: coalesced), one chunk
//     of TC samples ahead of the chunk being multiplied; rows past the time
//     range read 0 through the buffer descriptor's range check;
//   - registers -> LDS: 4x4 byte transposes (time-major -> input-major), bias,
//     A-operand bytes [u(t..t+3), w(t..t+3), u(t+4..t+7), w(t+4..t+7)] per
//     16-byte chunk, XOR swizzled across rows for conflict-free ds_write_b128 /
//     ds_read_b128; invalid codes only raise a flag, and a rare fix-up pass
//     over the stage buffer zeroes those samples;
//   - LDS -> MFMA: each wave owns a (NB/2) x (NB/WC) block of G_b in
//     accumulators (v_mfma_i32_32x32x32_i8); row fragments are read as
//     A-operands, column fragments are read and converted to B-operands in
//     registers (3 ALU ops per 4 samples); the unpack of the next chunk is
//     split into phases placed between the K-steps;
//   - epilogue: per-input sums reduced in LDS, quadrants of G_b exchanged
//     through LDS so that each lower-triangle element meets its transpose,
//     then acc += (Re, Im) (read-modify-write, or atomics for time splits).

#include "corrx_internal.h"

namespace corrx {

template <int NB, int TC, int WC>
struct Diag {
  static constexpr int WR = 2;                       // wave rows
  static constexpr int NW = WR * WC;                 // waves per workgroup
  static constexpr int NT = 64 * NW;                 // threads per workgroup
  static constexpr int TM = NB / WR;                 // wave tile rows
  static constexpr int TN = NB / WC;                 // wave tile columns
  static constexpr int FM = TM / 32;                 // 32x32 MFMA tiles along rows
  static constexpr int FN = TN / 32;                 // ... along columns
  static constexpr int ROWB = 2 * TC;                // staged bytes per input and chunk
  static constexpr int CHUNKS = ROWB / 16;           // 16-byte chunks per row (8 samples each)
  static constexpr int KSTEPS = TC / 16;             // K=32 (16-sample) MFMA steps per chunk
  static constexpr int QUADS = NB / 4;
  static constexpr int GROUPS = TC / 8;              // 8-row groups per chunk
  static constexpr int ITEMS = QUADS * GROUPS;       // unpack items (8 rows x 4 inputs)
  static constexpr int ITER = ITEMS >= NT ? ITEMS / NT : 1;
  static constexpr bool PARTIAL = ITEMS < NT;        // some threads idle in the unpack
  static constexpr int STAGE = NB * ROWB;            // bytes of one stage buffer
  static constexpr int H = NB / 2;                   // quadrant side
  static constexpr int XPITCH = H + 1;
  static constexpr int XAREA = H * XPITCH;           // int32 words of one exchange area
  static constexpr int LDS = (2 * STAGE > 2 * XAREA * 4) ? 2 * STAGE : 2 * XAREA * 4;
  static_assert(TM % 32 == 0 && TN % 32 == 0, "wave tiles are made of 32x32 MFMA tiles");
  static_assert(PARTIAL || ITEMS % NT == 0, "unpack work must divide evenly");
  static_assert(KSTEPS == 4, "the unpack is split into four phases, one per K-step");
  static_assert(CHUNKS == 8, "swizzle assumes 8 chunks per row");
  static_assert(WC % 2 == 0, "quadrants are made of whole wave tiles");
};

// Row-dependent XOR swizzle of 16-byte chunks: conflict-free for the unpack
// writes (rows 4l + c across lanes) and the fragment reads (rows r0 + m).
__device__ inline int swz(int row) { return (row ^ (row >> 2)) & 7; }

// Map the hardware workgroup id so that consecutive logical units land on the
// same XCD (ids are dealt round-robin over 8 XCDs): neighbouring channels then
// share an L2.
__device__ inline int xcd_remap(int b, int n) {
  if (n % 8) return b;
  return (b % 8) * (n / 8) + b / 8;
}

template <int NB, int TC, int WC>
struct DiagUnit {
  using D = Diag<NB, TC, WC>;

  __device__ static bool has_item(int k) { return !D::PARTIAL || (int)threadIdx.x + k * D::NT < D::ITEMS; }

  // Load the 8 rows x 4 inputs of this thread's unpack items of chunk c.
  //   ALIGNED (N % 4 == 0, 4-byte aligned buffer): raw buffer loads through a
  //   descriptor that starts at the chunk's first row and ends at the end of
  //   the channel's last valid row, so rows past the unit's time range read 0
  //   in hardware; quads past N use an out-of-range offset.  No branch and no
  //   select follows a load, so all loads stay in flight.
  //   Otherwise: byte loads (slow path).
  template <bool ALIGNED>
  __device__ static void load_chunk(const Problem& p, int f, int t0, int t1, int c, int64_t stride,
                                    uint32_t (&ld)[D::ITER][8]) {
    const int tb = t0 + c * TC;
    if constexpr (ALIGNED) {
      const int rows = min(t1 - tb, TC);
      const uint32_t nrec = (uint32_t)((rows - 1) * stride + p.n_inputs);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t*>(p.in + row_offset(p, f, tb)), (short)0, (int)nrec, kBufferRsrcWord3);
#pragma unroll
      for (int k = 0; k < D::ITER; ++k) {
        const int item = threadIdx.x + k * D::NT;
        const int q = item % D::QUADS, g = item / D::QUADS;
        const uint32_t off0 =
            (4 * q < p.n_inputs && has_item(k)) ? (uint32_t)(8 * g * stride + 4 * q) : 0x80000000u;
#pragma unroll
        for (int r = 0; r < 8; ++r)
          ld[k][r] = __builtin_amdgcn_raw_buffer_load_b32(rs, off0 + (uint32_t)(r * stride), 0, 0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < D::ITER; ++k) {
        const int item = threadIdx.x + k * D::NT;
        const int q = item % D::QUADS, g = item / D::QUADS;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int t = tb + 8 * g + r;
          uint32_t v = 0;
          if (t < t1 && has_item(k)) {
            const uint8_t* row = p.in + row_offset(p, f, t);
            for (int b = 0; b < 4; ++b)
              if (4 * q + b < p.n_inputs) v |= uint32_t(row[4 * q + b]) << (8 * b);
          }
          ld[k][r] = v;
        }
      }
    }
  }

  // Unpack of one chunk, in four phases (one per K-step of the previous
  // chunk).  Phases 0/1: transpose rows 0-3 / 4-7 (time-major -> input-major)
  // and bias; phases 2/3: inputs 0-1 / 2-3 of each quad -- byte sums and one
  // 16-byte store per input [u(4), w(4), u(4), w(4)].  Invalid codes only set
  // `bad`; a later fix-up pass zeroes those samples.
  template <int PH>
  __device__ static void unpack_phase(const uint32_t (&ld)[D::ITER][8], uint32_t (&y)[D::ITER][8], uint8_t* st,
                                      uint32_t (&sy)[D::ITER][4], uint32_t (&sw)[D::ITER][4], uint32_t& bad) {
#pragma unroll
    for (int k = 0; k < D::ITER; ++k) {
      if (!has_item(k)) continue;
      if constexpr (PH < 2) {
        uint32_t e0, e1, e2, e3;
        transpose4x4(ld[k][4 * PH], ld[k][4 * PH + 1], ld[k][4 * PH + 2], ld[k][4 * PH + 3], e0, e1, e2, e3);
        // y[k][2*c + PH]: input c, time quad PH
        y[k][PH] = bias4(e0);
        y[k][2 + PH] = bias4(e1);
        y[k][4 + PH] = bias4(e2);
        y[k][6 + PH] = bias4(e3);
#pragma unroll
        for (int c = 0; c < 4; ++c) bad |= (y[k][2 * c + PH] - 0x11111111u) & ~y[k][2 * c + PH];
      } else {
        const int item = threadIdx.x + k * D::NT;
        const int q = item % D::QUADS, g = item / D::QUADS;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          const int c = 2 * (PH - 2) + cc;
          const int row = 4 * q + c;
          const uint32_t ya = y[k][2 * c], yb = y[k][2 * c + 1];
          const uint32_t ra = bre4(ya), ia = bim4(ya), rb = bre4(yb), ib = bim4(yb);
          sy[k][c] = bytesum(yb, bytesum(ya, sy[k][c]));
          sw[k][c] = bytesum(ib, bytesum(ia, sw[k][c]));
          v4i v;
          v.x = (int)ra;
          v.y = (int)ia;
          v.z = (int)rb;
          v.w = (int)ib;
          *reinterpret_cast<v4i*>(st + row * D::ROWB + ((g ^ swz(row)) << 4)) = v;
        }
      }
    }
  }

  __device__ static void unpack_all(const uint32_t (&ld)[D::ITER][8], uint8_t* st, uint32_t (&sy)[D::ITER][4],
                                    uint32_t (&sw)[D::ITER][4], uint32_t& bad) {
    uint32_t y[D::ITER][8];
    unpack_phase<0>(ld, y, st, sy, sw, bad);
    unpack_phase<1>(ld, y, st, sy, sw, bad);
    unpack_phase<2>(ld, y, st, sy, sw, bad);
    unpack_phase<3>(ld, y, st, sy, sw, bad);
  }

  // Rare path: replace every invalid sample of a stage buffer (a biased part
  // of 0, i.e. the code 8) by a zero sample (u = w = 8) and correct the
  // per-input sums.  All threads of the workgroup take part.
  __device__ static void fixup_invalid(uint8_t* st, uint32_t* s_sy, uint32_t* s_sw) {
    for (int gi = threadIdx.x; gi < NB * D::ROWB / 8; gi += D::NT) {
      uint2* gp = reinterpret_cast<uint2*>(st) + gi;
      uint2 v = *gp;
      const uint32_t ok = (v.x + 0x7F7F7F7Fu) & (v.y + 0x7F7F7F7Fu) & 0x80808080u;
      if (ok == 0x80808080u) continue;
      const int row = (gi * 8) / D::ROWB;
      uint32_t dy = 0, dw = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if ((ok >> (8 * b + 7)) & 1u) continue;
        const uint32_t u = (v.x >> (8 * b)) & 0xFFu, w = (v.y >> (8 * b)) & 0xFFu;
        dy += 136u - (16u * u + w);
        dw += 8u - w;
        v.x = (v.x & ~(0xFFu << (8 * b))) | (8u << (8 * b));
        v.y = (v.y & ~(0xFFu << (8 * b))) | (8u << (8 * b));
      }
      *gp = v;
      atomicAdd(&s_sy[row], dy);
      atomicAdd(&s_sw[row], dw);
    }
  }

  // End of an unpack: raise the workgroup flag of stage buffer `slot` if any
  // lane saw an invalid code.
  __device__ static void publish_bad(uint32_t bad, uint32_t* s_bad, int slot) {
    if (__any((bad & 0x88888888u) != 0u) && (threadIdx.x & 63) == 0) s_bad[slot] = 1u;
  }

  // After the barrier that ends an unpack: fix the stage buffer if flagged.
  __device__ static void check_bad(uint8_t* st, uint32_t* s_bad, int slot, uint32_t* s_sy, uint32_t* s_sw) {
    if (s_bad[slot]) {
      fixup_invalid(st, s_sy, s_sw);
      __syncthreads();
      if (threadIdx.x == 0) s_bad[slot] = 0u;
    }
  }

  __device__ static v4i read_frag(const uint8_t* st, int row, int chunk) {
    return *reinterpret_cast<const v4i*>(st + row * D::ROWB + ((chunk ^ swz(row)) << 4));
  }

  __device__ static v4i to_b(v4i a) {
    v4i b;
    b.x = (int)op_s((uint32_t)a.x, (uint32_t)a.y);
    b.y = (int)op_d((uint32_t)a.x, (uint32_t)a.y);
    b.z = (int)op_s((uint32_t)a.z, (uint32_t)a.w);
    b.w = (int)op_d((uint32_t)a.z, (uint32_t)a.w);
    return b;
  }

  // One chunk of the main loop: the MFMAs of chunk c from its stage buffer,
  // with the four unpack phases of chunk c+1 (held in `ld`) into the other
  // stage buffer placed between the K-steps, and the loads of chunk c+2 issued
  // once `ld` is consumed.  MORE1 / MORE2: chunks c+1 / c+2 exist.  Ends with a
  // barrier (and the rare invalid-code fix-up of the new stage buffer).
  template <bool ALIGNED, bool MORE1, bool MORE2>
  __device__ static void chunk_step(const Problem& p, int f, int t0, int t1, int c, int64_t stride, uint8_t* lds,
                                    int rrow, int crow, uint32_t (&ld)[D::ITER][8], v16i (&acc)[D::FM][D::FN],
                                    uint32_t (&sy)[D::ITER][4], uint32_t (&sw)[D::ITER][4], uint32_t* s_bad,
                                    uint32_t* s_sy, uint32_t* s_sw) {
    const int half = (threadIdx.x & 63) >> 5;
    const uint8_t* st = lds + (c & 1) * D::STAGE;
    uint8_t* nst = lds + ((c + 1) & 1) * D::STAGE;
    uint32_t bad = 0;
    uint32_t y[D::ITER][8];
#pragma unroll
    for (int ks = 0; ks < D::KSTEPS; ++ks) {
      v4i a[D::FM], b[D::FN];
#pragma unroll
      for (int x = 0; x < D::FM; ++x) a[x] = read_frag(st, rrow + 32 * x, 2 * ks + half);
#pragma unroll
      for (int x = 0; x < D::FN; ++x) b[x] = to_b(read_frag(st, crow + 32 * x, 2 * ks + half));
#pragma unroll
      for (int x = 0; x < D::FM; ++x)
#pragma unroll
        for (int z = 0; z < D::FN; ++z)
          acc[x][z] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[x], b[z], acc[x][z], 0, 0, 0);
      if constexpr (MORE1) {
        if (ks == 0) unpack_phase<0>(ld, y, nst, sy, sw, bad);
        if (ks == 1) unpack_phase<1>(ld, y, nst, sy, sw, bad);
        if (ks == 2) unpack_phase<2>(ld, y, nst, sy, sw, bad);
        if (ks == 3) unpack_phase<3>(ld, y, nst, sy, sw, bad);
      }
      if constexpr (MORE2) {
        if (ks == 1) load_chunk<ALIGNED>(p, f, t0, t1, c + 2, stride, ld);
      }
    }
    if constexpr (MORE1) publish_bad(bad, s_bad, (c + 1) & 1);
    __syncthreads();
    if constexpr (MORE1) check_bad(nst, s_bad, (c + 1) & 1, s_sy, s_sw);
  }

  // Row (within a 32x32 tile) held by accumulator register r of this lane.
  __device__ static int acc_row(int r, int lane) { return ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3); }

  // Write this wave's tile into an exchange area at column offset col0.
  __device__ static void store_tile(int* xa, int col0, const v16i (&acc)[D::FM][D::FN], int lane) {
#pragma unroll
    for (int x = 0; x < D::FM; ++x)
#pragma unroll
      for (int z = 0; z < D::FN; ++z)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          xa[(32 * x + acc_row(r, lane)) * D::XPITCH + col0 + 32 * z + (lane & 31)] = acc[x][z][r];
  }

  // All threads: combine the quadrant of G_b at rows ib.., columns jb.. (in
  // `own`) with its mirror quadrant at rows jb.., columns ib.. (in `mir`; the
  // same area for a diagonal quadrant) and write the lower triangle into the
  // accumulator.  s_e / s_g: per-input correction terms.  Eight elements per
  // thread are in flight at a time, so read-modify-write latencies overlap.
  __device__ static void combine(const Problem& p, int f, const int* own, const int* mir, int ib, int jb,
                                 const int* s_e, const int* s_g, uint32_t tproc, int mode) {
    constexpr int UN = 8;
    const int64_t nb = tri_index(p.n_inputs, 0);
    int2* out = reinterpret_cast<int2*>(p.acc) + (int64_t)f * nb;
    for (int base = threadIdx.x; base < D::H * D::H; base += D::NT * UN) {
      int2 val[UN];
      int64_t pos[UN];
      bool ok[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int idx = base + u * D::NT;
        const int il = (idx / D::H) % D::H, jl = idx % D::H;
        const int i = ib + il, j = jb + jl;
        ok[u] = idx < D::H * D::H && i >= j && i < p.n_inputs;
        const uint32_t gij = (uint32_t)own[il * D::XPITCH + jl];
        const uint32_t gji = (uint32_t)mir[jl * D::XPITCH + il];
        const int ii = min(i, NB - 1), jj = min(j, NB - 1);
        const int re2 = (int)(gij + gji - (uint32_t)s_e[ii] - (uint32_t)s_e[jj] + 256u * tproc);
        const int im2 = (int)(gji - gij + (uint32_t)s_g[ii] - (uint32_t)s_g[jj]);
        val[u] = make_int2(re2 >> 1, im2 >> 1);
        pos[u] = ok[u] ? tri_index(i, j) : 0;
      }
      if (mode == kWriteStore) {
#pragma unroll
        for (int u = 0; u < UN; ++u)
          if (ok[u]) out[pos[u]] = val[u];
      } else if (mode == kWriteAdd) {
        int2 old[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) old[u] = out[pos[u]];
#pragma unroll
        for (int u = 0; u < UN; ++u)
          if (ok[u]) out[pos[u]] = make_int2(old[u].x + val[u].x, old[u].y + val[u].y);
      } else {
#pragma unroll
        for (int u = 0; u < UN; ++u)
          if (ok[u]) {
            __hip_atomic_fetch_add(&out[pos[u]].x, val[u].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&out[pos[u]].y, val[u].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
      }
    }
  }
};

template <int NT>
constexpr int diag_min_blocks = NT >= 512 ? 1 : 2;

template <int NB, int TC, int WC, bool ALIGNED>
__global__ __launch_bounds__(128 * WC, diag_min_blocks<128 * WC>) void xmac_diag_i8(Problem p, int nsplit,
                                                                                  int tsplit, int mode) {
  using D = Diag<NB, TC, WC>;
  using U = DiagUnit<NB, TC, WC>;
  static_assert(D::NT == 128 * WC, "thread count must match the launch bounds");
  __shared__ __attribute__((aligned(16))) uint8_t lds[D::LDS];
  __shared__ uint32_t s_sy[NB], s_sw[NB];
  __shared__ uint32_t s_bad[2];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
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
  if (tid < 2) s_bad[tid] = 0;
  __syncthreads();

  v16i acc[D::FM][D::FN];
#pragma unroll
  for (int x = 0; x < D::FM; ++x)
#pragma unroll
    for (int z = 0; z < D::FN; ++z) acc[x][z] = v16i{0};
  uint32_t sy[D::ITER][4], sw[D::ITER][4];
#pragma unroll
  for (int k = 0; k < D::ITER; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) sy[k][c] = sw[k][c] = 0;

  uint32_t ld[D::ITER][8];
  if (nchunks > 0) {
    uint32_t bad = 0;
    U::template load_chunk<ALIGNED>(p, f, t0, t1, 0, stride, ld);
    U::unpack_all(ld, lds, sy, sw, bad);
    U::publish_bad(bad, s_bad, 0);
    if (nchunks > 1) U::template load_chunk<ALIGNED>(p, f, t0, t1, 1, stride, ld);
  }
  __syncthreads();
  if (nchunks > 0) U::check_bad(lds, s_bad, 0, s_sy, s_sw);

  const int rrow = wr * D::TM + (lane & 31), crow = wc * D::TN + (lane & 31);
  int c = 0;
  for (; c + 2 < nchunks; ++c)
    U::template chunk_step<ALIGNED, true, true>(p, f, t0, t1, c, stride, lds, rrow, crow, ld, acc, sy, sw, s_bad,
                                                s_sy, s_sw);
  if (c + 1 < nchunks) {
    U::template chunk_step<ALIGNED, true, false>(p, f, t0, t1, c, stride, lds, rrow, crow, ld, acc, sy, sw, s_bad,
                                                 s_sy, s_sw);
    ++c;
  }
  if (c < nchunks)
    U::template chunk_step<ALIGNED, false, false>(p, f, t0, t1, c, stride, lds, rrow, crow, ld, acc, sy, sw, s_bad,
                                                  s_sy, s_sw);

  // Per-input sums of this unit, then the correction terms
  // e_k = Sy_k + 30 Sw_k and g_k = Sy_k - 2 Sw_k (in place).
#pragma unroll
  for (int k = 0; k < D::ITER; ++k) {
    if (!U::has_item(k)) continue;
    const int q = (tid + k * D::NT) % D::QUADS;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      atomicAdd(&s_sy[4 * q + cc], sy[k][cc]);
      atomicAdd(&s_sw[4 * q + cc], sw[k][cc]);
    }
  }
  __syncthreads();
  for (int k = tid; k < NB; k += D::NT) {
    const uint32_t y = s_sy[k], w = s_sw[k];
    s_sy[k] = y + 30u * w;
    s_sw[k] = y - 2u * w;
  }
  __syncthreads();
  const int* s_e = reinterpret_cast<const int*>(s_sy);
  const int* s_g = reinterpret_cast<const int*>(s_sw);

  const uint32_t tproc = (uint32_t)(nchunks * TC);
  const int wmode = nsplit > 1 ? kWriteAtomic : mode;
  int* xa = reinterpret_cast<int*>(lds);
  int* xb = xa + D::XAREA;
  constexpr int HW = WC / 2;  // wave columns per quadrant
  // Round 1: quadrant (1,0) against its mirror (0,1).
  if (wr == 0 && wc >= HW) U::store_tile(xa, (wc - HW) * D::TN, acc, lane);
  if (wr == 1 && wc < HW) U::store_tile(xb, wc * D::TN, acc, lane);
  __syncthreads();
  U::combine(p, f, xb, xa, D::H, 0, s_e, s_g, tproc, wmode);
  __syncthreads();
  // Round 2: the diagonal quadrants (0,0) and (1,1), each against itself.
  if (wr == 0 && wc < HW) U::store_tile(xa, wc * D::TN, acc, lane);
  if (wr == 1 && wc >= HW) U::store_tile(xb, (wc - HW) * D::TN, acc, lane);
  __syncthreads();
  U::combine(p, f, xa, xa, 0, 0, s_e, s_g, tproc, wmode);
  U::combine(p, f, xb, xb, D::H, D::H, s_e, s_g, tproc, wmode);
}

template <int NB, int TC, int WC>
static int launch_diag(const Problem& p, int nsplit, int mode, hipStream_t s) {
  using D = Diag<NB, TC, WC>;
  const int tsplit = (p.n_time + nsplit - 1) / nsplit;
  const int64_t grid = (int64_t)p.n_chan * nsplit;
  if (grid > 0x7FFFFFFF) return CORRX_EINVAL;
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;
  const bool aligned = (p.n_inputs % 4 == 0) && ((reinterpret_cast<uintptr_t>(p.in) & 3) == 0) &&
                       (int64_t)TC * stride + p.n_inputs < 0x7FFFFFFF;
  if (aligned)
    hipLaunchKernelGGL((xmac_diag_i8<NB, TC, WC, true>), dim3((unsigned)grid), dim3(D::NT), 0, s, p, nsplit,
                       tsplit, mode);
  else
    hipLaunchKernelGGL((xmac_diag_i8<NB, TC, WC, false>), dim3((unsigned)grid), dim3(D::NT), 0, s, p, nsplit,
                       tsplit, mode);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

int launch_mfma(const Problem& p, int engine, int nsplit, int mode, int tile_cfg, hipStream_t s) {
  if (engine != CORRX_ENGINE_MFMA_I8) return CORRX_EUNSUPPORTED;
  (void)tile_cfg;
  if (p.n_inputs <= 64) return launch_diag<64, 64, 2>(p, nsplit, mode, s);
  if (p.n_inputs <= 128) return launch_diag<128, 64, 2>(p, nsplit, mode, s);
  if (p.n_inputs <= 256) return launch_diag<256, 64, 4>(p, nsplit, mode, s);
  return CORRX_EUNSUPPORTED;
}

}  // namespace corrx
