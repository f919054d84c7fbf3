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
// Work units.  A channel's N x N square of G_b is tiled by blocks of 256
// inputs.  A diagonal unit computes one diagonal block (NB = 64, 128 or 256
// inputs) in full and pairs each element with its transpose through LDS.  The
// off-diagonal blocks use the direct complex form instead (two real products
// per baseline that share the column operand, no transpose): a cross unit
// takes 128 rows I of an off-diagonal block and its 256 columns J.  Units run
// as standalone grids (one launch per unit kind) or inside the persistent
// batch kernel.
//
// Unit structure (one workgroup = one unit x one time range, 8 waves for the
// 256-input units, two waves per SIMD so that one wave's vector-ALU and LDS
// work overlaps the other's MFMAs):
//   - global -> registers: raw buffer loads of 8 time rows x 4 inputs per
//     thread (lanes cover consecutive inputs of one row: coalesced), one chunk
//     of TC samples ahead of the chunk being multiplied; rows past the time
//     range read 0 through the buffer descriptor's range check;
//   - registers -> LDS: 4x4 byte transposes (time-major -> input-major), bias,
//     A-operand bytes [u(t..t+3), w(t..t+3), u(t+4..t+7), w(t+4..t+7)] per
//     16-byte chunk, XOR swizzled across rows for conflict-free ds_write_b128 /
//     ds_read_b128; an item holding an invalid code has those samples
//     replaced by the biased zero sample in registers (a branch only such
//     items take) before it is summed and stored;
//   - LDS -> MFMA: each wave owns a (NB/2) x (NB/WC) block of G_b in
//     accumulators (v_mfma_i32_32x32x32_i8); row fragments are read as
//     A-operands, column fragments are read and converted to B-operands in
//     registers (3 ALU ops per 4 samples); the unpack of the next chunk is
//     split into phases placed between the K-steps;
//   - epilogue: per-input sums reduced in LDS, quadrants of G_b exchanged
//     through LDS so that each lower-triangle element meets its transpose,
//     then acc += (Re, Im) (read-modify-write, or atomics for time splits).

#include <algorithm>

#include "corrx_internal.h"

namespace corrx {

// ---- staging of packed samples into LDS ---------------------------------------

// ROWS inputs staged per chunk of TC samples by NT threads.  Stage row r holds
// the A-operand bytes of one input: 16-byte granule k = samples 8k..8k+7 as
// [u(4), w(4), u(4), w(4)] (biased parts u = re + 8, w = im + 8), granules
// XOR-swizzled per row.  With QROWS > 0 the first QROWS rows are also stored
// in the form Q = [w(4), 15 - u(4), w(4), 15 - u(4)] in a second area after the
// ROWS rows (the cross units' imaginary-part operand).
//
// Per-input sums Su = sum u and Sw = sum w are kept in byte lanes: every
// store adds two words of at most 15 per byte, so a byte accumulator takes
// FLUSH chunks (8, or 4 when a thread's two items share their inputs) before it
// is folded into the LDS totals s_su / s_sw with one v_dot4 per word.
//
// SCALAR_RSRC: read the load descriptors from the first lane (for units whose
// block indices the compiler cannot prove uniform; a descriptor in vector
// registers costs a loop per load).
template <int ROWS, int TC, int NT, int QROWS = 0, bool SCALAR_RSRC = false>
struct Stage {
  static constexpr int QUADS = ROWS / 4;
  static constexpr int GROUPS = TC / 8;              // 8-row groups per chunk
  static constexpr int ITEMS = QUADS * GROUPS;       // unpack items (8 rows x 4 inputs)
  static constexpr int ITER = (ITEMS + NT - 1) / NT;
  static constexpr bool EXACT = ITEMS % NT == 0;
  // Split item order (cross units): item slot 0 of every thread holds one
  // item of the quads without the Q form, slot 1 of the first threads one
  // item of the Q quads.  Each slot is then wholly Q or wholly not, and slot
  // 1 exists for whole waves, so neither test needs a per-lane branch.
  static constexpr int QQUADS = QROWS / 4;
  static constexpr int PQUADS = QUADS - QQUADS;
  static constexpr bool SPLIT =
      QROWS > 0 && PQUADS * GROUPS == NT && QQUADS * GROUPS <= NT && (QQUADS * GROUPS) % 64 == 0;
  // When NT is a multiple of QUADS, all items of a thread cover the same
  // four inputs and share one set of per-input sums.
  static constexpr bool SHARED_Q = NT % QUADS == 0;
  static constexpr int SUMS = SHARED_Q ? 1 : ITER;
  static constexpr int ROWB = 2 * TC;                // bytes per row and chunk
  static constexpr int PBYTES = ROWS * ROWB;         // the A-form rows of one stage buffer
  static constexpr int BYTES = (ROWS + QROWS) * ROWB;  // one stage buffer
  static constexpr int GRAN = ROWB / 16;             // 16-byte granules per row and chunk
  static constexpr int KSTEPS = TC / 16;             // K=32 (16-sample) MFMA steps per chunk
  static constexpr int FLUSH = 255 / (30 * (SHARED_Q ? ITER : 1)) >= 8 ? 8 : 4;
  static_assert(30 * (SHARED_Q ? ITER : 1) * FLUSH <= 255, "byte sums must not carry");
  static_assert(TC == 64 || TC == 128 || TC == 256, "the unpack is split into four phases over the K-steps of a chunk");
  static_assert(QROWS % 4 == 0 && QROWS <= ROWS, "Q rows are whole quads of stage rows");
  static constexpr bool FP8 = false;

  // Stage quad q -> first input: the first `split` quads start at base0, the
  // rest at base1.
  struct Map {
    int base0, split, base1;
    __device__ int input(int q) const { return q < split ? base0 + 4 * q : base1 + 4 * (q - split); }
  };

  // Granule swizzle: a bijection over any GRAN consecutive rows and over the
  // rows 4q + c of GRAN consecutive quads q, so that fragment reads (one
  // granule of consecutive rows) and unpack stores (one granule of every
  // fourth row) are free of bank conflicts.
  __device__ static int swz(int row) { return (row ^ (row >> 2)) & (GRAN - 1); }
  __device__ static bool has_item(int tid, int k) {
    if constexpr (SPLIT) return k == 0 || __builtin_amdgcn_readfirstlane(tid) < QQUADS * GROUPS;
    return EXACT || tid + k * NT < ITEMS;
  }
  // Stage quad and 8-row group of item slot k of thread tid.
  __device__ static int quad(int tid, int k) {
    if constexpr (SPLIT) return k == 0 ? QQUADS + tid % PQUADS : tid % QQUADS;
    return (tid + k * NT) % QUADS;
  }
  __device__ static int group(int tid, int k) {
    if constexpr (SPLIT) return k == 0 ? tid / PQUADS : tid / QQUADS;
    return (tid + k * NT) / QUADS;
  }
  // Whether slot k's rows also take the Q form.
  __device__ static bool q_rows(int tid, int k) {
    if constexpr (SPLIT) return k == 1;
    return 4 * quad(tid, k) < QROWS;
  }

  // Load the 8 rows x 4 inputs of this thread's items of chunk c.
  //   ALIGNED (N % 4 == 0, 4-byte aligned buffer): raw buffer loads; quads
  //   past N use an out-of-range offset and read 0 in hardware.  FULL (every
  //   row of the chunk lies in the unit's time range): one descriptor for the
  //   chunk, row r of an item at scalar offset r rows.  Otherwise row r of an
  //   item uses a descriptor whose base is advanced by r rows and whose range
  //   ends at the channel's last valid row, so rows past the unit's time
  //   range read 0 in hardware.  Either way the per-lane offset is the same
  //   for all 8 rows of the item, and no branch and no select follows a
  //   load, so all loads stay in flight.
  //   Otherwise: byte loads (slow path).
  template <bool ALIGNED, bool FULL = false>
  __device__ static void load(const Problem& p, const Map& m, int f, int t0, int t1, int c, int64_t stride, int tid,
                              uint32_t (&ld)[ITER][8]) {
    const int tb = t0 + c * TC;
    if constexpr (ALIGNED) {
      const int rows = FULL ? TC : min(t1 - tb, TC);
      // TC rows of a channel span less than 2^31 bytes (checked on the host),
      // so the range arithmetic stays in 32-bit scalar registers.
      const int stride32 = (int)stride;
      const int nrec0 = (rows - 1) * stride32 + p.n_inputs;
      // the unit's first row (loop-invariant) advanced by c chunks of TC rows
      const uint8_t* base = p.in + row_offset(p, f, t0) + (int64_t)c * (TC * stride32);
      uint32_t off[ITER];
#pragma unroll
      for (int k = 0; k < ITER; ++k) {
        const int g = group(tid, k);
        const int i = m.input(quad(tid, k));
        off[k] = (i < p.n_inputs && has_item(tid, k)) ? (uint32_t)(8 * g * stride + i) : 0x80000000u;
      }
      if constexpr (FULL) {
        const uint8_t* rb = base;
        int nr = nrec0;
        if constexpr (SCALAR_RSRC) {
          nr = __builtin_amdgcn_readfirstlane(nr);
          const uint64_t a = reinterpret_cast<uint64_t>(rb);
          rb = reinterpret_cast<const uint8_t*>(
              ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
              (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a));
        }
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(rb), (short)0, nr, kBufferRsrcWord3);
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int k = 0; k < ITER; ++k) ld[k][r] = __builtin_amdgcn_raw_buffer_load_b32(rs, off[k], r * stride32, 0);
        return;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        int nr = max(nrec0 - r * stride32, 0);
        const uint8_t* rb = base + (int64_t)r * stride;
        if constexpr (SCALAR_RSRC) {
          nr = __builtin_amdgcn_readfirstlane(nr);
          const uint64_t a = reinterpret_cast<uint64_t>(rb);
          rb = reinterpret_cast<const uint8_t*>(
              ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
              (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a));
        }
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(rb), (short)0, nr, kBufferRsrcWord3);
#pragma unroll
        for (int k = 0; k < ITER; ++k) ld[k][r] = __builtin_amdgcn_raw_buffer_load_b32(rs, off[k], 0, 0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < ITER; ++k) {
        const int g = group(tid, k);
        const int i = m.input(quad(tid, k));
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int t = tb + 8 * g + r;
          uint32_t v = 0;
          if (t < t1 && has_item(tid, k)) {
            const uint8_t* row = p.in + row_offset(p, f, t);
            for (int b = 0; b < 4; ++b)
              if (i + b < p.n_inputs) v |= uint32_t(row[i + b]) << (8 * b);
          }
          ld[k][r] = v;
        }
      }
    }
  }

  // Unpack of one chunk, in four phases (one per K-step of the previous
  // chunk).  One item per thread: phases 0/1 transpose rows 0-3 / 4-7
  // (time-major -> input-major); phases 2/3 handle inputs 0-1 / 2-3 of the
  // quad -- biased parts, byte sums and one 16-byte store per input.  Two
  // items per thread: phases 0/1 transpose / store item 0, phases 2/3 item 1,
  // so only one item's transposed words are live at a time.  The transposes
  // flag invalid codes in `bad`; the item's store phase then masks them (a
  // branch taken only by items that hold one).  The transposed words x stay
  // raw (unbiased): the bias is folded into the nibble extraction.
  static_assert(ITER <= 2, "at most two unpack items per thread");
  static constexpr int LOAD_PHASE = ITER == 1 ? 1 : 2;  // last phase that reads the loaded words

  __device__ static void transpose_tq(const uint32_t (&ld)[ITER][8], uint32_t (&x)[8], int k, int tq, uint32_t& bad) {
    uint32_t e0, e1, e2, e3;
    transpose4x4(ld[k][4 * tq], ld[k][4 * tq + 1], ld[k][4 * tq + 2], ld[k][4 * tq + 3], e0, e1, e2, e3);
    x[tq] = e0;  // x[2*c + tq]: input c, time quad tq
    x[2 + tq] = e1;
    x[4 + tq] = e2;
    x[6 + tq] = e3;
    const uint32_t kc = vconst(0xEEEEEEEFu);
    bad = or_invalid_flags_raw(e0, kc, bad);
    bad = or_invalid_flags_raw(e1, kc, bad);
    bad = or_invalid_flags_raw(e2, kc, bad);
    bad = or_invalid_flags_raw(e3, kc, bad);
  }

  __device__ static void store_input(const uint32_t (&x)[8], uint8_t* st, int k, int c, uint32_t (&bu)[SUMS][4],
                                     uint32_t (&bw)[SUMS][4], int tid) {
    const int q = quad(tid, k), g = group(tid, k);
    const int row = 4 * q + c;
    const uint32_t xa = x[2 * c], xb = x[2 * c + 1];
    const uint32_t ra = bu4(xa), ia = bw4(xa), rb = bu4(xb), ib = bw4(xb);
    const int ks = SHARED_Q ? 0 : k;
    bu[ks][c] += ra + rb;
    bw[ks][c] += ia + ib;
    const int off = row * ROWB + ((g ^ swz(row)) << 4);
    *reinterpret_cast<v4i*>(st + off) = v4i{(int)ra, (int)ia, (int)rb, (int)ib};
    if constexpr (QROWS > 0) {
      if (q_rows(tid, k))
        *reinterpret_cast<v4i*>(st + PBYTES + off) =
            v4i{(int)bw4(xa), (int)(ra ^ 0x0F0F0F0Fu), (int)bw4(xb), (int)(rb ^ 0x0F0F0F0Fu)};
    }
  }

  // Rare path: some sample of the item holds the invalid code; replace each
  // such sample by a zero sample (raw 0x00, biased 0x88) before it is stored
  // and summed.
  __device__ static void mask_item(uint32_t (&x)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = mask_invalid_raw(x[q]);
  }

  template <int PH>
  __device__ static void unpack_phase(const uint32_t (&ld)[ITER][8], uint32_t (&x)[8], uint8_t* st,
                                      uint32_t (&bu)[SUMS][4], uint32_t (&bw)[SUMS][4], uint32_t& bad, int tid) {
    if constexpr (ITER == 1) {
      if (!has_item(tid, 0)) return;
      if constexpr (PH < 2) {
        transpose_tq(ld, x, 0, PH, bad);
      } else {
        if (PH == 2 && (bad & 0x88888888u)) mask_item(x);
        store_input(x, st, 0, 2 * (PH - 2), bu, bw, tid);
        store_input(x, st, 0, 2 * (PH - 2) + 1, bu, bw, tid);
      }
    } else {
      constexpr int k = PH / 2;
      if (!has_item(tid, k)) return;
      if constexpr (PH % 2 == 0) {
        transpose_tq(ld, x, k, 0, bad);
        transpose_tq(ld, x, k, 1, bad);
      } else {
        if (bad & 0x88888888u) mask_item(x);
        bad = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) store_input(x, st, k, c, bu, bw, tid);
      }
    }
  }

  __device__ static void unpack_all(const uint32_t (&ld)[ITER][8], uint8_t* st, uint32_t (&bu)[SUMS][4],
                                    uint32_t (&bw)[SUMS][4], uint32_t& bad, int tid) {
    uint32_t x[8];
    unpack_phase<0>(ld, x, st, bu, bw, bad, tid);
    unpack_phase<1>(ld, x, st, bu, bw, bad, tid);
    unpack_phase<2>(ld, x, st, bu, bw, bad, tid);
    unpack_phase<3>(ld, x, st, bu, bw, bad, tid);
  }

  __device__ static v4i read_frag(const uint8_t* st, int row, int chunk) {
    return *reinterpret_cast<const v4i*>(st + row * ROWB + ((chunk ^ swz(row)) << 4));
  }

  // Fold the byte accumulators into the LDS totals of Su and Sw and clear them.
  __device__ static void flush(uint32_t (&bu)[SUMS][4], uint32_t (&bw)[SUMS][4], uint32_t* s_su, uint32_t* s_sw,
                               int tid) {
#pragma unroll
    for (int k = 0; k < SUMS; ++k) {
      if (has_item(tid, k)) {
        const int q = quad(tid, k);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          atomicAdd(&s_su[4 * q + c], bytesum(bu[k][c], 0u));
          atomicAdd(&s_sw[4 * q + c], bytesum(bw[k][c], 0u));
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) bu[k][c] = bw[k][c] = 0;
    }
  }
};

__device__ inline v4i to_b(v4i a) {
  v4i b;
  b.x = (int)op_s((uint32_t)a.x, (uint32_t)a.y);
  b.y = (int)op_d((uint32_t)a.x, (uint32_t)a.y);
  b.z = (int)op_s((uint32_t)a.z, (uint32_t)a.w);
  b.w = (int)op_d((uint32_t)a.z, (uint32_t)a.w);
  return b;
}

// Row (within a 32x32 tile) held by accumulator register r of this lane.
__device__ inline int acc_row(int r, int lane) { return ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3); }

// Write UN baselines per thread (element pos[u] of the channel's accumulator
// out, nb baselines) with one of the write modes.  Store and read-modify-write
// go through a buffer descriptor over the channel: an element not to be
// written gets an offset past its end, which the hardware range check drops
// (stores) or reads as zero (loads), so no branch follows the lane masks.  RMW
// loads are all issued before any store so their latencies overlap.
template <int UN>
__device__ inline void write_out(int2* out, int64_t nb, const uint32_t (&pos)[UN], const bool (&ok)[UN],
                                 const int2 (&val)[UN], int mode) {
  if (mode == kWriteStore || mode == kWriteAdd) {
    // The channel's base is uniform; reading it from the first lane keeps the
    // descriptor in scalar registers where the compiler cannot prove that.
    // n_inputs <= 4096: a channel holds at most 8,390,656 baselines (67 MB).
    const uint64_t a = reinterpret_cast<uint64_t>(out);
    int2* base = reinterpret_cast<int2*>(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) << 32) |
                                         (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a));
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(base, (short)0, __builtin_amdgcn_readfirstlane((int)(8 * nb)), kBufferRsrcWord3);
    uint32_t off[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) off[u] = ok[u] ? 8u * pos[u] : 0x80000000u;
    if (mode == kWriteAdd) {
      v2i old[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) old[u] = __builtin_amdgcn_raw_buffer_load_b64(rs, off[u], 0, 0);
#pragma unroll
      for (int u = 0; u < UN; ++u)
        __builtin_amdgcn_raw_buffer_store_b64(v2i{old[u].x + val[u].x, old[u].y + val[u].y}, rs, off[u], 0, 0);
    } else {
#pragma unroll
      for (int u = 0; u < UN; ++u) __builtin_amdgcn_raw_buffer_store_b64(v2i{val[u].x, val[u].y}, rs, off[u], 0, 0);
    }
  } else if (mode == kWriteAtomic) {
#pragma unroll
    for (int u = 0; u < UN; ++u)
      if (ok[u]) {
        __hip_atomic_fetch_add(&out[pos[u]].x, val[u].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&out[pos[u]].y, val[u].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
  }
}

// Main loop shared by all unit kinds: prologue (chunk 0 unpacked, chunk 1
// loaded), then for every chunk the K-steps of the unit (kstep(st, ks)) with
// the four unpack phases of the next chunk placed after them and the loads of
// the chunk after that issued once the registers are free.  The int8 stages
// also add every input's sums of u and w into s_su / s_sw (zeroed by the
// caller); they are complete once the caller has synchronised after the loop.
template <class S, bool ALIGNED, class KStep>
__device__ inline void run_chunks(const Problem& p, const typename S::Map& m, int f, int t0, int t1, int64_t stride,
                                  int tid, uint8_t* lds, uint32_t* s_su, uint32_t* s_sw, int nchunks, KStep&& kstep) {
  uint32_t ld[S::ITER][8];
  uint32_t bu[S::SUMS][4], bw[S::SUMS][4];
#pragma unroll
  for (int k = 0; k < S::SUMS; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) bu[k][c] = bw[k][c] = 0;
  if (nchunks > 0) {
    uint32_t bad = 0;
    S::template load<ALIGNED>(p, m, f, t0, t1, 0, stride, tid, ld);
    S::unpack_all(ld, lds, bu, bw, bad, tid);
    if (nchunks > 1) S::template load<ALIGNED>(p, m, f, t0, t1, 1, stride, tid, ld);
  }
  __syncthreads();

  // full2: chunk c + 2 lies wholly in [t0, t1).  parity: c & 1 when known
  // at compile time (the stage buffers' offset then folds into the LDS
  // instructions' immediate offsets), else -1.
  auto step = [&](int c, auto more1, auto more2, auto full2, auto parity) {
    constexpr bool M1 = decltype(more1)::value, M2 = decltype(more2)::value, F2 = decltype(full2)::value;
    constexpr int P = decltype(parity)::value;
    const int cur = P < 0 ? (c & 1) : P;
    const uint8_t* st = lds + cur * S::BYTES;
    uint8_t* nst = lds + (cur ^ 1) * S::BYTES;
    uint32_t bad = 0;
    uint32_t x[8];
#pragma unroll
    for (int ks = 0; ks < S::KSTEPS; ++ks) {
      kstep(st, ks);
      // unpack phase PH runs after K-step PH * KSTEPS / 4
      if constexpr (M1) {
        if (ks == 0 * S::KSTEPS / 4) S::template unpack_phase<0>(ld, x, nst, bu, bw, bad, tid);
        if (ks == 1 * S::KSTEPS / 4) S::template unpack_phase<1>(ld, x, nst, bu, bw, bad, tid);
        if (ks == 2 * S::KSTEPS / 4) S::template unpack_phase<2>(ld, x, nst, bu, bw, bad, tid);
        if (ks == 3 * S::KSTEPS / 4) S::template unpack_phase<3>(ld, x, nst, bu, bw, bad, tid);
      }
      if constexpr (M2) {
        if (ks == S::LOAD_PHASE * S::KSTEPS / 4)
          S::template load<ALIGNED, F2>(p, m, f, t0, t1, c + 2, stride, tid, ld);
      }
    }
    if constexpr (M1 && !S::FP8) {
      // c + 2 chunks unpacked so far
      if (((c + 2) & (S::FLUSH - 1)) == 0) S::flush(bu, bw, s_su, s_sw, tid);
    }
    __syncthreads();
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  using P0 = std::integral_constant<int, 0>;
  using P1 = std::integral_constant<int, 1>;
  using PX = std::integral_constant<int, -1>;
  int c = 0;
  // every chunk but the last is whole; the main loop takes two per pass
  for (; c + 4 < nchunks; c += 2) {
    step(c, T_{}, T_{}, T_{}, P0{});
    step(c + 1, T_{}, T_{}, T_{}, P1{});
  }
  if (c + 3 < nchunks) {
    step(c, T_{}, T_{}, T_{}, PX{});
    ++c;
  }
  if (c + 2 < nchunks) {
    step(c, T_{}, T_{}, F_{}, PX{});
    ++c;
  }
  if (c + 1 < nchunks) {
    step(c, T_{}, F_{}, F_{}, PX{});
    ++c;
  }
  if (c < nchunks) step(c, F_{}, F_{}, F_{}, PX{});
  if constexpr (!S::FP8) S::flush(bu, bw, s_su, s_sw, tid);
}

// ---- diagonal unit -----------------------------------------------------------

// Samples per chunk of a standalone diagonal unit.  64 for 128 and 256 inputs
// (128 would halve the barriers per sample, but the extra loads in flight
// exceed the registers of two waves per SIMD); 128 for 64 inputs, whose units
// are HBM-bound and have registers to spare.
template <int NB>
constexpr int diag_tc = NB == 64 ? 128 : 64;

template <int NB, int WC, int TC_ = diag_tc<NB>>
struct DiagGeom {
  static constexpr int WR = 2;                       // wave rows
  static constexpr int NW = WR * WC;                 // waves
  static constexpr int NT = 64 * NW;                 // threads
  static constexpr int TM = NB / WR;                 // wave tile rows
  static constexpr int TN = NB / WC;                 // wave tile columns
  static constexpr int FM = TM / 32;                 // 32x32 MFMA tiles along rows
  static constexpr int FN = TN / 32;                 // ... along columns
  static constexpr int H = NB / 2;                   // quadrant side
  static constexpr int XPITCH = H + 1;
  static constexpr int XAREA = H * XPITCH;           // int32 words of one exchange area
  static constexpr int TC = TC_;                     // samples per chunk
  static constexpr int STAGE = NB * 2 * TC;          // one stage buffer
  static constexpr int LDS = (2 * STAGE > 2 * XAREA * 4) ? 2 * STAGE : 2 * XAREA * 4;
  static_assert(TM % 32 == 0 && TN % 32 == 0, "wave tiles are made of 32x32 MFMA tiles");
  static_assert(WC % 2 == 0, "quadrants are made of whole wave tiles");
};

// Write this wave's tile into an exchange area at column offset col0.
template <class G>
__device__ inline void store_tile(int* xa, int col0, const v16i (&acc)[G::FM][G::FN], int lane) {
#pragma unroll
  for (int x = 0; x < G::FM; ++x)
#pragma unroll
    for (int z = 0; z < G::FN; ++z)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        xa[(32 * x + acc_row(r, lane)) * G::XPITCH + col0 + 32 * z + (lane & 31)] = acc[x][z][r];
}

// Combine the quadrant of G_b at local rows ib.., columns jb.. (in `own`) with
// its mirror quadrant (in `mir`; the same area for a diagonal quadrant) and
// write the lower triangle; local row r is input ibase + r.  Each thread keeps
// one column jl and walks the rows jl's wave shares, NT / H rows apart: the
// column's correction terms are read once, and for H >= 64 the row, its
// correction terms and its triangle offset are the same in the whole wave
// (scalar registers); consecutive lanes write consecutive baselines.
template <class G>
__device__ inline void combine_quadrant(const Problem& p, int f, int ibase, const int* own, const int* mir, int ib,
                                        int jb, const uint32_t* s_e, const uint32_t* s_g, uint32_t tproc, int mode,
                                        int tid) {
  constexpr int H = G::H, RSTEP = G::NT / H, NPASS = H / RSTEP, UN = NPASS < 8 ? NPASS : 8;
  static_assert(G::NT % H == 0 && NPASS % UN == 0, "whole passes of whole rows");
  const bool diag = ib == jb;
  const int jl = tid % H, lj = jb + jl, j = ibase + lj;
  int r0 = tid / H;
  int jwave = 0;  // smallest column of the wave, when the wave shares its rows
  if constexpr (H >= 64) {
    r0 = __builtin_amdgcn_readfirstlane(r0);
    jwave = __builtin_amdgcn_readfirstlane(jl & ~63);
  }
  const int64_t nb = tri_index(p.n_inputs, 0);
  int2* out = reinterpret_cast<int2*>(p.acc) + (int64_t)f * nb;
  const uint32_t cre = 256u * tproc - s_e[lj], gj = s_g[lj];
  const int* ownp = own + r0 * G::XPITCH + jl;
  const int* mirp = mir + jl * G::XPITCH + r0;
#pragma unroll 1
  for (int k0 = 0; k0 < NPASS; k0 += UN) {
    // diagonal quadrant: passes whose rows all lie above the wave's columns write nothing
    if (diag && r0 + RSTEP * (k0 + UN - 1) < jwave) continue;
    int2 val[UN];
    uint32_t pos[UN];
    bool ok[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int il = r0 + RSTEP * (k0 + u);
      const int li = ib + il, i = ibase + li;
      ok[u] = (!diag || il >= jl) && i < p.n_inputs;
      const uint32_t gij = (uint32_t)ownp[RSTEP * (k0 + u) * G::XPITCH], gji = (uint32_t)mirp[RSTEP * (k0 + u)];
      // 2 Re = G_b[i][j] + G_b[j][i] - e_i - e_j + 256 T,  2 Im = G_b[j][i] - G_b[i][j] + g_i - g_j
      val[u] = make_int2((int)(gij + gji - s_e[li] + cre) >> 1, (int)(gji - gij + s_g[li] - gj) >> 1);
      // n_inputs <= 4096: the offset within the channel fits 32 bits
      pos[u] = ((uint32_t)i * (uint32_t)(i + 1) >> 1) + (uint32_t)j;
    }
    write_out<UN>(out, nb, pos, ok, val, mode);
  }
}

// One diagonal unit: inputs ibase .. ibase+NB-1 of channel f over samples
// [t0, t1), run by the NT threads whose local index is tid.  lds: G::LDS
// bytes; s_sy, s_sw: NB words each (the inputs' sums, then the correction
// terms e and g).
template <int NB, int WC, bool ALIGNED, int TC = diag_tc<NB>>
__device__ void run_diag(const Problem& p, int f, int ibase, int t0, int t1, int tid, uint8_t* lds, uint32_t* s_sy,
                         uint32_t* s_sw, int mode) {
  // Values derived from the thread index are recomputed for every unit: when
  // units run in a loop (the persistent kernel), hoisting them out of it would
  // keep them live across the whole unit and exhaust the registers.
  asm volatile("" : "+v"(tid));
  using G = DiagGeom<NB, WC, TC>;
  using S = Stage<NB, G::TC, G::NT>;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int nchunks = t1 > t0 ? (t1 - t0 + G::TC - 1) / G::TC : 0;
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;

  for (int k = tid; k < NB; k += G::NT) {
    s_sy[k] = 0;
    s_sw[k] = 0;
  }
  __syncthreads();

  v16i acc[G::FM][G::FN];
#pragma unroll
  for (int x = 0; x < G::FM; ++x)
#pragma unroll
    for (int z = 0; z < G::FN; ++z) acc[x][z] = v16i{0};

  const int half = lane >> 5;
  const int rrow = wr * G::TM + (lane & 31), crow = wc * G::TN + (lane & 31);
  const typename S::Map m{ibase, NB / 4, ibase};
  // fragments of K-steps ks (slot ks & 1) and ks + 1 (the other slot): the
  // next K-step's reads are issued before this one's MFMAs
  v4i fa[2][G::FM], fb[2][G::FN];
  run_chunks<S, ALIGNED>(p, m, f, t0, t1, stride, tid, lds, s_sy, s_sw, nchunks,
                         [&](const uint8_t* st, int ks) {
                           const int cb = ks & 1, nb = cb ^ 1;
                           if (ks == 0) {
#pragma unroll
                             for (int x = 0; x < G::FM; ++x) fa[cb][x] = S::read_frag(st, rrow + 32 * x, half);
#pragma unroll
                             for (int x = 0; x < G::FN; ++x) fb[cb][x] = to_b(S::read_frag(st, crow + 32 * x, half));
                           }
                           if (ks + 1 < S::KSTEPS) {
#pragma unroll
                             for (int x = 0; x < G::FM; ++x)
                               fa[nb][x] = S::read_frag(st, rrow + 32 * x, 2 * (ks + 1) + half);
#pragma unroll
                             for (int x = 0; x < G::FN; ++x)
                               fb[nb][x] = S::read_frag(st, crow + 32 * x, 2 * (ks + 1) + half);
                           }
#pragma unroll
                           for (int x = 0; x < G::FM; ++x)
#pragma unroll
                             for (int z = 0; z < G::FN; ++z)
                               acc[x][z] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[cb][x], fb[cb][z], acc[x][z], 0, 0, 0);
                           if (ks + 1 < S::KSTEPS) {
#pragma unroll
                             for (int x = 0; x < G::FN; ++x) fb[nb][x] = to_b(fb[nb][x]);
                           }
                         });

  // correction terms in place: e_k = 16 Su_k + 31 Sw_k, g_k = 16 Su_k - Sw_k
  // (with Sy = 16 Su + Sw these are Sy + 30 Sw and Sy - 2 Sw)
  __syncthreads();
  for (int k = tid; k < NB; k += G::NT) {
    const uint32_t su = s_sy[k], sw = s_sw[k];
    s_sy[k] = 16u * su + 31u * sw;
    s_sw[k] = 16u * su - sw;
  }
  __syncthreads();
  const uint32_t tproc = (uint32_t)(nchunks * G::TC);
  int* xa = reinterpret_cast<int*>(lds);
  int* xb = xa + G::XAREA;
  constexpr int HW = WC / 2;  // wave columns per quadrant
  // Pass 1: quadrant (1,0) against its mirror (0,1).
  if (wr == 0 && wc >= HW) store_tile<G>(xa, (wc - HW) * G::TN, acc, lane);
  if (wr == 1 && wc < HW) store_tile<G>(xb, wc * G::TN, acc, lane);
  __syncthreads();
  combine_quadrant<G>(p, f, ibase, xb, xa, G::H, 0, s_sy, s_sw, tproc, mode, tid);
  __syncthreads();
  // Pass 2: the diagonal quadrants (0,0) and (1,1), each against itself.
  if (wr == 0 && wc < HW) store_tile<G>(xa, wc * G::TN, acc, lane);
  if (wr == 1 && wc >= HW) store_tile<G>(xb, (wc - HW) * G::TN, acc, lane);
  __syncthreads();
  combine_quadrant<G>(p, f, ibase, xa, xa, 0, 0, s_sy, s_sw, tproc, mode, tid);
  combine_quadrant<G>(p, f, ibase, xb, xb, G::H, G::H, s_sy, s_sw, tproc, mode, tid);
  __syncthreads();
}

// ---- cross unit ---------------------------------------------------------------
//
// Rows I0 .. I0+127 against columns J0 .. J0+255 of an off-diagonal block
// pair (every row input above every column input), in the direct complex
// form rather than the single biased GEMM: with the staged bytes
// P_k = (u_k, w_k) of every input and the rows also staged as
// Q_i = (w_i, 15 - u_i),
//     R_ij = P_i . P_j = Re V_ij + 8 S_i + 8 S_j - 128 T
//     M_ij = Q_i . P_j = Im V_ij + 8 (Sw_i - Su_i) + 8 Su_j + 7 Sw_j
//                      = Im V_ij + 16 Sw_i - 8 S_i + 8 S_j - Sw_j
// with S_k = Su_k + Sw_k (Su, Sw the sums of u and w over the T processed
// samples).  Both products share the column operand, so a K-step reads six
// fragments for eight MFMAs and converts none.  8 waves as 2 x 4 tiles of
// 64 x 64 baselines, each holding R and M.
struct CrossGeom {
  static constexpr int NT = 512;
  static constexpr int ROWS = 384;                   // stage rows: 128 of I, then 256 of J
  static constexpr int QROWS = 128;                  // the I rows, also in the Q form
  static constexpr int LDS = 2 * (ROWS + QROWS) * 128;
};

template <bool ALIGNED>
__device__ void run_cross(const Problem& p, int f, int I0, int J0, int t0, int t1, int tid, uint8_t* lds,
                          uint32_t* s_sy, uint32_t* s_sw, int mode) {
  // Values derived from the thread index are recomputed for every unit: when
  // units run in a loop (the persistent kernel), hoisting them out of it would
  // keep them live across the whole unit and exhaust the registers.
  asm volatile("" : "+v"(tid));
  // The unit's coordinates are uniform, but the block decode (a float square
  // root) leaves them in vector registers: move them to scalar registers so
  // that the load descriptors and their row arithmetic stay scalar.
  f = __builtin_amdgcn_readfirstlane(f);
  I0 = __builtin_amdgcn_readfirstlane(I0);
  J0 = __builtin_amdgcn_readfirstlane(J0);
  t0 = __builtin_amdgcn_readfirstlane(t0);
  t1 = __builtin_amdgcn_readfirstlane(t1);
  using S = Stage<CrossGeom::ROWS, 64, CrossGeom::NT, CrossGeom::QROWS>;
  static_assert(2 * S::BYTES == CrossGeom::LDS, "two stage buffers");
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / 4, wc = wave % 4;
  const int nchunks = t1 > t0 ? (t1 - t0 + 63) / 64 : 0;
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;

  for (int k = tid; k < CrossGeom::ROWS; k += CrossGeom::NT) {
    s_sy[k] = 0;
    s_sw[k] = 0;
  }
  __syncthreads();

  v16i re[2][2], im[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z) re[x][z] = im[x][z] = v16i{0};

  const int half = lane >> 5;
  const int irow = wr * 64 + (lane & 31), jrow = 128 + wc * 64 + (lane & 31);
  const typename S::Map m{I0, 32, J0};
  run_chunks<S, ALIGNED>(p, m, f, t0, t1, stride, tid, lds, s_sy, s_sw, nchunks,
                         [&](const uint8_t* st, int ks) {
                           v4i a[2], q[2], b[2];
#pragma unroll
                           for (int x = 0; x < 2; ++x) {
                             a[x] = S::read_frag(st, irow + 32 * x, 2 * ks + half);
                             q[x] = S::read_frag(st + S::PBYTES, irow + 32 * x, 2 * ks + half);
                             b[x] = S::read_frag(st, jrow + 32 * x, 2 * ks + half);
                           }
#pragma unroll
                           for (int x = 0; x < 2; ++x)
#pragma unroll
                             for (int z = 0; z < 2; ++z) {
                               re[x][z] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[x], b[z], re[x][z], 0, 0, 0);
                               im[x][z] = __builtin_amdgcn_mfma_i32_32x32x32_i8(q[x], b[z], im[x][z], 0, 0, 0);
                             }
                         });

  // Correction terms in place: A_k = -8 S_k in s_sy, B_k = 8 S_k - 16 Sw_k in
  // s_sw, so that Re V = R + A_i + (128 T + A_j) and
  // Im V = M + B_i + (Sw_j - 8 S_j), with Sw_j = (-A_j - B_j) / 16 exactly.
  __syncthreads();
  for (int k = tid; k < CrossGeom::ROWS; k += CrossGeom::NT) {
    const uint32_t s8 = 8u * (s_sy[k] + s_sw[k]);
    s_sw[k] = s8 - 16u * s_sw[k];
    s_sy[k] = 0u - s8;
  }
  __syncthreads();
  const uint32_t tproc = (uint32_t)(nchunks * 64);
  const int64_t nb = tri_index(p.n_inputs, 0);
  int2* out = reinterpret_cast<int2*>(p.acc) + (int64_t)f * nb;
  // Column terms once per column tile.
  uint32_t cre[2], cim[2];
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    const int lj = 128 + wc * 64 + 32 * z + (lane & 31);  // stage row of j
    const uint32_t a = s_sy[lj], b = s_sw[lj];
    cre[z] = 128u * tproc + a;
    cim[z] = ((0u - a - b) >> 4) + a;
  }
  // Accumulator register r of this lane holds row (r >> 2) * 8 + (lane >> 5) * 4
  // + (r & 3) of its 32 x 32 tile: per (x, rh) eight rows in two runs of four
  // consecutive rows, whose terms are read with one 16-byte LDS load each and
  // whose triangle offsets follow from one multiply.
  const int lrow = wr * 64 + ((lane >> 5) << 2);
  const uint32_t jl = (uint32_t)(J0 + wc * 64 + (lane & 31));
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int rh = 0; rh < 2; ++rh) {
      uint32_t ra[8], rb[8], rt[8];
      bool ok[8];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int l0 = lrow + 32 * x + 16 * rh + 8 * g;  // stage row of the run's first row
        const uint4 a4 = *reinterpret_cast<const uint4*>(s_sy + l0);
        const uint4 b4 = *reinterpret_cast<const uint4*>(s_sw + l0);
        const uint32_t i0 = (uint32_t)(I0 + l0);
        // n_inputs <= 4096: triangle offsets within the channel fit 32 bits
        uint32_t t = i0 * (i0 + 1) >> 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ra[4 * g + q] = q == 0 ? a4.x : q == 1 ? a4.y : q == 2 ? a4.z : a4.w;
          rb[4 * g + q] = q == 0 ? b4.x : q == 1 ? b4.y : q == 2 ? b4.z : b4.w;
          rt[4 * g + q] = t;
          ok[4 * g + q] = (int)(i0 + q) < p.n_inputs;
          t += i0 + q + 1;
        }
      }
#pragma unroll
      for (int z = 0; z < 2; ++z) {
        int2 val[8];
        uint32_t pos[8];
        const uint32_t j = jl + 32u * z;
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
          const int r = 8 * rh + rr;
          val[rr] = make_int2((int)((uint32_t)re[x][z][r] + ra[rr] + cre[z]),
                              (int)((uint32_t)im[x][z][r] + rb[rr] + cim[z]));
          pos[rr] = rt[rr] + j;
        }
        write_out<8>(out, nb, pos, ok, val, mode);
      }
    }
  __syncthreads();
}

// ---- fp8 (E4M3) staging and diagonal unit -------------------------------------
//
// The fp8 engine multiplies the unbiased operands
//     A_i = (re_i, im_i)            in [-7, 7]
//     B_j = (re_j + im_j, im_j - re_j) in [-14, 14]
// all exactly representable in E4M3, so G = A B^T needs no correction terms:
// 2 Re V_ij = G[i][j] + G[j][i], 2 Im V_ij = G[j][i] - G[i][j].  Products are
// integers of magnitude <= 98 per sample, accumulated in fp32 by
// v_mfma_f32_32x32x64_f8f6f4; a work unit spans at most kMaxUnitTimeF8 samples
// so every partial sum is an integer below 2^24 (exact), and the epilogue
// folds it into the int32 accumulator by an exact conversion.
//
// Stage row layout (per input, TC = 64 samples): A bytes then B bytes, 128
// each; 16-byte chunk k holds samples 8k..8k+7 as four dwords of two samples,
// [re(t), re(t+1), im(t), im(t+1)] in A and [s(t), s(t+1), d(t), d(t+1)] in B
// (the K order is the same in both operands, which is all the product needs).
template <int ROWS, int NT>
struct StageF8 {
  using L = Stage<ROWS, 64, NT>;  // same loads and item geometry as int8
  static constexpr int SUMS = L::SUMS;
  static constexpr int QUADS = L::QUADS;
  static constexpr int ITER = L::ITER;
  static constexpr int ROWB = 128;
  static constexpr int BYTES = 2 * ROWS * ROWB;      // A then B
  static constexpr int KSTEPS = 2;                   // K=64 (32-sample) MFMA steps per chunk
  static constexpr int LOAD_PHASE = L::LOAD_PHASE;
  static constexpr bool FP8 = true;
  static constexpr int FLUSH = 8;  // no sums: the unbiased operands need no correction terms
  __device__ static void flush(uint32_t (&)[SUMS][4], uint32_t (&)[SUMS][4], uint32_t*, uint32_t*, int) {}
  static_assert(ITER == 1, "one unpack item per thread");
  using Map = typename L::Map;

  template <bool ALIGNED, bool FULL = false>
  __device__ static void load(const Problem& p, const Map& m, int f, int t0, int t1, int c, int64_t stride, int tid,
                              uint32_t (&ld)[ITER][8]) {
    L::template load<ALIGNED, FULL>(p, m, f, t0, t1, c, stride, tid, ld);
  }

  // Two samples (bytes 2h, 2h+1 of the raw word x) of one input -> one A
  // dword and one B dword of E4M3 codes.  u = re + 8, w = im + 8 become f16
  // via 1024 + u.
  __device__ static void to_fp8(uint32_t x, int h, uint32_t& a, uint32_t& b) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef short s2 __attribute__((ext_vector_type(2)));
    const uint32_t sel = h ? 0x04030402u : 0x04010400u;
    const uint32_t u = bu4(x), w = bw4(x);
    const h2 bias = {(_Float16)1032.0f, (_Float16)1032.0f};
    const h2 re = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0x64646464u, u, sel)) - bias;
    const h2 im = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0x64646464u, w, sel)) - bias;
    const h2 sm = re + im, df = im - re;
    s2 va = {0, 0}, vb = {0, 0};
    va = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(va, re, 1.0f, false);
    va = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(va, im, 1.0f, true);
    vb = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(vb, sm, 1.0f, false);
    vb = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(vb, df, 1.0f, true);
    a = __builtin_bit_cast(uint32_t, va);
    b = __builtin_bit_cast(uint32_t, vb);
  }

  // Phases 0/1: transpose rows 0-3 / 4-7; phases 2/3: inputs 0-1 / 2-3 --
  // invalid samples zeroed (rare branch), conversion, one 16-byte store of A
  // and one of B per input.
  template <int PH>
  __device__ static void unpack_phase(const uint32_t (&ld)[ITER][8], uint32_t (&y)[8], uint8_t* st,
                                      uint32_t (&)[SUMS][4], uint32_t (&)[SUMS][4], uint32_t& bad, int tid) {
    if (!L::has_item(tid, 0)) return;
    if constexpr (PH < 2) {
      L::transpose_tq(ld, y, 0, PH, bad);
    } else {
      if (PH == 2 && (bad & 0x88888888u)) L::mask_item(y);
      const int q = tid % QUADS, g = tid / QUADS;
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int c = 2 * (PH - 2) + cc;
        const int row = 4 * q + c;
        v4i va, vb;
        uint32_t a0, b0, a1, b1, a2, b2, a3, b3;
        to_fp8(y[2 * c], 0, a0, b0);
        to_fp8(y[2 * c], 1, a1, b1);
        to_fp8(y[2 * c + 1], 0, a2, b2);
        to_fp8(y[2 * c + 1], 1, a3, b3);
        va = v4i{(int)a0, (int)a1, (int)a2, (int)a3};
        vb = v4i{(int)b0, (int)b1, (int)b2, (int)b3};
        const int off = row * ROWB + ((g ^ L::swz(row)) << 4);
        *reinterpret_cast<v4i*>(st + off) = va;
        *reinterpret_cast<v4i*>(st + ROWS * ROWB + off) = vb;
      }
    }
  }

  __device__ static void unpack_all(const uint32_t (&ld)[ITER][8], uint8_t* st, uint32_t (&sy)[SUMS][4],
                                    uint32_t (&sw)[SUMS][4], uint32_t& bad, int tid) {
    uint32_t y[8];
    unpack_phase<0>(ld, y, st, sy, sw, bad, tid);
    unpack_phase<1>(ld, y, st, sy, sw, bad, tid);
    unpack_phase<2>(ld, y, st, sy, sw, bad, tid);
    unpack_phase<3>(ld, y, st, sy, sw, bad, tid);
  }

  // 32 bytes (16 samples) of one input for a K=64 step; `part` = 2 ks + half.
  __device__ static v8i read_frag(const uint8_t* arr, int row, int part) {
    const uint8_t* base = arr + row * ROWB;
    const v4i lo = *reinterpret_cast<const v4i*>(base + (((2 * part) ^ L::swz(row)) << 4));
    const v4i hi = *reinterpret_cast<const v4i*>(base + (((2 * part + 1) ^ L::swz(row)) << 4));
    return v8i{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  }
};

// One fp8 diagonal unit of 256 inputs (inputs ibase ..), 8 waves.
template <bool ALIGNED>
__device__ void run_diag_f8(const Problem& p, int f, int ibase, int t0, int t1, int tid, uint8_t* lds,
                            uint32_t* s_sy, uint32_t* s_sw, int mode) {
  // Values derived from the thread index are recomputed for every unit: when
  // units run in a loop (the persistent kernel), hoisting them out of it would
  // keep them live across the whole unit and exhaust the registers.
  asm volatile("" : "+v"(tid));
  using G = DiagGeom<256, 4>;
  using S = StageF8<256, G::NT>;
  static_assert(2 * S::BYTES <= G::LDS, "two fp8 stage buffers fit in the unit's LDS");
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / 4, wc = wave % 4;
  const int nchunks = t1 > t0 ? (t1 - t0 + 63) / 64 : 0;
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;

  for (int k = tid; k < 256; k += G::NT) {
    s_sy[k] = 0;  // no correction terms in the unbiased formulation
    s_sw[k] = 0;
  }
  __syncthreads();

  v16f acc[G::FM][G::FN];
#pragma unroll
  for (int x = 0; x < G::FM; ++x)
#pragma unroll
    for (int z = 0; z < G::FN; ++z) acc[x][z] = v16f{0.0f};

  const int half = lane >> 5;
  const int rrow = wr * G::TM + (lane & 31), crow = wc * G::TN + (lane & 31);
  const typename S::Map m{ibase, 64, ibase};
  run_chunks<S, ALIGNED>(p, m, f, t0, t1, stride, tid, lds, s_sy, s_sw, nchunks,
                         [&](const uint8_t* st, int ks) {
                           v8i a[G::FM], b[G::FN];
#pragma unroll
                           for (int x = 0; x < G::FM; ++x) a[x] = S::read_frag(st, rrow + 32 * x, 2 * ks + half);
#pragma unroll
                           for (int x = 0; x < G::FN; ++x)
                             b[x] = S::read_frag(st + 256 * S::ROWB, crow + 32 * x, 2 * ks + half);
#pragma unroll
                           for (int x = 0; x < G::FM; ++x)
#pragma unroll
                             for (int z = 0; z < G::FN; ++z)
                               acc[x][z] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[x], b[z], acc[x][z], 0,
                                                                                           0, 0, 0, 0, 0);
                         });

  // Exact fold: every accumulator holds an integer below 2^24.
  v16i iacc[G::FM][G::FN];
#pragma unroll
  for (int x = 0; x < G::FM; ++x)
#pragma unroll
    for (int z = 0; z < G::FN; ++z)
#pragma unroll
      for (int r = 0; r < 16; ++r) iacc[x][z][r] = (int)acc[x][z][r];

  __syncthreads();
  int* xa = reinterpret_cast<int*>(lds);
  int* xb = xa + G::XAREA;
  constexpr int HW = 2;
  if (wr == 0 && wc >= HW) store_tile<G>(xa, (wc - HW) * G::TN, iacc, lane);
  if (wr == 1 && wc < HW) store_tile<G>(xb, wc * G::TN, iacc, lane);
  __syncthreads();
  combine_quadrant<G>(p, f, ibase, xb, xa, G::H, 0, s_sy, s_sw, 0u, mode, tid);
  __syncthreads();
  if (wr == 0 && wc < HW) store_tile<G>(xa, wc * G::TN, iacc, lane);
  if (wr == 1 && wc >= HW) store_tile<G>(xb, (wc - HW) * G::TN, iacc, lane);
  __syncthreads();
  combine_quadrant<G>(p, f, ibase, xa, xa, 0, 0, s_sy, s_sw, 0u, mode, tid);
  combine_quadrant<G>(p, f, ibase, xb, xb, G::H, G::H, s_sy, s_sw, 0u, mode, tid);
  __syncthreads();
}

// ---- standalone grids -----------------------------------------------------------

// Map the hardware workgroup id so that consecutive logical units land on the
// same XCD (ids are dealt round-robin over 8 XCDs): neighbouring channels then
// share an L2.
__device__ inline int xcd_remap(int b, int n) {
  if (n % 8) return b;
  return (b % 8) * (n / 8) + b / 8;
}

template <int NT>
constexpr int unit_min_blocks = NT >= 512 ? 1 : 2;

// Diagonal units: unit id -> (channel, diagonal block, time split).
// Where time split sp of a unit writes.  part == nullptr: every split adds
// atomically into the accumulator.  Otherwise split 0 writes the accumulator
// in the caller's mode and split sp > 0 stores into partial sum sp - 1 (a
// whole accumulator image at part + (sp - 1) * accumulator words), which
// combine_partials adds in a second launch.
__device__ inline int split_target(Problem& q, int* part, int nsplit, int sp, int mode) {
  if (nsplit == 1) return mode;
  if (part == nullptr) return kWriteAtomic;
  if (sp == 0) return mode;
  q.acc = part + (int64_t)(sp - 1) * ((int64_t)q.n_chan * tri_index(q.n_inputs, 0) * 2);
  return kWriteStore;
}

template <int NB, int WC, bool ALIGNED, int TC>
__global__ __launch_bounds__(128 * WC, unit_min_blocks<128 * WC>) void xmac_diag_i8(Problem p, int nblk, int nsplit,
                                                                                  int tsplit, int mode, int* part) {
  using G = DiagGeom<NB, WC, TC>;
  static_assert(G::NT == 128 * WC, "thread count must match the launch bounds");
  __shared__ __attribute__((aligned(16))) uint8_t lds[G::LDS];
  __shared__ uint32_t s_sy[NB], s_sw[NB];
  int u = xcd_remap(blockIdx.x, gridDim.x);
  const int sp = u % nsplit;
  u /= nsplit;
  const int blk = u % nblk, f = u / nblk;
  const int t0 = sp * tsplit, t1 = min(p.n_time, t0 + tsplit);
  Problem q = p;
  const int m = split_target(q, part, nsplit, sp, mode);
  run_diag<NB, WC, ALIGNED, TC>(q, f, blk * NB, t0, t1, threadIdx.x, lds, s_sy, s_sw, m);
}

// Cross units: unit id -> (channel, (block pair, half), time split).
__device__ inline void pair_decode(int pu, int& I0, int& J0) {
  const int half = pu & 1, pr = pu >> 1;  // pr -> (bi, bj), bi > bj, row-major
  int bi = (int)((sqrtf(8.0f * pr + 1.0f) + 1.0f) * 0.5f);
  while (bi * (bi - 1) / 2 > pr) --bi;
  while ((bi + 1) * bi / 2 <= pr) ++bi;
  const int bj = pr - bi * (bi - 1) / 2;
  I0 = 256 * bi + 128 * half;
  J0 = 256 * bj;
}

template <bool ALIGNED>
__global__ __launch_bounds__(512, 1) void xmac_cross_i8(Problem p, int npair, int nsplit, int tsplit, int mode,
                                                         int* part) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[CrossGeom::LDS];
  __shared__ __attribute__((aligned(16))) uint32_t s_sy[CrossGeom::ROWS], s_sw[CrossGeom::ROWS];
  int u = xcd_remap(blockIdx.x, gridDim.x);
  const int sp = u % nsplit;
  u /= nsplit;
  const int pu = u % npair, f = u / npair;
  int I0, J0;
  pair_decode(pu, I0, J0);
  const int t0 = sp * tsplit, t1 = min(p.n_time, t0 + tsplit);
  Problem q = p;
  const int m = split_target(q, part, nsplit, sp, mode);
  run_cross<ALIGNED>(q, f, I0, J0, t0, t1, threadIdx.x, lds, s_sy, s_sw, m);
}

// acc[i] += sum over s < n_part of part[s * n_words + i].  Four words per
// thread and step where every operand is 16-byte aligned.
__global__ __launch_bounds__(256) void combine_partials(int* acc, const int* part, int64_t n_words, int n_part,
                                                        int vec) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n4 = vec ? n_words / 4 : 0;
  for (int64_t i = i0; i < n4; i += stride) {
    v4i a = reinterpret_cast<const v4i*>(acc)[i];
    for (int s = 0; s < n_part; ++s) a += __builtin_nontemporal_load(reinterpret_cast<const v4i*>(part + s * n_words) + i);
    reinterpret_cast<v4i*>(acc)[i] = a;
  }
  for (int64_t i = 4 * n4 + i0; i < n_words; i += stride) {
    int a = acc[i];
    for (int s = 0; s < n_part; ++s) a += part[s * n_words + i];
    acc[i] = a;
  }
}

template <bool ALIGNED>
__global__ __launch_bounds__(512, 1) void xmac_diag_f8(Problem p, int nsplit, int tsplit, int mode) {
  using G = DiagGeom<256, 4>;
  __shared__ __attribute__((aligned(16))) uint8_t lds[G::LDS];
  __shared__ uint32_t s_sy[256], s_sw[256];
  int u = xcd_remap(blockIdx.x, gridDim.x);
  const int sp = u % nsplit, f = u / nsplit;
  const int t0 = sp * tsplit, t1 = min(p.n_time, t0 + tsplit);
  run_diag_f8<ALIGNED>(p, f, 0, t0, t1, threadIdx.x, lds, s_sy, s_sw, nsplit > 1 ? (int)kWriteAtomic : mode);
}

// The raw-buffer loads need N % 4 == 0, a 4-byte aligned input and a chunk of
// rows (up to 256, the longest chunk) spanning less than 2^31 bytes, so that
// their ranges and offsets stay in 32 bits.
static bool aligned_problem(const Problem& p) {
  const int64_t stride = p.layout == CORRX_LAYOUT_TFI ? (int64_t)p.n_chan * p.n_inputs : p.n_inputs;
  return (p.n_inputs % 4 == 0) && ((reinterpret_cast<uintptr_t>(p.in) & 3) == 0) &&
         256 * stride + p.n_inputs < 0x7FFFFFFF;
}

template <int NB, int WC, int TC>
static int launch_diag(const Problem& p, int nblk, int nsplit, int mode, int* part, hipStream_t s) {
  using G = DiagGeom<NB, WC, TC>;
  const int tsplit = (p.n_time + nsplit - 1) / nsplit;
  const int64_t grid = (int64_t)p.n_chan * nblk * nsplit;
  if (grid > 0x7FFFFFFF) return CORRX_EINVAL;
  if (aligned_problem(p))
    hipLaunchKernelGGL((xmac_diag_i8<NB, WC, true, TC>), dim3((unsigned)grid), dim3(G::NT), 0, s, p, nblk, nsplit,
                       tsplit, mode, part);
  else
    hipLaunchKernelGGL((xmac_diag_i8<NB, WC, false, TC>), dim3((unsigned)grid), dim3(G::NT), 0, s, p, nblk, nsplit,
                       tsplit, mode, part);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

// Diagonal units of NB inputs with TC-sample chunks (tc == 0: the default).
template <int NB, int WC>
static int launch_diag_tc(const Problem& p, int nblk, int nsplit, int mode, int* part, int tc, hipStream_t s) {
  if (tc == 0) tc = diag_tc<NB>;
  // 256-input units hold their loads in flight for 64-sample chunks only
  // (longer chunks spill registers); 64-input units take up to 256.
  switch (tc) {
    case 64: return launch_diag<NB, WC, 64>(p, nblk, nsplit, mode, part, s);
    case 128:
      if constexpr (NB <= 128) return launch_diag<NB, WC, 128>(p, nblk, nsplit, mode, part, s);
      return CORRX_EUNSUPPORTED;
    case 256:
      if constexpr (NB == 64) return launch_diag<NB, WC, 256>(p, nblk, nsplit, mode, part, s);
      return CORRX_EUNSUPPORTED;
    default: return CORRX_EUNSUPPORTED;
  }
}

static int launch_cross(const Problem& p, int npair, int nsplit, int mode, int* part, hipStream_t s) {
  const int tsplit = (p.n_time + nsplit - 1) / nsplit;
  const int64_t grid = (int64_t)p.n_chan * npair * nsplit;
  if (grid > 0x7FFFFFFF) return CORRX_EINVAL;
  if (aligned_problem(p))
    hipLaunchKernelGGL((xmac_cross_i8<true>), dim3((unsigned)grid), dim3(CrossGeom::NT), 0, s, p, npair, nsplit,
                       tsplit, mode, part);
  else
    hipLaunchKernelGGL((xmac_cross_i8<false>), dim3((unsigned)grid), dim3(CrossGeom::NT), 0, s, p, npair, nsplit,
                       tsplit, mode, part);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

static int launch_combine(const Problem& p, int n_part, const int* part, hipStream_t s) {
  const int64_t n_words = (int64_t)p.n_chan * tri_index(p.n_inputs, 0) * 2;
  const int vec = ((reinterpret_cast<uintptr_t>(p.acc) | reinterpret_cast<uintptr_t>(part)) & 15) == 0 &&
                  n_words % 4 == 0;
  const int64_t items = vec ? n_words / 4 : n_words;
  const int64_t grid = std::min<int64_t>((items + 255) / 256, 4096);
  hipLaunchKernelGGL(combine_partials, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(256), 0, s, p.acc, part,
                     n_words, n_part, vec);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

int mfma_units_per_channel(int n_inputs) {
  if (n_inputs <= 256) return 1;
  const int nb = (n_inputs + 255) / 256;
  return nb + nb * (nb - 1);
}

static int launch_f8(const Problem& p, int nsplit, int mode, hipStream_t s) {
  if (p.n_inputs > 256) return CORRX_EUNSUPPORTED;
  const int tsplit = (p.n_time + nsplit - 1) / nsplit;
  if (tsplit > kMaxUnitTimeF8) return CORRX_EINVAL;
  const int64_t grid = (int64_t)p.n_chan * nsplit;
  if (grid > 0x7FFFFFFF) return CORRX_EINVAL;
  if (aligned_problem(p))
    hipLaunchKernelGGL((xmac_diag_f8<true>), dim3((unsigned)grid), dim3(512), 0, s, p, nsplit, tsplit, mode);
  else
    hipLaunchKernelGGL((xmac_diag_f8<false>), dim3((unsigned)grid), dim3(512), 0, s, p, nsplit, tsplit, mode);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

int mfma_unit_inputs(int n_inputs, int tile_cfg) {
  switch (tile_cfg & 0xFF) {
    case CORRX_TILE_DEFAULT: return n_inputs <= 64 ? 64 : n_inputs <= 128 ? 128 : 256;
    case CORRX_TILE_UNIT64: return n_inputs <= 64 ? 64 : 0;
    case CORRX_TILE_UNIT128: return n_inputs <= 128 ? 128 : 0;
    case CORRX_TILE_UNIT256: return 256;
    default: return 0;
  }
}

bool mfma_tile_supported(int n_inputs, int tile_cfg) {
  const int nb = mfma_unit_inputs(n_inputs, tile_cfg);
  const int tc = tile_chunk_samples(tile_cfg);
  if (nb == 0 || (tile_cfg >> 28) != 0) return false;
  if (tc == 0) return true;
  if (tc != 64 && tc != 128 && tc != 256) return false;
  if (nb == 256) return tc == 64;
  return tc <= (nb == 64 ? 256 : 128);
}

int launch_mfma(const Problem& p, int engine, int nsplit, int mode, int tile_cfg, int* part, hipStream_t s) {
  if (engine == CORRX_ENGINE_MFMA_F8) return launch_f8(p, nsplit, mode, s);
  if (engine != CORRX_ENGINE_MFMA_I8) return CORRX_EUNSUPPORTED;
  if (!mfma_tile_supported(p.n_inputs, tile_cfg)) return CORRX_EUNSUPPORTED;
  if (nsplit == 1) part = nullptr;
  const int unit = mfma_unit_inputs(p.n_inputs, tile_cfg), tc = tile_chunk_samples(tile_cfg);
  int rc;
  if (unit == 64) {
    rc = launch_diag_tc<64, 2>(p, 1, nsplit, mode, part, tc, s);
  } else if (unit == 128) {
    rc = launch_diag_tc<128, 2>(p, 1, nsplit, mode, part, tc, s);
  } else {
    const int nb = (p.n_inputs + 255) / 256;
    rc = launch_diag_tc<256, 4>(p, nb, nsplit, mode, part, tc, s);
    if (rc == CORRX_OK && nb > 1) rc = launch_cross(p, nb * (nb - 1), nsplit, mode, part, s);
  }
  if (rc == CORRX_OK && part) rc = launch_combine(p, nsplit - 1, part, s);
  return rc;
}

// ---- persistent batch kernels ---------------------------------------------------
//
// One persistent launch per unit kind: one workgroup per compute unit pulls
// the kind's work items (a contiguous segment of the work list, longest first)
// from the segment's counter until the segment is exhausted.  A kernel per
// kind keeps each unit inlined with its own register allocation; one kernel
// switching between kinds would either share one allocation (and spill) or
// call the units out of line and save their registers on every call.

template <int KIND>
constexpr int batch_nb = (KIND == kUnitDiag64 || KIND == kUnitDiag64K256) ? 64
                         : (KIND == kUnitDiag128x2 || KIND == kUnitDiag128x2K128) ? 128 : 256;
template <int KIND>
constexpr int batch_tc = KIND == kUnitDiag64K256 ? 256 : (KIND == kUnitDiag64 || KIND == kUnitDiag128x2K128) ? 128 : 64;
template <int KIND>
constexpr int batch_lds = KIND == kUnitDiag256 ? DiagGeom<256, 4>::LDS
                          : KIND == kUnitPair  ? CrossGeom::LDS
                                               : 2 * DiagGeom<batch_nb<KIND>, 2, batch_tc<KIND>>::LDS;
template <int KIND>
constexpr int batch_rows = KIND == kUnitPair ? CrossGeom::ROWS : 256;

// Work queues per XCD.  Queue x holds the x-th eighth of a segment's items
// (a contiguous run: neighbouring channels, and the units of one channel).
// Workgroups are dealt to the 8 XCDs round-robin by id, so workgroup b takes
// items from queue b % 8 first, then from the others in turn once that one
// is empty.  Items that share input rows then run on one XCD, at about the
// same time, and share its L2 -- as the unit order of the standalone grids
// does.  Any queue order is correct: every item is taken exactly once.
constexpr int kQueues = 8;

// Next work item of the persistent kernel (same value in every thread), or
// n_items once every queue is empty.  ctr: kQueues counters, zero at launch.
__device__ inline int batch_fetch(int* ctr, int n_items, int* s_item) {
  if (threadIdx.x == 0) {
    const int x0 = (int)(blockIdx.x % kQueues);
    int it = n_items;
    for (int d = 0; d < kQueues; ++d) {
      const int x = (x0 + d) % kQueues;
      const int b = (int)((int64_t)x * n_items / kQueues), e = (int)((int64_t)(x + 1) * n_items / kQueues);
      const int k = atomicAdd(&ctr[x], 1);
      if (k < e - b) {
        it = b + k;
        break;
      }
    }
    *s_item = it;
  }
  __syncthreads();
  const int it = *s_item;
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(it);
}

__device__ inline WorkItem batch_item(const WorkItem* items, int it) {
  WorkItem w;
  w.array = __builtin_amdgcn_readfirstlane(items[it].array);
  w.channel = __builtin_amdgcn_readfirstlane(items[it].channel);
  w.tile = __builtin_amdgcn_readfirstlane(items[it].tile);
  w.t0 = __builtin_amdgcn_readfirstlane(items[it].t0);
  w.t1 = __builtin_amdgcn_readfirstlane(items[it].t1);
  w.kind = __builtin_amdgcn_readfirstlane(items[it].kind);
  w.atomic = __builtin_amdgcn_readfirstlane(items[it].atomic);
  return w;
}

// 64-input units (HBM-bound): 256-thread workgroups, two per compute unit,
// one channel per item, so that each unit's chunk barriers are its own and
// one workgroup's loads are in flight while the other computes.
template <int TC>
__global__ __launch_bounds__(256, 2) void xmac_batch64_i8(BatchArgs args, const WorkItem* items, int n_items,
                                                           int* counter, int base_mode) {
  using G = DiagGeom<64, 2, TC>;
  __shared__ __attribute__((aligned(16))) uint8_t lds[G::LDS];
  __shared__ uint32_t s_sy[64], s_sw[64];
  __shared__ int s_item;
  (void)args;
  const Problem* table = (const Problem*)__builtin_amdgcn_kernarg_segment_ptr();
  int it = batch_fetch(counter, n_items, &s_item);
  while (it < n_items) {
    const WorkItem w = batch_item(items, it);
    const Problem p = table[w.array];
    run_diag<64, 2, true, TC>(p, w.channel, 0, w.t0, w.t1, threadIdx.x, lds, s_sy, s_sw,
                              w.atomic ? (int)kWriteAtomic : base_mode);
    it = batch_fetch(counter, n_items, &s_item);
  }
}

// items / n_items: the kind's segment of the work list.  All arrays must be
// aligned.  The 128x2 kinds run two units side by side, on channels f and f+1
// of the same array (the second writes nothing past the last channel).
template <int KIND>
__global__ __launch_bounds__(512, 1) void xmac_batch_i8(BatchArgs args, const WorkItem* items, int n_items,
                                                         int* counter, int base_mode) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[batch_lds<KIND>];
  __shared__ __attribute__((aligned(16))) uint32_t s_sy[batch_rows<KIND>], s_sw[batch_rows<KIND>];
  __shared__ int s_item;
  // The problem table is the first kernel argument: read it in place in the
  // kernel-argument segment (taking the address of the by-value parameter
  // would copy it to private memory).
  (void)args;
  const Problem* table = (const Problem*)__builtin_amdgcn_kernarg_segment_ptr();
  int it = batch_fetch(counter, n_items, &s_item);
  while (it < n_items) {
    const WorkItem w = batch_item(items, it);
    const Problem p = table[w.array];
    const int mode = w.atomic ? (int)kWriteAtomic : base_mode;
    if constexpr (KIND == kUnitDiag256) {
      run_diag<256, 4, true>(p, w.channel, w.tile * 256, w.t0, w.t1, threadIdx.x, lds, s_sy, s_sw, mode);
    } else if constexpr (KIND == kUnitPair) {
      int I0, J0;
      pair_decode(w.tile, I0, J0);
      run_cross<true>(p, w.channel, I0, J0, w.t0, w.t1, threadIdx.x, lds, s_sy, s_sw, mode);
    } else {
      constexpr int NB = batch_nb<KIND>;
      constexpr int TC = batch_tc<KIND>;
      const int tid = threadIdx.x;
      const int g = tid >> 8, f = w.channel + g;
      run_diag<NB, 2, true, TC>(p, min(f, p.n_chan - 1), 0, w.t0, w.t1, tid & 255,
                                lds + g * DiagGeom<NB, 2, TC>::LDS, s_sy + NB * g, s_sw + NB * g,
                                f < p.n_chan ? mode : (int)kWriteNone);
    }
    it = batch_fetch(counter, n_items, &s_item);
  }
}

__global__ void reset_counters(int* counters, int n) {
  if ((int)threadIdx.x < n) counters[threadIdx.x] = 0;
}

int launch_batch(const BatchArgs& args, const WorkItem* d_items, const BatchSegment* segs, int n_segs, int* d_counters,
                 int grid, int base_mode, hipStream_t s) {
  if (n_segs < 0 || n_segs > kMaxSegments) return CORRX_EINVAL;
  if (n_segs == 0) return CORRX_OK;  // no work items
  static_assert(kBatchCounters == kMaxSegments * kQueues, "queue counters per segment");
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(kBatchCounters), 0, s, d_counters, n_segs * kQueues);
  for (int k = 0; k < n_segs; ++k) {
    const WorkItem* it = d_items + segs[k].begin;
    int* ctr = d_counters + k * kQueues;
    switch (segs[k].kind) {
      case kUnitDiag256:
        hipLaunchKernelGGL(xmac_batch_i8<kUnitDiag256>, dim3(grid), dim3(512), 0, s, args, it, segs[k].count, ctr,
                           base_mode);
        break;
      case kUnitPair:
        hipLaunchKernelGGL(xmac_batch_i8<kUnitPair>, dim3(grid), dim3(512), 0, s, args, it, segs[k].count, ctr,
                           base_mode);
        break;
      case kUnitDiag128x2:
        hipLaunchKernelGGL(xmac_batch_i8<kUnitDiag128x2>, dim3(grid), dim3(512), 0, s, args, it, segs[k].count, ctr,
                           base_mode);
        break;
      case kUnitDiag64:
        hipLaunchKernelGGL(xmac_batch64_i8<128>, dim3(2 * grid), dim3(256), 0, s, args, it, segs[k].count, ctr,
                           base_mode);
        break;
      case kUnitDiag128x2K128:
        hipLaunchKernelGGL(xmac_batch_i8<kUnitDiag128x2K128>, dim3(grid), dim3(512), 0, s, args, it, segs[k].count,
                           ctr, base_mode);
        break;
      case kUnitDiag64K256:
        hipLaunchKernelGGL(xmac_batch64_i8<256>, dim3(2 * grid), dim3(256), 0, s, args, it, segs[k].count, ctr,
                           base_mode);
        break;
      default:
        return CORRX_EINVAL;
    }
  }
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

}  // namespace corrx
