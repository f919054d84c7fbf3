// corrx_internal.h -- shared definitions of the gfx950 X-engine kernels and
// the host library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/corrx.h"

namespace corrx {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Word 3 of a raw buffer descriptor on gfx9-family parts (32-bit data format,
// no swizzle): loads past num_records return 0.
constexpr int kBufferRsrcWord3 = 0x00020000;

// Largest time range one work unit integrates.  Bounds the biased int32 sums
// of the MFMA engines (|G_b| <= 900 per sample) well inside int32.
constexpr int kMaxUnitTime = 1 << 20;
// Same for the fp8 engine: fp32 partial sums stay exact integers while
// 98 * samples <= 2^24; 2^17 samples keep a margin.
constexpr int kMaxUnitTimeF8 = 1 << 17;

// int32 bound of the accumulator: |Re|, |Im| <= 2 * 7 * 7 = 98 per sample.
constexpr int64_t kMaxAccSamples = 21913098;  // floor((2^31 - 1) / 98)
// float32 exactness of a dump: |value| <= 2^24.
constexpr int64_t kMaxF32Samples = 171196;    // floor(2^24 / 98)

// Description of one correlation problem as seen by a kernel.
struct Problem {
  const uint8_t* in;   // packed samples
  int* acc;            // int32 [f][b][2]
  int n_inputs;
  int n_chan;
  int n_time;
  int layout;          // CORRX_LAYOUT_*
};

__host__ __device__ inline int64_t row_offset(const Problem& p, int f, int t) {
  return p.layout == CORRX_LAYOUT_TFI ? ((int64_t)t * p.n_chan + f) * p.n_inputs
                                      : ((int64_t)f * p.n_time + t) * p.n_inputs;
}

__host__ __device__ inline int64_t tri_index(int i, int j) {
  return (int64_t)i * (i + 1) / 2 + j;
}

// ---- packed-sample helpers (device) ---------------------------------------

// 4x4 byte transpose: d_r holds byte c = sample (time r, input c); the result
// e_c holds byte r = sample (time r, input c).  v_perm_b32 picks bytes of
// {S0:S1}, selector values 0-3 from S1 and 4-7 from S0.
__device__ inline void transpose4x4(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3,
                                    uint32_t& e0, uint32_t& e1, uint32_t& e2, uint32_t& e3) {
  const uint32_t t01l = __builtin_amdgcn_perm(d1, d0, 0x05010400u);
  const uint32_t t01h = __builtin_amdgcn_perm(d1, d0, 0x07030602u);
  const uint32_t t23l = __builtin_amdgcn_perm(d3, d2, 0x05010400u);
  const uint32_t t23h = __builtin_amdgcn_perm(d3, d2, 0x07030602u);
  e0 = __builtin_amdgcn_perm(t23l, t01l, 0x05040100u);
  e1 = __builtin_amdgcn_perm(t23l, t01l, 0x07060302u);
  e2 = __builtin_amdgcn_perm(t23h, t01h, 0x05040100u);
  e3 = __builtin_amdgcn_perm(t23h, t01h, 0x07060302u);
}

// Bias four packed samples: y = x ^ 0x88 per byte, so that each nibble holds
// its 4-bit two's complement value plus 8 (range 0..15).  A nibble of 0 in y is
// the invalid code.
__device__ inline uint32_t bias4(uint32_t x) { return x ^ 0x88888888u; }

// Nonzero (in bits 3 and 7 of some byte) iff some nibble of y is zero, i.e.
// some sample of the four is invalid.  Exact as an "any" test.
__device__ inline uint32_t invalid_flags(uint32_t y) {
  return (y - 0x11111111u) & ~y & 0x88888888u;
}

// The same test on the raw (unbiased) word x, before masking with 0x88888888:
// bit 3 of ~y equals bit 3 of x, and y - 0x11111111 = (x ^ 0x88888888) +
// 0xEEEEEEEF.  k is 0xEEEEEEEF held in a vector register (see vconst): a VOP3
// instruction on this target reads at most one scalar operand, and with the
// second constant in a vector register the compiler forms one v_xad_u32.
__device__ inline uint32_t invalid_flags_raw(uint32_t x, uint32_t k) { return ((x ^ 0x88888888u) + k) & x; }

// acc | invalid_flags_raw(x, k) with the AND and the OR in one v_bitop3_b32:
// table 0xEC is (S0 & S2) | S1, the same function whichever of S0 and S2 the
// hardware takes as the table's high index bit.
__device__ inline uint32_t or_invalid_flags_raw(uint32_t x, uint32_t k, uint32_t acc) {
  return __builtin_amdgcn_bitop3_b32((x ^ 0x88888888u) + k, acc, x, 0xEC);
}

// A constant the compiler must hold in a vector register: the empty asm
// statement emits no instruction, it only hides the value.  It is not
// volatile, so the compiler may hoist it out of loops.
__device__ inline uint32_t vconst(uint32_t c) {
  asm("" : "+v"(c));
  return c;
}

// Replace every byte of y that has a zero nibble by 0x88 (a valid 0 + 0j):
// an invalid sample contributes nothing.
__device__ inline uint32_t mask_invalid(uint32_t y) {
  const uint32_t nz = (((y & 0x77777777u) + 0x77777777u) | y) & 0x88888888u;  // bit 3 per nonzero nibble
  const uint32_t both = nz & (nz >> 4) & 0x08080808u;                          // bit 3 per valid byte
  const uint32_t one = both >> 3;                                              // 0x01 per valid byte
  const uint32_t m = (one << 8) - one;                                         // 0xFF per valid byte
  return (y & m) | (0x88888888u & ~m);
}

// The same on raw words: with y = x ^ 0x88888888, y & 0x77777777 =
// x & 0x77777777 and bit 3 of y is bit 3 of ~x; the masked sample returns to
// raw 0x00, so the result is x with every invalid byte cleared.
__device__ inline uint32_t mask_invalid_raw(uint32_t x) {
  const uint32_t nz = (((x & 0x77777777u) + 0x77777777u) | ~x) & 0x88888888u;  // bit 3 per nonzero nibble of y
  const uint32_t both = nz & (nz >> 4) & 0x08080808u;                           // bit 3 per valid byte
  const uint32_t one = both >> 3;                                               // 0x01 per valid byte
  return x & ((one << 8) - one);                                                // 0xFF per valid byte
}

// Biased real / imaginary parts (0..15) of four samples, one per byte, from
// biased words y ...
__device__ inline uint32_t bre4(uint32_t y) { return (y >> 4) & 0x0F0F0F0Fu; }
__device__ inline uint32_t bim4(uint32_t y) { return y & 0x0F0F0F0Fu; }
// ... and from raw words x (the bias folded into the mask: one v_bitop3 each).
__device__ inline uint32_t bu4(uint32_t x) { return ((x >> 4) & 0x0F0F0F0Fu) ^ 0x08080808u; }
__device__ inline uint32_t bw4(uint32_t x) { return (x & 0x0F0F0F0Fu) ^ 0x08080808u; }

// Second GEMM operand from the first, for four samples per dword:
//   s = (re+8) + (im+8)      = re + im + 16   in 0..30
//   d = (im+8) - (re+8) + 15 = im - re + 15   in 0..30
// Bytes never carry or borrow into each other; 15 - r = r ^ 15 for a byte
// r <= 15, so d is one v_xad_u32.
__device__ inline uint32_t op_s(uint32_t r, uint32_t i) { return r + i; }
__device__ inline uint32_t op_d(uint32_t r, uint32_t i) { return (r ^ 0x0F0F0F0Fu) + i; }

// Sum of the four bytes of x, added to acc.
__device__ inline uint32_t bytesum(uint32_t x, uint32_t acc) {
  return __builtin_amdgcn_udot4(x, 0x01010101u, acc, false);
}

// ---- launchers (defined in the kernel translation units) ------------------

struct LaunchStatus {
  int status;
};

// How a kernel writes its results into the accumulator.
enum WriteMode {
  kWriteStore = 0,   // accumulator known to be zero and one writer per element: plain store
  kWriteAdd = 1,     // one writer per element: read-modify-write
  kWriteAtomic = 2,  // several writers per element (time splits): atomic add
  kWriteNone = 3     // padding unit: compute, write nothing
};

// int8 / fp8 MFMA engine over one problem.  nsplit: time splits per channel
// (each at most kMaxUnitTime samples).  With nsplit > 1 the int8 engine
// stores splits 1..nsplit-1 into part (nsplit - 1 accumulator images, fully
// overwritten) and adds them into the accumulator in a second launch; with
// part == nullptr, and always for fp8, the splits add atomically.
int launch_mfma(const Problem& p, int engine, int nsplit, int mode, int tile_cfg, int* part, hipStream_t s);
// Work units per channel of the MFMA engine (diagonal blocks + cross units).
int mfma_units_per_channel(int n_inputs);
// Tile codes (include/corrx.h): the inputs of the diagonal unit a code
// selects for n_inputs (0 if it cannot hold them), whether the int8 engine
// serves the code, and the code's chunk length in samples (0 = default).
int mfma_unit_inputs(int n_inputs, int tile_cfg);
bool mfma_tile_supported(int n_inputs, int tile_cfg);
inline int tile_chunk_samples(int tile_cfg) {
  const int k = (tile_cfg >> 24) & 0xF;
  return k == 0 ? 0 : 32 << k;
}
inline int tile_splits(int tile_cfg) { return (tile_cfg >> 8) & 0xFFFF; }
// vector-ALU engine.
int launch_plain(const Problem& p, int nsplit, int mode, hipStream_t s);
// accumulator fill, dump and incoherent beam.
int launch_zero(int* acc, int64_t n_words, hipStream_t s);
int launch_dump(const int* acc, int n_inputs, int n_chan, int order, int dtype, int f_avg, float scale, void* dst,
                hipStream_t s);

// Lane payload pointers of up to four PFBs (8 lanes each), passed by value.
struct PfbLanes {
  const uint8_t* p[32];
};
int launch_pfb_ingest(const PfbLanes& lanes, uint8_t* out, int n_pfb, int n_coarse, int n_time, int natural,
                      hipStream_t s);
int launch_pfb_remap(const int* src, int* dst, int n_inputs, int n_chan, hipStream_t s);
int launch_beam(const Problem& p, int* out, hipStream_t s);

// ---- persistent batched engine ---------------------------------------------

// Unit kinds of the batch kernel.
enum UnitKind {
  kUnitDiag256 = 0,        // one 256-input diagonal block (tile = block index), 64-sample chunks
  kUnitPair = 1,           // one cross unit (tile = pair index: block pair * 2 + half), 64-sample chunks
  kUnitDiag128x2 = 2,      // two 128-input channels (f, f+1) side by side, 64-sample chunks
  kUnitDiag64 = 3,         // one 64-input channel (256-thread workgroups, two per CU), 128-sample chunks
  kUnitDiag128x2K128 = 4,  // as kUnitDiag128x2 with 128-sample chunks
  kUnitDiag64K256 = 5      // as kUnitDiag64 with 256-sample chunks
};
constexpr int kUnitKinds = 6;

constexpr int kMaxBatch = 64;

// One work item of the persistent kernel.
struct WorkItem {
  int array;    // index into BatchArgs::arrays
  int channel;  // channel (first of two for the x2 kinds)
  int tile;     // block / pair index within the channel
  int t0, t1;   // sample range
  int kind;     // UnitKind
  int atomic;   // several items write the same elements (time splits)
};

struct BatchArgs {
  Problem arrays[kMaxBatch];
};

// A contiguous run of the work list holding the items of one unit kind.
struct BatchSegment {
  int kind;
  int begin;
  int count;
};
constexpr int kMaxSegments = kUnitKinds;  // one per unit kind
constexpr int kBatchCounters = kMaxSegments * 8;  // eight queues (one per XCD) per segment

// One persistent launch per segment (after one launch that resets the
// segments' queue counters: kBatchCounters ints at d_counters).  base_mode: kWriteStore (all accumulators freshly
// zeroed) or kWriteAdd; items with time splits always add atomically.
int launch_batch(const BatchArgs& args, const WorkItem* d_items, const BatchSegment* segs, int n_segs, int* d_counters,
                 int grid, int base_mode, hipStream_t s);

}  // namespace corrx
