// fpfb.hip -- fine polyphase filterbank (the F-engine stage before the
// X-engine, Sec. 3.2.1): 12 taps x 128 points, critically sampled, producing
// the packed 4+4-bit samples of 128 fine channels per coarse channel.
//
// Fixed point throughout, so the result is an exact function of the input:
//   FIR   v[k][p] = sum_j h[128 j + p] * x[128 (k + j) + p]   (int32, complex)
//   v8    = clip(round_shift(v, s1), -127, 127)
//   DFT   Y[k][q] = sum_p v8[k][p] * W[p q mod 128]            (int32, complex)
//   out   = clip(round_shift(Y, s2), -7, 7), channel f = (q + 64) mod 128
// with round_shift(v, s) = floor((v + 2^(s-1)) / 2^s), int16 taps h (a
// Hann-windowed sinc scaled to a peak of 32767) and int8 twiddles
// W[n] = rint(127 e^(-2 pi i n / 128)).  The paper gives no filter or
// quantiser; these are this implementation's.
//
// Kernels: fpfb_fir (vector ALU; one thread per (coarse channel, input, pair
// of polyphase branches) over 32 frames, the 12-tap sums as packed int16 dot
// products, output v8 to a workspace) and fpfb_dft (int8 MFMA: the 128-point
// complex DFT of 256 (frame, input) rows at a time as one real GEMM
// [v8r v8i] x [[Wr Wi], [-Wi Wr]], the twiddle matrix held in LDS for the
// whole launch, then requantised, packed and written as TFI rows through LDS).

#include <math.h>
#include <string.h>

#include <new>

#include "corrx_internal.h"

namespace corrx {

namespace {

constexpr int kM = 128, kTaps = 12, kL = kM * kTaps;
constexpr int kFirFrames = 32;  // frames per FIR thread
constexpr int kDftRows = 256;  // GEMM rows per DFT tile: NI inputs x 256 / NI frames

typedef short v2s __attribute__((ext_vector_type(2)));

// Sign-extended int16 pair (lo, hi) from a byte of each of two words, by
// v_perm_b32 (bytes 0..3 of src1, 4..7 of src0; selectors 8..11 give the sign
// of bytes 1, 3, 5, 7).  odd = 0 takes byte 1 of each word, odd = 1 byte 3.
template <int odd>
__device__ inline v2s pair16(uint32_t lo_word, uint32_t hi_word) {
  return __builtin_bit_cast(v2s, __builtin_amdgcn_perm(hi_word, lo_word, odd ? 0x0B070903u : 0x0A050801u));
}

// Filter: thread (c, i, branch pair p, p+1) for frames k0 .. k0 + kFirFrames
// - 1, so that each load and store moves two branches at once.  in: complex
// int8 pairs [c][i][n]; work: [c][i][k][256] with re in bytes 0..127 and im
// in 128..255 (the GEMM's K axis).  The 12-tap sums run as 6 packed int16
// dot products over tap pairs (j, j + 1), the samples of frames m and m + 1
// paired the same way.
__global__ __launch_bounds__(64) void fpfb_fir(const uint32_t* in, int8_t* work, const int16_t* taps, int n_frames,
                                               int s1, int runs) {
  const int p = 2 * threadIdx.x;
  const int run = blockIdx.x % runs;
  const int ci = blockIdx.x / runs;  // c * n_inputs + i
  const int k0 = run * kFirFrames;
  const int64_t ns2 = (int64_t)(kM / 2) * (n_frames + kTaps - 1);  // words (2 samples) per (c, i)
  const uint32_t* x = in + (int64_t)ci * ns2 + threadIdx.x;
  v2s h0[kTaps / 2], h1[kTaps / 2];  // (h[j][p], h[j + 1][p]) for even j
#pragma unroll
  for (int j = 0; j < kTaps; j += 2) {
    h0[j / 2] = v2s{taps[kM * j + p], taps[kM * (j + 1) + p]};
    h1[j / 2] = v2s{taps[kM * j + p + 1], taps[kM * (j + 1) + p + 1]};
  }
  // The whole run's samples are loaded up front so that all the loads are in
  // flight together; frames past the last are clamped to it and not stored.
  // Word m holds bytes (re p, im p, re p+1, im p+1) of frame k0 + m.
  uint32_t raw[kFirFrames + kTaps - 1];
#pragma unroll
  for (int j = 0; j < kFirFrames + kTaps - 1; ++j)
    raw[j] = x[(int64_t)(kM / 2) * min(k0 + j, n_frames + kTaps - 2)];
  // Pairs of frames (m, m + 1) for each of the four components.
  v2s pr0[kFirFrames + kTaps - 2], pi0[kFirFrames + kTaps - 2], pr1[kFirFrames + kTaps - 2],
      pi1[kFirFrames + kTaps - 2];
#pragma unroll
  for (int m = 0; m < kFirFrames + kTaps - 2; ++m) {
    pr0[m] = pair16<0>(raw[m] << 8, raw[m + 1] << 8);
    pr1[m] = pair16<1>(raw[m] << 8, raw[m + 1] << 8);
    pi0[m] = pair16<0>(raw[m], raw[m + 1]);
    pi1[m] = pair16<1>(raw[m], raw[m + 1]);
  }
  const int bias = s1 > 0 ? 1 << (s1 - 1) : 0;  // the rounding term of round_shift
  int8_t* out = work + ((int64_t)ci * n_frames + k0) * 256 + p;
#pragma unroll
  for (int k = 0; k < kFirFrames; ++k) {
    int ar0 = bias, ai0 = bias, ar1 = bias, ai1 = bias;
#pragma unroll
    for (int j = 0; j < kTaps; j += 2) {
      ar0 = __builtin_amdgcn_sdot2(h0[j / 2], pr0[k + j], ar0, false);
      ai0 = __builtin_amdgcn_sdot2(h0[j / 2], pi0[k + j], ai0, false);
      ar1 = __builtin_amdgcn_sdot2(h1[j / 2], pr1[k + j], ar1, false);
      ai1 = __builtin_amdgcn_sdot2(h1[j / 2], pi1[k + j], ai1, false);
    }
    const int vr0 = min(127, max(-127, ar0 >> s1)), vr1 = min(127, max(-127, ar1 >> s1));
    const int vi0 = min(127, max(-127, ai0 >> s1)), vi1 = min(127, max(-127, ai1 >> s1));
    if (k0 + k < n_frames) {
      *reinterpret_cast<uint16_t*>(out + (int64_t)k * 256) = (uint16_t)((vr0 & 0xFF) | ((vr1 & 0xFF) << 8));
      *reinterpret_cast<uint16_t*>(out + (int64_t)k * 256 + 128) = (uint16_t)((vi0 & 0xFF) | ((vi1 & 0xFF) << 8));
    }
  }
}

// GEMM geometry: 256 rows (row = k_l NI + i_l) x 256 columns (0..127 re q,
// 128..255 im q) x K = 256; 8 waves as 2 x 4 tiles of 128 x 64.
__device__ inline int swz16(int row) { return (row ^ (row >> 2)) & 15; }
// Granule swizzle of the transposed codes (one 256-byte row per output
// column): 16 consecutive columns land in 16 different granules for the
// 4-byte stores, and 4 consecutive columns in 4 different frame groups for
// the 16-byte reads of the write phase.
__device__ inline int swzc(int col) { return ((col & 3) << 2) | ((col >> 2) & 3); }

// NI inputs per tile (64, or 128 when the array allows it, so that each
// output row segment is a whole 128-byte line).
template <int NI>
__global__ __launch_bounds__(512, 1) void fpfb_dft(const int8_t* work, const int8_t* wmat, uint8_t* out,
                                                   int n_inputs, int n_coarse, int n_frames, int s2) {
  constexpr int NF = kDftRows / NI;  // frames per tile
  // lds: the A tile (256 rows of 256 bytes), reused for the transposed codes;
  // ldb: the twiddle matrix (the B operand, wmat[n][k], 256 x 256 int8) for
  // the whole launch.  Both are stored as 16 granules of 16 bytes per row,
  // swizzled.
  __shared__ __attribute__((aligned(16))) uint8_t lds[256 * 256];
  __shared__ __attribute__((aligned(16))) uint8_t ldb[256 * 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int half = lane >> 5;
  const int iblocks = n_inputs / NI;
  const int kblocks = (n_frames + NF - 1) / NF;
  const int bias = s2 > 0 ? 1 << (s2 - 1) : 0;
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    const int idx = tid + 512 * g, row = idx >> 4, gr = idx & 15;
    *reinterpret_cast<v4i*>(ldb + row * 256 + ((gr ^ swz16(row)) << 4)) =
        *reinterpret_cast<const v4i*>(wmat + row * 256 + 16 * gr);
  }

  // Tile t: frames NF (t % kblocks) .., inputs NI ((t / kblocks) % iblocks)
  // .., coarse channel t / (kblocks iblocks).  Each thread loads 8 granules of
  // 16 bytes of the A tile: row k_l NI + i_l = work[c][i0 + i_l][k0 + k_l][..]
  // (granule g belongs to frame k_l = g / (NI / 32)); frames past the end are
  // loaded clamped and zeroed when staged.  The next tile's granules are loaded into
  // registers while the current one is multiplied.
  const int tiles = n_coarse * iblocks * kblocks;  // < 2^31, checked by the host
  auto load_tile = [&](int t, v4i* v) {
    const int kb = t % kblocks, rest = t / kblocks;
    const int ib = rest % iblocks, c = rest / iblocks;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int idx = tid + 512 * g;  // 4096 granules
      const int row = idx >> 4, gr = idx & 15;
      const int kl = row / NI, il = row % NI;
      const int k = kb * NF + kl;
      v[g] = *reinterpret_cast<const v4i*>(
          work + (((int64_t)c * n_inputs + ib * NI + il) * n_frames + min(k, n_frames - 1)) * 256 + 16 * gr);
    }
  };
  v4i next[8];
  if ((int)blockIdx.x < tiles) load_tile(blockIdx.x, next);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int kb = tile % kblocks, rest = tile / kblocks;
    const int ib = rest % iblocks, c = rest / iblocks;
    const int i0 = ib * NI, k0 = kb * NF;
    // Stage the A tile.
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int idx = tid + 512 * g;
      const int row = idx >> 4, gr = idx & 15;
      *reinterpret_cast<v4i*>(lds + row * 256 + ((gr ^ swz16(row)) << 4)) =
          k0 + g / (NI / 32) < n_frames ? next[g] : v4i{0, 0, 0, 0};
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) load_tile(tile + gridDim.x, next);
    v16i acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 2; ++z)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[x][z][r] = bias;  // the rounding term of round_shift
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      v4i a[4], b[2];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int row = 128 * wr + 32 * x + (lane & 31);
        a[x] = *reinterpret_cast<const v4i*>(lds + row * 256 + (((2 * ks + half) ^ swz16(row)) << 4));
      }
#pragma unroll
      for (int z = 0; z < 2; ++z) {
        const int row = 64 * wc + 32 * z + (lane & 31);
        b[z] = *reinterpret_cast<const v4i*>(ldb + row * 256 + (((2 * ks + half) ^ swz16(row)) << 4));
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z)
          acc[x][z] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[x], b[z], acc[x][z], 0, 0, 0);
    }
    __syncthreads();
    // Requantise into 4-bit codes, stored transposed: codes[col][row] bytes;
    // accumulator registers 4m .. 4m+3 hold four consecutive rows.
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 2; ++z) {
        const int col = 64 * wc + 32 * z + (lane & 31);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          int q[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) q[r] = min(7, max(-7, acc[x][z][4 * m + r] >> s2));
          // low bytes of q0..q3 into one word (v_perm_b32: 0..3 select src1's
          // bytes, 4..7 src0's, 12 gives zero)
          const uint32_t word = __builtin_amdgcn_perm(q[1], q[0], 0x0C0C0400u) |
                                __builtin_amdgcn_perm(q[3], q[2], 0x04000C0Cu);
          const int row = 128 * wr + 32 * x + 8 * m + 4 * half;
          *reinterpret_cast<uint32_t*>(lds + col * 256 + (((row >> 4) ^ swzc(col)) << 4) + (row & 15)) = word;
        }
      }
    __syncthreads();
    // Pack and write: thread -> (q, segment s mod 4), four (k_l, s) in turn:
    // bytes (re << 4) | (im & 15) for inputs i0 + 16 s .. +15 of row
    // (k0 + k_l, channel 128 c + (q + 64) % 128).
    {
      const int s4 = tid & 3, q = tid >> 2;
      const int n_chan = 128 * n_coarse;
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int kl = it / (NI / 64), s = s4 + 4 * (it % (NI / 64));
        if (k0 + kl >= n_frames) break;
        const int g = ((kl * (NI / 16) + s) ^ swzc(q)) << 4;  // swzc(128 + q) == swzc(q)
        const uint4 re = *reinterpret_cast<const uint4*>(lds + q * 256 + g);
        const uint4 im = *reinterpret_cast<const uint4*>(lds + (128 + q) * 256 + g);
        uint4 o;
        o.x = ((re.x << 4) & 0xF0F0F0F0u) | (im.x & 0x0F0F0F0Fu);
        o.y = ((re.y << 4) & 0xF0F0F0F0u) | (im.y & 0x0F0F0F0Fu);
        o.z = ((re.z << 4) & 0xF0F0F0F0u) | (im.z & 0x0F0F0F0Fu);
        o.w = ((re.w << 4) & 0xF0F0F0F0u) | (im.w & 0x0F0F0F0Fu);
        const int f = 128 * c + ((q + 64) & 127);
        *reinterpret_cast<uint4*>(out + ((int64_t)(k0 + kl) * n_chan + f) * n_inputs + i0 + 16 * s) = o;
      }
    }
  }
}

}  // namespace

}  // namespace corrx

using namespace corrx;

struct corrx_fpfb {
  int n_inputs, n_coarse, n_frames;
  int device;
  int n_cu;
  int16_t* d_taps;
  int8_t* d_wmat;
  int16_t h_taps[kL];
  int8_t h_wmat[256 * 256];
};

namespace {

// Tables from their definitions (double precision, ties to even).
void make_tables(int16_t* taps, int8_t* wmat) {
  const double pi = 3.14159265358979323846;
  double proto[kL], peak = 0.0;
  for (int m = 0; m < kL; ++m) {
    const double w = 0.5 - 0.5 * cos(2.0 * pi * (m + 0.5) / kL);
    const double u = (m - (kL - 1) / 2.0) / kM;
    const double s = u == 0.0 ? 1.0 : sin(pi * u) / (pi * u);
    proto[m] = w * s;
    peak = fmax(peak, fabs(proto[m]));
  }
  for (int m = 0; m < kL; ++m) taps[m] = (int16_t)nearbyint(32767.0 * proto[m] / peak);
  int wr[kM], wi[kM];
  for (int n = 0; n < kM; ++n) {
    wr[n] = (int)nearbyint(127.0 * cos(2.0 * pi * n / kM));
    wi[n] = (int)nearbyint(-127.0 * sin(2.0 * pi * n / kM));
  }
  // wmat[n][k]: column n of B = [[Wr, Wi], [-Wi, Wr]] (k: re p then im p;
  // n: re q then im q), stored row n = output column.
  for (int q = 0; q < kM; ++q)
    for (int p = 0; p < kM; ++p) {
      const int t = (p * q) % kM;
      wmat[q * 256 + p] = (int8_t)wr[t];
      wmat[q * 256 + kM + p] = (int8_t)(-wi[t]);
      wmat[(kM + q) * 256 + p] = (int8_t)wi[t];
      wmat[(kM + q) * 256 + kM + p] = (int8_t)wr[t];
    }
}

}  // namespace

extern "C" {

int corr_fpfb_create(int n_inputs, int n_coarse, int n_frames, corrx_fpfb_t* out) {
  if (!out) return CORRX_EINVAL;
  *out = nullptr;
  if (n_inputs < 1 || n_coarse < 1 || n_frames < 1) return CORRX_EINVAL;
  if (n_inputs % 64) return CORRX_EUNSUPPORTED;
  if ((double)n_coarse * n_inputs * (n_frames + kTaps - 1) * kM * 2 >= 1099511627776.0) return CORRX_EINVAL;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return CORRX_EDEVICE;
  corrx_fpfb* h = new (std::nothrow) corrx_fpfb;
  if (!h) return CORRX_ENOMEM;
  h->n_inputs = n_inputs;
  h->n_coarse = n_coarse;
  h->n_frames = n_frames;
  h->device = dev;
  h->n_cu = prop.multiProcessorCount;
  make_tables(h->h_taps, h->h_wmat);
  h->d_taps = nullptr;
  h->d_wmat = nullptr;
  if (hipMalloc(&h->d_taps, sizeof(h->h_taps)) != hipSuccess || hipMalloc(&h->d_wmat, sizeof(h->h_wmat)) != hipSuccess) {
    (void)hipFree(h->d_taps);
    delete h;
    return CORRX_ENOMEM;
  }
  if (hipMemcpy(h->d_taps, h->h_taps, sizeof(h->h_taps), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_wmat, h->h_wmat, sizeof(h->h_wmat), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(h->d_taps);
    (void)hipFree(h->d_wmat);
    delete h;
    return CORRX_EDEVICE;
  }
  *out = h;
  return CORRX_OK;
}

int corr_fpfb_destroy(corrx_fpfb_t h) {
  if (!h) return CORRX_OK;
  (void)hipFree(h->d_taps);
  (void)hipFree(h->d_wmat);
  delete h;
  return CORRX_OK;
}

size_t corr_fpfb_workspace_bytes(corrx_fpfb_t h) {
  return h ? (size_t)h->n_coarse * h->n_inputs * h->n_frames * 256 : 0;
}

int corr_fpfb_tables(corrx_fpfb_t h, int16_t* taps, int8_t* twiddle_matrix) {
  if (!h) return CORRX_EINVAL;
  if (taps) memcpy(taps, h->h_taps, sizeof(h->h_taps));
  if (twiddle_matrix) memcpy(twiddle_matrix, h->h_wmat, sizeof(h->h_wmat));
  return CORRX_OK;
}

int corr_fpfb(corrx_fpfb_t h, const void* in, int s1, int s2, void* work, void* out, void* stream) {
  if (!h || !in || !work || !out) return CORRX_EINVAL;
  if (s1 < 0 || s1 > 30 || s2 < 0 || s2 > 30) return CORRX_EINVAL;
  if ((reinterpret_cast<uintptr_t>(in) & 3) || (reinterpret_cast<uintptr_t>(work) & 15) ||
      (reinterpret_cast<uintptr_t>(out) & 15))
    return CORRX_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device) return CORRX_EDEVICE;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int runs = (h->n_frames + kFirFrames - 1) / kFirFrames;
  const int64_t fir_blocks = (int64_t)h->n_coarse * h->n_inputs * runs;
  if (fir_blocks > 0x7FFFFFFF) return CORRX_EINVAL;
  hipLaunchKernelGGL(fpfb_fir, dim3((unsigned)fir_blocks), dim3(64), 0, s, static_cast<const uint32_t*>(in),
                     static_cast<int8_t*>(work), h->d_taps, h->n_frames, s1, runs);
  if (hipGetLastError() != hipSuccess) return CORRX_EDEVICE;
  const int ni = h->n_inputs % 128 == 0 ? 128 : 64;
  const int64_t tiles =
      (int64_t)h->n_coarse * (h->n_inputs / ni) * ((h->n_frames + kDftRows / ni - 1) / (kDftRows / ni));
  if (tiles > (1LL << 30)) return CORRX_EINVAL;  // cannot happen below the input size bound
  // One resident block per compute unit (128 KB of LDS), each walking its
  // tiles with the next one's loads in flight.
  const int64_t grid = tiles < h->n_cu ? tiles : h->n_cu;
  if (ni == 128)
    hipLaunchKernelGGL(fpfb_dft<128>, dim3((unsigned)grid), dim3(512), 0, s, static_cast<const int8_t*>(work),
                       h->d_wmat, static_cast<uint8_t*>(out), h->n_inputs, h->n_coarse, h->n_frames, s2);
  else
    hipLaunchKernelGGL(fpfb_dft<64>, dim3((unsigned)grid), dim3(512), 0, s, static_cast<const int8_t*>(work),
                       h->d_wmat, static_cast<uint8_t*>(out), h->n_inputs, h->n_coarse, h->n_frames, s2);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

}  // extern "C"
