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
// Kernels: fpfb_fir (vector ALU; one thread per (coarse channel, input,
// polyphase branch p) sliding a 12-sample window over 32 frames, output v8 to
// a workspace) and fpfb_dft (int8 MFMA: the 128-point complex DFT of 256
// frames at a time as one real GEMM [v8r v8i] x [[Wr Wi], [-Wi Wr]], the
// twiddle matrix held in registers for the whole launch, then requantised,
// packed and written as TFI rows through LDS).

#include <math.h>
#include <string.h>

#include <new>

#include "corrx_internal.h"

namespace corrx {

namespace {

constexpr int kM = 128, kTaps = 12, kL = kM * kTaps;
constexpr int kFirFrames = 32;  // frames per FIR thread
constexpr int kDftInputs = 64;  // inputs per DFT tile
constexpr int kDftFrames = 4;   // frames per DFT tile: 256 GEMM rows

__device__ inline int round_shift(int v, int s) { return s > 0 ? (v + (1 << (s - 1))) >> s : v; }

// Filter: thread (c, i, p) for frames k0 .. k0 + kFirFrames - 1.  in: complex
// int8 pairs [c][i][n]; work: [c][i][k][256] with re in bytes 0..127 and im
// in 128..255 (the GEMM's K axis).
__global__ __launch_bounds__(128) void fpfb_fir(const char2* in, int8_t* work, const int16_t* taps, int n_inputs,
                                                int n_frames, int s1, int runs) {
  const int p = threadIdx.x;
  const int run = blockIdx.x % runs;
  const int ci = blockIdx.x / runs;  // c * n_inputs + i
  const int k0 = run * kFirFrames;
  const int64_t ns = (int64_t)kM * (n_frames + kTaps - 1);
  const char2* x = in + (int64_t)ci * ns + p;
  int h[kTaps];
#pragma unroll
  for (int j = 0; j < kTaps; ++j) h[j] = taps[kM * j + p];
  int wr[kTaps], wi[kTaps];
#pragma unroll
  for (int j = 0; j < kTaps - 1; ++j) {
    const char2 v = x[(int64_t)kM * (k0 + j)];
    wr[j] = v.x;
    wi[j] = v.y;
  }
  int8_t* out = work + ((int64_t)ci * n_frames + k0) * 256 + p;
#pragma unroll
  for (int k = 0; k < kFirFrames; ++k) {
    if (k0 + k >= n_frames) break;
    const char2 v = x[(int64_t)kM * (k0 + k + kTaps - 1)];
    wr[(k + kTaps - 1) % kTaps] = v.x;
    wi[(k + kTaps - 1) % kTaps] = v.y;
    int ar = 0, ai = 0;
#pragma unroll
    for (int j = 0; j < kTaps; ++j) {
      ar += h[j] * wr[(k + j) % kTaps];
      ai += h[j] * wi[(k + j) % kTaps];
    }
    out[(int64_t)k * 256] = (int8_t)min(127, max(-127, round_shift(ar, s1)));
    out[(int64_t)k * 256 + 128] = (int8_t)min(127, max(-127, round_shift(ai, s1)));
  }
}

// GEMM geometry: 256 rows (row = k_l * 64 + i_l) x 256 columns (0..127 re q,
// 128..255 im q) x K = 256; 8 waves as 2 x 4 tiles of 128 x 64.
__device__ inline int swz16(int row) { return (row ^ (row >> 2)) & 15; }

__global__ __launch_bounds__(512, 1) void fpfb_dft(const int8_t* work, const int8_t* wmat, uint8_t* out,
                                                   int n_inputs, int n_coarse, int n_frames, int s2) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[256 * 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int half = lane >> 5;
  const int iblocks = n_inputs / kDftInputs;
  const int kblocks = (n_frames + kDftFrames - 1) / kDftFrames;

  // Twiddle fragments (the B operand) for this wave's 64 columns and all of
  // K, kept in registers: wmat is [n][k], 256 x 256 int8.
  v4i bfrag[2][8];
#pragma unroll
  for (int z = 0; z < 2; ++z)
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
      bfrag[z][ks] = *reinterpret_cast<const v4i*>(wmat + (64 * wc + 32 * z + (lane & 31)) * 256 + 32 * ks + 16 * half);

  const int64_t tiles = (int64_t)n_coarse * iblocks * kblocks;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int kb = (int)(tile % kblocks);
    const int64_t rest = tile / kblocks;
    const int ib = (int)(rest % iblocks), c = (int)(rest / iblocks);
    const int i0 = ib * kDftInputs, k0 = kb * kDftFrames;
    // Stage the A tile: row (k_l, i_l) = work[c][i0 + i_l][k0 + k_l][0..255],
    // 16 granules of 16 bytes, swizzled; frames past the end are zero.
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int idx = tid + 512 * g;  // 4096 granules
      const int row = idx >> 4, gr = idx & 15;
      const int kl = row >> 6, il = row & 63;
      v4i v = v4i{0, 0, 0, 0};
      if (k0 + kl < n_frames)
        v = *reinterpret_cast<const v4i*>(work + (((int64_t)c * n_inputs + i0 + il) * n_frames + k0 + kl) * 256 + 16 * gr);
      *reinterpret_cast<v4i*>(lds + row * 256 + ((gr ^ swz16(row)) << 4)) = v;
    }
    __syncthreads();
    v16i acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 2; ++z) acc[x][z] = v16i{0};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      v4i a[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int row = 128 * wr + 32 * x + (lane & 31);
        a[x] = *reinterpret_cast<const v4i*>(lds + row * 256 + (((2 * ks + half) ^ swz16(row)) << 4));
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z)
          acc[x][z] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[x], bfrag[z][ks], acc[x][z], 0, 0, 0);
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
          uint32_t word = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = min(7, max(-7, round_shift(acc[x][z][4 * m + r], s2)));
            word |= (uint32_t)(q & 0xFF) << (8 * r);
          }
          const int row = 128 * wr + 32 * x + 8 * m + 4 * half;
          *reinterpret_cast<uint32_t*>(lds + col * 256 + row) = word;
        }
      }
    __syncthreads();
    // Pack and write: thread -> (k_l, q, 16-input segment): bytes
    // (re << 4) | (im & 15) for inputs i0 + 16 s .. +15 of row (k0 + k_l,
    // channel 128 c + (q + 64) % 128).
    {
      const int s = tid & 3, q = (tid >> 2) & 127;
      const int n_chan = 128 * n_coarse;
#pragma unroll
      for (int kl = 0; kl < kDftFrames; ++kl) {
        if (k0 + kl >= n_frames) break;
        const uint4 re = *reinterpret_cast<const uint4*>(lds + q * 256 + 64 * kl + 16 * s);
        const uint4 im = *reinterpret_cast<const uint4*>(lds + (128 + q) * 256 + 64 * kl + 16 * s);
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
  if (n_inputs % kDftInputs) return CORRX_EUNSUPPORTED;
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
  if ((reinterpret_cast<uintptr_t>(in) & 1) || (reinterpret_cast<uintptr_t>(work) & 15) ||
      (reinterpret_cast<uintptr_t>(out) & 15))
    return CORRX_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device) return CORRX_EDEVICE;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int runs = (h->n_frames + kFirFrames - 1) / kFirFrames;
  const int64_t fir_blocks = (int64_t)h->n_coarse * h->n_inputs * runs;
  if (fir_blocks > 0x7FFFFFFF) return CORRX_EINVAL;
  hipLaunchKernelGGL(fpfb_fir, dim3((unsigned)fir_blocks), dim3(128), 0, s, static_cast<const char2*>(in),
                     static_cast<int8_t*>(work), h->d_taps, h->n_inputs, h->n_frames, s1, runs);
  if (hipGetLastError() != hipSuccess) return CORRX_EDEVICE;
  const int64_t tiles =
      (int64_t)h->n_coarse * (h->n_inputs / kDftInputs) * ((h->n_frames + kDftFrames - 1) / kDftFrames);
  const int64_t grid = tiles < 4LL * h->n_cu ? tiles : 4LL * h->n_cu;
  hipLaunchKernelGGL(fpfb_dft, dim3((unsigned)grid), dim3(512), 0, s, static_cast<const int8_t*>(work),
                     h->d_wmat, static_cast<uint8_t*>(out), h->n_inputs, h->n_coarse, h->n_frames, s2);
  return hipGetLastError() == hipSuccess ? CORRX_OK : CORRX_EDEVICE;
}

}  // extern "C"
