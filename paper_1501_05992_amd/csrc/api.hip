// api.hip -- the C ABI of include/corrx.h: argument validation, device check,
// engine dispatch, time-split planning.  No C++ exception crosses the ABI.

#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "corrx_internal.h"

using namespace corrx;

struct corrx_ctx {
  int n_inputs, n_chan, n_time, layout;
  int engine;      // requested (may be AUTO)
  int device;
  int n_cu;
  int64_t samples; // since the last corr_zero
  void* zeroed;    // accumulator last set to zero by corr_zero (while samples == 0)
  int tile;        // int8 engine tile code (corr_set_tile)
  int* part;       // time-split partial sums of the int8 engine (device), or NULL
  int64_t part_bytes;  // its size
};

namespace {

bool device_ok(int* dev, int* n_cu) {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d) != hipSuccess) return false;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return false;
  *dev = d;
  *n_cu = prop.multiProcessorCount;
  return true;
}

int resolve_engine(int e) { return e == CORRX_ENGINE_AUTO ? CORRX_ENGINE_MFMA_I8 : e; }

// Time splits per channel: enough work units to reach `target` (at least 512
// samples per split, at most max_unit per unit).  A split unit adds its output
// with atomics, so units with a large output (256-input blocks: 263 KB per
// channel) split only while fewer than half the compute units would have work;
// small units (64/128-input blocks, the plain engine's 64 x 64 tiles) aim at
// about two per compute unit.
int plan_splits(int n_chan, int units_per_chan, int n_time, int64_t target, int max_unit = kMaxUnitTime) {
  const int64_t units = (int64_t)n_chan * units_per_chan;
  int split = 1;
  while (units * split < target && n_time / (2 * split) >= 512) split *= 2;
  while ((n_time + split - 1) / split > max_unit) ++split;
  return split;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t acc_bytes_of(int n_inputs, int n_chan) { return (int64_t)n_chan * tri_index(n_inputs, 0) * 2 * sizeof(int); }

// Largest partial-sum buffer a handle allocates; beyond it time splits of the
// int8 engine add atomically.
constexpr int64_t kMaxHandlePartBytes = 1LL << 30;

// Time splits of the int8 MFMA engine.  With room for nsplit - 1 partial sums
// (part_cap bytes) a split writes its own image and a second launch adds them,
// so 256-input units (263 KB of output per channel) split until every compute
// unit has one; without, splits add atomically and such units split only
// while fewer than half the compute units would have work.
struct XmacPlan {
  int nsplit;
  int64_t part_bytes;  // 0: no partial sums (one split, or atomic splits)
};

// forced > 0: that many time ranges (more if a range would exceed the
// largest unit), whatever the device.
XmacPlan plan_i8(int n_inputs, int n_chan, int n_time, int n_cu, int64_t part_cap, int forced = 0) {
  const int units = mfma_units_per_channel(n_inputs);
  const bool large = n_inputs > 128;
  int ns = forced;
  if (ns > 0) {
    ns = std::min(ns, n_time);
    while ((n_time + ns - 1) / ns > kMaxUnitTime) ++ns;
  } else {
    ns = plan_splits(n_chan, units, n_time, large ? n_cu : 2LL * n_cu);
  }
  if (ns == 1) return {1, 0};
  const int64_t need = (int64_t)(ns - 1) * acc_bytes_of(n_inputs, n_chan);
  if (need <= part_cap) return {ns, need};
  if (forced > 0) return {ns, 0};
  return {plan_splits(n_chan, units, n_time, large ? n_cu / 2 : 2LL * n_cu), 0};
}

bool valid_shape(int n_inputs, int n_chan, int n_time, int layout) {
  if (n_inputs < 1 || n_inputs > 4096 || n_chan < 1 || n_time < 1) return false;
  if (layout != CORRX_LAYOUT_TFI && layout != CORRX_LAYOUT_FTI) return false;
  return (double)n_inputs * n_chan * n_time < 1099511627776.0;
}

}  // namespace

// ---- library-held scratch of corr_xmac_noalloc ----------------------------------

// Partial sums of corr_xmac_noalloc, one copy per device (the code object is
// loaded once per device).  In host code this name is only a stand-in for
// the device array: kernels get the device address looked up below.
constexpr int64_t kScratchBytes = CORRX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) int scratch[kScratchBytes / sizeof(int)];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceSetup {
  bool done;
  int status;    // CORRX_OK once the address is known
  int n_cu;
  int* scratch;  // this device's copy of `scratch`
};

std::mutex g_setup_mutex;
DeviceSetup g_setup[kMaxDevices];

// Once per device, with that device current: check it and look up the device
// address of its copy of `scratch`.
const DeviceSetup* device_setup() {
  int d = 0, n_cu = 0;
  if (!device_ok(&d, &n_cu) || d < 0 || d >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_setup_mutex);
  DeviceSetup& e = g_setup[d];
  if (!e.done) {
    void* ptr = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    e.status = (rc == hipSuccess && ptr != nullptr) ? CORRX_OK : CORRX_EDEVICE;
    e.scratch = static_cast<int*>(ptr);
    e.n_cu = n_cu;
    e.done = true;
  }
  return &e;
}

}  // namespace

extern "C" {

int corr_abi_version(void) { return CORRX_ABI_VERSION; }

const char* corr_strerror(int status) {
  switch (status) {
    case CORRX_OK: return "ok";
    case CORRX_EINVAL: return "invalid argument";
    case CORRX_ENOMEM: return "out of memory";
    case CORRX_EDEVICE: return "no usable gfx950 device or a HIP call failed";
    case CORRX_EUNSUPPORTED: return "unsupported request";
    case CORRX_EOVERFLOW: return "int32 accumulator could overflow";
    case CORRX_ESCRATCH: return "problem needs more scratch memory than the no-allocation entry point holds";
    default: return "unknown status";
  }
}

int corr_create(int n_inputs, int n_chan, int n_time, int layout, corrx_t* out) {
  if (!out) return CORRX_EINVAL;
  *out = nullptr;
  if (!valid_shape(n_inputs, n_chan, n_time, layout)) return CORRX_EINVAL;
  int dev = 0, n_cu = 0;
  if (!device_ok(&dev, &n_cu)) return CORRX_EDEVICE;
  const XmacPlan plan = plan_i8(n_inputs, n_chan, n_time, n_cu, kMaxHandlePartBytes);
  int* part = nullptr;
  if (plan.part_bytes > 0 && hipMalloc(&part, (size_t)plan.part_bytes) != hipSuccess) return CORRX_ENOMEM;
  corrx_ctx* h = new (std::nothrow) corrx_ctx;
  if (!h) {
    (void)hipFree(part);
    return CORRX_ENOMEM;
  }
  h->tile = CORRX_TILE_DEFAULT;
  h->part = part;
  h->part_bytes = plan.part_bytes;
  h->n_inputs = n_inputs;
  h->n_chan = n_chan;
  h->n_time = n_time;
  h->layout = layout;
  h->engine = CORRX_ENGINE_AUTO;
  h->device = dev;
  h->n_cu = n_cu;
  h->samples = 0;
  h->zeroed = nullptr;
  *out = h;
  return CORRX_OK;
}

int corr_destroy(corrx_t h) {
  if (h && h->part) (void)hipFree(h->part);
  delete h;
  return CORRX_OK;
}

int corr_set_engine(corrx_t h, int engine) {
  if (!h) return CORRX_EINVAL;
  if (engine < CORRX_ENGINE_AUTO || engine > CORRX_ENGINE_MFMA_F8) return CORRX_EINVAL;
  h->engine = engine;
  return CORRX_OK;
}

int corr_set_tile(corrx_t h, int tile_cfg) {
  if (!h || tile_cfg < 0 || (tile_cfg >> 28) != 0 || (tile_cfg & 0xFF) > CORRX_TILE_UNIT256) return CORRX_EINVAL;
  if (mfma_unit_inputs(h->n_inputs, tile_cfg) == 0) return CORRX_EINVAL;
  if (!mfma_tile_supported(h->n_inputs, tile_cfg)) return CORRX_EUNSUPPORTED;
  const XmacPlan plan =
      plan_i8(h->n_inputs, h->n_chan, h->n_time, h->n_cu, kMaxHandlePartBytes, tile_splits(tile_cfg));
  if (plan.part_bytes > h->part_bytes) {
    int* part = nullptr;
    if (hipMalloc(&part, (size_t)plan.part_bytes) != hipSuccess) return CORRX_ENOMEM;
    if (h->part) (void)hipFree(h->part);
    h->part = part;
    h->part_bytes = plan.part_bytes;
  }
  h->tile = tile_cfg;
  return CORRX_OK;
}

int corr_get_engine(corrx_t h) {
  if (!h) return CORRX_EINVAL;
  return resolve_engine(h->engine);
}

size_t corr_acc_bytes(corrx_t h) {
  if (!h) return 0;
  return (size_t)h->n_chan * (size_t)tri_index(h->n_inputs, 0) * 2 * sizeof(int);
}

size_t corr_dump_count(corrx_t h, int order) {
  if (!h) return 0;
  if (order == CORRX_TRI_INPUT) return (size_t)h->n_chan * (size_t)tri_index(h->n_inputs, 0) * 2;
  if (order == CORRX_TRI_STATION_POL) {
    if (h->n_inputs % 2) return 0;
    return (size_t)h->n_chan * (size_t)tri_index(h->n_inputs / 2, 0) * 8;
  }
  return 0;
}

int64_t corr_samples(corrx_t h) { return h ? h->samples : CORRX_EINVAL; }

int corr_zero(corrx_t h, void* acc, void* stream) {
  if (!h || !acc) return CORRX_EINVAL;
  const int rc = launch_zero(static_cast<int*>(acc), (int64_t)(corr_acc_bytes(h) / sizeof(int)), as_stream(stream));
  if (rc == CORRX_OK) {
    h->samples = 0;
    h->zeroed = acc;
  }
  return rc;
}

int corr_xmac(corrx_t h, const void* in, void* acc, void* stream) {
  if (!h || !in || !acc) return CORRX_EINVAL;
  if (h->samples + h->n_time > kMaxAccSamples) return CORRX_EOVERFLOW;
  Problem p;
  p.in = static_cast<const uint8_t*>(in);
  p.acc = static_cast<int*>(acc);
  p.n_inputs = h->n_inputs;
  p.n_chan = h->n_chan;
  p.n_time = h->n_time;
  p.layout = h->layout;
  const int engine = resolve_engine(h->engine);
  // A freshly zeroed accumulator (corr_zero on this handle and stream, no
  // correlation since) is overwritten instead of read and added to.
  const int mode = (h->samples == 0 && h->zeroed == acc) ? kWriteStore : kWriteAdd;
  int rc;
  if (engine == CORRX_ENGINE_PLAIN) {
    const int nbk = (h->n_inputs + 63) / 64;
    rc = launch_plain(p, plan_splits(h->n_chan, nbk * (nbk + 1) / 2, h->n_time, 2LL * h->n_cu), mode,
                      as_stream(stream));
  } else if (engine == CORRX_ENGINE_MFMA_F8) {
    rc = launch_mfma(p, engine, plan_splits(h->n_chan, 1, h->n_time, h->n_cu / 2, kMaxUnitTimeF8), mode,
                     CORRX_TILE_DEFAULT, nullptr, as_stream(stream));
  } else {
    const XmacPlan plan = plan_i8(h->n_inputs, h->n_chan, h->n_time, h->n_cu, h->part_bytes, tile_splits(h->tile));
    rc = launch_mfma(p, engine, plan.nsplit, mode, h->tile, plan.part_bytes ? h->part : nullptr, as_stream(stream));
  }
  if (rc == CORRX_OK) h->samples += h->n_time;
  return rc;
}

int corr_xmac_noalloc(const void* in, void* acc, int n_inputs, int n_chan, int n_time, int layout, int accumulate,
                      void* stream) {
  if (!in || !acc || (accumulate != 0 && accumulate != 1)) return CORRX_EINVAL;
  if (!valid_shape(n_inputs, n_chan, n_time, layout)) return CORRX_EINVAL;
  if (n_time > kMaxAccSamples) return CORRX_EOVERFLOW;
  const DeviceSetup* setup = device_setup();
  if (!setup || setup->status != CORRX_OK) return CORRX_EDEVICE;
  // corr_xmac's plan for a handle of this shape; its partial sums must fit.
  const XmacPlan plan = plan_i8(n_inputs, n_chan, n_time, setup->n_cu, kMaxHandlePartBytes);
  if (plan.part_bytes > kScratchBytes) return CORRX_ESCRATCH;
  Problem p;
  p.in = static_cast<const uint8_t*>(in);
  p.acc = static_cast<int*>(acc);
  p.n_inputs = n_inputs;
  p.n_chan = n_chan;
  p.n_time = n_time;
  p.layout = layout;
  int mode = accumulate ? kWriteAdd : kWriteStore;
  if (mode == kWriteStore && plan.nsplit > 1 && plan.part_bytes == 0) {
    // atomic splits add into the accumulator: clear it first (a kernel, no memset)
    const int rc = launch_zero(p.acc, acc_bytes_of(n_inputs, n_chan) / (int64_t)sizeof(int), as_stream(stream));
    if (rc != CORRX_OK) return rc;
    mode = kWriteAdd;
  }
  return launch_mfma(p, CORRX_ENGINE_MFMA_I8, plan.nsplit, mode, CORRX_TILE_DEFAULT,
                     plan.part_bytes ? setup->scratch : nullptr, as_stream(stream));
}

int corr_dump(corrx_t h, const void* acc, int order, int dtype, void* dst, void* stream) {
  if (!h || !acc || !dst) return CORRX_EINVAL;
  if (order != CORRX_TRI_INPUT && order != CORRX_TRI_STATION_POL) return CORRX_EINVAL;
  if (dtype != CORRX_I32 && dtype != CORRX_F32) return CORRX_EINVAL;
  if (order == CORRX_TRI_STATION_POL && h->n_inputs % 2) return CORRX_EINVAL;
  if (dtype == CORRX_F32 && h->samples > kMaxF32Samples) return CORRX_EOVERFLOW;
  const char* a = static_cast<const char*>(acc);
  const char* d = static_cast<const char*>(dst);
  const size_t na = corr_acc_bytes(h), nd = corr_dump_count(h, order) * 4;
  if (a < d + nd && d < a + na) return CORRX_EINVAL;
  return launch_dump(static_cast<const int*>(acc), h->n_inputs, h->n_chan, order, dtype, 1, 1.0f, dst,
                     as_stream(stream));
}

int corr_dump_avg(corrx_t h, const void* acc, int order, int dtype, int f_avg, int t_avg, void* dst, void* stream) {
  if (!h || !acc || !dst) return CORRX_EINVAL;
  if (order != CORRX_TRI_INPUT && order != CORRX_TRI_STATION_POL) return CORRX_EINVAL;
  if (dtype != CORRX_I32 && dtype != CORRX_F32) return CORRX_EINVAL;
  if (order == CORRX_TRI_STATION_POL && h->n_inputs % 2) return CORRX_EINVAL;
  if (f_avg < 1 || (f_avg & (f_avg - 1)) || h->n_chan % f_avg) return CORRX_EINVAL;
  if (t_avg < 1 || (t_avg & (t_avg - 1)) || (int64_t)f_avg * t_avg > 4096) return CORRX_EINVAL;
  // Integer sums of f_avg channels stay exact in int32, and in float32 while
  // |sum| <= 98 * samples * f_avg <= 2^24.
  if (h->samples * f_avg > kMaxAccSamples) return CORRX_EOVERFLOW;
  if (dtype == CORRX_F32 && h->samples * f_avg > kMaxF32Samples) return CORRX_EOVERFLOW;
  const char* a = static_cast<const char*>(acc);
  const char* d = static_cast<const char*>(dst);
  const size_t na = corr_acc_bytes(h), nd = corr_dump_count(h, order) / f_avg * 4;
  if (a < d + nd && d < a + na) return CORRX_EINVAL;
  return launch_dump(static_cast<const int*>(acc), h->n_inputs, h->n_chan, order, dtype, f_avg,
                     1.0f / (float)(f_avg * t_avg), dst, as_stream(stream));
}

int corr_pfb_ingest(corrx_t h, const void* const* lanes, int order, void* in, void* stream) {
  if (!h || !lanes || !in) return CORRX_EINVAL;
  if (order != CORRX_ORDER_PACKET && order != CORRX_ORDER_NATURAL) return CORRX_EINVAL;
  if (h->layout != CORRX_LAYOUT_TFI || h->n_inputs % 64 || h->n_inputs > 256 || h->n_chan % 128)
    return CORRX_EUNSUPPORTED;
  if (reinterpret_cast<uintptr_t>(in) & 15) return CORRX_EINVAL;
  const int n_pfb = h->n_inputs / 64;
  PfbLanes pl;
  memset(&pl, 0, sizeof(pl));
  for (int k = 0; k < 8 * n_pfb; ++k) {
    if (!lanes[k] || (reinterpret_cast<uintptr_t>(lanes[k]) & 15)) return CORRX_EINVAL;
    pl.p[k] = static_cast<const uint8_t*>(lanes[k]);
  }
  return launch_pfb_ingest(pl, static_cast<uint8_t*>(in), n_pfb, h->n_chan / 128, h->n_time,
                           order == CORRX_ORDER_NATURAL, as_stream(stream));
}

int corr_pfb_remap(corrx_t h, const void* acc_pkt, void* acc_nat, void* stream) {
  if (!h || !acc_pkt || !acc_nat) return CORRX_EINVAL;
  if (h->n_inputs % 64) return CORRX_EUNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(acc_pkt) & 7) || (reinterpret_cast<uintptr_t>(acc_nat) & 7)) return CORRX_EINVAL;
  const char* a = static_cast<const char*>(acc_pkt);
  const char* d = static_cast<const char*>(acc_nat);
  const size_t na = corr_acc_bytes(h);
  if (a < d + na && d < a + na) return CORRX_EINVAL;
  return launch_pfb_remap(static_cast<const int*>(acc_pkt), static_cast<int*>(acc_nat), h->n_inputs, h->n_chan,
                          as_stream(stream));
}

int corr_beam(corrx_t h, const void* in, void* out, void* stream) {
  if (!h || !in || !out) return CORRX_EINVAL;
  Problem p;
  p.in = static_cast<const uint8_t*>(in);
  p.acc = nullptr;
  p.n_inputs = h->n_inputs;
  p.n_chan = h->n_chan;
  p.n_time = h->n_time;
  p.layout = h->layout;
  return launch_beam(p, static_cast<int*>(out), as_stream(stream));
}

}  // extern "C"
