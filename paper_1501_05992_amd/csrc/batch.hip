// batch.hip -- uneven batch of arrays in one persistent launch: planning of
// the work list (unit kind, time splits, longest-first order) and the C ABI.

#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "corrx_internal.h"

using namespace corrx;

struct corrx_batch {
  int n;
  corrx_desc d[kMaxBatch];
  int kind[kMaxBatch];
  int splits[kMaxBatch];
  int device;
  int grid;
  int n_items;
  WorkItem* d_items;
  int* d_counter;  // the queue counters of every segment (kBatchCounters)
  int n_segs;
  BatchSegment segs[kMaxSegments];
  void* zeroed[kMaxBatch];  // accumulators set to zero by corr_batch_zero and not written since
  int64_t samples[kMaxBatch];  // samples accumulated per array since corr_batch_zero
};

namespace {

bool gfx950(int* dev, int* n_cu) {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d) != hipSuccess) return false;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return false;
  *dev = d;
  *n_cu = prop.multiProcessorCount;
  return true;
}

// Relative cost of one item: matrix-core work (square of the staged inputs
// times samples) against the bytes it streams, whichever dominates.  The
// constant converts bytes to the same unit at the int8 MFMA / HBM ridge.
double item_cost(int kind, int n_inputs, int samples) {
  double mfma, bytes;
  switch (kind) {
    case kUnitDiag64:
    case kUnitDiag64K256:
      mfma = 64.0 * 64 * samples;
      bytes = 1.0 * n_inputs * samples;
      break;
    case kUnitDiag128x2:
    case kUnitDiag128x2K128:
      mfma = 2.0 * 128 * 128 * samples;
      bytes = 2.0 * n_inputs * samples;
      break;
    case kUnitPair:
      mfma = 2.0 * 128 * 256 * samples;
      bytes = 384.0 * samples;
      break;
    default:
      mfma = 256.0 * 256 * samples;
      bytes = 256.0 * samples;
      break;
  }
  return std::max(mfma, bytes * 625.0 / 4.0);
}

// Unit kind of a tile code's unit and chunk length (tc == 0: default), or -1
// if the kernels have no such variant.
int unit_kind(int unit, int n_inputs, int tc) {
  if (unit == CORRX_TILE_UNIT64 || (unit == CORRX_TILE_DEFAULT && n_inputs <= 64)) {
    if (tc == 0 || tc == 128) return kUnitDiag64;
    return tc == 256 ? kUnitDiag64K256 : -1;
  }
  if (unit == CORRX_TILE_UNIT128 || (unit == CORRX_TILE_DEFAULT && n_inputs <= 128)) {
    if (tc == 0 || tc == 64) return kUnitDiag128x2;
    return tc == 128 ? kUnitDiag128x2K128 : -1;
  }
  return (tc == 0 || tc == 64) ? kUnitDiag256 : -1;
}

// Channels one work item covers: the 128-input kinds run two channels side
// by side in one 512-thread workgroup.
int items_channels(int kind) { return (kind == kUnitDiag128x2 || kind == kUnitDiag128x2K128) ? 2 : 1; }

int units_of(int kind, int n_inputs) {
  if (kind != kUnitDiag256) return 1;
  const int nb = (n_inputs + 255) / 256;
  return nb + nb * (nb - 1);  // diagonal blocks, then cross units
}

}  // namespace

extern "C" {

int corr_batch_create(const corrx_desc* descs, int n, int engine, const int* tile_cfg, corrx_batch_t* out) {
  if (!out) return CORRX_EINVAL;
  *out = nullptr;
  if (!descs || n < 1 || n > kMaxBatch) return CORRX_EINVAL;
  if (engine != CORRX_ENGINE_AUTO && engine != CORRX_ENGINE_MFMA_I8) return CORRX_EUNSUPPORTED;
  for (int a = 0; a < n; ++a) {
    const corrx_desc& d = descs[a];
    if (d.n_inputs < 1 || d.n_inputs > 4096 || d.n_chan < 1 || d.n_time < 1) return CORRX_EINVAL;
    if (d.layout != CORRX_LAYOUT_TFI && d.layout != CORRX_LAYOUT_FTI) return CORRX_EINVAL;
    if ((double)d.n_inputs * d.n_chan * d.n_time >= 1099511627776.0) return CORRX_EINVAL;
    const int64_t stride = d.layout == CORRX_LAYOUT_TFI ? (int64_t)d.n_chan * d.n_inputs : d.n_inputs;
    const int unit = tile_cfg ? (tile_cfg[a] & 0xFF) : CORRX_TILE_DEFAULT;
    if (tile_cfg) {
      const int spl = tile_splits(tile_cfg[a]);
      if (unit > CORRX_TILE_UNIT256 || spl > 4096 || (tile_cfg[a] >> 28) != 0) return CORRX_EINVAL;
      if ((unit == CORRX_TILE_UNIT64 && d.n_inputs > 64) || (unit == CORRX_TILE_UNIT128 && d.n_inputs > 128))
        return CORRX_EINVAL;
      if (unit_kind(unit, d.n_inputs, tile_chunk_samples(tile_cfg[a])) < 0) return CORRX_EUNSUPPORTED;
    }
    // one chunk of rows (256 for 64-input units, else 128 at most) must span
    // less than 2^31 bytes
    const bool unit64 = unit == CORRX_TILE_UNIT64 || (unit == CORRX_TILE_DEFAULT && d.n_inputs <= 64);
    if (d.n_inputs % 4 != 0 || (unit64 ? 256 : 128) * stride + d.n_inputs >= 0x7FFFFFFF) return CORRX_EUNSUPPORTED;
  }
  int dev = 0, n_cu = 0;
  if (!gfx950(&dev, &n_cu)) return CORRX_EDEVICE;
  corrx_batch* b = new (std::nothrow) corrx_batch;
  if (!b) return CORRX_ENOMEM;
  memset(b, 0, sizeof(*b));
  b->n = n;
  b->device = dev;
  b->grid = n_cu;

  // Unit kind per array.
  double total = 0.0;
  for (int a = 0; a < n; ++a) {
    const corrx_desc& d = descs[a];
    b->d[a] = d;
    const int unit = tile_cfg ? (tile_cfg[a] & 0xFF) : CORRX_TILE_DEFAULT;
    const int kind = unit_kind(unit, d.n_inputs, tile_cfg ? tile_chunk_samples(tile_cfg[a]) : 0);
    b->kind[a] = kind;
    const int per_item_chan = items_channels(kind);
    const int64_t items = (int64_t)((d.n_chan + per_item_chan - 1) / per_item_chan) * units_of(kind, d.n_inputs);
    total += (double)items * item_cost(kind, d.n_inputs, d.n_time);
  }
  // Time splits per array: requested, or enough that no item costs more than
  // half of a compute unit's fair share (load balance of the longest-first
  // schedule), with at least 512 samples per split and at most kMaxUnitTime.
  // Splits are not free: a split item adds its output with atomics, which
  // costs more than the imbalance of a few whole items per compute unit.
  const double target = total / (2.0 * n_cu);
  std::vector<WorkItem> items;
  for (int a = 0; a < n; ++a) {
    const corrx_desc& d = descs[a];
    const int kind = b->kind[a];
    int spl = tile_cfg ? tile_splits(tile_cfg[a]) : 0;
    if (spl == 0) {
      spl = 1;
      while (item_cost(kind, d.n_inputs, (d.n_time + spl - 1) / spl) > target && d.n_time / (2 * spl) >= 512)
        spl *= 2;
    }
    while ((d.n_time + spl - 1) / spl > kMaxUnitTime) ++spl;
    spl = std::min(spl, d.n_time);
    b->splits[a] = spl;
    const int tsplit = (d.n_time + spl - 1) / spl;
    const int per_item_chan = items_channels(kind);
    const int nb = (d.n_inputs + 255) / 256;
    for (int f = 0; f < d.n_chan; f += per_item_chan)
      for (int u = 0; u < units_of(kind, d.n_inputs); ++u)
        for (int sp = 0; sp < spl; ++sp) {
          WorkItem w;
          w.array = a;
          w.channel = f;
          w.t0 = sp * tsplit;
          w.t1 = std::min(d.n_time, w.t0 + tsplit);
          if (w.t0 >= w.t1) continue;
          w.atomic = spl > 1;
          if (kind == kUnitDiag256 && u >= nb) {
            w.kind = kUnitPair;
            w.tile = u - nb;
          } else {
            w.kind = kind;
            w.tile = u;
          }
          items.push_back(w);
        }
  }
  // Longest first within each unit kind (the dynamic queue then balances the
  // tail); the kinds form contiguous segments, one persistent launch each, in
  // the order of their most expensive item.
  std::stable_sort(items.begin(), items.end(), [&](const WorkItem& x, const WorkItem& y) {
    return item_cost(x.kind, b->d[x.array].n_inputs, x.t1 - x.t0) >
           item_cost(y.kind, b->d[y.array].n_inputs, y.t1 - y.t0);
  });
  int kind_rank[kMaxSegments];
  for (int k = 0; k < kMaxSegments; ++k) kind_rank[k] = kMaxSegments;
  int n_kinds = 0;
  for (const WorkItem& w : items)
    if (kind_rank[w.kind] == kMaxSegments) kind_rank[w.kind] = n_kinds++;
  std::stable_sort(items.begin(), items.end(),
                   [&](const WorkItem& x, const WorkItem& y) { return kind_rank[x.kind] < kind_rank[y.kind]; });
  b->n_segs = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    if (b->n_segs == 0 || b->segs[b->n_segs - 1].kind != items[k].kind)
      b->segs[b->n_segs++] = BatchSegment{items[k].kind, (int)k, 0};
    ++b->segs[b->n_segs - 1].count;
  }
  if (items.size() > 0x7FFFFFFF) {
    delete b;
    return CORRX_EINVAL;
  }
  b->n_items = (int)items.size();
  if (hipMalloc(&b->d_items, sizeof(WorkItem) * items.size()) != hipSuccess ||
      hipMalloc(&b->d_counter, sizeof(int) * kBatchCounters) != hipSuccess) {
    (void)hipFree(b->d_items);
    delete b;
    return CORRX_ENOMEM;
  }
  if (hipMemcpy(b->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_counter);
    delete b;
    return CORRX_EDEVICE;
  }
  *out = b;
  return CORRX_OK;
}

int corr_batch_destroy(corrx_batch_t b) {
  if (!b) return CORRX_OK;
  (void)hipFree(b->d_items);
  (void)hipFree(b->d_counter);
  delete b;
  return CORRX_OK;
}

int64_t corr_batch_items(corrx_batch_t b) { return b ? b->n_items : CORRX_EINVAL; }

int corr_batch_plan(corrx_batch_t b, int array, int* kind, int* splits) {
  if (!b || array < 0 || array >= b->n) return CORRX_EINVAL;
  if (kind) *kind = b->kind[array];
  if (splits) *splits = b->splits[array];
  return CORRX_OK;
}

int corr_batch_zero(corrx_batch_t b, void* const* accs, void* stream) {
  if (!b || !accs) return CORRX_EINVAL;
  for (int a = 0; a < b->n; ++a)
    if (!accs[a]) return CORRX_EINVAL;
  for (int a = 0; a < b->n; ++a) {
    const int64_t words = (int64_t)b->d[a].n_chan * tri_index(b->d[a].n_inputs, 0) * 2;
    const int rc = launch_zero(static_cast<int*>(accs[a]), words, reinterpret_cast<hipStream_t>(stream));
    if (rc != CORRX_OK) return rc;
    b->zeroed[a] = accs[a];
    b->samples[a] = 0;
  }
  return CORRX_OK;
}

int64_t corr_batch_samples(corrx_batch_t b, int array) {
  if (!b || array < 0 || array >= b->n) return CORRX_EINVAL;
  return b->samples[array];
}

int corr_batch_xmac(corrx_batch_t b, const void* const* ins, void* const* accs, void* stream) {
  if (!b || !ins || !accs) return CORRX_EINVAL;
  BatchArgs args;
  memset(&args, 0, sizeof(args));
  int fresh = 1;
  for (int a = 0; a < b->n; ++a) {
    if (!ins[a] || !accs[a]) return CORRX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(ins[a]) & 3) || (reinterpret_cast<uintptr_t>(accs[a]) & 7)) return CORRX_EINVAL;
    Problem& p = args.arrays[a];
    p.in = static_cast<const uint8_t*>(ins[a]);
    p.acc = static_cast<int*>(accs[a]);
    p.n_inputs = b->d[a].n_inputs;
    p.n_chan = b->d[a].n_chan;
    p.n_time = b->d[a].n_time;
    p.layout = b->d[a].layout;
    fresh &= b->zeroed[a] == accs[a];
    // |Re|, |Im| <= 98 per sample: refuse before any int32 accumulator could wrap
    if (b->samples[a] + b->d[a].n_time > kMaxAccSamples) return CORRX_EOVERFLOW;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return CORRX_EDEVICE;
  // Freshly zeroed accumulators (all of them) are overwritten, not added to.
  const int rc = launch_batch(args, b->d_items, b->segs, b->n_segs, b->d_counter, b->grid,
                              fresh ? kWriteStore : kWriteAdd, reinterpret_cast<hipStream_t>(stream));
  for (int a = 0; a < b->n; ++a) b->zeroed[a] = nullptr;
  if (rc == CORRX_OK)
    for (int a = 0; a < b->n; ++a) b->samples[a] += b->d[a].n_time;
  return rc;
}

}  // extern "C"
