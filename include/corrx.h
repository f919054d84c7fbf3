/*
 * corrx.h -- C ABI of the MI355X (gfx950) X-engine.
 *
 * The X-engine is the cross-multiply-accumulate stage of an FX correlator
 * (Ord et al., "The Murchison Widefield Array Correlator", Sec. 2 eq. (3) and
 * Sec. 3.4).  For every fine frequency channel f and every input pair
 * 0 <= j <= i < N it forms
 *
 *     V_f[i][j] = sum_t x_i(f,t) * conj(x_j(f,t))
 *
 * from packed 4+4-bit complex samples, keeping the lower triangle of the
 * Hermitian matrix including the autocorrelations (Appendix C, "GPU Output").
 * All sums are exact integers: the library accumulates in int32.
 *
 * Conventions shared by every entry point:
 *   - Sample byte (Appendix A, data-format list): high nibble = real part,
 *     low nibble = imaginary part, 4-bit two's complement.  The code 8 (-8)
 *     marks invalid data; a sample with the code in either nibble contributes
 *     nothing (it is treated as 0 + 0j).
 *   - Input index i = 2*station + polarisation (Appendix C, "GPU Input":
 *     station, then polarisation, fastest last).
 *   - Pointers named in, acc, dst, bufs are DEVICE pointers (HIP device memory,
 *     e.g. torch tensors) owned by the caller; they must stay valid until the
 *     work queued on `stream` has completed.  `stream` is a hipStream_t (NULL =
 *     the null stream).  Calls enqueue work and return without synchronising;
 *     device-side faults surface at the caller's next synchronisation.
 *   - Every entry point returns CORRX_OK or a negative status.  Argument errors
 *     are detected before anything is enqueued.  No C++ exception crosses the ABI.
 *   - A handle is used by one host thread and one stream at a time.  Distinct
 *     handles may be used concurrently on different streams.
 *   - Calls other than the *_create / *_destroy ones and corr_set_tile (a
 *     set-up call) allocate nothing and enqueue only kernels on `stream` (no
 *     memset, no synchronisation), so they may be captured into a HIP graph.  The handle's host-side state (samples
 *     since corr_zero, whether the accumulator was just zeroed, which selects
 *     overwrite or add) advances when a call is made, not when a graph replays
 *     it: capture whole integrations (corr_zero ... corr_dump) so that every
 *     replay starts from a zeroed accumulator.
 */
#ifndef CORRX_H
#define CORRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CORRX_ABI_VERSION 1

typedef struct corrx_ctx *corrx_t;
typedef struct corrx_batch *corrx_batch_t;
typedef struct corrx_fpfb *corrx_fpfb_t;

/* Status codes. */
enum {
    CORRX_OK = 0,
    CORRX_EINVAL = -1,       /* bad argument: null pointer, size, enum value */
    CORRX_ENOMEM = -2,       /* host or device allocation failed */
    CORRX_EDEVICE = -3,      /* no usable gfx950 device, or a HIP call / launch failed */
    CORRX_EUNSUPPORTED = -4, /* valid request this library does not serve */
    CORRX_EOVERFLOW = -5,    /* the int32 accumulator could overflow: zero it first */
    CORRX_ESCRATCH = -6      /* corr_xmac_noalloc: the problem needs more than its scratch */
};

/* Input layouts of the packed sample buffer (N*F*T bytes). */
enum {
    CORRX_LAYOUT_TFI = 0, /* byte (t*F + f)*N + i: the paper's GPU input order (App. C) */
    CORRX_LAYOUT_FTI = 1  /* byte (f*T + t)*N + i: one contiguous block per channel */
};

/* Output orders of corr_dump. */
enum {
    /* f, then b = i*(i+1)/2 + j for i >= j, then {re, im}: N(N+1)/2 per channel. */
    CORRX_TRI_INPUT = 0,
    /* Appendix C "GPU Output": f, then s1 >= s2 packed as s1*(s1+1)/2 + s2, then
     * p1, p2 in {0,1}, then {re, im}; element = V[2*s1+p1][2*s2+p2].  For s1 == s2
     * the (p1=0, p2=1) element is conj(V[2*s1+1][2*s1]).  2N(N/2+1) per channel
     * (33024 for N = 256, Sec. 3.4.3).  Needs an even N. */
    CORRX_TRI_STATION_POL = 1
};

/* Element types of corr_dump (both exact at the sizes corr_dump accepts). */
enum { CORRX_I32 = 0, CORRX_F32 = 1 };

/* Compute engines.  All are bit-exact; they differ in speed only. */
enum {
    CORRX_ENGINE_AUTO = 0,    /* currently MFMA_I8 */
    CORRX_ENGINE_PLAIN = 1,   /* vector ALU only (no matrix cores) */
    CORRX_ENGINE_MFMA_I8 = 2, /* int8 MFMA, int32 accumulation */
    CORRX_ENGINE_MFMA_F8 = 3  /* fp8 E4M3 MFMA, fp32 accumulation in exact chunks folded to int32 */
};

/* Library version, for checking the binding against the header. */
int corr_abi_version(void);

/* Human-readable text of a status code (static storage, never NULL). */
const char *corr_strerror(int status);

/*
 * Create a correlator for n_inputs inputs, n_chan fine channels and n_time
 * samples per corr_xmac call, with the given input layout (Sec. 1.1: the
 * problem is fixed by the number of inputs, channels and the integration).
 * Selects the current HIP device, which must be gfx950; allocates the
 * host-side handle and, when the int8 engine splits the handle's samples into
 * several time ranges to fill the device (few channels, long integrations),
 * a device buffer of up to 1 GiB for the partial sums of those ranges
 * (nsplit - 1 accumulator images; larger needs fall back to atomic adds).
 * Sizes: 1 <= n_inputs <= 4096, n_chan >= 1, n_time >= 1, N*F*T < 2^40.
 * Errors: CORRX_EINVAL, CORRX_EDEVICE (no gfx950 device), CORRX_ENOMEM.  On
 * error *out is set to NULL.
 */
int corr_create(int n_inputs, int n_chan, int n_time, int layout, corrx_t *out);

/* Free the handle and its device buffer (NULL is accepted).  Does not touch
 * caller memory; work queued with the handle must have completed. */
int corr_destroy(corrx_t h);

/* Choose the compute engine (CORRX_ENGINE_*); default AUTO. */
int corr_set_engine(corrx_t h, int engine);

/*
 * Choose how the int8 engine divides corr_xmac's work (Sec. 3.4.2: the tile
 * a work unit computes sets its arithmetic intensity), with the tile codes of
 * corr_batch_create (CORRX_TILE_*, below): the diagonal unit's inputs (64,
 * 128 or 256; CORRX_EINVAL if it cannot hold n_inputs), time_splits 0 for
 * the built-in plan or the number of time ranges per channel, and the chunk
 * length: 64, 128 or 256 samples for 64-input units, 64 or 128 for 128-input
 * units, 64 for 256-input units (CORRX_EUNSUPPORTED otherwise).
 * Default 0 (built-in choice); other engines ignore it.  A set-up call: it may
 * grow the handle's partial-sum buffer for the requested time splits, so work
 * queued with the handle must have completed.  tune.py picks codes by
 * measurement.
 */
int corr_set_tile(corrx_t h, int tile_cfg);
/* Engine that corr_xmac will run (AUTO resolved), or a negative status. */
int corr_get_engine(corrx_t h);

/* Bytes of the accumulator: n_chan * N(N+1)/2 * 2 * 4 (int32 re, im). */
size_t corr_acc_bytes(corrx_t h);
/* Elements (re and im counted separately) of a corr_dump in `order`, or 0 if
 * the order is invalid for this handle. */
size_t corr_dump_count(corrx_t h, int order);

/*
 * Set the accumulator to zero (start of an integration, Sec. 3.4.3: the
 * accumulation length is chosen by the operator).  acc: device, corr_acc_bytes.
 */
int corr_zero(corrx_t h, void *acc, void *stream);

/*
 * acc += V(in): cross-multiply all input pairs of every channel over the
 * handle's n_time samples and add the lower triangle into acc (Sec. 3.4:
 * products are accumulated on the device).
 *   in:  device, N*F*T bytes in the handle's layout.
 *   acc: device, corr_acc_bytes(h) bytes, int32 [f][b][re, im], b = i(i+1)/2 + j.
 * The handle counts samples since the last corr_zero on the host; a call that
 * could overflow int32 (more than 21,913,098 samples, |Re|,|Im| <= 98 per
 * sample) returns CORRX_EOVERFLOW and enqueues nothing.  The first corr_xmac
 * after corr_zero on the same accumulator writes V instead of adding it (the
 * accumulator is known to be zero), so the caller must not modify the
 * accumulator between corr_zero and that call.
 */
int corr_xmac(corrx_t h, const void *in, void *acc, void *stream);

/* Size of the device scratch the library holds for corr_xmac_noalloc. */
#define CORRX_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)

/*
 * corr_xmac for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  No
 * handle and no allocation: computes what corr_create(n_inputs, n_chan,
 * n_time, layout) followed by corr_xmac computes, with the int8 MFMA engine
 * and the same work plan, and keeps the partial sums of time splits in a
 * scratch array the library holds on each device (CORRX_NOALLOC_SCRATCH_BYTES,
 * held until the process ends) instead of a handle's buffer.
 *   in, acc, stream: as for corr_xmac; acc has n_chan * N(N+1)/2 * 2 int32.
 *   accumulate: 0 = acc is overwritten with V(in) (no corr_zero needed),
 *               1 = acc += V(in).
 * Sizes as for corr_create (CORRX_EINVAL otherwise).  The caller counts the
 * samples in acc: the int32 bound of corr_xmac applies to the running total,
 * and one call of more than 21,913,098 samples returns CORRX_EOVERFLOW.  A
 * shape whose plan needs more partial-sum memory than the scratch returns
 * CORRX_ESCRATCH; errors enqueue nothing.  Every call on a device shares that
 * device's scratch, which keeps the last call's contents (each call
 * overwrites what it reads, so nothing needs clearing): calls that may
 * overlap on one device, on different streams or from different threads,
 * race; order them on one stream.
 */
int corr_xmac_noalloc(const void *in, void *acc, int n_inputs, int n_chan, int n_time, int layout,
                      int accumulate, void *stream);

/*
 * Write the visibilities in acc to dst in `order` (CORRX_TRI_*) as `dtype`
 * (CORRX_I32 / CORRX_F32), Appendix C "GPU Output".  dst: device,
 * corr_dump_count(h, order) * 4 bytes; must not overlap acc.  CORRX_F32 is
 * exact while |values| <= 2^24, which holds for integrations of up to 171,196
 * samples; past that it returns CORRX_EOVERFLOW.
 */
int corr_dump(corrx_t h, const void *acc, int order, int dtype, void *dst, void *stream);

/*
 * corr_dump with channel averaging (Sec. 3.4.3: the archived products may be
 * averaged by two in time and in frequency).  Time averaging is done by
 * accumulating t_avg integrations into acc before the dump; this call sums
 * f_avg adjacent channels: output channel g = channels g*f_avg .. g*f_avg +
 * f_avg - 1, in the given order.  CORRX_I32 writes the integer sum;
 * CORRX_F32 writes sum / (f_avg * t_avg), exact because both factors must be
 * powers of two (f_avg dividing n_chan, f_avg * t_avg <= 4096) and the sum is
 * checked to stay within 2^24 (CORRX_EOVERFLOW otherwise).  dst: device,
 * corr_dump_count(h, order) / f_avg values of 4 bytes; must not overlap acc.
 */
int corr_dump_avg(corrx_t h, const void *acc, int order, int dtype, int f_avg, int t_avg, void *dst,
                  void *stream);

/* ---- PFB packet order (Appendix A, B, C) ------------------------------- */

/*
 * Input order of the X-engine buffer built from PFB packets.  PACKET keeps the
 * order of the antenna samples inside a packet, as the paper's XMAC servers
 * do (input 64 b + k for position k of PFB b); NATURAL undoes the PFB's
 * permutation on the way in (position k holds PFB input 16 (k % 4) + k / 4,
 * Appendix A), so input 64 b + a is PFB b's input a.
 */
enum { CORRX_ORDER_PACKET = 0, CORRX_ORDER_NATURAL = 1 };

/*
 * Corner turn of PFB lane payloads into the handle's input buffer (layout
 * TFI; n_inputs = 64 per PFB, at most 4 PFBs; n_chan a multiple of 128, i.e.
 * whole coarse channels).  lanes: HOST array of 8 * n_pfb DEVICE pointers
 * (16-byte aligned), lane (PFB b, fibre n) at index 8 b + n.  Each lane buffer
 * holds that lane's packet payloads (header, counters and checksum removed)
 * for the handle's coarse channels in stream order (Appendix A): packet
 * (c, s, t) at byte offset ((c * 4 + s) * n_time + t) * 256 for coarse
 * channel c, group s (0..3) and time t, and inside a packet byte 64 f2 + k is
 * fine channel f2 (0..3) of position k (0..63).  That byte becomes sample
 * (time t, channel 128 c + 16 n + 4 s + f2, input per `order`) of `in`
 * (device, 16-byte aligned, n_time * n_chan * n_inputs bytes).
 */
int corr_pfb_ingest(corrx_t h, const void *const *lanes, int order, void *in, void *stream);

/*
 * Remap visibilities correlated in PACKET order to NATURAL order (Appendix C,
 * "GPU Output": products of permuted inputs, some of them conjugated).  For
 * natural inputs i >= j at packet indices P(i), P(j) (P(64 b + a) = 64 b +
 * 4 (a % 16) + a / 16): acc_nat[f][i][j] = acc_pkt[f][P(i)][P(j)] if
 * P(i) >= P(j), else its conjugate taken from acc_pkt[f][P(j)][P(i)].  Both
 * are device accumulators of the handle's shape (corr_acc_bytes, 8-byte
 * aligned, not overlapping); n_inputs must be a multiple of 64.
 */
int corr_pfb_remap(corrx_t h, const void *acc_pkt, void *acc_nat, void *stream);

/* ---- Fine polyphase filterbank, the F-engine stage (Sec. 3.2.1) ------- */

/*
 * 12-tap, 128-point critically sampled polyphase filterbank turning complex
 * coarse-channel samples into the packed 4+4-bit samples of 128 fine channels
 * (the input of corr_xmac).  Fixed point, so the output is an exact function
 * of the input (the paper gives no filter or quantiser; these are ours):
 *   v[k][p] = sum_{j<12} h[128 j + p] x[128 (k + j) + p]      (complex, int32)
 *   v8 = clip(round_shift(v, s1), -127, 127)
 *   Y[k][q] = sum_{p<128} v8[k][p] W[p q mod 128]             (complex, int32)
 *   sample = clip(round_shift(Y, s2), -7, 7) at fine channel (q + 64) mod 128
 * with round_shift(v, s) = floor((v + 2^(s-1)) / 2^s), h = rint(32767 w sinc /
 * peak) (w the 1536-point Hann window, sinc centred at 767.5 with period 128),
 * W[n] = rint(127 exp(-2 pi i n / 128)).
 * corr_fpfb_create: n_inputs a multiple of 64 (else CORRX_EUNSUPPORTED),
 * n_coarse coarse channels, n_frames output samples per fine channel; builds
 * the tables on the host and copies them to the current device (owned by the
 * handle, 67 KB).
 */
int corr_fpfb_create(int n_inputs, int n_coarse, int n_frames, corrx_fpfb_t *out);
int corr_fpfb_destroy(corrx_fpfb_t h);

/* Bytes of the device workspace corr_fpfb needs: n_coarse * n_inputs * n_frames * 256. */
size_t corr_fpfb_workspace_bytes(corrx_fpfb_t h);

/* Copy the handle's tables to HOST memory (either pointer may be NULL):
 * taps[1536]; twiddle_matrix[256 * 256] = row n, column k of the real GEMM
 * operand [[Wr, Wi], [-Wi, Wr]] transposed (k < 128: real part of input p = k,
 * else imaginary part of p = k - 128; n < 128: real part of output q = n, else
 * imaginary part of q = n - 128). */
int corr_fpfb_tables(corrx_fpfb_t h, int16_t *taps, int8_t *twiddle_matrix);

/*
 * in: device, complex int8 pairs (re, im) laid out [c][i][n], n = 0 ..
 * 128 (n_frames + 11) - 1 (each frame needs the 11 before it), 4-byte
 * aligned.  work: device workspace (corr_fpfb_workspace_bytes, 16-byte
 * aligned).  out: device, TFI packed samples n_frames * (128 n_coarse) *
 * n_inputs bytes, 16-byte aligned: byte (k, 128 c + f, i).  Two launches on
 * `stream` (filter, then DFT and requantisation).  0 <= s1, s2 <= 30.
 */
int corr_fpfb(corrx_fpfb_t h, const void *in, int s1, int s2, void *work, void *out, void *stream);

/* Samples accumulated since the last corr_zero (host-side count). */
int64_t corr_samples(corrx_t h);

/*
 * Incoherent beam (Sec. 3.4, other XMAC modes): out[f][t] = sum_i |x_i(f,t)|^2
 * as int32 for the handle's shape; invalid samples contribute nothing.
 * in: device, as for corr_xmac; out: device, n_chan * n_time * 4 bytes,
 * [f][t].  Any N and alignment; N a multiple of 16 with a 16-byte aligned
 * input takes the fast path (whole rows per 16 lanes).
 */
int corr_beam(corrx_t h, const void *in, void *out, void *stream);

/* ---- Uneven batch in one persistent launch ---------------------------- */

/* One array of a batch: its own shape and input layout. */
typedef struct {
    int n_inputs;
    int n_chan;
    int n_time;
    int layout;
} corrx_desc;

/*
 * Plan a batch of n arrays (1 <= n <= 64) of uneven shapes, run by one
 * persistent launch per kind of work unit present: one workgroup per compute
 * unit pulls work items (array, channel, tile, time range) from device
 * queues (eight per kind, one per XCD), longest first.  The paper's
 * correlator fixes the number of stations, channels and samples when it is
 * compiled (Sec. 3.3.3, footnote on compile-time parameters); here every
 * array of the batch has its own run-time shape.  Each array needs
 * n_inputs % 4 == 0 and 4-byte aligned input (else CORRX_EUNSUPPORTED).
 * engine: CORRX_ENGINE_MFMA_I8 or AUTO.  Allocates the device work list and
 * its queue counters (freed by corr_batch_destroy).
 * tile_cfg: NULL (built-in choice) or one code per array, chosen by the
 * autotuner: (unit) | (time_splits << 8) | (chunk << 24), with unit a
 * CORRX_TILE_* value (the input block a work item stages), time_splits 0 for
 * automatic or the number of time ranges per channel (at most 4096), and
 * chunk the samples a work item stages at a time: 0 for the unit's default,
 * 1, 2, 3 for 64, 128, 256.  The batch kernels have 128 (default) and 256 for
 * 64-input units, 64 (default) and 128 for 128-input units, 64 for 256-input
 * units; other chunks return CORRX_EUNSUPPORTED, malformed codes
 * CORRX_EINVAL.
 */
enum {
    CORRX_TILE_DEFAULT = 0, /* smallest unit that holds the array's inputs */
    CORRX_TILE_UNIT64 = 1,  /* 64-input units, one channel per work item (N <= 64) */
    CORRX_TILE_UNIT128 = 2, /* 128-input units, two channels per work item (N <= 128) */
    CORRX_TILE_UNIT256 = 3  /* 256-input diagonal blocks plus cross units (any N) */
};
int corr_batch_create(const corrx_desc *descs, int n, int engine, const int *tile_cfg,
                      corrx_batch_t *out);
int corr_batch_destroy(corrx_batch_t b);

/* Work items in the plan (for reporting). */
int64_t corr_batch_items(corrx_batch_t b);

/* The plan of one array: internal unit kind (0: 256-input blocks, 2: 128-input
 * pairs of channels, 3: 64-input channels, 4: 128-input pairs with 128-sample
 * chunks, 5: 64-input channels with 256-sample chunks) and time splits. */
int corr_batch_plan(corrx_batch_t b, int array, int *kind, int *splits);

/*
 * Set every accumulator of the batch to zero (one fill launch per array;
 * Sec. 3.4.3: the accumulation length is the operator's choice).  The
 * next corr_batch_xmac with the same accumulators then writes instead of
 * adding, as corr_xmac does after corr_zero; the caller must not modify them
 * in between.  accs: HOST array of n DEVICE pointers.
 */
int corr_batch_zero(corrx_batch_t b, void *const *accs, void *stream);

/*
 * For every array a: accs[a] += V(ins[a]) (Sec. 2 eq. (3), Sec. 3.4, as
 * corr_xmac).  ins and accs are HOST arrays of n DEVICE pointers (same
 * meaning as for corr_xmac, one per array; accs 8-byte aligned).  One
 * persistent launch per unit kind (plus a one-block queue reset) on `stream`.  The handle
 * counts each array's samples since corr_batch_zero; a call that would take
 * any array past 21,913,098 samples (the int32 bound, |Re|, |Im| <= 98 per
 * sample) returns CORRX_EOVERFLOW and enqueues nothing.
 */
int corr_batch_xmac(corrx_batch_t b, const void *const *ins, void *const *accs, void *stream);

/* Samples accumulated for one array of the batch since corr_batch_zero
 * (host-side count), or a negative status. */
int64_t corr_batch_samples(corrx_batch_t b, int array);

#ifdef __cplusplus
}
#endif

#endif /* CORRX_H */
