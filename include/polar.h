/*
 * libpolar -- Fast-SSC and SC decoding of polar codes on AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes, no exceptions cross it.
 *
 * The decoder is the one of Giard et al., "Low-Latency Software Polar
 * Decoders": a depth-first walk of the pruned decoder tree (Sec. II-B, II-C)
 * with the min-sum f of eq. (1), the g of eq. (2) and the combine of eq. (3),
 * stopping at Rate-0 and Rate-1 nodes (Sec. II-D) and at repetition and
 * single-parity-check nodes (Sec. II-E).  LLRs are 8-bit saturating fixed
 * point (Sec. III-A.1, Listing 4: values in [-127, 127], g saturates) or
 * IEEE binary32.
 *
 * Conventions shared by every entry point:
 *   - natural (not bit-reversed) indexing (Sec. II-A); frozen bits are 0;
 *   - an LLR is ln P(x=0)/P(x=1): positive favours bit 0; the hard decision
 *     of a value v is 1 iff v < 0 (so zero decides 0);
 *   - packed bit rows are LSB first: bit j of a row is (row[j/8] >> (j%8)) & 1;
 *   - N is a power of two in [2, 32768] and 1 <= K <= N;
 *   - functions returning polar_code* return NULL on error and record the
 *     reason for polar_last_status() (thread local); functions returning
 *     polar_status record it too.
 * All functions are thread safe on distinct codes, and on one code once it
 * is prepared (decode/encode/introspection only read it).
 */
#ifndef POLAR_H
#define POLAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct polar_code polar_code; /* opaque; owned by the library */

typedef enum {
  POLAR_OK = 0,
  POLAR_EINVAL = 1,  /* bad argument: size, range, NULL pointer, alignment */
  POLAR_ENOMEM = 2,  /* host or device allocation failed, or the code needs
                        more on-chip memory than the device offers */
  POLAR_EDEVICE = 3, /* a HIP call failed (launch error, no device) */
  POLAR_ESTATE = 4,  /* call out of order: e.g. decode before prepare,
                        configure after prepare */
  POLAR_ECOMPILE = 5, /* the code's unrolled kernel failed to compile */
  POLAR_EAGAIN = 6    /* no room right now (request server): poll, then retry */
} polar_status;

typedef enum { POLAR_ALGO_FASTSSC = 0, POLAR_ALGO_SC = 1 } polar_algo;
typedef enum { POLAR_LLR_I8 = 0, POLAR_LLR_F32 = 1 } polar_llr;

/* Which kernel decodes a code (Sec. III-A vs III-B: instruction-based vs
 * unrolled decoder).  Both run the same node functions and give identical
 * results; the unrolled kernels of N >= 16384 also lay out the widest LLR
 * stages differently (registers, or recomputed from the channel) to fit
 * more frames on a compute unit.
 *   POLAR_KERNEL_SCHEDULE: one kernel for every code reads the code's
 *     schedule from device memory at run time; prepare is immediate.
 *   POLAR_KERNEL_UNROLLED: a kernel generated for this one code, with the
 *     schedule compiled in (no run-time dispatch).  It is compiled with the
 *     HIP run-time compiler the first time a code needs it (seconds to a
 *     minute for N = 32768) and kept in an on-disk cache: the directory in
 *     the environment variable POLAR_KERNEL_CACHE, else "kernels" next to
 *     the library file. */
typedef enum { POLAR_KERNEL_SCHEDULE = 0, POLAR_KERNEL_UNROLLED = 1 } polar_kernel;

/* Node functions reported by polar_schedule(), named after Listing 1. */
typedef enum {
  POLAR_OP_F = 0,          /* eq. (1) to the left child */
  POLAR_OP_G = 1,          /* eq. (2) to the right child */
  POLAR_OP_G_0R = 2,       /* eq. (2) when the left child is Rate-0 */
  POLAR_OP_COMBINE = 3,    /* eq. (3) */
  POLAR_OP_COMBINE_0R = 4, /* eq. (3) when the left child is Rate-0 */
  POLAR_OP_INFO = 5,       /* Rate-1 node: eq. (4) on every bit */
  POLAR_OP_REP = 6,        /* repetition node (Sec. II-E) */
  POLAR_OP_SPC = 7         /* single-parity-check node (Sec. II-E) */
} polar_op_kind;

/* Builds an (N, K) code: the N-K least reliable bit channels are frozen
 * (Sec. II-A), reliability being the Bhattacharyya parameter of BPSK over
 * AWGN at the design Eb/N0 (dB) propagated through the polarising kernel
 * (z -> 2z - z^2 for the first child, z -> z^2 for the second; ties go to
 * the higher index as information bit).  Also builds the decoder schedule.
 * The code starts configured as Fast-SSC with int8 LLRs.  Host only.
 * Errors: POLAR_EINVAL (N not a power of two in [2, 32768], K outside
 * [1, N]), POLAR_ENOMEM. */
polar_code* polar_construct(int n, int k, double design_ebn0_db);

/* Builds a code from an explicit frozen mask: frozen[i] in {0, 1} for
 * i < N (1 = frozen, e.g. Fig. 2's (8,5) code is {1,1,0,0,1,0,0,0}).
 * K = N - sum(frozen) must be >= 1.  The mask is copied. */
polar_code* polar_construct_mask(int n, const uint8_t* frozen);

/* Selects the algorithm (Fast-SSC, Sec. II-E, or plain SC, Sec. II-B) and
 * the LLR type (8-bit fixed point, Sec. III-A.1, or binary32).  Must be
 * called before polar_prepare(); POLAR_ESTATE afterwards, POLAR_EINVAL for
 * a value outside the enums. */
polar_status polar_configure(polar_code* code, polar_algo algo, polar_llr llr_type);

/* Fast-SSC only: enable (1, the default) or disable (0) the fused nodes of
 * the Fast-SSC function library (Sec. II-E): every internal node of size
 * <= 64 whose children are a Rate-0 or repetition node (left) and a Rate-1
 * or SPC node (right) -- the P_01, 0SPC and RepSPC functions, and the
 * repetition / Rate-1 pair -- runs as one device op instead of five (or
 * three).  The decoded bits and the trace are identical either way; the
 * switch exists to measure the effect.  Ignored by plain SC.  Must be
 * called before polar_prepare(); POLAR_ESTATE afterwards, POLAR_EINVAL for
 * another value. */
polar_status polar_set_fused_nodes(polar_code* code, int enable);

/* Selects the kernel (polar_kernel); default POLAR_KERNEL_SCHEDULE.  Must
 * be called before polar_prepare(); POLAR_ESTATE afterwards, POLAR_EINVAL
 * for a value outside the enum. */
polar_status polar_set_kernel(polar_code* code, polar_kernel kernel);

/* Layouts of an unrolled kernel's widest alpha stages (how many stages sit
 * in registers instead of LDS, whether the stage below the root is
 * recomputed from the channel instead of stored, and -- float codes of
 * N = 32768 -- whether the stage below the register stage is recomputed
 * from it instead of stored): the choices the
 * autotuner times, a per-code analogue of the threads-per-block,
 * blocks-per-kernel and shared-memory sweeps of Sec. V (Sec. V-B, V-C,
 * V-E).  Index 0 is the default rule;
 * every layout gives identical results.  polar_layout_count returns how
 * many there are for the code as configured (LLR type; 0 on NULL),
 * polar_layout_info describes one (any output pointer may be NULL;
 * virtual_top, virtual_mid: 0 or 1 for the two recomputed stages;
 * wave_lds_bytes: LDS per frame).  Errors: POLAR_EINVAL. */
int polar_layout_count(const polar_code* code);
polar_status polar_layout_info(const polar_code* code, int index, int* reg_stages, int* virtual_top,
                               int* wave_lds_bytes, int* virtual_mid);

/* Selects layout `index` for the code's unrolled kernel (and for batches
 * created from the code afterwards).  Before polar_prepare; polar_configure
 * and polar_set_fused_nodes reset it to 0, since the candidates depend on
 * the LLR type and the schedule.  Errors:
 * POLAR_EINVAL (index out of range), POLAR_ESTATE (prepared). */
polar_status polar_set_layout(polar_code* code, int index);

/* Autotuner for one code: loads the kernel of every layout (compiling
 * kernels not yet in the cache), times decodes of the given frames with
 * each in rounds (device buffers as for polar_decode; bits is
 * overwritten): warm-up rounds until 30 ms of decoding, then 3 timed
 * rounds of a burst of 5 back-to-back launches per layout, each layout
 * keeping its fastest burst; and leaves the code prepared with the
 * fastest; *chosen (may be NULL) receives its index.  The code must use the unrolled kernel and not be
 * prepared.  Synchronous.  Errors: POLAR_EINVAL, POLAR_ESTATE,
 * POLAR_ECOMPILE, POLAR_EDEVICE, POLAR_ENOMEM (the code is then left
 * unprepared, with the default layout). */
polar_status polar_tune_layout(polar_code* code, const void* llr, int nframes, uint8_t* bits, void* stream,
                               int* chosen);

/* Generates and compiles the unrolled kernel of the code as configured
 * (algorithm and LLR type) into the kernel cache, unless it is there
 * already.  Host only: needs no device, so kernels can be built ahead of
 * time.  Synchronous.  Errors: POLAR_ECOMPILE, POLAR_ENOMEM. */
polar_status polar_build_kernel(const polar_code* code);

/* Uploads the schedule (or loads the unrolled kernel, building it first if
 * the cache lacks it) on the current HIP device and sizes the launch.
 * Synchronous; allocates device memory; call it before any capture.
 * Errors: POLAR_EDEVICE (no device / HIP failure), POLAR_ENOMEM (device
 * allocation, or the decoder's on-chip working set does not fit the
 * device's LDS), POLAR_ECOMPILE, POLAR_ESTATE (already prepared). */
polar_status polar_prepare(polar_code* code);

/* Frees host and device memory of the code.  NULL is a no-op.  The caller
 * must make sure no decode on the code is still running. */
void polar_destroy(polar_code* code);

polar_status polar_last_status(void);
const char* polar_strerror(polar_status status);

/* Details of the last failure on this thread, e.g. the compiler log after
 * POLAR_ECOMPILE; "" when there are none.  Valid until the next call into
 * the library on this thread. */
const char* polar_last_message(void);

/* Test hook (failure handling): after `after` more allocations succeed, the
 * next allocation the library makes -- a code, batch or server object,
 * device memory or pinned host memory -- fails as if memory ran out (once;
 * then allocations succeed again).  The call that makes it returns
 * POLAR_ENOMEM (or NULL with polar_last_status() == POLAR_ENOMEM) and keeps
 * nothing it allocated.  after < 0 disarms the hook.  Process wide. */
polar_status polar_debug_fail_allocations(int after);

int polar_n(const polar_code* code); /* 0 for NULL */
int polar_k(const polar_code* code); /* 0 for NULL */

/* Copies the frozen mask (N bytes of 0/1) to host memory out. */
polar_status polar_frozen_mask(const polar_code* code, uint8_t* out);

/* The node functions one decode runs, in order (the form of Listing 1):
 * kinds[i] is a polar_op_kind, sizes[i] the node size N_v, offsets[i] the
 * index of the node's first bit.  Plain SC reports its full walk.  Writes at
 * most cap entries to each non-NULL array and sets *n_ops to the total. */
polar_status polar_schedule(const polar_code* code, int32_t* kinds, int32_t* sizes,
                            int32_t* offsets, int cap, int* n_ops);

/* Device ops: what the kernels actually run (polar_device_schedule).  One
 * 32-bit word per op: op | stage << 8 | node offset << 16, where stage is
 * log2 of the node size.  F / G / G_0R read the node at that stage and write
 * its child; leaves, combines and fused nodes act on the node itself. */
typedef enum {
  POLAR_DOP_F = 0, POLAR_DOP_G = 1, POLAR_DOP_G_0R = 2,
  POLAR_DOP_COMBINE = 3, POLAR_DOP_COMBINE_0R = 4,
  POLAR_DOP_COMBINE_R0 = 5,  /* right child Rate-0: clear its estimate */
  POLAR_DOP_INFO = 6, POLAR_DOP_REP = 7, POLAR_DOP_SPC = 8,
  POLAR_DOP_FLUSH = 9,       /* a finished size-64 estimate to LDS */
  POLAR_DOP_P01 = 11,        /* fused: left Rate-0, right Rate-1 */
  POLAR_DOP_0SPC = 12,       /* fused: left Rate-0, right SPC */
  POLAR_DOP_REPSPC = 13,     /* fused: left repetition, right SPC */
  POLAR_DOP_REPR1 = 14       /* fused: left repetition, right Rate-1 */
} polar_dev_op;

/* The device schedule (polar_dev_op words, in execution order) of the code
 * as configured.  Writes at most cap words to ops (may be NULL) and sets
 * *n_ops to the total.  Host only. */
polar_status polar_device_schedule(const polar_code* code, uint32_t* ops, int cap, int* n_ops);

/* Host encoder: x = u G_N (Sec. II-A) with u_A taken from info (packed
 * rows of ceil(K/8) bytes, information bits in increasing index order) and
 * u_F = 0.  Writes packed rows of ceil(N/8) bytes to x.  Host memory. */
polar_status polar_encode(const polar_code* code, const uint8_t* info, int nframes, uint8_t* x);

/* Decodes nframes frames on the given HIP stream (hipStream_t, NULL = the
 * default stream): for each frame, the successive-cancellation walk of the
 * decoder tree (Sec. II-B, II-C: f of eq. (1) to the left child, g of
 * eq. (2) to the right child, the combine of eq. (3)), pruned at Rate-0 and
 * Rate-1 nodes (Sec. II-D) and, for Fast-SSC, at repetition and SPC nodes
 * (Sec. II-E), in the order of Listing 1.  The output is the information
 * part of u_hat = x_hat G_N (Sec. II-A).  Asynchronous: never allocates,
 * frees or synchronises, so it can be captured in a HIP graph.
 *   llr : device memory, [nframes][N] of int8 or float (as configured),
 *         natural index order.  int8 follows Listing 4's symmetric range:
 *         -128 is read as -127.  int8 rows must start on a 4-byte boundary
 *         (16 recommended), float rows on a 16-byte boundary (the kernels
 *         read 128-bit words).
 *   bits: device memory, [nframes][ceil(K/8)] bytes: u_hat over the
 *         information set in increasing index order, LSB first, pad bits 0.
 * Both buffers belong to the caller and must stay alive until the stream
 * has run the decode; their contents must be ready in stream order.
 * nframes == 0 is a no-op.  Errors: POLAR_EINVAL (NULL buffers with
 * nframes > 0, nframes < 0, misaligned llr), POLAR_ESTATE (not prepared,
 * or the current device is not the one the code was prepared on),
 * POLAR_EDEVICE (the launch itself failed; an error left on the thread by
 * an earlier call is not reported).  Kernel faults surface at the
 * caller's next synchronisation. */
polar_status polar_decode(const polar_code* code, const void* llr, int nframes, uint8_t* bits,
                          void* stream);

/* polar_decode plus a trace of the intermediate LLRs: for every frame,
 * trace[frame][i] (int8 or float, [nframes][N], device memory) receives the
 * LLR input alpha_v of the decision node (Rate-1, repetition or SPC leaf,
 * or single bit in SC) that covers index i; indices under Rate-0 nodes are
 * left untouched.  Slower; meant for parity tests. */
polar_status polar_decode_trace(const polar_code* code, const void* llr, int nframes, uint8_t* bits,
                                void* trace, void* stream);

/* ------------------------------------------------------------------------
 * Batches of mixed codes: one persistent launch decodes frames of several
 * codes (lengths and rates) together.  Each code's decoder is its unrolled
 * kernel (Sec. III-B) compiled into one generated kernel; every wavefront
 * walks the frame list with a stride and decodes one frame at a time with
 * the decoder of that frame's code, in an LDS slot sized for the largest
 * code.  Results are identical to polar_decode on each code.
 * ------------------------------------------------------------------------ */
typedef struct polar_batch polar_batch; /* opaque; owned by the library */

/* Builds a batch over ncodes (1..255) codes that share one LLR type (as
 * configured; each code keeps its own algorithm).  The codes' schedules are
 * copied; the codes may be destroyed afterwards.  Host only.
 * Errors: POLAR_EINVAL (NULL, count, mixed LLR types), POLAR_ENOMEM. */
polar_batch* polar_batch_create(const polar_code* const* codes, int ncodes);

/* Compiles the batch kernel into the kernel cache unless it is there
 * (host only; about a minute for fifteen codes up to N = 32768).
 * Errors: POLAR_ECOMPILE, POLAR_ENOMEM. */
polar_status polar_batch_build_kernel(const polar_batch* batch);

/* Loads the batch kernel on the current device (building it first if the
 * cache lacks it) and sets a default launch shape.  Synchronous.
 * Errors: POLAR_EDEVICE, POLAR_ENOMEM, POLAR_ECOMPILE, POLAR_ESTATE. */
polar_status polar_batch_prepare(polar_batch* batch);

/* Describes the frames that polar_batch_decode() decodes: for frame i,
 * code_index[i] (index into the codes given to polar_batch_create),
 * llr_offset[i] (elements from the llr base pointer of the decode; the
 * frame's N LLRs follow contiguously) and bits_offset[i] (bytes from the
 * bits base pointer; the frame's ceil(K/8) output bytes follow).  Host
 * arrays, copied.  The library orders frames longest code first, frames
 * of one code together (in their given order), and keeps the descriptors in device memory it owns (allocated here, grown when
 * needed).  Synchronous: waits for the device to finish its work first
 * (decodes in flight read the previous descriptors), so not for use under
 * stream capture.  Errors: POLAR_EINVAL (index or offset out of
 * range), POLAR_ESTATE (not prepared), POLAR_ENOMEM, POLAR_EDEVICE. */
polar_status polar_batch_set_frames(polar_batch* batch, int nframes, const int32_t* code_index,
                                    const int64_t* llr_offset, const int64_t* bits_offset);

/* Decodes the frames of the last polar_batch_set_frames() in one launch on
 * the given stream.  Asynchronous; never allocates or synchronises, so it
 * can be captured in a HIP graph (the descriptors must not change between
 * capture and replay).  llr: device memory of the batch's LLR type, aligned
 * as for polar_decode (4 bytes int8, 16 bytes float); bits: device memory.  Errors: POLAR_EINVAL, POLAR_ESTATE (not
 * prepared, or the current device is not the batch's), POLAR_EDEVICE. */
polar_status polar_batch_decode(const polar_batch* batch, const void* llr, uint8_t* bits, void* stream);

/* As polar_batch_decode with caller-owned descriptors in device memory:
 * desc[2i] = code index | bits byte offset << 8, desc[2i+1] = LLR offset in
 * elements, for i < nframes (no ordering is applied; waves take frames i,
 * i + W, i + 2W, ...).  The descriptors are not validated: indices and
 * offsets must be in range. */
polar_status polar_batch_decode_desc(const polar_batch* batch, const uint64_t* desc, int nframes,
                                     const void* llr, uint8_t* bits, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): decodes nframes
 * frames described by three arrays in DEVICE memory -- code_index[i] (int32),
 * llr_offset[i] (elements) and bits_offset[i] (bytes), as for
 * polar_batch_set_frames() -- in one launch, with the same results as
 * polar_batch_set_frames() + polar_batch_decode() on those frames.  Calls
 * no hipMalloc/hipFree: the descriptor queue is a fixed device array of the
 * library (4 MiB per device, held until the process ends), filled by a small
 * kernel on the stream, so at most 262144 frames per call (more:
 * POLAR_EINVAL).  Frames are decoded in the given order (no longest-first
 * ordering).  A frame whose code index is out of range, or whose offset is
 * negative (bits offset >= 2^56), is skipped and its output row is not
 * written; offsets must otherwise index inside llr and bits.  Every call on
 * one device shares the one array: calls that overlap on a device (other
 * streams, other threads) race and must be ordered by the caller.
 * Asynchronous, capturable (two kernel launches, no memset).  Errors:
 * POLAR_EINVAL, POLAR_ESTATE (not prepared, other device), POLAR_EDEVICE. */
polar_status polar_batch_decode_frames_noalloc(const polar_batch* batch, int nframes, const int32_t* code_index,
                                               const int64_t* llr_offset, const int64_t* bits_offset,
                                               const void* llr, uint8_t* bits, void* stream);

/* Autotuner: times launch shapes (1, 2 or 4 frames per workgroup; a grid
 * that fills the chip's wave slots once or twice, or one wave per frame)
 * on the frames of the last polar_batch_set_frames() and keeps the
 * fastest.  Runs decodes on the given buffers and synchronises.  Errors:
 * POLAR_EINVAL, POLAR_ESTATE, POLAR_EDEVICE. */
polar_status polar_batch_tune(polar_batch* batch, const void* llr, uint8_t* bits, void* stream);

/* The current launch shape (any pointer may be NULL). */
polar_status polar_batch_launch_shape(const polar_batch* batch, int* waves_per_block, int* blocks,
                                      int* wave_lds_bytes);

/* Frees the batch and its device memory.  NULL is a no-op. */
void polar_batch_destroy(polar_batch* batch);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of decode requests over a prepared
 * batch.  A request is 1..n frames of one of the batch's codes; its LLRs
 * and its results each live in host or in device memory.  Requests are
 * admitted first come, first served as soon as the device memory they need
 * is free: LLR slots of the server's pool for host LLRs, bits slots for
 * host results, and for buffers already in device memory a share of a
 * byte budget of caller memory that admitted, unfinished requests may
 * reference (the bytes the request pins on the device).  Every poll
 * retires finished steps (in whatever order they finish), admits what fits
 * and launches steps (batch decodes) over the admitted frames not yet
 * launched while server streams are free: one step per frame length, the
 * length of the oldest admitted request first (at most two steps of one
 * length in flight, so one busy length cannot hold every stream), so steps
 * overlap on the device, short codes do not wait for long ones, and
 * requests that arrive while steps run join the next.  Each frame is decoded exactly as
 * polar_decode would decode it alone.
 * Not thread safe: one thread drives a server, with the server's device
 * current.  After a HIP failure (POLAR_EDEVICE from a poll) the requests in
 * flight are lost and every later submit or poll returns POLAR_EDEVICE:
 * destroy the server.
 * ------------------------------------------------------------------------ */
typedef struct polar_server polar_server; /* opaque; owned by the library */

/* Creates a server on the current device for a prepared batch; codes /
 * ncodes must be the codes the batch was created from, in the same order.
 * slots_per_class (>= 0): frame slots for each distinct frame length N in
 * the server's LLR pool and in its bits pool, used by requests whose LLRs
 * or results are in host memory (device memory: slots x (N x LLR size +
 * ceil(K/8)) per length); device_bytes: the budget of caller device
 * memory (LLR and result bytes) that admitted, unfinished requests with
 * device-resident buffers may reference; at least one of the two must be
 * non-zero.  streams: steps in flight at once (1..8); staging_bytes:
 * pinned host memory holding submitted LLRs until their step has copied
 * them.  Allocates device and pinned host memory.  NULL on error (see
 * polar_last_status: POLAR_EINVAL, POLAR_ESTATE if the batch is not
 * prepared or was prepared on another device, POLAR_ENOMEM,
 * POLAR_EDEVICE). */
polar_server* polar_server_create(const polar_batch* batch, const polar_code* const* codes, int ncodes,
                                  int slots_per_class, int streams, size_t staging_bytes, size_t device_bytes);

/* Where the buffers of a request live (flags for polar_server_submit). */
enum { POLAR_SERVER_LLR_DEVICE = 1, POLAR_SERVER_BITS_DEVICE = 2 };

/* Queues a request of nframes frames of code code_index (an index into
 * the batch's codes).  llr: [nframes][N] LLRs of the batch's type in host
 * memory (copied to pinned staging before the call returns, then to a
 * device slot by the request's step) or, with POLAR_SERVER_LLR_DEVICE in
 * `where`, in device memory of the server's device (read in place, no
 * copy).  bits: [nframes][ceil(K/8)] results, in host memory (written by
 * the poll that reports the request done) or, with
 * POLAR_SERVER_BITS_DEVICE, in device memory (written in place by the
 * decode).  Buffers must stay valid until the request is reported done.
 * Readiness: the server's streams do not wait for any other stream, so
 * device buffers must be ready when submit is called -- the LLRs written
 * and any earlier work on the result buffer finished (synchronise the
 * stream that produced them first).
 * *id receives the request id (> 0).  Errors: POLAR_EINVAL (bad arguments,
 * or a request that could never be admitted: more frames than its length
 * class has slots, or more device bytes than the budget), POLAR_EAGAIN
 * (staging memory full: poll, then submit again), POLAR_EDEVICE (the
 * server has failed). */
polar_status polar_server_submit(polar_server* server, int code_index, int nframes, const void* llr, int where,
                                 uint8_t* bits, int64_t* id);

/* Replays a timed request trace against the server on the calling thread,
 * as a load generator: request i (code code_index[i], nframes[i] frames,
 * device LLRs llr[i], device results bits[i]) is submitted once
 * arrival_s[i] seconds have passed since the call began (arrival_s
 * non-decreasing), and the server is polled continuously;
 * completion_s[i] receives the time (same clock) at which a poll saw it
 * done.  Returns when every request is done.  Errors: POLAR_EINVAL,
 * POLAR_ESTATE (another device is current), POLAR_EDEVICE. */
polar_status polar_server_run_trace(polar_server* server, int nreq, const double* arrival_s,
                                    const int32_t* code_index, const int32_t* nframes, const void* const* llr,
                                    uint8_t* const* bits, double* completion_s);

/* Makes progress without blocking: retires finished steps (writing their
 * requests' bits), admits waiting requests, launches a step.  Writes the
 * ids of requests completed by this call to done_ids (at most cap; *ndone
 * receives the count).  Errors: POLAR_EINVAL, POLAR_ESTATE (another device
 * is current), POLAR_EDEVICE. */
polar_status polar_server_poll(polar_server* server, int64_t* done_ids, int cap, int* ndone);

/* Device bytes of caller memory referenced by admitted, unfinished
 * requests, and the budget (any pointer may be NULL). */
polar_status polar_server_device_bytes(const polar_server* server, size_t* in_use, size_t* budget);

/* Requests waiting for memory, admitted but not launched, and steps in
 * flight (any pointer may be NULL). */
polar_status polar_server_pending(const polar_server* server, int* waiting, int* admitted, int* inflight_steps);

/* Waits for the server's streams, then frees it.  Requests not yet
 * reported by a poll are dropped.  NULL is a no-op. */
void polar_server_destroy(polar_server* server);

#ifdef __cplusplus
}
#endif

#endif /* POLAR_H */
