/*
 * hicr.h -- C ABI of the MI355X (gfx950) communication-manager data path.
 *
 * Operations follow HiCR (arXiv 2509.01425):
 *   Sec. 3.1.2  memory spaces            -> HICR_MEM_*
 *   Sec. 3.1.3  local memory slots       -> hicr_slot_register / _deregister
 *   Sec. 3.1.4  memcpy(dst, dstOff, src, srcOff, size), rejection of an
 *               unsupported memory-space pair, asynchronous completion,
 *               fence on the expected number of incoming and outgoing
 *               transfers               -> hicr_memcpy, hicr_memcpy_batch,
 *                                          hicr_fence, hicr_fence_slot,
 *                                          hicr_slot_counters
 *   Sec. 4.3    Channels frontend: circular buffers at the consumer, the
 *               producer waits while the buffer is full, SPSC and MPSC
 *               (locking / non-locking)  -> hicr_channel_*, and inside the
 *                                          caller's kernels hicr_device.h
 *   Sec. 4.3    Data Objects frontend   -> hicr_dobj_*
 *   Sec. 5      Test Case 1 (ping-pong) -> hicr_pingpong
 *   Growth directions beyond the paper: persistent batches (hicr_plan_*),
 *   schedule selection (hicr_autotune, hicr_tune_*, hicr_mlp_*) and a
 *   continuous-batching server (hicr_serve).
 *
 * General conventions
 *   - Every function returns 0 (HICR_OK) or a negative HICR_E* code and never
 *     throws: a host allocation that fails inside a call returns
 *     HICR_ENOMEM.  hicr_last_error() gives a human-readable reason for the
 *     last failure on a context.
 *   - Pointers named *_dev are device (HBM) addresses; all other pointers are
 *     host addresses (a slot's own memory may be HBM or pinned host memory).
 *     "stream" arguments are hipStream_t values passed as void*; NULL selects
 *     the context's own stream.
 *   - The caller owns every registered allocation and must keep it alive
 *     until the slot is deregistered.  The library owns its internal buffers.
 *   - Transfers are asynchronous: a successful return means the request was
 *     accepted and enqueued, not that a byte has moved.  Only a fence (or an
 *     observed counter) guarantees completion and visibility.
 *   - Within one epoch (between two fences) no byte may be written by two
 *     requests, or written by one and read by another; such a batch has an
 *     undefined result, as overlapping C memcpy does.  The library does not
 *     check this.
 *   - One context serialises its host calls with a mutex.  GPU code that
 *     faults or a device-side error surfaces as HICR_EDEVICE at the next fence.
 */
#ifndef HICR_H
#define HICR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define HICR_OK 0
#define HICR_EINVAL (-1)       /* bad argument                                   */
#define HICR_ERANGE (-2)       /* offset/size outside the slot                   */
#define HICR_EBADSLOT (-3)     /* unknown or deregistered slot                   */
#define HICR_EUNSUPPORTED (-4) /* memory-space pair not supported (Sec. 3.1.4)   */
#define HICR_EAGAIN (-5)       /* channel full (push) or empty (peek/pop)        */
#define HICR_ENOMEM (-6)       /* allocation of an internal buffer failed        */
#define HICR_ETIMEDOUT (-7)    /* expectation not met within the time limit      */
#define HICR_EHAZARD (-8)      /* reserved for debug hazard checks               */
#define HICR_EDEVICE (-9)      /* HIP runtime or device-side error               */
#define HICR_EBUSY (-10)       /* object still has transfers in flight           */

/* Memory spaces (Sec. 3.1.2): the GPU's HBM and pinned host memory.  The
 * copy kernel reaches both (host memory over the host link), so memcpy
 * supports every pair by default; hicr_ctx_set_pairs narrows the set, and a
 * request whose pair is outside it is rejected with HICR_EUNSUPPORTED
 * (Sec. 3.1.4).  Channels and ping-pong rings are HBM only. */
#define HICR_MEM_HBM 0u
#define HICR_MEM_HOST 1u
/* bit (2 * dst_space + src_space) of a pair mask: that pair is supported */
#define HICR_PAIR(dst_space, src_space) (1u << (2u * (dst_space) + (src_space)))
#define HICR_PAIRS_ALL 0xfu

typedef struct hicr_ctx_s *hicr_ctx;
typedef uint32_t hicr_slot;

/* One memcpy request in the argument order of Sec. 3.1.4 (32 bytes). */
typedef struct {
  uint32_t dst_slot;
  uint32_t src_slot;
  uint64_t dst_off;
  uint64_t src_off;
  uint64_t size;
} hicr_desc;

/* Copy schedule.  A batch is cut into pieces of at most chunk_bytes; a
 * request is spread over at least wgs_per_desc pieces (of at least 1 KiB)
 * when it is large enough; unroll sets the depth of the copy loop: a lane
 * moves rounds of 4 x unroll 16-byte vectors, two rounds in flight.  The
 * schedule never changes a byte of the result.
 * mode: HICR_SCHED_FIXED uses the fields as given; HICR_SCHED_TUNED looks the
 * batch up in the context's autotuned table; HICR_SCHED_LEARNED lets the
 * schedule network pick the class from the batch's size histogram: for a
 * submission on the host (the device kernels' arithmetic, from the
 * parameters last written by the device), for a plan once at creation by
 * the device forward kernel.  Without a network LEARNED falls back to the
 * tuned table, then to the context default. */
#define HICR_SCHED_FIXED 0u
#define HICR_SCHED_TUNED 1u
#define HICR_SCHED_LEARNED 2u
typedef struct {
  uint32_t chunk_bytes;  /* multiple of 128, in [128, 1 GiB]  */
  uint32_t wgs_per_desc; /* 1..64                             */
  uint32_t unroll;       /* 2 or 4                            */
  uint32_t mode;
} hicr_sched;

#define HICR_NUM_CLASSES 12
/* Class c in [0, 12) -> (chunk, wgs, unroll) with chunk in {4 KiB, 64 KiB,
 * 1 MiB} (c / 4), wgs in {1, 4} ((c / 2) % 2), unroll in {2, 4} (c % 2). */
int hicr_sched_class(uint32_t cls, hicr_sched *out);

/* --------------------------------------------------------------- context */
/* Create a context on HIP device `device`.  `stream` (hipStream_t or NULL)
 * becomes the default stream; with NULL the context creates its own
 * non-blocking stream. */
int hicr_ctx_create(int device, void *stream, hicr_ctx *out);
/* Fences, then frees every library-owned resource. */
int hicr_ctx_destroy(hicr_ctx ctx);
/* Static description of a return code. */
const char *hicr_strerror(int code);
/* Copy the last error message of `ctx` into buf (NUL-terminated, at most n). */
int hicr_last_error(hicr_ctx ctx, char *buf, size_t n);
/* Default schedule used when hicr_memcpy_batch gets s_or_null == NULL. */
int hicr_ctx_set_sched(hicr_ctx ctx, const hicr_sched *s);
/* Copy workgroups launched per compute unit (the persistent grid is at most
 * CUs x this, capped by what fits).  0 (the default) picks by schedule: 4 for
 * chunks of 4 KiB or less, 1 for chunks above 16 KiB up to 32 KiB, otherwise
 * 2; at least 4 for a launch of more than 4,096 requests whose chunks are
 * 16 KiB or less or whose average request is under 16 KiB.  Never changes a
 * byte.
 * wgs_per_cu > 64 -> HICR_EINVAL. */
int hicr_ctx_set_copy_grid(hicr_ctx ctx, uint32_t wgs_per_cu);
/* Memory-space pairs memcpy accepts from now on (HICR_PAIR bits; default
 * HICR_PAIRS_ALL).  Requests already accepted are not re-checked.  Bits
 * outside HICR_PAIRS_ALL -> HICR_EINVAL. */
int hicr_ctx_set_pairs(hicr_ctx ctx, uint32_t pair_mask);

/* ----------------------------------------------------------------- slots */
/* Sec. 3.1.3: register the existing allocation [ptr, ptr+size) of memory
 * space `memspace` as a slot.  For HICR_MEM_HBM the range must lie inside one
 * device allocation of this context's device; for HICR_MEM_HOST it must be
 * pinned host memory (hipHostMalloc, torch pin_memory) that the device can
 * address -- pageable or device memory -> HICR_EINVAL.  size == 0 ->
 * HICR_EINVAL.  Slots may alias.  Counters start at zero. */
int hicr_slot_register(hicr_ctx ctx, void *ptr, uint64_t size, uint32_t memspace,
                       hicr_slot *out);
/* Forget a slot.  HICR_EBUSY while any submitted transfer is unfenced. */
int hicr_slot_deregister(hicr_ctx ctx, hicr_slot slot);
/* Completed outgoing (sent: slot was the source) and incoming (recv: slot
 * was the destination) transfers since registration (Sec. 3.1.4).  A
 * counter is raised only after the transfer's bytes are visible on the
 * device.  Without a fence the values may lag. */
int hicr_slot_counters(hicr_ctx ctx, hicr_slot slot, uint64_t *sent, uint64_t *recv);

/* ---------------------------------------------------------------- memcpy */
/* Sec. 3.1.4 memcpy(dst, dstOff, src, srcOff, size).  Checked at once (slot
 * ids, bounds without overflow, supported memory-space pair); accepted
 * requests are queued on the context and launched together, as one fused
 * batch, at the next fence or batch submission.  size == 0 is a valid
 * transfer that moves nothing and still counts once. */
int hicr_memcpy(hicr_ctx ctx, hicr_slot dst, uint64_t dst_off, hicr_slot src, uint64_t src_off,
                uint64_t size);
/* Submit n requests as one fused launch on `stream`.  The whole batch is
 * checked first; on the first invalid request nothing is enqueued, the code
 * of that request is returned and its index stored in *bad_index_or_null.
 * `descs` is copied before the call returns.  s_or_null NULL selects the
 * context default.  A batch of 8,192 requests or more is uploaded on a
 * private stream that `stream` waits for (so the upload overlaps earlier
 * copies); 16,384 or more are checked by several host threads.  A
 * submission stages through host memory and is not meant for HIP graph
 * capture: persistent plans (below) are. */
int hicr_memcpy_batch(hicr_ctx ctx, const hicr_desc *descs, uint64_t n,
                      const hicr_sched *s_or_null, void *stream, uint64_t *bad_index_or_null);
/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): hicr_memcpy_batch with the same
 * arguments, validation, result and counters, that allocates nothing.  The
 * packed requests and piece tables go to a fixed per-device workspace
 * (2.5 MiB, held by every device the library runs on until the process
 * ends), staged through pinned memory the context allocated at creation.
 *   n > 65,536 requests, a total of 2^38 bytes or more, or a schedule whose
 *   mode is not HICR_SCHED_FIXED -> HICR_EINVAL, nothing enqueued.
 * Every call on one device shares the workspace: calls of one context are
 * ordered (a call on another stream waits for the previous one's launches),
 * but calls of two contexts on one device that overlap in time race, and
 * their results are undefined.  Completion and visibility as for
 * hicr_memcpy_batch (fences).  Pending hicr_memcpy requests stay queued for
 * the next fence. */
int hicr_memcpy_batch_noalloc(hicr_ctx ctx, const hicr_desc *descs, uint64_t n,
                              const hicr_sched *s_or_null, void *stream,
                              uint64_t *bad_index_or_null);
/* Sec. 3.1.4 fence: return once every transfer submitted on this context
 * (any stream) has completed and its bytes and counters are visible.
 * HICR_EDEVICE if the device reported an error. */
int hicr_fence(hicr_ctx ctx);
/* Fence on expected counts (Sec. 3.1.4 "expected number of incoming and
 * outgoing transfers"): wait until the slot's counters reach at least
 * (exp_sent, exp_recv).  HICR_ETIMEDOUT when timeout_ns passes first, or at
 * once when nothing is in flight that could still raise them. */
int hicr_fence_slot(hicr_ctx ctx, hicr_slot slot, uint64_t exp_sent, uint64_t exp_recv,
                    uint64_t timeout_ns);

/* ------------------------------------------ persistent batch plans (growth) */
/* Sec. 3.1.4 memcpy batches that repeat unchanged (a halo exchange, a fixed
 * gather): the batch is validated, resolved to addresses and uploaded once;
 * every hicr_plan_launch queues its fused copy launches and counter kernel
 * again -- directly, or, with HICR_PLAN_GRAPH, as one launch of a HIP graph
 * captured at creation.  One replay moves every request once
 * and raises each request's sent/recv counters once, like one
 * hicr_memcpy_batch of the same requests; hicr_fence (and fence_slot) wait
 * for replays as for any other transfer.
 *   d[0..n): requests as for hicr_memcpy_batch (copied; the caller may reuse
 *   the array at once).  s_or_null: FIXED, TUNED (resolved now) or LEARNED
 *   (the network's device forward kernel runs once now; every replay uses
 *   its choice).  On a rejected request: its code, *bad_index set, no
 *   plan.  n = 0 gives a plan whose launches move nothing.
 * While a plan exists the slots it names cannot be deregistered (HICR_EBUSY).
 * Replays of one plan are serialised: a launch on another stream than the
 * previous one first waits for the previous replay.  Slot contents may change
 * between replays; slot addresses may not (they are resolved at creation). */
typedef struct hicr_plan_s *hicr_plan;
#define HICR_PLAN_GRAPH 1u /* flags: replay as one captured HIP graph */
/* flags other than HICR_PLAN_GRAPH -> HICR_EINVAL. */
int hicr_plan_create(hicr_ctx ctx, const hicr_desc *d, uint64_t n, const hicr_sched *s_or_null,
                     uint32_t flags, hicr_plan *out, uint64_t *bad_index_or_null);
/* Replay once on `stream` (NULL: the context stream).  Asynchronous. */
int hicr_plan_launch(hicr_plan plan, void *stream);
/* Wait for the plan's last replay, then free it and release its slots. */
int hicr_plan_destroy(hicr_plan plan);



/* ------------------------------------------- schedule selection (growth) */
/* The batch feature used to pick a schedule: bin b of 32 counts the requests
 * with floor(log2 size) == b (bins above 31 fold into 31, size 0 into bin 0);
 * out32[b] = log2(1 + count).  Host-only; needs no context. */
int hicr_sched_features(const hicr_desc *descs, uint64_t n, float *out32);

/* Autotuner: run the batch under each of the 12 classes, `reps` timed runs
 * (1..64) after one warm-up, and store the median copy-kernel time of each
 * class in times_ms[12] (and the fastest class, ties to the lowest, in
 * *best_or_null).  The bytes really move (12 * (reps + 1) times in all),
 * so the batch must be hazard-free: its result is then that of one
 * application.  Slot counters are not raised.  Synchronous.  descs NULL, n
 * == 0, reps outside 1..64 or times_ms NULL -> HICR_EINVAL. */
int hicr_autotune(hicr_ctx ctx, const hicr_desc *descs, uint64_t n, uint32_t reps,
                  float *times_ms, uint32_t *best_or_null);
/* Tuned table used by HICR_SCHED_TUNED: each entry is an autotuned batch's
 * feature and its best class; a batch takes the class of the nearest entry
 * (squared distance of features).  With an empty table the context default
 * schedule is used. */
int hicr_tune_add(hicr_ctx ctx, const hicr_desc *descs, uint64_t n, uint32_t cls);
int hicr_tune_clear(hicr_ctx ctx);
/* The class HICR_SCHED_TUNED would give this batch (ties: the earliest
 * entry); an empty table -> HICR_EINVAL. */
int hicr_tune_lookup(hicr_ctx ctx, const hicr_desc *descs, uint64_t n, uint32_t *cls);

/* The schedule network, 32 -> 64 -> 64 -> 12 with ReLU, fp32, parameters in
 * the flat layout W1[64][32] b1[64] W2[64][64] b2[64] W3[12][64] b3[12]
 * (7,052 floats).  Training runs on the GPU (the kernels below); loading
 * parameters enables HICR_SCHED_LEARNED, in which every submission (or plan
 * creation) evaluates the network on the batch feature on the host -- the
 * sizes are there already -- and takes the argmax class (ties to the lowest);
 * after device training steps the parameters are read back once, at the next
 * learned submission.  Without a network HICR_SCHED_LEARNED falls back to the
 * tuned table.  x_dev: [batch][32] features, y_dev: [batch] class
 * labels, logits_dev: [batch][12], grad_dev: [7052] (all device memory).
 * Labels lie in [0, 12); a sample with a label outside that range gets a NaN
 * loss and contributes no gradient.  The kernels read and write these buffers
 * on the context stream: the caller orders their producers before the call
 * (same stream, or a synchronisation) and keeps them alive until the call's
 * work has completed. */
int hicr_mlp_set_params(hicr_ctx ctx, const float *params); /* also resets Adam */
int hicr_mlp_get_params(hicr_ctx ctx, float *params_out);
int hicr_mlp_forward(hicr_ctx ctx, const float *x_dev, uint32_t batch, float *logits_dev);
/* Class the network chose for the most recent HICR_SCHED_LEARNED submission
 * or plan; HICR_EINVAL before the first. */
int hicr_last_choice(hicr_ctx ctx, uint32_t *cls);
/* Gradient of the mean softmax cross-entropy (and the mean loss, if loss_dev). */
int hicr_mlp_grad(hicr_ctx ctx, const float *x_dev, const int32_t *y_dev, uint32_t batch,
                  float *grad_dev, float *loss_dev);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on one mini-batch; asynchronous
 * on the context stream, completed by hicr_fence. */
int hicr_mlp_train_step(hicr_ctx ctx, const float *x_dev, const int32_t *y_dev, uint32_t batch,
                        float lr, float *loss_dev);

/* --------------------------------------------------- data objects (growth) */
/* Sec. 4.3 Data Objects: a block [offset, offset+size) of a local slot is
 * published under an identifier that is unique within the context and never
 * reused; whoever holds the identifier (it may travel through a channel)
 * obtains a handle -- the object's metadata -- and starts an asynchronous
 * get, a memcpy of the whole object into its own slot that completes at the
 * next fence and counts on both slots like any memcpy.  A published object
 * keeps its slot from being deregistered (HICR_EBUSY).  Its bytes are read
 * when the get runs: the publisher keeps them unchanged until the getter's
 * fence. */
typedef struct {
  uint64_t id;
  uint64_t size;     /* bytes */
  uint64_t offset;   /* in the publishing slot */
  hicr_slot slot;    /* publishing slot */
  uint32_t memspace; /* memory space of the publishing slot */
} hicr_dobj_handle;
/* size == 0 or [offset, offset+size) outside the slot -> HICR_ERANGE. */
int hicr_dobj_publish(hicr_ctx ctx, hicr_slot slot, uint64_t offset, uint64_t size,
                      uint64_t *id_out);
/* Unknown or withdrawn id -> HICR_EINVAL. */
int hicr_dobj_get_handle(hicr_ctx ctx, uint64_t id, hicr_dobj_handle *out);
/* Queue the copy of the object into dst at dst_off (the rules of
 * hicr_memcpy).  A handle whose object was withdrawn -> HICR_EINVAL. */
int hicr_dobj_get(hicr_ctx ctx, const hicr_dobj_handle *h, hicr_slot dst, uint64_t dst_off);
/* Withdraw an object; gets already queued still run.  Unknown id -> HICR_EINVAL. */
int hicr_dobj_unpublish(hicr_ctx ctx, uint64_t id);

/* -------------------------------------------------------------- channels */
/* Sec. 4.3 Channels: circular buffers pre-allocated at the consumer.  The
 * caller registers the payload ring(s) and the entry ring(s) as HBM slots;
 * the library owns the coordination counters.  Counters are monotone, so a
 * ring of C tokens holds C tokens (no wasted slot).
 *
 *   kind      HICR_CH_FIXED: tokens of token_bytes; capacity = C tokens;
 *                            `entries` ignored (one entry per token).
 *             HICR_CH_VAR:   messages of 0..capacity bytes; capacity = P
 *                            payload bytes per ring; `entries` = E messages;
 *                            a message crossing the ring end continues at
 *                            the ring start.
 *   mode      HICR_CH_SPSC (producers = 1), HICR_CH_MPSC_LOCK (one shared
 *             ring; exclusive access for the room check and reservation, so
 *             the ring holds one total order), HICR_CH_MPSC_NOLOCK (one ring
 *             per producer, more memory, no exclusive access).
 *   endpoints HICR_CH_HOST: producer and consumer call the host API below;
 *             HICR_CH_DEVICE: producer and consumer are GPU workgroups of
 *             hicr_channel_pump (the host API then returns HICR_EINVAL).
 *   payload   slot of at least rings * ring_bytes bytes (ring r at r * ring_bytes);
 *   entries   slot of at least rings * E * 8 bytes, 8-byte aligned
 *             (rings = producers for MPSC_NOLOCK, else 1; ring_bytes = C * T or P).
 * The channel starts empty.  A channel must not outlive its context. */
#define HICR_CH_FIXED 0u
#define HICR_CH_VAR 1u
#define HICR_CH_SPSC 0u
#define HICR_CH_MPSC_LOCK 1u
#define HICR_CH_MPSC_NOLOCK 2u
#define HICR_CH_HOST 0u
#define HICR_CH_DEVICE 1u
#define HICR_CH_MAX_PRODUCERS 64u

typedef struct hicr_channel_s *hicr_channel;
typedef struct {
  uint32_t kind;
  uint32_t mode;
  uint32_t producers;
  uint32_t endpoints;
  uint64_t token_bytes; /* FIXED: T                     */
  uint64_t capacity;    /* FIXED: C tokens; VAR: P bytes */
  uint64_t entries;     /* VAR: E messages per ring      */
  hicr_slot payload;
  hicr_slot entries_slot;
} hicr_channel_cfg;

int hicr_channel_create(hicr_ctx ctx, const hicr_channel_cfg *cfg, hicr_channel *out);
/* Waits for the channel's pushes in flight, then frees it. */
int hicr_channel_destroy(hicr_channel ch);
/* Producer `producer` pushes `count` tokens (FIXED; all or nothing) or one
 * message of `count` bytes (VAR) read from slot `src` at `src_off`.  The
 * producer may not push while the ring lacks room: HICR_EAGAIN (retry after
 * the consumer pops).  count > C (FIXED) or > P (VAR): HICR_EINVAL.  The
 * payload moves asynchronously on the context stream; the consumer sees the
 * message once the device has published it. */
int hicr_channel_push(hicr_channel ch, uint32_t producer, hicr_slot src, uint64_t src_off,
                      uint64_t count);
/* The i-th oldest published message of ring `ring` (the producer index for
 * MPSC_NOLOCK, else 0): its byte offset inside the payload slot, its size
 * and its producer.  HICR_EAGAIN if fewer than i + 1 messages are visible. */
int hicr_channel_peek(hicr_channel ch, uint32_t ring, uint64_t i, uint64_t *payload_off,
                      uint64_t *bytes, uint32_t *producer);
/* Consume the n oldest messages of `ring`: the notification that frees their
 * room.  Reads of their bytes must be complete (e.g. a hicr_memcpy from the
 * payload slot followed by hicr_fence) before the call.  HICR_EAGAIN if fewer
 * than n are visible. */
int hicr_channel_pop(hicr_channel ch, uint32_t ring, uint64_t n);
/* Messages and bytes visible to the consumer in `ring`. */
int hicr_channel_depth(hicr_channel ch, uint32_t ring, uint64_t *msgs, uint64_t *bytes);

/* One producer stream of a pump: `n_msgs` messages, message j read from slot
 * `src` at msg_src_off[first_msg + j] with msg_size[first_msg + j] bytes,
 * pushed by producer `producer` of `channel`; the consumer appends the
 * stream's messages, in order, to slot `out` from offset 0. */
typedef struct {
  hicr_channel channel;
  uint32_t producer;
  hicr_slot src;
  hicr_slot out;
  uint32_t pad;
  uint64_t first_msg;
  uint64_t n_msgs;
} hicr_stream;

typedef struct {
  const uint64_t *msg_src_off; /* array [n_msgs]: host memory, or device memory with
                                  HICR_PUMP_DEVICE_TABLES                          */
  const uint64_t *msg_size;    /* array [n_msgs]; FIXED channels: token_bytes      */
  uint64_t n_msgs;
  uint32_t *trace_dev;   /* optional device array: for every consumed message, its
                            stream index; channels in order of first appearance in
                            the stream list.  A locking MPSC channel's part is the
                            order its consumer took the messages from the shared
                            ring; SPSC and non-locking MPSC rings are consumed
                            independently, so their part lists producer 0's
                            messages, then producer 1's, ...                     */
  uint64_t *ts_dev;      /* optional device array [2 * n_msgs]: publish time, then
                            consume time of every message (100 MHz device clock)    */
  uint64_t timeout_ns;   /* a wait that sees no progress for this long ends the
                            pump with HICR_ETIMEDOUT at the next fence (0: 10 s)    */
  uint32_t flags;        /* HICR_PUMP_* bits                                       */
  uint32_t reserved;     /* 0                                                      */
} hicr_pump_io;

/* msg_src_off and msg_size are device arrays the caller keeps valid (and
 * unchanged) until the pump has finished: nothing is copied from the host.
 * Variable-size channels only.  The host then cannot check the messages;
 * every producer checks each of its messages before moving a byte (size at
 * most the ring's payload, the source range inside its source slot, the
 * stream's output inside its output slot) and a bad one ends the pump with
 * HICR_EDEVICE at the next fence.  Rings are balanced over consumer
 * workgroups by message count instead of bytes. */
#define HICR_PUMP_DEVICE_TABLES 0x1u

/* Run every stream through its device-endpoint channel in one persistent
 * launch on `stream`: one GPU wave per producer stream.  The consumer side
 * of each channel is a team of workgroups: a locking MPSC channel's shared
 * ring is drained in its total order by up to 16 workgroups that take turns
 * (rounds of consecutive messages, ring room released in order); the rings
 * with a single producer (SPSC rings, non-locking MPSC sub-rings) are spread
 * over the remaining workgroups the device holds, balanced by bytes.  Validated on the host (slots, ranges, sizes, one stream per
 * (channel, producer)); HICR_EINVAL if the launch would not fit on the device
 * at once.  Asynchronous; hicr_fence reports a time-out or abort.  Pumps of
 * one context never overlap unsafely: a pump queued on another stream than
 * an unfinished earlier one first waits for it if they share a channel (a
 * ring has one producer and one consumer), and waits for the oldest others
 * until all pumps that can run together fit the device at once (every
 * workgroup of a pump must be resident).  Pumps of two contexts on one
 * device are not coordinated. */
int hicr_channel_pump(hicr_ctx ctx, const hicr_stream *streams, uint32_t n_streams,
                      const hicr_pump_io *io, void *stream);
/* Ask running pumps of this context to stop (they end at their next wait;
 * a waiting wave reads the request within ~10 ms of its own waiting, the
 * waves staggered, and passes it on to the others within 10 us).  A store
 * into each pump's pinned abort word:
 * it never waits for the device, and it reaches a pump even when every
 * stream of the process shares the pump's hardware queue. */
int hicr_channel_abort(hicr_ctx ctx);

/* Device view of one ring, for producers and consumers written in the
 * caller's own kernels with hicr_device.h (device addresses). */
typedef struct {
  uint64_t payload;  /* P payload bytes */
  uint64_t P;
  uint64_t entries;  /* E u64 entries: size | producer << 48 */
  uint64_t E;
  uint64_t coord;    /* the ring's coordination block (library memory) */
  uint32_t producer; /* tag a producer writes into this ring's entries */
  uint32_t pad;
} hicr_dev_ring;
/* Ring `ring` of a device-endpoint SPSC (ring 0) or non-locking MPSC (ring =
 * producer) channel.  Host-endpoint channels and bad ring numbers ->
 * HICR_EINVAL; locking MPSC -> HICR_EUNSUPPORTED (its producers take a lock
 * that only the pump implements).  From then on the channel belongs to user
 * kernels: hicr_channel_pump refuses it (HICR_EINVAL). */
int hicr_channel_device_view(hicr_channel ch, uint32_t ring, hicr_dev_ring *out);

/* ---------------------------------------------------- ping-pong (growth) */
/* Sec. 5, Test Case 1 on one GPU: a pinger and a ponger, each a group of W
 * workgroups, joined by two opposing channels of one-message capacity (rings
 * ring_a and ring_b).  For every size, `reps` round trips: the pinger pushes
 * sizes[i] bytes of `src` into A and waits for the echo in B, which it reads
 * into `dst`; the ponger takes each message from A into `buf`, frees A, and
 * pushes `buf` into B.  rtt_ticks[i * reps + k] receives round trip k of size
 * i in 100 MHz device-clock ticks.  All five slots: HBM, 16-byte aligned, at
 * least max(sizes) bytes.  wgs_per_endpoint 0 picks max(1, min(256,
 * size / 64 KiB)).  Synchronous. */
int hicr_pingpong(hicr_ctx ctx, hicr_slot src, hicr_slot dst, hicr_slot ring_a, hicr_slot ring_b,
                  hicr_slot buf, const uint64_t *sizes, uint32_t n_sizes, uint32_t reps,
                  uint32_t wgs_per_endpoint, uint64_t *rtt_ticks);

/* ------------------------------------------------------ serving (growth) */
/* A continuous-batching server on one context.  Requests arrive over time
 * (arrival_ns from the start of the run, non-decreasing); each is a memcpy
 * batch or a channel burst and needs hbm_bytes of the arena (an HBM slot that
 * is the serving budget) for its destinations.  In arrival order, a request
 * is admitted as soon as its destinations fit in the arena; every request
 * admitted since the last launch is fused into one copy launch (memcpy
 * batches, with the given schedule) and one pump launch (bursts; a burst
 * waits, and with it every later request, while a launch in flight still
 * drives its channel); up to `streams` launches are in flight so new work
 * overlaps work already running.  When a launch completes, each of
 * its requests is timestamped and passed to on_complete while its results
 * are still in the arena; then its arena space is freed.  on_complete runs on
 * the calling thread and must not call into the library on this context.
 *
 *   HICR_REQ_COPY:  descs[first .. first+count): dst_off relative to the
 *                   request's arena block, src_off in slot `src`; slot ids in
 *                   the descriptors are ignored.  hbm_bytes >= every
 *                   dst_off + size.
 *   HICR_REQ_BURST: messages first .. first+count of msg_src_off/msg_size, read
 *                   from slot `src` and pushed through channels[channel] (a
 *                   device-endpoint channel, producer 0); the consumer writes
 *                   them back to back at the start of the request's block.
 * Synchronous: returns when every request has completed (or on the first
 * error, after draining the launches in flight). */
#define HICR_REQ_COPY 0u
#define HICR_REQ_BURST 1u
typedef struct {
  uint32_t kind;
  uint32_t channel;
  uint64_t first;
  uint64_t count;
  uint64_t hbm_bytes;
  uint64_t arrival_ns;
} hicr_request;

typedef struct {
  hicr_slot arena;
  hicr_slot src;
  uint32_t streams;        /* launches in flight, 1..4 */
  uint32_t max_batch_reqs; /* requests fused into one launch, >= 1 */
  const hicr_desc *descs;
  uint64_t n_descs;
  const uint64_t *msg_src_off;
  const uint64_t *msg_size;
  uint64_t n_msgs;
  const hicr_channel *channels;
  uint32_t n_channels;
  uint32_t pad;
  const hicr_sched *sched_or_null; /* copy schedule; TUNED / LEARNED allowed */
  void (*on_complete)(void *user, uint64_t request, uint64_t arena_off);
  void *user;
  uint64_t *admit_ns;  /* optional [n]: when each request was admitted    */
  uint64_t *done_ns;   /* optional [n]: when its completion was observed  */
} hicr_serve_cfg;

typedef struct {
  uint64_t completed;
  uint64_t peak_arena_bytes;
  uint64_t copy_launches;
  uint64_t pump_launches;
  uint64_t max_inflight_requests;
  uint64_t wall_ns;
} hicr_serve_stats;

int hicr_serve(hicr_ctx ctx, const hicr_request *requests, uint64_t n, const hicr_serve_cfg *cfg,
               hicr_serve_stats *stats_or_null);

#ifdef __cplusplus
}
#endif
#endif /* HICR_H */
