/*
 * hh.h -- C ABI of libhh.so: batched HighwayHash on AMD Instinct MI355X (gfx950).
 *
 * HighwayHash is the keyed hash / pseudo-random function of "Fast keyed
 * hash/pseudo-random function using SIMD multiply and permute" (Alakuijala,
 * Cox, Wassenberg; arXiv:1612.06257).  A 256-bit key and a byte string of any
 * length (including 0) give a 64-, 128- or 256-bit result (Sec. 1 and 4.3):
 *   Reset(key) (Sec. 4.4); Update(packet) for every full 32-byte packet
 *   (Sec. 4.1, 4.2); if size mod 32 != 0, the size-injected, v1-rotated padded
 *   remainder packet (Sec. 4.5); four rounds of Update(Permute(v0)) and the
 *   sum v0 + v1 + mul0 + mul1 of the four state vectors (Sec. 4.3).
 * The 64-bit hash is lane 0 of that sum, the 128-bit hash lanes 0..1 and the
 * 256-bit hash lanes 0..3.
 *
 * Conventions for every entry point:
 *   - Pointers named in the argument list are DEVICE pointers unless noted:
 *     addresses the GPU can access, which includes the device address of
 *     pinned host memory (hh_pinned_device_pointer) for the small index,
 *     length and output arrays.  The caller owns every buffer and keeps it alive until the work enqueued
 *     on `stream` has finished; the library keeps no reference after return.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work; results are visible after stream or event
 *     synchronisation.
 *   - A key is four uint64 words; word i is lane i (a 32-byte key read
 *     little-endian).  keys[4*k + i] is lane i of key k.
 *   - Message j is data[offsets[j] .. offsets[j] + lengths[j]), bytes at any
 *     alignment and of any 64-bit length (offsets and messages beyond 4 GiB
 *     included); offsets[j] + lengths[j] <= data_bytes is the caller's
 *     contract.  The kernels never read outside [data, data + data_bytes):
 *     a message that violates the contract is clamped to the buffer and
 *     hashed truncated, it never faults.
 *   - key_idx[j] selects message j's key; NULL means key 0 for every message.
 *     An index >= n_keys is clamped to n_keys - 1.
 *   - Outputs are uint64 words, message-major, lane 0 first:
 *     out[w*j + i] is word i of message j's w-word hash.
 *   - `out` must not overlap any input.  n_msgs == 0 is a valid no-op.
 *   - Threads: calls on different streams are independent.  Several host
 *     threads may call on one stream (the null stream included): each call
 *     enqueues its launches as one unit while holding the stream's library
 *     workspace, so the calls run on the stream one after another, in the
 *     order in which they took it.  (hh_hash_noalloc is the exception: see
 *     there.)
 *   - Argument errors are reported synchronously (HH_ERR_INVALID_ARG) before
 *     any device call.  A device that is not gfx950 gives
 *     HH_ERR_UNSUPPORTED_DEVICE.  Faults of enqueued work surface at stream
 *     synchronisation.
 */
#ifndef HH_H_
#define HH_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HH_OK = 0,
    HH_ERR_INVALID_ARG = 1,
    HH_ERR_UNSUPPORTED_DEVICE = 2,
    HH_ERR_OUT_OF_MEMORY = 3,
    HH_ERR_LAUNCH = 4,
    HH_ERR_BUSY = 5
} hh_status;

/* Human-readable text for a status code (static storage, never NULL). */
const char* hh_status_string(hh_status status);

/* Library version as 10000*major + 100*minor + patch. */
int hh_version(void);

/* The two initialization constants of Sec. 4.4 (host pointers, 4 words each,
 * lane 0 first), as the kernels use them. */
void hh_get_constants(uint64_t c0[4], uint64_t c1[4]);

/* Batched one-shot hashing (Sec. 4.2-4.5), 64-, 128- or 256-bit results.
 * The library picks the kernel: a planner buckets messages by length
 * (longest first) and a persistent kernel hashes long messages with four
 * threads per message and short ones with one thread per message. */
hh_status hh_hash64(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                    const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                    const uint64_t* lengths, uint64_t n_msgs, uint64_t* out, void* stream);
hh_status hh_hash128(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                     const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                     const uint64_t* lengths, uint64_t n_msgs, uint64_t* out, void* stream);
hh_status hh_hash256(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                     const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                     const uint64_t* lengths, uint64_t n_msgs, uint64_t* out, void* stream);

/* Explicit kernel choice, same arguments plus the output width in words
 * (1, 2 or 4).  The result never depends on the path:
 *   HH_PATH_AUTO        what hh_hash64/128/256 do;
 *   HH_PATH_LANE1       one launch, one thread per message (all 4 lanes in
 *                       registers), messages in index order;
 *   HH_PATH_LANE4       one launch, four threads per message (one lane each,
 *                       DPP exchanges), messages in index order;
 *   HH_PATH_BUCKETED    length planner + persistent kernel (the AUTO path). */
typedef enum {
    HH_PATH_AUTO = 0,
    HH_PATH_LANE1 = 1,
    HH_PATH_LANE4 = 2,
    HH_PATH_BUCKETED = 3
} hh_path;

hh_status hh_hash_path(hh_path path, uint32_t width_words, const uint64_t* keys,
                       uint32_t n_keys, const uint32_t* key_idx, const uint8_t* data,
                       uint64_t data_bytes, const uint64_t* offsets, const uint64_t* lengths,
                       uint64_t n_msgs, uint64_t* out, void* stream);

/* Allocation-free batched hashing, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, argument checks and results as
 * hh_hash_path(HH_PATH_BUCKETED, ...), but the length planner's plan and
 * index lists live in one fixed array of device memory per GPU, part of the
 * library's code object (HH_NOALLOC_SCRATCH_BYTES, about 8 MiB, held by every
 * GPU the library runs on until the process ends), instead of a workspace
 * the library allocates.  The call allocates nothing (no hipMalloc, no
 * graph), launches its kernels directly on `stream` and is not seen by the
 * measurement hook.  Its first call on a device looks up that device's copy
 * of the array (no allocation); later calls only enqueue kernels.
 *   - n_msgs above HH_NOALLOC_MAX_MSGS gives HH_ERR_INVALID_ARG (split larger
 *     batches over several calls on one stream).
 *   - Each call clears the part of the array that must start at zero, so it
 *     does not depend on what the previous call left there.
 *   - Every call on one GPU uses that GPU's one array: calls whose work
 *     overlaps in time on the same GPU (other streams, other host threads)
 *     race on it and give wrong results.  The caller orders them (one
 *     stream, or events between streams).  Calls of the other entry points
 *     do not touch the array. */
#define HH_NOALLOC_MAX_MSGS (1u << 20)
#define HH_NOALLOC_SCRATCH_BYTES (256u * 9u + 8u * HH_NOALLOC_MAX_MSGS)
hh_status hh_hash_noalloc(uint32_t width_words, const uint64_t* keys, uint32_t n_keys,
                          const uint32_t* key_idx, const uint8_t* data, uint64_t data_bytes,
                          const uint64_t* offsets, const uint64_t* lengths, uint64_t n_msgs,
                          uint64_t* out, void* stream);

/* The "plain" kernel: every message has the same `length`, one thread per
 * message, one launch.  Hashing a batch of mixed lengths with it takes one
 * call per distinct length (the baseline the batched path is measured
 * against).  64-bit results. */
hh_status hh_hash64_uniform(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                            const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                            uint64_t length, uint64_t n_msgs, uint64_t* out, void* stream);

/* Counter-mode keyed PRF (the random-number use case of Sec. 1): message j
 * (j < n) is the 8-byte little-endian encoding of c = counter_base + j
 * (mod 2^64), hashed under key c mod n_keys; out[w*j ..] receives its
 * width_words-word hash.  Identical to hh_hash* over those messages, but no
 * input buffer or offsets/lengths exist: each thread builds its message in
 * registers. */
hh_status hh_prf(uint32_t width_words, const uint64_t* keys, uint32_t n_keys,
                 uint64_t counter_base, uint64_t n, uint64_t* out, void* stream);

/* ---------------------------------------------------------------------------
 * Incremental hashing (Sec. 4.5: only size mod 32 enters the hash, so a stream
 * is fully described by the 1024-bit state once whole packets are consumed).
 * A state is HH_STATE_WORDS uint64 words in device memory, caller-owned:
 * v0[0..3], v1[0..3], mul0[0..3], mul1[0..3].
 */
#define HH_STATE_WORDS 16

/* The state array holds n_states states (16*n_states words).  An item whose
 * state index is n_states or more is skipped: it reads and writes nothing.
 *
 * For k < n: states[16*t ..] = Reset(keys[key_idx[k]]) (Sec. 4.4), where
 * t = state_idx[k] (state_idx NULL: t = k; key_idx NULL: key 0; key indices
 * are clamped to n_keys - 1). */
hh_status hh_state_init(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                        uint64_t* states, uint64_t n_states, const uint32_t* state_idx, uint64_t n,
                        void* stream);

/* Item k folds the whole packets of data[offsets[k] .. + lengths[k]) into
 * state state_idx[k] (state_idx NULL: state k) and stores the state back.
 * lengths[k] should be a multiple of 32; only its whole packets are consumed
 * (lengths[k] rounded down to a multiple of 32).  Two items must not name the
 * same state in one call.  Byte ranges are clamped to data_bytes. */
hh_status hh_state_update(uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                          const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                          const uint64_t* lengths, uint64_t n, void* stream);

/* Item k takes state state_idx[k], folds in its bytes (any length: whole
 * packets, then the remainder step with r = lengths[k] mod 32, which is the
 * stream's total size mod 32 because earlier updates were whole packets),
 * finalizes (Sec. 4.3) and writes width_words[k] (1, 2 or 4; NULL = 1) words
 * to out[out_offsets[k] ..] (out_offsets NULL: out[4*k ..]); words at index
 * out_words or beyond are not written, and an item whose width is not 1, 2
 * or 4 writes nothing.  The stored state is not modified, so a stream can be
 * finished more than once. */
hh_status hh_state_final(uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                         const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                         const uint64_t* lengths, const uint8_t* width_words, uint64_t* out,
                         uint64_t out_words, const uint64_t* out_offsets, uint64_t n,
                         void* stream);

/* One launch of mixed items (a serving iteration): item k with
 * width_words[k] == 0 is an update exactly as in hh_state_update; any other
 * width finishes as in hh_state_final (widths other than 1, 2 and 4 leave
 * the state as it is and write nothing).  width_words is required; out may be
 * NULL when no item finishes (out_words is then taken as 0). */
hh_status hh_state_step(uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                        const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                        const uint64_t* lengths, const uint8_t* width_words, uint64_t* out,
                        uint64_t out_words, const uint64_t* out_offsets, uint64_t n,
                        void* stream);

/* Device byte copies for request ingress (the serving loop moves many
 * payloads into its arena with one launch): for k < n,
 * dst[dst_offs[k] .. + lens[k]) = src[src_offs[k] .. + lens[k]), each
 * segment clamped to both buffers.  Segments must not overlap each other in
 * dst or overlap src.  max_len (the longest lens[k]) only sizes the launch:
 * any value gives the same bytes. */
hh_status hh_copy_segments(uint8_t* dst, uint64_t dst_bytes, const uint8_t* src,
                           uint64_t src_bytes, const uint64_t* src_offs, const uint64_t* dst_offs,
                           const uint64_t* lens, uint64_t n, uint64_t max_len, void* stream);

/* ---------------------------------------------------------------------------
 * Continuous hashing of long messages (serving): a persistent kernel takes
 * messages from a queue in host memory while it runs and hashes each one
 * whole (Sec. 4.2-4.5, four threads per message), so that a message submitted
 * while others are being hashed starts without waiting for a launch.  Each
 * hashing wave holds up to 16 messages at a time, taking a new one whenever
 * one of its places is free (it looks every 2048 packets); results reach host
 * memory directly.  One feed serves one caller thread at a time (calls on one
 * feed are serialised by a lock).
 *
 * hh_feed_open: keys (device, n_keys x 4 words) and the byte buffer
 * data[0 .. data_bytes) (device) are fixed for the feed's life; the caller
 * keeps them alive, and unmodified where submitted messages lie until their
 * results are seen.  `slots` result rows (1 .. HH_FEED_MAX_SLOTS) live in
 * pinned host memory owned by the feed, and at most `slots` messages are in
 * flight.  `waves` (2 .. HH_FEED_MAX_WAVES) one-wave workgroups are launched
 * on `stream` (which then carries nothing else while the feed is open): one
 * dispatcher and waves - 1 hashing waves, which fill up in index order (an
 * idle wave takes a message only while no lower one has a free place), so
 * that few CUs carry the long chains beside other work.  Each launch stops
 * taking messages after max_ms (1 .. HH_FEED_MAX_MS) milliseconds and ends
 * once it has finished those it holds; hh_feed_submit and hh_feed_poll
 * launch again while submitted messages wait (so a message submitted as a
 * launch ends waits for the longest message that launch still holds:
 * choose max_ms well above the longest message's hashing time).  Allocates
 * host and device memory (HH_ERR_OUT_OF_MEMORY). */
#define HH_FEED_MAX_SLOTS 65536u
#define HH_FEED_MAX_WAVES 65u
#define HH_FEED_MAX_MS 60000u
typedef struct hh_feed hh_feed;
hh_status hh_feed_open(const uint64_t* keys, uint32_t n_keys, const uint8_t* data,
                       uint64_t data_bytes, uint32_t slots, uint32_t waves, uint32_t max_ms,
                       void* stream, hh_feed** feed);

/* Queue n (1 .. slots) messages, taken in this order; the arrays are HOST
 * arrays of n entries, read before the call returns.  Message i is
 * data[offsets[i] .. + lengths[i]) (clamped to data_bytes) under key
 * key_idx[i] (NULL: key 0; clamped to n_keys - 1), and its width_words[i]
 * (1, 2 or 4) hash words go to result row slot[i] (< slots).  *first_ticket
 * receives the ticket of message 0; message i has ticket first + i (tickets
 * start at 1 and never repeat in a feed).  A slot must not be submitted
 * again until its result has been seen.  HH_ERR_BUSY (nothing queued): the
 * queue has no room for n more messages until the kernel has read earlier
 * ones; submit again later. */
hh_status hh_feed_submit(hh_feed* feed, uint32_t n, const uint64_t* offsets,
                         const uint64_t* lengths, const uint32_t* key_idx,
                         const uint8_t* width_words, const uint32_t* slot,
                         uint64_t* first_ticket);

/* Launch the kernel again if its last launch has ended while submitted
 * messages wait.  Call it from the loop that watches the results. */
hh_status hh_feed_poll(hh_feed* feed);

/* Result rows (host memory, 5 words per slot): row s holds the hash words of
 * the message last hashed for slot s, then that message's ticket.  The
 * words of a message are in place once its ticket is: read the ticket, then
 * the words.  Valid until hh_feed_close; NULL for a null feed. */
const volatile uint64_t* hh_feed_results(const hh_feed* feed);

/* Stop taking messages, wait for the kernel to finish those it holds and
 * free the feed. */
hh_status hh_feed_close(hh_feed* feed);

/* ---------------------------------------------------------------------------
 * Avalanche statistics (the strengthened avalanche test of Sec. 6.1 and the
 * finalization-round study of Sec. 4.3).  For every sample s < n_samples it
 * hashes (64-bit, `rounds` finalization rounds, 1..4; the hash proper uses 4)
 * a message of msg_bytes (1..32) bytes and the same message with input bit
 * b flipped, for b in [bit_first, bit_first + bit_count) (bit_count <= 32,
 * bit_first + bit_count <= 8*msg_bytes; bit b is bit b%8 of byte b/8), and
 * adds to counts[64*(b - bit_first) + k] (device, uint64, caller-zeroed) the
 * number of samples whose output bit k changed.
 *   mode 0: key word w (0..3) and message word w (4..7, little-endian, bytes
 *           beyond msg_bytes cleared) of sample s are output 8s+w+1 of
 *           SplitMix64 (Steele, Lea, Flood 2014) seeded with `seed`;
 *   mode 1: the message is the little-endian encoding of s (bytes beyond
 *           msg_bytes cleared) under the one key `key` (host, 4 words): with
 *           n_samples = 2^(8*msg_bytes) every input is enumerated. */
hh_status hh_avalanche(int mode, uint32_t msg_bytes, uint32_t rounds, uint64_t seed,
                       const uint64_t key[4], uint64_t n_samples, uint32_t bit_first,
                       uint32_t bit_count, uint64_t* counts, void* stream);

/* ---------------------------------------------------------------------------
 * Tuning of the bucketed path (host-side settings, process-wide). */
typedef struct {
    uint32_t lane4_min_bytes;   /* messages at least this long go to the persistent
                                   kernel (four threads each); shorter ones are
                                   hashed one thread each while the plan is built */
    uint32_t waves_per_cu;      /* persistent grid: CUs x waves_per_cu waves (4, 8, ...) */
    uint32_t use_graph;         /* capture planner + hash launches in a hipGraph */
    uint32_t long_ring;         /* packets in flight per thread in the persistent
                                   kernel: 36, 48, 72 or 96 */
    uint32_t isolate_long;      /* 1: the items that set the critical path (first
                                   message within 2x of the longest, at most a
                                   quarter of the CUs' worth) run on CUs whose
                                   other waves take no short dynamic items;
                                   0: off.  Only with waves_per_cu <= 4. */
} hh_tuning;

void hh_get_tuning(hh_tuning* t);
hh_status hh_set_tuning(const hh_tuning* t);

/* Free the library's per-device workspaces and cached graphs.  Call it after
 * synchronising the streams the library was called on, and while no other
 * host thread is inside a library call; later calls allocate afresh. */
hh_status hh_release(void);

/* Device address of pinned host memory (hipHostMalloc'd, e.g. a pinned
 * torch tensor), for kernels that read item lists from or write results to
 * host memory directly (the serving loop passes such addresses to
 * hh_state_init, hh_state_step and hh_hash_path, so that no copy runs for
 * them).  Returns
 * HH_ERR_INVALID_ARG for a null pointer and for memory the runtime does not
 * know as pinned. */
hh_status hh_pinned_device_pointer(const void* host, void** device);

/* ---------------------------------------------------------------------------
 * Measurement hook (benchmarks, profilers).  While enabled, every call of the
 * bucketed path records a pair of HIP events on its stream around its
 * persistent long-message kernel, the path's dominant kernel.
 * hh_timing_collect waits for every recorded pair, returns how many launches
 * were recorded and their summed duration in milliseconds, and forgets them.
 * Recording stops at 4096 pending pairs.  Process-wide; not for concurrent
 * use from several threads. */
hh_status hh_timing_enable(int enable);
hh_status hh_timing_collect(uint32_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HH_H_ */
