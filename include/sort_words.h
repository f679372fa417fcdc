/*
 * sort_words.h -- C ABI of the MI355X (gfx950) length-bucketed word sort.
 *
 * The operation (arXiv:1411.5283, "Parallelize Bubble and Merge Sort
 * Algorithms Using MPI"):
 *   - words go into one sub-array per character count, shorter words first,
 *     each sub-array sized by the number of words of that length (Abstract;
 *     section 3, "Pre-processing", phase 2);
 *   - each sub-array is put in alphabetical order by bubble sort (section 2;
 *     phase 3);
 *   - in the parallel form a sub-array is cut into chunks, each chunk is
 *     bubble-sorted on its own and the sorted chunks are merged (section 3.2;
 *     section 4, "MPI Implementation"; section 5).
 * On the GPU the chunk sort is odd-even transposition (the data-parallel form
 * of bubble sort's adjacent compare-exchanges) on chunks held in registers,
 * followed by merge-path merges, first in LDS and then across HBM.
 *
 * Result: the unique order of the word indices by the key
 *     (length, bytes compared as unsigned, original index).
 * Ties between equal words keep input order, as bubble sort (which never
 * exchanges equal items) does.
 *
 * Conventions shared by every entry point
 *   - Word i is chars[offsets[i] .. offsets[i+1]).  `offsets` has n+1 entries,
 *     must not decrease, and offsets[0] need not be 0.  Total characters must
 *     be below 2^32, and n at most 2^32 - 2 (a workspace for more words is
 *     refused).  Any byte value is allowed.
 *   - Lengths 0..SW_MAX_LEN are accepted.  A longer word is an error
 *     (SW_ERR_WORD_TOO_LONG); offsets that decrease are SW_ERR_INVALID_ARG,
 *     which takes precedence.  On any error the outputs are unspecified.
 *   - out_perm[k] = index of the word at sorted position k (gather form).
 *   - out_bucket_offsets[L] = number of words shorter than L, for
 *     L = 0..SW_MAX_LEN+1 (SW_NUM_OFFSETS entries; the last one is n).  The
 *     words of length L are out_perm[out_bucket_offsets[L] ..
 *     out_bucket_offsets[L+1]).
 *   - Pointers named chars/offsets/doc_offsets/out_* are DEVICE pointers;
 *     the device offsets and doc_offsets must be 4-byte aligned (as a
 *     uint32_t array is), else SW_ERR_INVALID_ARG.  The
 *     caller owns every buffer; the library keeps no reference to one after
 *     the work on the stream has completed.  Inputs and outputs must not
 *     alias.  Outputs are fully overwritten.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Return values are sw_status codes.  sort_words_last_error() gives a
 *     thread-local message for the last non-OK return of the calling thread.
 */
#ifndef SORT_WORDS_H
#define SORT_WORDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_MAX_LEN 32
#define SW_NUM_OFFSETS (SW_MAX_LEN + 2)
#define SW_NUM_CLASSES 5   /* key classes: lengths 0-4, 5-8, 9-16, 17-24, 25-32 */

typedef enum {
    SW_OK = 0,
    SW_ERR_INVALID_ARG = -1,   /* null or misaligned pointer, bad size, offsets that decrease */
    SW_ERR_WORD_TOO_LONG = -2, /* a word longer than SW_MAX_LEN bytes */
    SW_ERR_WORKSPACE = -3,     /* workspace too small for the request */
    SW_ERR_OOM = -4,           /* device allocation failed */
    SW_ERR_HIP = -5            /* a HIP runtime call failed */
} sw_status;

/* Simple form.  Sorts n words on the null stream with a library-owned,
 * cached workspace and returns when the result is ready, including errors the
 * device detects.  Abstract and section 3 ("Pre-processing", phases 2-3).
 *   chars     device, the characters (may be NULL when the total is 0)
 *   offsets   device, n+1 entries
 *   out_perm  device, n entries; out_bucket_offsets device, SW_NUM_OFFSETS */
int sort_words(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
               uint32_t *out_perm, uint32_t *out_bucket_offsets);

/* Bytes of device workspace that sort_words_ex / sort_words_batch /
 * sort_words_plain need for up to max_words words in up to max_docs
 * documents.  Returns 0 if the sizes are out of range. */
size_t sort_words_workspace_size(uint32_t max_words, uint32_t max_docs);

/* Asynchronous form of sort_words: enqueues the whole sort on `stream` and
 * returns without waiting.  Argument errors found on the host are returned
 * at once; errors found on the device are read with sort_words_status().
 * `workspace` (device, caller-owned, at least
 * sort_words_workspace_size(n, 1) bytes) must not be used by another call
 * until this one has completed on the stream. */
int sort_words_ex(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                  uint32_t *out_perm, uint32_t *out_bucket_offsets,
                  void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): sort_words_ex with
 * the library's own fixed scratch array as its workspace.  It calls no
 * hipMalloc, hipFree or other allocating routine, and every kernel goes on
 * `stream` in order (no side streams, no events).
 *   out_status  device, 1 word: receives the device status word of the run
 *               (0 when it sorted; sort_words_decode_status() turns it into
 *               an sw_status), written on `stream` after the sort
 * The scratch is SW_NOALLOC_SCRATCH_BYTES of device memory, one copy per
 * GPU, held from the library's load until the process ends.  n is limited to
 * the largest count whose sort_words_workspace_size(n, 1) fits it (about 460
 * thousand words); a larger n is SW_ERR_WORKSPACE, returned at once.  Every
 * call on one GPU uses that GPU's one scratch, which keeps the last call's
 * contents (each call rewrites what it reads): calls that overlap on one GPU
 * (two streams or two threads) race, so the caller must serialize them.
 * Other arguments as sort_words_ex; asynchronous. */
#define SW_NOALLOC_SCRATCH_BYTES (32u << 20)
int sort_words_noalloc(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                       uint32_t *out_perm, uint32_t *out_bucket_offsets,
                       uint32_t *out_status, void *stream);

/* Batched form: n_docs independent documents sorted in one pass; every
 * (document, length) pair is one segment (section 3.2: each sub-array is
 * given to its own worker).
 *   offsets      device, N+1 entries over all documents (N total words)
 *   doc_offsets  device, n_docs+1 entries into the word list, doc_offsets[0]
 *                must be 0 and entries must not decrease; document d holds
 *                words doc_offsets[d] .. doc_offsets[d+1]
 *   out_perm     device, N entries; positions doc_offsets[d] ..
 *                doc_offsets[d+1] hold document d's result as
 *                DOCUMENT-LOCAL word indices
 *   out_bucket_offsets  device, n_docs * SW_NUM_OFFSETS entries, row d is
 *                document d's bucket offsets (document-local)
 * Asynchronous like sort_words_ex.  N is read on the device; N above the
 * workspace capacity is SW_ERR_WORKSPACE (reported by sort_words_status). */
int sort_words_batch(const uint8_t *chars, const uint32_t *offsets,
                     const uint32_t *doc_offsets, uint32_t n_docs,
                     uint32_t *out_perm, uint32_t *out_bucket_offsets,
                     void *workspace, size_t workspace_bytes, void *stream);

/* Per-bucket-launch form of sort_words_batch, the comparison baseline for
 * the batched form: the length histogram is read back to the host, then the
 * chunk sort and every merge level are launched separately for each
 * (document, length) segment.  Same arguments and result as
 * sort_words_batch; SYNCHRONOUS (returns device-detected errors). */
int sort_words_plain(const uint8_t *chars, const uint32_t *offsets,
                     const uint32_t *doc_offsets, uint32_t n_docs,
                     uint32_t *out_perm, uint32_t *out_bucket_offsets,
                     void *workspace, size_t workspace_bytes, void *stream);

/* The chunk step alone (section 4: each slave bubble-sorts its chunk; the
 * master's merge is left out): every length list is cut into chunks of
 * `chunk` words from its start (the last chunk shorter), and each chunk is
 * sorted by odd-even transposition on its own.  out_perm holds, for every
 * length list in length order, its chunks one after another, each chunk's
 * indices in sorted order; the chunks are NOT merged.  A power of two in
 * [2, 1024]; the tile configuration is the current sw_config's.  Arguments
 * otherwise as sort_words_ex (one document); SYNCHRONOUS (the host reads the
 * length histogram back, like sort_words_plain). */
int sort_words_chunks(const uint8_t *chars, const uint32_t *offsets, uint32_t n, uint32_t chunk,
                      uint32_t *out_perm, uint32_t *out_bucket_offsets,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Baseline without length lists (the whole-file sorts of Table 2): every word
 * becomes one 32-byte key (its length in the top byte, then its bytes) and
 * the whole list is chunk-sorted and merged as one sequence.  The order is the
 * same total order, so the result equals sort_words'.  Words of at most 31
 * bytes (a 32-byte word is SW_ERR_WORD_TOO_LONG here).  Arguments as
 * sort_words_ex; asynchronous, device errors via sort_words_status(). */
int sort_words_unbucketed(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                          uint32_t *out_perm, uint32_t *out_bucket_offsets,
                          void *workspace, size_t workspace_bytes, void *stream);

/* Waits for `stream`, then returns the status the device recorded in
 * `workspace` for the last call enqueued with it (SW_OK or an error). */
int sort_words_status(const void *workspace, void *stream);

/* Asynchronous status read for callers that must not block: enqueues on
 * `stream` a copy of the device status word of the last call enqueued with
 * `workspace` into *status_dst (pinned host or device memory, caller-owned,
 * 4 bytes); once the stream has reached it, sort_words_decode_status() turns
 * the word into an sw_status.  Returns SW_OK or a host-side error. */
int sort_words_status_async(const void *workspace, uint32_t *status_dst, void *stream);
int sort_words_decode_status(uint32_t status_word);

/* Persistent plan for repeated batched sorts (serving, benchmarks): owns its
 * workspace and a captured HIP graph of the whole pass, so one run is one
 * small descriptor kernel plus one hipGraphLaunch on the plan's stream.
 *   sw_plan_create  capacity max_words words, max_docs documents and
 *                   max_chars characters (the span offsets[N] - offsets[0]
 *                   of a run, below 2^32); `stream` as above; *out receives
 *                   the plan (NULL on error)
 *   sw_plan_run     same arguments and result as sort_words_batch, plus
 *                   n_words: doc_offsets may be NULL, and the run is then one
 *                   document of n_words words (with doc_offsets, n_words is
 *                   not read: the total is doc_offsets[n_docs], read on the
 *                   device); asynchronous; a run above any capacity is
 *                   SW_ERR_WORKSPACE (documents and, without doc_offsets,
 *                   words checked on the host; the device checks the total
 *                   words and characters), device errors via sw_plan_status
 *   sw_plan_status  waits for the plan's stream, returns the device status
 *   sw_plan_destroy frees the plan (waits for its stream first)
 * A plan is not thread-safe; distinct plans may be used from distinct
 * threads. */
typedef struct sw_plan sw_plan;
int sw_plan_create(uint32_t max_words, uint32_t max_docs, uint64_t max_chars, void *stream, sw_plan **out);
int sw_plan_run(sw_plan *plan, const uint8_t *chars, const uint32_t *offsets,
                const uint32_t *doc_offsets, uint32_t n_docs, uint32_t n_words,
                uint32_t *out_perm, uint32_t *out_bucket_offsets);
/* Sort and sorted text in one pass (section 4 prints the merged result):
 * sw_plan_run's arguments and outputs, and out_text receives the words in
 * sorted order, each followed by the byte `sep` (0..255) or back to back when
 * sep < 0, in exactly the layout sort_words_materialize writes (documents one
 * after another; out_text holds (offsets[N] - offsets[0]) + (sep >= 0 ? N : 0)
 * bytes, N the total words).  Every word fits its key (at most 32 bytes), so
 * the text is written from the sorted keys: no word is read again from
 * chars.  The first call captures a second graph (the pass plus the text
 * writer); later calls launch it.  Asynchronous; device errors via
 * sw_plan_status (on an error out_text is unspecified, and no byte outside
 * it is written). */
int sw_plan_run_text(sw_plan *plan, const uint8_t *chars, const uint32_t *offsets,
                     const uint32_t *doc_offsets, uint32_t n_docs, uint32_t n_words,
                     uint32_t *out_perm, uint32_t *out_bucket_offsets, int sep,
                     uint8_t *out_text);
int sw_plan_status(sw_plan *plan);
/* sort_words_status_async for a plan (copy enqueued on the plan's stream). */
int sw_plan_status_async(sw_plan *plan, uint32_t *status_dst);
void sw_plan_destroy(sw_plan *plan);

/* Tuning knobs, process-wide, read when work is enqueued (and when a plan's
 * graph is captured).  chunk[c] is the odd-even chunk size of key class c
 * (section 5: chunk size = array size / processors; here a power of two in
 * [2, 1024], used as given by every tile configuration: a chunk may lie
 * inside one thread's registers, span lanes of a wave or span waves);
 * variant[c] selects a compiled tile configuration of class c
 * (0 .. sw_num_variants(c)-1).  Results never depend on these values. */
typedef struct {
    uint32_t chunk[SW_NUM_CLASSES];
    uint32_t variant[SW_NUM_CLASSES];
    uint32_t flags;   /* SW_FLAG_* */
    /* merge[c]: how class c merges the sorted tiles across HBM.  0: two-way
     * merge-path levels (each pass doubles the run length, tiles of the
     * variant's merge tile); k >= 1: four-way passes with compiled
     * configuration k-1 (each pass merges four runs into one through LDS, two
     * doublings per HBM read and write).  0 .. sw_num_merges(c)-1. */
    uint32_t merge[SW_NUM_CLASSES];
} sw_config;
/* Run the key classes one after another on the caller's stream instead of on
 * parallel streams (for per-kernel measurement; results are identical). */
#define SW_FLAG_SERIAL_CLASSES 1u
/* Enqueue each key class's short-segment sort (segments of at most 1024
 * words, several to a tile) before the class's chunk sort instead of after
 * it.  Results are identical; which order is faster depends on the workload
 * (measured: first is faster for thousands of small documents, after for one
 * large one), so the autotuner chooses it per workload. */
#define SW_FLAG_PACKED_FIRST 2u
/* Run the segment scheduling (the counting sort of (document, length)
 * segments and the tile prefixes, which the bucket scatter does not read) on
 * a side stream beside the scatter instead of before it.  Results are
 * identical; it pays with thousands of documents (many segments) and costs
 * with one large document, so the autotuner chooses it per workload.  Plans
 * and the batched entry points with parallel classes only. */
#define SW_FLAG_SCHEDULE_BESIDE_SCATTER 4u
/* Bits SW_FLAG_ORDER_SHIFT.. of flags: the order in which the key classes'
 * work is enqueued, as an index 0..119 into the 120 orders of the five
 * classes taken in lexicographic order (0: 0-1-2-3-4, 1: 0-1-2-4-3, ...,
 * 119: 4-3-2-1-0).
 * The classes' chains run concurrently either way; the order decides which
 * chunk sorts start first and hold the LDS.  Results are identical; the
 * autotuner chooses it per workload.  Larger indices are rejected. */
#define SW_FLAG_ORDER_SHIFT 8
#define SW_FLAG_ORDER_MASK (127u << SW_FLAG_ORDER_SHIFT)
int sw_get_config(sw_config *out);
int sw_set_config(const sw_config *cfg);
/* Number of compiled variants of class c, and the chunk-sort tile (words per
 * workgroup) and merge tile of a variant. */
int sw_num_variants(int cls);
/* Number of merge choices of class c (two-way, then the four-way
 * configurations): the range of sw_config.merge[c]. */
int sw_num_merges(int cls);
int sw_variant_tiles(int cls, int variant, uint32_t *sort_tile, uint32_t *merge_tile);

/* Kernel timing for measurement: while enabled, every kernel the library
 * enqueues on the eager path (sort_words*, not plan graphs) is bracketed by
 * HIP events on its own stream.  sw_profile_read waits for the recorded
 * work and returns, per kernel family, the launch count and the summed
 * device time in milliseconds; names are static strings. */
int sw_profile_enable(int on);
int sw_profile_reset(void);
int sw_profile_read(int max_entries, const char **names, uint32_t *launches, double *ms);

/* ------------------------------------------------------------ around the sort
 * Tokenizer: the first pre-processing phase of section 3 (special characters
 * removed from the text before the words are listed).  A word is a run of
 * bytes between ASCII whitespace (tab, line feed, vertical tab, form feed,
 * carriage return, space); inside a run the ASCII letters are kept in order
 * and every other byte is dropped without ending the run; a run left without
 * letters is no word.  With SW_TOK_LOWER capitals become lower case.
 *   text         device, n_bytes bytes (n_bytes < 2^32; any pointer alignment)
 *   out_chars    device, n_bytes bytes of capacity: the kept letters
 *   out_offsets  device, max_words+1 entries: word w is
 *                out_chars[out_offsets[w] .. out_offsets[w+1]), out_offsets[0] = 0
 *   out_n_words  device, 1 word: the number of words
 *   workspace    device, sort_words_tokenize_workspace_size(n_bytes) bytes
 * The result is the word list sort_words* take.  Asynchronous on `stream`;
 * more words than max_words is SW_ERR_WORKSPACE, read with
 * sort_words_status(workspace, stream) (outputs then unspecified). */
#define SW_TOK_LOWER 1u
size_t sort_words_tokenize_workspace_size(uint64_t n_bytes);
int sort_words_tokenize(const uint8_t *text, uint64_t n_bytes, uint32_t flags,
                        uint8_t *out_chars, uint32_t *out_offsets, uint32_t max_words,
                        uint32_t *out_n_words, void *workspace, size_t workspace_bytes,
                        void *stream);

/* Sorted text: section 4 prints the merged result.  Writes the words in
 * sorted order, each followed by the byte `sep` (0..255), or back to back
 * when sep < 0.
 *   chars, offsets, doc_offsets, n_docs  the word list given to the sort
 *                (doc_offsets NULL with n_docs = 1: one document)
 *   n_words      total words N
 *   perm, bucket_offsets  the sort's outputs (document-local indices,
 *                n_docs * SW_NUM_OFFSETS offsets)
 *   out_text     device, (offsets[N] - offsets[0]) + (sep >= 0 ? N : 0) bytes;
 *                document d's text starts at byte
 *                (offsets[doc_offsets[d]] - offsets[0]) + (sep >= 0 ? doc_offsets[d] : 0)
 *   out_status   device, 1 word: set to 0, then nonzero if a word fails a
 *                check (index outside its document, offsets outside the word
 *                list, length unlike its bucket's, bytes past the output); such
 *                a word is not written and no byte outside out_text ever is.
 * Asynchronous on `stream`; host-side argument errors are returned. */
int sort_words_materialize(const uint8_t *chars, const uint32_t *offsets,
                           const uint32_t *doc_offsets, uint32_t n_docs, uint32_t n_words,
                           const uint32_t *perm, const uint32_t *bucket_offsets, int sep,
                           uint8_t *out_text, uint32_t *out_status, void *stream);

/* ------------------------------------------------------------ serving
 * Continuous batching of sort requests (not in the paper; the serving form of
 * the batched sort).  sw_server_create allocates budget_bytes of device
 * memory.  A host thread admits requests in arrival order while a block of
 * that memory is free for each (its characters and offsets, each part
 * rounded up to 256 bytes: swsrv::footprint); an admitted request is copied
 * into its block at once by the upload threads (copy_threads of them, at
 * least one; pinned staging, one upload stream), so requests wait for their
 * batch on the device and their uploads overlap the batches running.  Every
 * admitted, uploaded request that is not running is packed into the next
 * batch (up to the batch limits) on the device, from the blocks into the
 * slot's word list, and the batch runs as one sw_plan_run on a free slot
 * (each slot: its own stream, plan and buffers), so batches on different
 * slots overlap on the device.  While a batch runs, the next one starts once
 * it holds min_batch_words words or max_batch_docs requests, or its oldest
 * request has waited max_wait_us.  A request's block is freed when its batch
 * completes; its results are copied out to the caller's buffers by the
 * calling thread and copy_threads helpers.  Device memory taken by the
 * server beside the budget (plans and slot buffers) is
 * sw_server_fixed_bytes(cfg). */
typedef struct sw_server sw_server;
typedef struct {
    uint32_t slots;             /* 1..8 concurrent batches */
    uint32_t max_batch_words;
    uint32_t max_batch_docs;
    uint32_t copy_threads;      /* 0..64 */
    uint64_t max_batch_chars;   /* < 2^32 */
    uint64_t budget_bytes;
    uint32_t min_batch_words;
    uint32_t max_wait_us;
} sw_server_config;
typedef struct {
    uint64_t completed, failed, words, batches, bytes_in_use, max_bytes_in_use;
} sw_server_counts;
int sw_server_create(const sw_server_config *cfg, sw_server **out);
/* One request (one document), HOST pointers: chars/offsets (n_words+1
 * entries, any first offset) must stay valid, and out_perm (n_words) /
 * out_bucket_offsets (SW_NUM_OFFSETS) untouched, until sw_server_wait
 * returns for its ticket.  A malformed request (SW_ERR_INVALID_ARG,
 * SW_ERR_WORD_TOO_LONG) or one that can never fit the budget or a batch
 * (SW_ERR_WORKSPACE) is refused here, alone, and gets no ticket. */
int sw_server_submit(sw_server *srv, const uint8_t *chars, const uint32_t *offsets, uint32_t n_words,
                     uint32_t *out_perm, uint32_t *out_bucket_offsets, uint64_t *out_ticket);
/* Blocks until the request completes; returns its status (a batch that failed
 * on the device fails all its requests) and its latency from submission to
 * the completion seen by the server thread.  A ticket is waited for once:
 * waiting for an unknown ticket, or for one another thread is already
 * waiting for or has waited for, is SW_ERR_INVALID_ARG. */
int sw_server_wait(sw_server *srv, uint64_t ticket, double *latency_s);
int sw_server_stats(sw_server *srv, sw_server_counts *out);
size_t sw_server_fixed_bytes(const sw_server_config *cfg);
/* Bytes of the budget a request of n_words words and n_chars characters
 * holds from its admission until its batch completes (characters, then the
 * n_words+1 offsets, each rounded up to 256 bytes). */
uint64_t sw_server_request_bytes(uint32_t n_words, uint64_t n_chars);
/* Finishes every submitted request, then frees the server. */
void sw_server_destroy(sw_server *srv);

const char *sort_words_last_error(void);
const char *sort_words_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SORT_WORDS_H */
