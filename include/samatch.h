/*
 * samatch.h -- suffix-array matching of short DNA reads on an AMD MI355X (gfx950).
 *
 * The problem follows Sections III and IV of Liao et al., "Ultra-fast Multiple
 * Genome Sequence Matching Using GPU": a reference S over {a,c,g,t} (Section
 * III) is indexed by its suffix array SA (Section III, Table I); each query P
 * is located by binary searches over SA that find the row range of the
 * suffixes that start with P (Section IV, Algorithm 1: LB and RB).
 *
 * Conventions
 *   - positions and SA rows are 0-based; bases order a < c < g < t; a suffix
 *     that is a proper prefix of another sorts first (Table I);
 *   - upper and lower case are the same base;
 *   - a read byte outside ACGTacgt matches no reference base.
 *
 * Result per read P[0..m): the longest matched prefix length len (the
 * largest k <= m such that P[0..k) occurs in S) and the half-open row range
 * [lo, hi) of the suffixes that start with P[0..len).  When len == m the
 * read occurs exactly, hi - lo is its number of occurrences, and the paper's
 * pair is LB = lo, RB = hi - 1.  When P does not occur the paper reports
 * "NULL"; this library reports the longest prefix that does occur instead
 * (len = 0 gives [0, n)).
 *
 * Return codes: SA_OK (0) on success, a negative SA_E* code on failure,
 * and SA_PENDING (> 0) only from match_poll.  After a failure,
 * sa_last_error() returns a thread-local message with detail (for
 * SA_EDEVICE the HIP error string).  No function aborts the process.
 */
#ifndef SAMATCH_H
#define SAMATCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SA_OK = 0,
    SA_PENDING = 1,        /* match_poll: request not finished yet            */
    SA_EINVAL = -1,        /* null pointer, bad size, bad offsets, bad option */
    SA_EALPHABET = -2,     /* reference byte outside ACGTacgt                 */
    SA_ETOOBIG = -3,       /* n > 2^31-1, or a read longer than SA_MAX_READ   */
    SA_ENOMEM = -4,        /* host allocation failed                          */
    SA_EDEVICE = -5,       /* HIP runtime error (see sa_last_error)           */
    SA_ENOSPC = -6,        /* a request can never fit in device memory        */
    SA_ECANCELED = -7,     /* request cancelled (server destroyed)            */
    SA_EIO = -8,           /* index file could not be read or written         */
    SA_EFORMAT = -9,       /* index file is corrupt or of another version     */
    SA_ENOTFOUND = -10     /* unknown ticket                                  */
};

/* Longest read the search kernels take (32 packed 64-bit words: the
 * paper's 1024-base queries, Section V).  Reads of up to 320 bases are
 * searched with their words in registers; longer ones are packed into LDS
 * and searched from there by a kernel of their own. */
#define SA_MAX_READ 1024

typedef struct sa_index sa_index;     /* host index: n, 2-bit packed text, int32 SA */
typedef struct sa_dindex sa_dindex;   /* the same index resident in device memory    */
typedef struct sa_server sa_server;   /* request loop over resident indexes          */

/* One result, 16 bytes, written with one store per read. */
typedef struct {
    int32_t lo;       /* first SA row of the suffixes starting with P[0..len)  */
    int32_t hi;       /* one past the last such row                            */
    int32_t len;      /* longest matched prefix length                         */
    uint32_t flags;   /* SA_HIT_EXACT, SA_HIT_TOOLONG                          */
} sa_hit;

#define SA_HIT_EXACT   1u  /* len == m: the whole read occurs                    */
#define SA_HIT_TOOLONG 2u  /* device entry points only: the read is longer than
                              SA_MAX_READ (or its offsets decrease); lo, hi and
                              len are 0 and the read was not searched           */

/* ------------------------------------------------------------------ index */

/* Build the suffix array of text[0..n) on the host by the DC3 (skew)
 * construction of Section III, and pack the text at 2 bits per base.
 * text: host bytes, ACGTacgt only (else SA_EALPHABET); 1 <= n <= 2^31-1
 * (else SA_EINVAL / SA_ETOOBIG).  The text is copied; *out is owned by the
 * caller and released with sa_free. */
int sa_build(const char *text, int64_t n, sa_index **out);

/* Build from a suffix array the caller already has (no check beyond ranges:
 * sa must be the suffix array of text; values outside [0,n) -> SA_EINVAL). */
int sa_build_from_sa(const char *text, int64_t n, const int32_t *sa, sa_index **out);

int64_t sa_index_length(const sa_index *ix);          /* n, or -1 for NULL         */
/* Copy the int32 suffix array (n entries) into host memory at sa_out. */
int sa_index_copy_sa(const sa_index *ix, int32_t *sa_out);

/* Persist / restore an index (magic, version, n, packed text, SA, FNV-1a
 * checksum).  sa_load returns SA_EIO / SA_EFORMAT for unreadable or corrupt
 * files. */
int sa_save(const sa_index *ix, const char *path);
int sa_load(const char *path, sa_index **out);
void sa_free(sa_index *ix);                           /* NULL is a no-op            */

/* Copy the index to device `device` and keep it resident: the packed text
 * (with zero padding words after the end), the int32 SA, a 16-byte record per SA
 * row holding the first 32 bases of its suffix with the suffix's position
 * and length (so that most probes of the tuned kernel load one record and
 * never touch the text), the table of the top levels of the
 * implicit binary-search tree that the tuned kernel stages in LDS (the tile
 * of Section IV), and, for n >= 4096, a prefix table: for every string v of
 * k = round(log4 n) + 2 bases (4 <= k <= 16, fewer while the table would
 * take more than a quarter of the free device memory), the first SA row
 * whose suffix is not below v with the bracket of rows that start with v,
 * or the result of the reads that start with v when there are none (4^k + 1
 * entries of 16 bytes; see sa_set_prefix_table).  The host index may be
 * freed afterwards.  Released with sa_dfree (NULL is a no-op). */
int sa_upload(const sa_index *ix, int device, sa_dindex **out);
void sa_dfree(sa_dindex *d);
int64_t sa_dindex_length(const sa_dindex *d);

/* Resident index of text[0..n) with its suffix array built on the device
 * (the array of Section III; the paper builds it with DC3, here the device
 * sorts suffixes by prefix doubling with radix sorts).  The result is the
 * same array sa_build gives and the same resident index sa_upload makes
 * from it.  Same validation and errors as sa_build; SA_EDEVICE /
 * SA_ENOMEM when the device fails or runs out of memory (scratch about
 * 29 bytes per base during construction, freed before returning).  The text
 * buffer is the caller's and is not kept. */
int sa_build_device(const char *text, int64_t n, int device, sa_dindex **out);

/* Device bytes of a resident index by part: bytes[0] packed text (with its
 * padding words), bytes[1] suffix array, bytes[2] row records, bytes[3]
 * prefix table (0 without one), bytes[4] LDS tile table.  The plain kernel
 * reads the first two; the tuned kernels all of them. */
int sa_dindex_bytes(const sa_dindex *d, int64_t bytes[5]);

/* Rebuild the prefix table of a resident index for strings of k bases
 * (4 <= k <= 16, texts of at least 4096 bases), or drop it (k = 0).  The
 * default is k = round(log4 n) + 2, at most 16 (see sa_upload).  Entries
 * are 16 bytes, one per k-base string v (4^k + 1 in all): the first SA row
 * not below v, and either the size of the bracket of rows that start with v
 * with the position and
 * bases k .. k+15 of the suffix at its first search pivot, or, when no
 * suffix starts with v, the result every read starting with v gets (its
 * longest matched prefix is shorter than k and depends on v alone).
 * Resets the index's default search start and sort (prefix table and input
 * order with a table, tile and prefix sort without); results never change.
 * Not to be called while batches on this index are in flight. */
int sa_set_prefix_table(sa_dindex *d, int k);

/* Host copy (packed text and suffix array) of a resident index, e.g. to
 * save one built on the device with sa_save.  Free with sa_free. */
int sa_download(const sa_dindex *d, sa_index **out);

/* For an index from sa_build_device: *steps = sorting rounds (the 21-base
 * keys, then one per doubling), *sorted_pairs = (key, value) pairs sorted
 * over all rounds.  Both 0 for an index from sa_upload.  Nullable outputs. */
int sa_dindex_build_info(const sa_dindex *d, int *steps, int64_t *sorted_pairs);

/* ------------------------------------------------------------------ batches */

enum { SA_KERNEL_TUNED = 0, SA_KERNEL_PLAIN = 1 };

/* Launch configuration.  A NULL configuration means the index's defaults
 * (sa_tune's choice once it has run, else built-in ones).  In a given one,
 * a zero tile_levels, block, blocks_per_cu, group, nbuckets or max_words
 * takes the index's default; every other field is used as given. */
typedef struct {
    int kernel;          /* SA_KERNEL_TUNED or SA_KERNEL_PLAIN                     */
    int tile_levels;     /* tuned: levels of the search tree held in LDS (1..13)   */
    int block;           /* tuned: threads per workgroup: 256, 512 or 1024         */
    int blocks_per_cu;   /* tuned: persistent workgroups per compute unit          */
    int nbuckets;        /* tuned: length buckets (1..8)                           */
    int bucket_edge[8];  /* tuned: bucket b holds reads with m <= bucket_edge[b];
                            ascending; the last bucket takes every longer read   */
    int sort;            /* tuned: sort reads by prefix first: 1 = on the top 8, 16
                            or 24 prefix bits, the fewest with 2^bits >= reads/64;
                            8, 16 or 24 = on that many bits; 0 = input order     */
    int use_graph;       /* 1 = match_batch_dev replays the batch's launch sequence
                            as a hipGraph captured on first use for the same
                            buffers, size and settings (not on the null stream;
                            up to 8 per stream are kept)                         */
    int profile;         /* 1 = record HIP events between the stages (pack, sort,
                            search) for sa_stage_times                           */
    int count;           /* 1 = run the instrumented search kernel that counts
                            probes and text words for sa_probe_counts (slower;
                            results are the same)                                */
    int group;           /* tuned: 64-read chunks per block of the work split
                            (1..64): workgroup rank r takes blocks r, r+G, ... */
    int prefix_table;    /* tuned: 1 = start each search from the prefix table
                            (when the index has one), 0 = from the LDS tile     */
    int inline_pack;     /* tuned, reads in input order (sort 0) given by CSR
                            offsets: 1 = the search kernel converts its reads
                            from ASCII itself (no separate pack pass), when its
                            tile and packing areas fit in LDS (160 KB);
                            0 = a pack pass first                               */
    int max_words;       /* tuned, with inline_pack: 64-bit words of a read the
                            search kernel holds in registers, 5 or 10 (reads of
                            up to 160 or 320 bases; longer ones go to the
                            long-read kernel).  5 keeps fewer registers live so
                            that more waves fit a compute unit; 0 = the
                            index's default                                     */
    int defer;           /* tuned, with inline_pack: a read whose binary searches
                            take more than this many probes of row records is
                            set aside and searched again, without a limit,
                            together with 63 other such reads, so that one long
                            search does not keep 63 lanes of its wave idle
                            (0..1024; 0 = never; the index default is 3).
                            Results never change.                              */
} sa_match_cfg;

/* Fill cfg with the index's current defaults. */
int sa_default_cfg(const sa_dindex *d, sa_match_cfg *cfg);

/* Match a batch held in host memory and wait for it: for every read, the
 * two binary searches of Section IV (Algorithm 1: LB, then RB) over the
 * suffix array, or, when the read does not occur, the longest prefix that
 * does and its row range (see "Result per read" above).  reads: concatenated
 * read bytes; offs[nreads+1]: read i is reads[offs[i] .. offs[i+1]) (offs[0]
 * may be nonzero, offsets must not decrease); out[nreads]: results in input
 * order.  Reads longer than SA_MAX_READ -> SA_ETOOBIG before any work.
 * hip_stream: a hipStream_t or NULL for the null stream.  cfg may be NULL.
 * The batch streams through pinned staging in chunks of whole reads (at most
 * 32 MiB of bytes or 2^19 reads each): the host copies one chunk in while the
 * device searches the one before, so the device sees each chunk as a batch
 * of its own (stage times and counts report the last chunk).
 * Thread-safe for distinct streams. */
int match_batch(const sa_dindex *d, const char *reads, const int64_t *offs, int64_t nreads,
                sa_hit *out, void *hip_stream, const sa_match_cfg *cfg);

/* The same searches (Section IV, Algorithm 1) on device memory,
 * asynchronous on hip_stream: d_reads, d_offs
 * and d_out are device pointers of the index's device; the call returns
 * after enqueueing.  Per-read errors (SA_HIT_TOOLONG) are reported in the
 * flags of out.  Scratch memory is kept per (index, stream) and grows on
 * demand; concurrent calls on one stream must be serialised by the caller. */
int match_batch_dev(const sa_dindex *d, const uint8_t *d_reads, const int64_t *d_offs,
                    int64_t nreads, sa_hit *d_out, void *hip_stream, const sa_match_cfg *cfg);

/* Entry point without allocation, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, hosts that forbid
 * hipMalloc): the pipeline of match_batch_dev with the same arguments and
 * results, but its scratch comes from one fixed array of
 * SA_NOALLOC_SCRATCH_BYTES per device, set aside when the library is loaded
 * and kept until the process ends, and it calls no allocating routine.  Its
 * size bounds the batch only on the path with a pack pass (cfg.sort != 0,
 * the plain kernel, or inline_pack = 0): sa_noalloc_max_reads(1) reads;
 * inline packing (the default with a prefix table) needs a few counters
 * whatever the batch size (sa_noalloc_max_reads(0)).  A larger batch ->
 * SA_ENOSPC before any work.  cfg.use_graph is ignored (launches go to the
 * stream directly); cfg.profile and cfg.count -> SA_EINVAL.  Every call on
 * one device shares that device's array and leaves its contents behind (the
 * kernels clear what must start at zero): calls that overlap on one device,
 * on any streams, race and must be serialised by the caller. */
#define SA_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int match_batch_dev_noalloc(const sa_dindex *d, const uint8_t *d_reads, const int64_t *d_offs,
                            int64_t nreads, sa_hit *d_out, void *hip_stream, const sa_match_cfg *cfg);
/* Largest batch match_batch_dev_noalloc takes on the path with a pack pass
 * (pack_pass = 1) or with inline packing (0). */
int64_t sa_noalloc_max_reads(int pack_pass);

/* Stage times in milliseconds of the last batch enqueued with cfg.profile
 * on this (index, stream): ms[0] pack, ms[1] prefix sort, ms[2] search,
 * ms[3] whole pipeline.  Waits for that batch.  SA_EINVAL if there is none. */
int sa_stage_times(const sa_dindex *d, void *hip_stream, double ms[4]);

/* Counts of the last batch enqueued with cfg.count on this (index, stream):
 * c[0] global-memory probes (one SA row each), c[1] 64-bit text words
 * those probes compare, c[2] probes answered from the LDS tile, c[3] reads
 * searched, c[4] packed query words loaded, c[5] 8-byte words loaded from
 * row records (the first 32 bases of each probe included), c[6]
 * prefix-table lookups (one 16-byte entry each), c[7] bytes
 * touched by the search kernels: for every global load or store of a wave,
 * the distinct 64-byte segments its active lanes address, times 64; c[8]
 * the part of c[7] / 64 that the loads from the index make (prefix table,
 * row records, suffix array, text: scattered addresses), the memory
 * requests of the searches; c[9] those index loads counted per lane.
 * Waits for that batch. */
int sa_probe_counts(const sa_dindex *d, void *hip_stream, int64_t c[10]);

/* Autotuner: time candidate configurations (tile depth, workgroups per CU,
 * block size, bucket edges) on the given device batch, keep the fastest as
 * the index's default, and return it in best (nullable).  best_ms receives
 * its time per batch (nullable).  If cache_path is non-NULL the result is
 * read from / appended to that JSON-lines file keyed by (device name, n,
 * length histogram).  Every candidate's results are compared on the device
 * with the first candidate's; a difference fails the call (SA_EDEVICE). */
int sa_tune(sa_dindex *d, const uint8_t *d_reads, const int64_t *d_offs, int64_t nreads,
            void *hip_stream, const char *cache_path, sa_match_cfg *best, double *best_ms);

/* The configurations sa_tune would time on a batch with these offsets:
 * every tile depth and workgroup shape of its first stage, then the
 * variants of its later stages (work-split block size, search start, sort
 * width, packing pass, bucket layouts) taken around `around` (NULL: the
 * index's current defaults; bucket layouts as if sorted).  Each one must
 * give the same results (the intervals of Section IV are unique), which
 * the parity tests check.  Writes min(*count, capacity) of them to out;
 * *count receives the total. */
int sa_tune_candidates(const sa_dindex *d, const int64_t *d_offs, int64_t nreads, void *hip_stream,
                       const sa_match_cfg *around, sa_match_cfg *out, int capacity, int *count);

/* ------------------------------------------------------------------ locate */

/* Text positions of the occurrences (Section IV lists a read's occurrences
 * as the suffix-array entries of its row interval).  A read is selected when
 * its hit is exact (min_len == 0), or when its matched length h.len >=
 * min_len (min_len > 0, which also locates the longest matched prefix of
 * reads that do not occur).  A selected read emits SA[h.lo], SA[h.lo + 1],
 * ... for its first min(h.hi - h.lo, cap) rows, in suffix-array order;
 * other reads emit nothing.
 *
 * Device form: d_hits[nreads] as written by match_batch_dev; d_offs
 * [nreads + 1] (int64) receives CSR offsets, so read i's positions are
 * d_pos[d_offs[i] .. d_offs[i + 1]).  *total receives d_offs[nreads].  When
 * *total > pos_capacity the offsets are still written, no position is, and
 * the call returns SA_ENOSPC (call again with a buffer of *total entries).
 * Enqueued on hip_stream; waits for it to read the total, the positions are
 * written asynchronously after return.  SA_EINVAL for a selected hit whose
 * interval is not inside [0, n].  Allocates a small scratch per call. */
int sa_locate_dev(const sa_dindex *d, const sa_hit *d_hits, int64_t nreads, int32_t cap, int32_t min_len,
                  int64_t *d_offs, int32_t *d_pos, int64_t pos_capacity, void *hip_stream, int64_t *total);

/* Host form of sa_locate_dev: hits, offs and pos are host buffers; waits
 * for completion. */
int sa_locate(const sa_dindex *d, const sa_hit *hits, int64_t nreads, int32_t cap, int32_t min_len,
              int64_t *offs, int32_t *pos, int64_t pos_capacity, int64_t *total);

/* ------------------------------------------------------------ suffix tree */

/* The suffix tree the paper compares the suffix array with (Sections III
 * and V; it transmits the tree to the GPU as a flattened array and gives
 * no layout).  Built on the host from a host index (its suffix array and
 * the LCP array) as the tree of lcp-intervals, flattened into 32-byte nodes
 * {lb, rb, depth, 0, child[a], child[c], child[g], child[t]}: the node's
 * suffix-array rows [lb, rb) share `depth` leading bases; child[b] is the
 * node index of the child continuing with base b, -2 - row for a leaf, -1
 * for none.  The search walks it from the root and gives the same
 * (lo, hi, len, flags) as match_batch. */
typedef struct st_index st_index;    /* host tree                                  */
typedef struct st_dindex st_dindex;  /* the same tree resident in device memory    */

int st_build(const sa_index *ix, st_index **out);
void st_free(st_index *t);
int64_t st_node_count(const st_index *t);
int32_t st_root(const st_index *t);
/* Copies the nodes (st_node_count x 8 int32) into out. */
int st_copy_nodes(const st_index *t, int32_t *out);
/* Device bytes of the tree as searched: nodes, suffix array, 2-bit text. */
int64_t st_index_bytes(const st_index *t);
/* Uploads the nodes; the search reads the text and suffix array of d, which
 * must be an index of the same text and must outlive the tree. */
int st_upload(const st_index *t, const sa_dindex *d, st_dindex **out);
void st_dfree(st_dindex *s);
/* Device batch as match_batch_dev (reads of up to SA_MAX_READ bases; longer
 * ones get SA_HIT_TOOLONG), one read per lane in input order.  Async. */
int st_match_batch_dev(const st_dindex *s, const uint8_t *d_reads, const int64_t *d_offs, int64_t nreads,
                       sa_hit *d_out, void *hip_stream);

/* ------------------------------------------------------------------ serving */

typedef struct {
    int64_t hbm_reserve_bytes;   /* device memory left free for others (default 1 GiB)   */
    int64_t max_batch_reads;     /* reads per device batch (default 1,048,576)           */
    int64_t max_inflight_reads;  /* admitted but unfinished reads (default 8,388,608)    */
    int nstreams;                /* device streams used round-robin (default 2, max 8)   */
    int64_t test_fake_free_hbm;  /* < 0: ask the device; >= 0: pretend this much is free */
    int test_echo;               /* 1: no device work, results are a deterministic echo  */
    int test_fail_batch;         /* > 0: the n-th executed batch fails (error injection) */
    int64_t host_pool_bytes;     /* pinned host memory, mapped for the device, that submit
                                    copies reads into (0: default 1 GiB, < 0: none); when it
                                    is full, submit waits for room; a request larger than the
                                    whole pool (or any request without a pool) is copied to
                                    pageable memory instead.  Every admitted request is copied
                                    into a device arena (from the pool by an upload kernel,
                                    else by the runtime) and searched there */
    int measure;                 /* 0: off; 1: time each batch's search stage with events;
                                    2: also run the instrumented search kernels and add up
                                    the bytes they touch (slower); see sa_server_get_stats */
    int64_t batch_linger_us;     /* 0 (default): a free stream starts a batch with whatever
                                    reads are waiting; > 0 (at most 1,000,000): it waits
                                    until a reference has max_batch_reads unscheduled reads
                                    or its oldest one has waited this long, so that batches
                                    are larger (the device busier per launch) at the price
                                    of latency */
} sa_server_opts;

/* Totals of a server since it started.  upload_bytes: request images copied
 * into the device arena; search_ms (measure >= 1): device time of the
 * batches' search stages; touched_bytes (measure == 2): bytes touched by the
 * search kernels, as c[7] of sa_probe_counts. */
typedef struct {
    int64_t batches, reads;
    int64_t upload_bytes;
    double search_ms;
    int64_t touched_bytes;
} sa_server_stats;

typedef struct {
    int64_t t_submit_ns, t_admit_ns, t_done_ns;  /* steady-clock timestamps          */
    int status;                                  /* SA_OK, SA_PENDING or an SA_E*    */
    int64_t nreads;
} sa_req_stats;

/* Start a request loop over nrefs resident indexes (all on one device).
 * At start the server takes, as its device arena, the device memory then
 * free (hipMemGetInfo, or test_fake_free_hbm) less hbm_reserve_bytes and
 * its streams' own buffers (at most 16 GiB); requests are admitted in
 * arrival order while the arena has room for their reads and offsets and
 * max_inflight_reads allows (a request that could never fit finishes with
 * SA_ENOSPC), copied into the arena, batched per reference across requests
 * (continuous batching) on nstreams streams, and their results scattered
 * back by a thread of their own.  The indexes must outlive the server.
 * opts may be NULL (defaults). */
int sa_server_create(const sa_dindex *const *refs, int nrefs, const sa_server_opts *opts,
                     sa_server **out);

/* Queue nreads host reads against refs[ref].  The reads are copied into the
 * server's pinned pool before the call returns (waiting for room while the
 * pool is full: backpressure on the caller); out[nreads] must stay valid
 * until match_poll reports the request finished.  *ticket identifies the
 * request.  SA_ECANCELED when the server is being destroyed.  Thread-safe. */
int match_submit(sa_server *s, int ref, const char *reads, const int64_t *offs, int64_t nreads,
                 sa_hit *out, uint64_t *ticket);

/* Measurement helper (an open-loop client in native threads, so that a
 * load test measures the server and not its caller): submits request i
 * (reference ref[i], reads[i] with offsets offs[i][0..nreads[i]], results
 * into out[i]) at arrival_ns[i] nanoseconds after a start about 20 ms after
 * the call, from nthreads threads (1..64; thread t submits requests t,
 * t + nthreads, ...), then waits for every request.  sched_ns[i] receives
 * the scheduled submit time and stats[i] the request's timestamps and
 * status, on the steady clock of sa_req_stats.  arrival_ns must not
 * decrease within each thread's share.  Returns SA_OK, or the first error
 * of a submit (that request's status holds it; the others still run). */
int sa_server_replay(sa_server *s, int64_t nreq, const int32_t *ref, const char *const *reads,
                     const int64_t *const *offs, const int64_t *nreads, const int64_t *arrival_ns,
                     sa_hit *const *out, int nthreads, int64_t *sched_ns, sa_req_stats *stats);

/* Wait up to timeout_us (0: just look, < 0: forever) for a request.
 * Returns SA_PENDING while it runs, SA_OK once out[] is filled, or the
 * request's error code; st (nullable) receives its timestamps.  A finished
 * ticket may be polled again until sa_server_destroy. Thread-safe. */
int match_poll(sa_server *s, uint64_t ticket, int64_t timeout_us, sa_req_stats *st);

/* Copy the server's running totals (see sa_server_stats) into *out. */
int sa_server_get_stats(sa_server *s, sa_server_stats *out);

/* Cancel pending requests (they finish with SA_ECANCELED), wait for
 * in-flight batches, release everything. */
int sa_server_destroy(sa_server *s);

/* ------------------------------------------------------------------ errors */

const char *sa_strerror(int code);
const char *sa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SAMATCH_H */
