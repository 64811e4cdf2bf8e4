// Host-side launchers of the device kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "samatch.h"

namespace samatch {

constexpr int kWMax = 10;                 // packed words per read slot of the short-read path
constexpr int kShortWords = 5;            // query words of the search kernel's register-light instance
constexpr int kShortMax = kWMax * 32;     // longest read of the short-read path (320 bases)
constexpr int kLongWords = SA_MAX_READ / 32;  // words of a read on the long-read path
constexpr int kDefaultDefer = 3;          // probes before a read is set aside (sa_match_cfg.defer)
constexpr int kStatWords = 11;
constexpr int kLongFlag = 10;
constexpr int kMaxTileLevels = 13;        // 8191 nodes x 12 B = 96 KiB of LDS
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of a gfx950 compute unit
constexpr int kSortBlock = 256;           // radix sort: threads per workgroup
constexpr int kSortItems = 16;            // keys per thread per pass
constexpr int kSortTile = kSortBlock * kSortItems;

// Per SA row: the suffix's text position and length, then its first
// 32 * kRecWords bases as aligned 2-bit words (zero past the text end).  A
// probe loads the first 16 bytes (position, length, word 0) and further
// words only while they keep matching, from the same line.  One word (16
// bytes per row) is the default: on MI355X the 32- and 64-byte records cut
// the bytes touched per read by 8-10 % but made the search 3-5 % slower
// (a 2-4x larger array caches worse).
#ifndef SAMATCH_REC_WORDS
#define SAMATCH_REC_WORDS 1
#endif
constexpr int kRecWords = SAMATCH_REC_WORDS;
static_assert(kRecWords == 1 || kRecWords == 3 || kRecWords == 7, "row records are 16, 32 or 64 bytes");
struct alignas(8 + 8 * kRecWords) RowRec {
    int32_t pos;
    int32_t len;
    uint64_t key[kRecWords];
};
static_assert(sizeof(RowRec) == 8 + 8 * kRecWords, "row record layout");

// Node of the flattened suffix tree: its run of suffix-array rows [lb, rb),
// the bases its suffixes share (depth), and per base a, c, g, t the child
// that continues with it (node index, leaf -2 - row, or -1).
struct alignas(16) StNode {
    int32_t lb, rb, depth, pad;
    int32_t child[4];
};

// Prefix-table entry of a k-base string v, 16 bytes, so that one load
// answers a lookup.  row = T[v], the first SA row whose suffix is not below
// v.  When some suffix starts with v, its rows are the bracket [T[v],
// T[v] + size), size >= 1 (the suffixes shorter than k that sort right
// after them are left out), pos = text position of the suffix at the
// bracket's first pivot row, midpoint(T[v] - 1, T[v] + size), and next =
// that suffix's bases k .. k+15 (its first k are v).  When none does, every
// read that starts with v has the same result, fixed by v alone: size =
// kPtabAnswer | l, with l < k the longest prefix of v that occurs, and
// [pos, next) the row interval of v[0..l).
struct alignas(16) PrefixEntry {
    uint32_t row;
    uint32_t size;
    int32_t pos;
    uint32_t next;
};
constexpr uint32_t kPtabAnswer = 0x80000000u;

// Device view of a resident index, passed to kernels by value.
struct DevIndex {
    const uint64_t *text;      // packed text, 2 bits per base, zero padded
    const int32_t *sa;         // suffix array, n entries
    const uint64_t *tile_key;  // first 32 bases of the pivot suffix of each tree node
    const int32_t *tile_sa;    // text position of each tree node's pivot suffix
    const RowRec *rows;        // one record per SA row
    const PrefixEntry *ptab;   // prefix table, 4^ptab_k + 1 entries (NULL when ptab_k == 0)
    int32_t n;
    int32_t ptab_k;            // bases indexed by the prefix table (0: no table)
};
// Longest prefix a table may index: an entry holds the 16 bases after its
// k, which must lie in the suffix's first 32 (4^16 + 1 entries: 64 GiB).
constexpr int kMaxPrefixBases = 16;

struct BucketTable {
    int count;     // 1..8
    int edge[8];   // bucket b: m <= edge[b]
    int keys;      // 1: pack writes sort keys and read ids (the reads get sorted)
};

// Scratch buffers of one batch (device pointers).
struct BatchBuffers {
    uint64_t *qw;        // nreads * kWMax packed words
    int2 *qlm;           // per read: length, ACGT-prefix length, word offset (see ReadLen)
    uint32_t *key[2];    // sort keys (ping-pong)
    uint32_t *val[2];    // read ids (ping-pong)
    uint32_t *hist;      // 256 * sort blocks
    uint32_t *digit_total;  // 256
    unsigned long long *stats;  // kStatWords words zeroed by pack: 10 counters of the instrumented
                                // search, then kLongFlag (set when a batch holds a long read)
};

// Once per device before any launch (and before any graph capture): lets
// the tuned kernel use the LDS of the deepest tile.
hipError_t prepare_kernels();

hipError_t launch_build_rows(const uint64_t *text, const int32_t *sa, int32_t n, RowRec *rows, hipStream_t s);

// Fills the 4^k + 1 entries of a prefix table (see PrefixEntry); ix.rows
// must hold the row records.
hipError_t launch_build_prefix_table(const DevIndex &ix, int k, PrefixEntry *tab, hipStream_t s);

hipError_t launch_build_tile(const uint64_t *text, const int32_t *sa, int32_t n, int levels,
                             uint64_t *key, int32_t *tsa, hipStream_t s);

// Read i is reads[offs[i] .. offs[i+1]), or reads[offs[i] .. ends[i]) when
// ends is not NULL.
hipError_t launch_pack(const uint8_t *reads, const int64_t *offs, const int64_t *ends, int64_t nreads,
                       const BatchBuffers &b, const BucketTable &bt, hipStream_t s);

// LSD radix sort of (key, val) pairs on bits [lo_bit, hi_bit), 8 bits per
// pass (stable, so lower bits keep their input order); returns in *which the
// ping-pong slot that holds the result.
hipError_t launch_sort(const BatchBuffers &b, int64_t nreads, int lo_bit, int hi_bit, int *which, hipStream_t s);

// count = true runs the instrumented variant that fills b.stats.
// group: 64-read chunks per block of the work split (see the kernel).
// use_table: start LB searches from the prefix table (when the index has one).
// offs not NULL: the kernel packs the reads itself from reads/offs (and
// ends, when not NULL: read i is reads[offs[i] .. ends[i]), else CSR) in
// input order (order must be NULL; no pack kernel runs, and b.stats must be
// cleared before, see launch_clear_stats); the dynamic LDS is then
// tuned_lds_bytes(tile_levels, block, true), which must not exceed
// inline_lds_limit().
// words: query words a read may hold (kShortWords or kWMax); with offs,
// longer reads are left to launch_search_long (long_min = 32 * words).
// defer (with offs, > 0): a read whose searches take more than this many
// probes of row records is set aside and searched again, without a limit,
// in a chunk of such reads (0: never; the counting variant never does).
hipError_t launch_search_tuned(const DevIndex &ix, int tile_levels, int use_table, int block, int grid,
                               int group, int defer, const BatchBuffers &b, const uint32_t *order, const uint8_t *reads,
                               const int64_t *offs, const int64_t *ends, int64_t nreads, int words, void *out,
                               bool count, hipStream_t s);

// Most dynamic LDS an inline-packing tuned kernel may take on the device
// that prepare_kernels last ran on (0 before).
size_t inline_lds_limit();

// Zero b.stats (the pack kernel does it otherwise).
hipError_t launch_clear_stats(const BatchBuffers &b, hipStream_t s);

hipError_t launch_search_plain(const DevIndex &ix, const BatchBuffers &b, int64_t nreads,
                               void *out, bool count, hipStream_t s);

// Reads of kShortMax + 1 .. SA_MAX_READ bases (pack marks them, the kernels
// above skip them): packed in LDS by one wave per 64 reads and searched from
// there.  order / sorted_key: the sort's result (NULL when unsorted); the
// long reads sort last, from the first row whose key bits
// [key_shift, key_shift + bits(key_mask)) reach long_field.
// Read i starts at reads[offs[i]] (offs holds the start array in gather mode).
// lengths_from_offs: take each read's length from offs (and ends, when not
// NULL) instead of the pack kernel's record (when the search kernel packed
// its reads); a read is then long when it has more than long_min bases.
hipError_t launch_search_long(const DevIndex &ix, const uint8_t *reads, const int64_t *offs, const BatchBuffers &b,
                              const uint32_t *order, const uint32_t *sorted_key, int key_shift, uint32_t key_mask,
                              uint32_t long_field, int use_table, bool lengths_from_offs, int long_min,
                              const int64_t *ends, int grid, int64_t nreads, void *out, bool count, hipStream_t s);

// Suffix-tree search, one read per lane, reads in input order, each packed
// into LDS by its wave (reads of up to SA_MAX_READ bases).
hipError_t launch_search_st(const uint64_t *text, const int32_t *sa, int32_t n, const StNode *nodes, int32_t root,
                            const uint8_t *reads, const int64_t *offs, int64_t nreads, void *out, int grid,
                            hipStream_t s);

// Sort key of a long read: the last bucket and an all-ones prefix, so that
// long reads sort after every other read.
__host__ __device__ inline uint32_t long_read_key(int nbuckets) { return ((uint32_t)(nbuckets - 1) << 24) | 0xFFFFFFu; }

// Dynamic LDS bytes of the tuned kernel for a tile depth.
__host__ __device__ inline size_t tile_lds_bytes(int levels) {
    const size_t nodes = ((size_t)1 << levels) - 1;
    return nodes * (sizeof(uint64_t) + sizeof(int32_t));
}

// Start of the per-wave packing areas after the tile (16-byte aligned).
__host__ __device__ inline size_t inline_area_offset(int levels) { return (tile_lds_bytes(levels) + 15) & ~(size_t)15; }

// 16-byte pieces of ASCII a wave's packing area holds in the search kernel
// whose reads hold up to `words` query words: 64 slots of 2 * words + 1
// pieces, each the most a read of up to 32 * words bases can touch; a span
// of 64 consecutive such reads fits too.
__host__ __device__ constexpr int inline_slot(int words) { return 2 * words + 1; }
__host__ __device__ constexpr int inline_vec(int words) { return 64 * inline_slot(words); }

// Entries of a wave's queue of set-aside reads (it is drained at 64, and a
// chunk adds at most 64).
constexpr int kDeferCap = 128;

// LDS bytes of such an area: a 4-byte code word and a 2-byte flag word per
// piece (with four pieces of slack), then the queue of set-aside reads (4
// bytes each), rounded up to 16 bytes.
__host__ __device__ constexpr int inline_codes_bytes(int words) { return (((inline_vec(words) + 4) * 6 + 8) + 15) & ~15; }
__host__ __device__ constexpr int inline_wave_bytes(int words) { return inline_codes_bytes(words) + 4 * kDeferCap; }

// Dynamic LDS of the tuned kernel: the tile, plus one packing area per wave
// when it packs its reads itself.
inline size_t tuned_lds_bytes(int levels, int block, bool inline_pack, int words = kWMax) {
    return inline_pack ? inline_area_offset(levels) + (size_t)(block / 64) * inline_wave_bytes(words)
                       : tile_lds_bytes(levels);
}

}  // namespace samatch
