// Device kernels for suffix-array read matching on gfx950 (wave64).
//
// Text layout: 2 bits per base, a=0 c=1 g=2 t=3, base i at bits
// [63-2(i%32)-1, 63-2(i%32)] of word i/32, so comparing two aligned 32-base
// words as unsigned integers compares them lexicographically, and the first
// differing base of two words is clz(x ^ y) / 2.
//
// Search semantics (Section IV, Algorithm 1): with open bounds L = -1 and
// R = n, the LB search moves R to the pivot when the query is not greater
// than the pivot suffix (a prefix match counts as not greater) and ends with
// LB = R; the RB search moves R only when the query is strictly smaller and
// ends with RB = L, i.e. RB + 1 = R.  A suffix that runs out while matching
// is smaller than the query.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "kernels.h"
#include "pivot.h"
#include "radix_sort.h"

namespace samatch {
namespace {

constexpr uint32_t kHitExact = 1u;
constexpr uint32_t kHitTooLong = 2u;
// Internal result of a search that ran out of its probe budget (never
// written out: the read is searched again without a limit).
constexpr uint32_t kHitDeferred = 0x40000000u;
constexpr int kNoBudget = 0x7FFFFFFF;

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int min_i(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int max_i(int a, int b) { return a > b ? a : b; }

// Probe accounting.  The timed kernels use NoCount (compiles to nothing);
// the instrumented variant counts global probes (one SA entry each), the
// 64-bit text words each probe compares, and probes answered in LDS.
struct NoCount {
    __device__ __forceinline__ void table_probe() {}
    __device__ __forceinline__ void global_probe() {}
    __device__ __forceinline__ void key_probe() {}
    __device__ __forceinline__ void tile_probe() {}
    __device__ __forceinline__ void text_words(uint32_t, uint32_t) {}
    __device__ __forceinline__ void rec_word() {}
    __device__ __forceinline__ void touch(const void *, int) {}
    __device__ __forceinline__ void index_touch(const void *, int) {}
};
// touch(p, bytes): one global access of this lane; the 64-byte segments
// that the wave's active lanes address together are added to `touched`
// (credited to the first active lane), the bytes-touched measure of a
// wave instruction.  index_touch: the same for a load from the index
// (prefix table, row records, suffix array, text), whose addresses are
// scattered; its segments and the load itself are also counted apart
// (`scattered`, `index_loads`), the requests a search makes.
struct Count {
    uint32_t global = 0, words = 0, tile = 0, keys = 0, table = 0, index_loads = 0;
    unsigned long long touched = 0, scattered = 0;
    __device__ __forceinline__ void index_touch(const void *p, int bytes) {
        const unsigned long long before = touched;
        touch(p, bytes);
        scattered += (touched - before) >> 6;
        ++index_loads;
    }
    __device__ __forceinline__ void touch(const void *p, int bytes) {
        const uint64_t a = (uint64_t)(uintptr_t)p;
        const uint64_t s0 = a >> 6;
        const uint64_t active = __ballot(1);
        uint64_t todo = active;
        uint32_t segs = 0;
        while (todo) {
            const int l = __ffsll((unsigned long long)todo) - 1;
            const uint64_t seg = __shfl(s0, l, 64);
            todo &= ~__ballot(s0 == seg);
            ++segs;
        }
        segs += (uint32_t)__popcll(__ballot(((a + (uint64_t)bytes - 1) >> 6) != s0));  // straddling lanes
        if ((threadIdx.x & 63) == __ffsll((unsigned long long)active) - 1) touched += 64ull * segs;
    }
    __device__ __forceinline__ void table_probe() { ++table; }
    __device__ __forceinline__ void global_probe() { ++global; }
    __device__ __forceinline__ void key_probe() { ++global; ++keys; }
    __device__ __forceinline__ void tile_probe() { ++tile; }
    __device__ __forceinline__ void rec_word() { ++keys; }
    // bases [first, end) of the text were compared
    __device__ __forceinline__ void text_words(uint32_t first, uint32_t end) {
        if (end > first) words += ((end - 1) >> 5) - (first >> 5) + 1;
    }
};

// 32 bases of the text starting at base b (bases past the end read as 0; the
// caller never trusts them).  Two neighbouring words joined by a funnel
// shift; the shift by (63 - sh) after a shift by 1 is a shift by 64 - sh
// that also works for sh == 0.
__device__ __forceinline__ uint64_t text_word(const uint64_t *__restrict__ text, uint32_t b) {
    const uint32_t wi = b >> 5;
    const uint32_t sh = (b & 31u) << 1;
    const uint64_t lo = text[wi];
    const uint64_t hi = text[wi + 1];
    return (lo << sh) | ((hi >> 1) >> (63u - sh));
}

template <class Cnt>
__device__ __forceinline__ uint64_t text_word(const uint64_t *__restrict__ text, uint32_t b, Cnt &cnt) {
    cnt.index_touch(text + (b >> 5), 8);
    cnt.index_touch(text + (b >> 5) + 1, 8);
    return text_word(text, b);
}

// Two consecutive 64-bit words with one 16-byte load from an address that
// is only 8-byte aligned (global loads of several dwords need dword
// alignment on this device).
typedef uint64_t u64x2_a8 __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ u64x2_a8 load_u64x2(const uint64_t *p) { return *reinterpret_cast<const u64x2_a8 *>(p); }

// 16 bytes read once: a non-temporal load, so that the caches keep lines
// that are used again (the text) rather than prefix-table entries, row
// records and ASCII reads, which a search touches once (on MI355X this took
// the 250 Mbp / 64M-read batch from 6.47 to 5.93 ms, results unchanged).
__device__ __forceinline__ uint4 load_stream16(const void *p) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// A 16-byte result, written once and not read again by the kernels.
__device__ __forceinline__ void store_stream16(int4 *p, int4 r) {
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    const i32x4 v = {r.x, r.y, r.z, r.w};
    __builtin_nontemporal_store(v, reinterpret_cast<i32x4 *>(p));
}

// Two consecutive 32-bit words with one 8-byte load, 4-byte aligned.
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ u32x2_a4 load_u32x2(const uint32_t *p) { return *reinterpret_cast<const u32x2_a4 *>(p); }

// The words of one suffix taken in order: word k (bases p + 32k ..
// p + 32k + 31) joins text words wi + k and wi + k + 1 (wi = p / 32) by a
// funnel shift.  Text words come two per 16-byte load and each is loaded
// once per comparison, so k consecutive suffix words cost 1 + k/2 loads
// (the text carries zero padding words after its end for the loads past it).
struct TextRun {
    const uint64_t *base;  // text + p / 32
    uint32_t sh;           // 2 * (p % 32)
    uint64_t a, b, c;      // text words wi + k, wi + k + 1 and, when `spare`, wi + k + 2
    bool started, spare;

    __device__ __forceinline__ TextRun(const uint64_t *__restrict__ text, uint32_t p)
        : base(text + (p >> 5)), sh((p & 31u) << 1), a(0), b(0), c(0), started(false), spare(false) {}

    // word k of the suffix; successive calls take successive k
    template <class Cnt>
    __device__ __forceinline__ uint64_t word(int k, Cnt &cnt) {
        if (!started) {
            const u64x2_a8 v = load_u64x2(base + k);
            cnt.index_touch(base + k, 16);
            a = v.x;
            b = v.y;
            started = true;
        } else {
            a = b;
            if (spare) {
                b = c;
                spare = false;
            } else {
                const u64x2_a8 v = load_u64x2(base + k + 1);
                cnt.index_touch(base + k + 1, 16);
                b = v.x;
                c = v.y;
                spare = true;
            }
        }
        return (a << sh) | ((b >> 1) >> (63u - sh));
    }
};

// Compare the query P[0..plen) with the suffix at text position p, skipping
// the first 32*k0 bases (known to match).  Returns -1 when P sorts before
// the suffix, 0 when P[0..plen) is a prefix of it, +1 when P sorts after it
// (including when the suffix ends first); lcp gets the exact common-prefix
// length, capped at min(plen, n - p).  The word loop is unrolled over all W
// words and predicated, so the query stays in registers (a run-time index
// into q would move it to scratch memory).
template <int W, class Q, class Cnt>
__device__ __forceinline__ int compare_from(const uint64_t *__restrict__ text, int32_t n,
                                            const Q &q, int plen, int32_t p, int k0,
                                            int &lcp, Cnt &cnt) {
    const int lim = min_i(plen, n - p);
    int res = lim;
    int sign = (lim == plen) ? 0 : 1;
    bool done = false;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        if (!done && k >= k0 && (k << 5) < lim) {
            const uint64_t t = text_word(text, (uint32_t)p + ((uint32_t)k << 5), cnt);
            const uint64_t x = q[k] ^ t;
            if (x) {
                const int mm = (k << 5) + (int)(__clzll((long long)x) >> 1);
                if (mm < lim) {
                    res = mm;
                    sign = q[k] > t ? 1 : -1;
                }
                done = true;
            }
        }
    }
    lcp = res;
    cnt.text_words((uint32_t)p + ((uint32_t)k0 << 5), (uint32_t)p + (uint32_t)min_i(lim, res + 1));
    return sign;
}

// First 16 bytes of a row record: position, length, word 0 (one load).
struct RowHead {
    int32_t pos;
    int32_t len;
    uint64_t key0;
};

__device__ __forceinline__ RowHead row_head(const RowRec *__restrict__ rows, int r) {
    const uint4 v = load_stream16(rows + r);
    RowHead h;
    h.pos = (int32_t)v.x;
    h.len = (int32_t)v.y;
    h.key0 = ((uint64_t)v.w << 32) | v.z;
    return h;
}

// Probe of one suffix (text position p) whose first key_bases bases (key0,
// the rest of its first word zero) are in hand, with h bases known to
// match: like compare_from, but word 0 comes from key0 and words 1 ..
// kRecWords-1 from the row record (rec; NULL for a node of the LDS tile or
// a prefix-table pivot), loaded only while the words before them tie; later
// words come from the text, and so does word 0 when key0 holds fewer than
// 32 bases, ties on them, and the comparison reaches past them.
template <int W, class Q, class Cnt>
__device__ __forceinline__ int compare_row(const DevIndex &ix, const Q &q, int plen,
                                           const RowRec *__restrict__ rec, int32_t p, uint64_t key0, int h,
                                           int &lcp, Cnt &cnt, int key_bases = 32) {
    const int lim = min_i(plen, ix.n - p);
    const int k0 = h >> 5;
    int res = lim;
    int sign = (lim == plen) ? 0 : 1;
    bool done = false;
    uint32_t text_first = 0, text_end = 0;
    TextRun run(ix.text, (uint32_t)p);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        if (!done && k >= k0 && (k << 5) < lim) {
            uint64_t t;
            if (k == 0 && (key_bases >= 32 || lim <= key_bases ||
                           ((q[0] ^ key0) & (~0ull << (64 - 2 * key_bases))) != 0)) {
                t = key0;
            } else if (k > 0 && rec != nullptr && k < kRecWords) {
                t = reinterpret_cast<const uint64_t *>(rec)[1 + k];  // word k of the record
                cnt.rec_word();
                cnt.index_touch(reinterpret_cast<const uint64_t *>(rec) + 1 + k, 8);
            } else {
                t = run.word(k, cnt);
                if (text_end == 0) text_first = (uint32_t)p + ((uint32_t)k << 5);
                text_end = (uint32_t)p + (uint32_t)min_i(lim, (k << 5) + 32);
            }
            const uint64_t x = q[k] ^ t;
            if (x) {
                const int mm = (k << 5) + (int)(__clzll((long long)x) >> 1);
                if (mm < lim) {
                    res = mm;
                    sign = q[k] > t ? 1 : -1;
                }
                done = true;
                if (text_end) text_end = (uint32_t)p + (uint32_t)min_i(lim, mm + 1);
            }
        }
    }
    lcp = res;
    cnt.text_words(text_first, text_end);
    return sign;
}

// Binary search over rows (L, R] with known common-prefix lengths at the
// bounds (lcpL, lcpR, 0 for the open ends).  Every row strictly between
// them shares min(lcpL, lcpR) leading bases with the query, so each probe
// starts comparing at that word.  UPPER = false: first row whose suffix is
// not below P[0..plen) (LB); UPPER = true: first row strictly above every
// extension of P[0..plen) (RB + 1).
//
// left: probes the read may still take; a search that would take one more
// when none is left stops and returns -1 (every result is >= 0).
template <int W, bool UPPER, class Q, class Cnt>
__device__ __forceinline__ int bounded_search(const DevIndex &ix, const Q &q, int plen, int L, int R,
                              int lcpL, int lcpR, int &left, Cnt &cnt) {
    while (R > L + 1) {
        if (--left < 0) return -1;
        const int piv = midpoint(L, R);
        const RowHead row = row_head(ix.rows, piv);
        cnt.index_touch(ix.rows + piv, 16);
        int lcp;
        cnt.key_probe();
        const int sign = compare_row<W>(ix, q, plen, ix.rows + piv, row.pos, row.key0, min_i(lcpL, lcpR), lcp, cnt);
        const bool go_left = UPPER ? (sign < 0) : (sign <= 0);
        if (go_left) { R = piv; lcpR = lcp; }
        else { L = piv; lcpL = lcp; }
    }
    return R;
}

// State at the end of the LB search: adjacent rows L, R = L + 1 around the
// insertion point of P[0..plen), their common-prefix lengths with P, and for
// each side the last bound before its common-prefix length reached its final
// value (Llt / Rlt) with that bound's length.  Common-prefix lengths only
// grow towards the insertion point, so every row at or beyond Llt (Rlt) on
// that side shares fewer than lcpL (lcpR) bases with P.
struct LbState {
    int L, R, lcpL, lcpR, Llt, lcpLlt, Rlt, lcpRlt;
};

__device__ __forceinline__ void lb_update(LbState &st, int sign, int piv, int lcp) {
    if (sign <= 0) {
        if (lcp > st.lcpR) { st.Rlt = st.R; st.lcpRlt = st.lcpR; }
        st.R = piv; st.lcpR = lcp;
    } else {
        if (lcp > st.lcpL) { st.Llt = st.L; st.lcpLlt = st.lcpL; }
        st.L = piv; st.lcpL = lcp;
    }
}

// Full LB search of P[0..plen).  The first `levels` probes of every search
// from (-1, n) visit nodes of one fixed implicit binary tree; their pivot
// suffixes (first 32 bases and text position) sit in LDS.  A probe that
// ties on all 32 staged bases continues in global memory at word 1.
// Returns false when the global probes ran out of `left`.
template <int W, class Q, class Cnt>
__device__ __forceinline__ bool lb_search(const DevIndex &ix, const uint64_t *s_key, const int32_t *s_sa, int levels,
                          const Q &q, int plen, LbState &st, int &left, Cnt &cnt) {
    st.L = -1; st.R = ix.n; st.lcpL = 0; st.lcpR = 0;
    st.Llt = -1; st.lcpLlt = 0; st.Rlt = ix.n; st.lcpRlt = 0;
    int node = 0;
    for (int d = 0; d < levels && st.R > st.L + 1; ++d) {
        const uint64_t key = s_key[node];
        const int32_t p = s_sa[node];
        int lcp;
        cnt.tile_probe();
        const int sign = compare_row<W>(ix, q, plen, nullptr, p, key, min_i(st.lcpL, st.lcpR), lcp, cnt);
        const int piv = midpoint(st.L, st.R);
        lb_update(st, sign, piv, lcp);
        node = 2 * node + (sign <= 0 ? 1 : 2);
    }
    while (st.R > st.L + 1) {
        if (--left < 0) return false;
        const int piv = midpoint(st.L, st.R);
        const RowHead row = row_head(ix.rows, piv);
        cnt.index_touch(ix.rows + piv, 16);
        int lcp;
        cnt.key_probe();
        const int sign =
            compare_row<W>(ix, q, plen, ix.rows + piv, row.pos, row.key0, min_i(st.lcpL, st.lcpR), lcp, cnt);
        lb_update(st, sign, piv, lcp);
    }
    return true;
}

// ---- prefix table
// The table T[v] (v a k-base string) is the first SA row whose suffix is not
// below v.  For a query P with at least k leading ACGT bases and first k
// bases v, every row before T[v] is below P and every row of a suffix that
// does not start with v after them is above it, so the LB search of P runs
// inside the bracket of rows that start with v (see PrefixEntry).

// LB search of P[0..plen) inside the table bracket of its first k bases v.
// Returns false when no suffix starts with v: the entry then holds the
// read's result (ans); also when the record probes ran out of `left` (ans
// is then flagged kHitDeferred).  Otherwise st holds the LB search's final
// state.
// Rows inside the bracket share k bases with P, so when the search moves a
// bound inside, the other bound's common-prefix length (below k) never
// decides anything and starts as 0.  The first probe takes its pivot
// suffix's position and first k + 16 bases from the entry, with no load of
// its own.
template <int W, class Q, class Cnt>
__device__ __forceinline__ bool lb_search_table(const DevIndex &ix, const Q &q, int plen, LbState &st,
                                                int4 &ans, int &left, Cnt &cnt) {
    const int K = ix.ptab_k;
    const uint32_t v = (uint32_t)(q[0] >> (64 - 2 * K));
    const uint4 e4 = load_stream16(ix.ptab + v);
    const PrefixEntry ent{e4.x, e4.y, (int32_t)e4.z, e4.w};
    cnt.index_touch(ix.ptab + v, 16);
    cnt.table_probe();
    if (ent.size & kPtabAnswer) {
        ans = make_int4(ent.pos, (int)ent.next, (int)(ent.size & ~kPtabAnswer), 0);
        return false;
    }
    const int lo_k = (int)ent.row;
    const int hi_k = lo_k + (int)ent.size;
    st.L = lo_k - 1; st.R = hi_k; st.lcpL = 0; st.lcpR = 0;
    st.Llt = -1; st.lcpLlt = 0; st.Rlt = ix.n; st.lcpRlt = 0;
    {
        const int piv = midpoint(st.L, st.R);
        const uint64_t key = (q[0] & ~(~0ull >> (2 * K))) | ((uint64_t)ent.next << (32 - 2 * K));
        int lcp;
        cnt.global_probe();  // its position and bases came with the entry, not from a record
        const int sign = compare_row<W>(ix, q, plen, nullptr, ent.pos, key, 0, lcp, cnt, K + 16);
        lb_update(st, sign, piv, lcp);
    }
    while (st.R > st.L + 1) {
        if (--left < 0) {
            ans = make_int4(0, 0, 0, (int)kHitDeferred);
            return false;
        }
        const int piv = midpoint(st.L, st.R);
        const RowHead row = row_head(ix.rows, piv);
        cnt.index_touch(ix.rows + piv, 16);
        int lcp;
        cnt.key_probe();
        const int sign =
            compare_row<W>(ix, q, plen, ix.rows + piv, row.pos, row.key0, min_i(st.lcpL, st.lcpR), lcp, cnt);
        lb_update(st, sign, piv, lcp);
    }
    return true;
}

// One read: LB search of its ACGT prefix; exact reads finish with an RB
// search confined to (LB, Rlt]; other reads take the longest matched prefix
// l = max(lcpL, lcpR) from the two rows around the insertion point and find
// the interval of P[0..l) inside the bounds the LB search already bracketed.
// The empty prefix (an empty read, or one that starts with a non-base)
// matches every suffix.  `budget` bounds the probes of row records and of
// the global part of the tree; a read that needs more gets a result
// flagged kHitDeferred instead (kNoBudget: no bound).
template <int W, class Q, class Cnt>
__device__ __forceinline__ int4 match_read(const DevIndex &ix, const uint64_t *s_key, const int32_t *s_sa, int levels,
                           bool use_table, const Q &q, int m, int mv, int budget, Cnt &cnt) {
    if (mv == 0) return make_int4(0, ix.n, 0, m == 0 ? (int)kHitExact : 0);
    const int4 deferred = make_int4(0, 0, 0, (int)kHitDeferred);
    int left = budget;
    LbState st;
    if (use_table && ix.ptab_k > 0 && mv >= ix.ptab_k) {
        int4 ans;
        if (!lb_search_table<W>(ix, q, mv, st, ans, left, cnt)) return ans;
    } else {
        if (!lb_search<W>(ix, s_key, s_sa, levels, q, mv, st, left, cnt)) return deferred;
    }
    if (mv == m && st.lcpR == m) {
        const int hi = bounded_search<W, true>(ix, q, m, st.R, st.Rlt, m, st.lcpRlt, left, cnt);
        if (hi < 0) return deferred;
        return make_int4(st.R, hi, m, (int)kHitExact);
    }
    // (after a search inside a table bracket l >= k: one of the final
    // bounds is a probed row of the bracket, which shares the k bases)
    const int l = max_i(st.lcpL, st.lcpR);
    if (l == 0) return make_int4(0, ix.n, 0, 0);
    const int lo =
        (st.lcpL == l) ? bounded_search<W, false>(ix, q, l, st.Llt, st.L, st.lcpLlt, l, left, cnt) : st.R;
    const int hi = (st.lcpR == l) ? bounded_search<W, true>(ix, q, l, st.R, st.Rlt, l, st.lcpRlt, left, cnt) : st.R;
    if ((lo | hi) < 0) return deferred;
    return make_int4(lo, hi, l, 0);
}

template <int W>
__device__ __forceinline__ void load_query(const uint64_t *__restrict__ src, int nw, uint64_t (&q)[W]) {
#pragma unroll
    for (int k = 0; k < W; ++k) q[k] = k < nw ? src[k] : 0ull;
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// ------------------------------------------------------------------ row keys

// One record per SA row: the suffix's text position and length and its
// first 32 * kRecWords bases (zero past the text end), so that a probe
// fetches position and bases from one line.
__global__ void build_rows_kernel(const uint64_t *__restrict__ text, const int32_t *__restrict__ sa, int32_t n,
                                  RowRec *__restrict__ rows) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t p = sa[r];
    RowRec rec;
    rec.pos = p;
    rec.len = n - p;
#pragma unroll
    for (int k = 0; k < kRecWords; ++k) rec.key[k] = text_word(text, (uint32_t)p + ((uint32_t)k << 5));
    rows[r] = rec;
}

// ------------------------------------------------------------------ prefix table

// Order key of a row for a k-base table: 2 * (first k bases, zero-padded)
// + 1 for a suffix of at least k bases, without the +1 for a shorter one (it
// sorts before every k-base string it is a proper prefix of).  It does not
// decrease along the suffix array.
__device__ __forceinline__ uint64_t row_order_key(const DevIndex &ix, int k, int r) {
    const RowHead row = row_head(ix.rows, r);
    return 2 * (row.key0 >> (64 - 2 * k)) + (row.len >= k ? 1u : 0u);
}

// T[v] = first row whose order key reaches 2v + 1 (binary search per entry).
__global__ void build_prefix_table_kernel(DevIndex ix, int k, int64_t first, int64_t end,
                                          PrefixEntry *__restrict__ tab) {
    const int64_t v = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= end) return;
    const uint64_t target = 2 * (uint64_t)v + 1;
    int lo = 0, hi = ix.n;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (row_order_key(ix, k, mid) >= target) hi = mid;
        else lo = mid + 1;
    }
    tab[v].row = (uint32_t)lo;
}

// Second pass (after every T[v] is written): each entry's bracket size
// and first pivot suffix, or, for a string v no suffix starts with, the
// result of a search for v itself from the root (any read starting with v
// has it: its longest matched prefix is shorter than v).
__global__ void fill_prefix_entries_kernel(DevIndex ix, int k, int64_t first, int64_t end, int64_t entries,
                                           PrefixEntry *__restrict__ tab) {
    const int64_t v = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= end) return;
    if (v == entries - 1) {  // T[4^k] = n closes the last bracket; it is never looked up
        tab[v].size = 0;
        tab[v].pos = 0;
        tab[v].next = 0;
        return;
    }
    const int lo = (int)tab[v].row;
    // rows [lo, T[v+1]) have order key 2v + 1 (suffixes that start with v),
    // then 2v + 2 (suffixes shorter than k, at most k - 1, that are proper
    // prefixes of v + 1 padded with a's); the bracket ends before the latter
    int hi = (int)tab[v + 1].row;
    while (hi > lo && row_head(ix.rows, hi - 1).len < k) --hi;
    if (hi > lo) {
        const RowHead h = row_head(ix.rows, midpoint(lo - 1, hi));
        tab[v].size = (uint32_t)(hi - lo);
        tab[v].pos = h.pos;
        tab[v].next = (uint32_t)(h.key0 >> (32 - 2 * k));
    } else {
        const uint64_t q[1] = {(uint64_t)v << (64 - 2 * k)};
        NoCount none;
        const int4 r = match_read<1>(ix, nullptr, nullptr, 0, false, q, k, k, kNoBudget, none);
        tab[v].size = kPtabAnswer | (uint32_t)r.z;
        tab[v].pos = r.x;
        tab[v].next = (uint32_t)r.y;
    }
}

// ------------------------------------------------------------------ tile

__global__ void build_tile_kernel(const uint64_t *__restrict__ text, const int32_t *__restrict__ sa,
                                  int32_t n, int levels, uint64_t *key, int32_t *tsa) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nodes = (1 << levels) - 1;
    if (j >= nodes) return;
    // node j is reached by the bits of j+1 after its leading one: 0 = the
    // query was not above the pivot (R = pivot), 1 = it was (L = pivot)
    const int depth = 31 - __clz(j + 1);
    const int path = (j + 1) - (1 << depth);
    int L = -1, R = n;
    bool live = true;
    for (int i = depth - 1; i >= 0; --i) {
        if (R <= L + 1) { live = false; break; }
        const int piv = midpoint(L, R);
        if ((path >> i) & 1) L = piv; else R = piv;
    }
    if (!live || R <= L + 1) {  // no search reaches this node
        key[j] = 0;
        tsa[j] = 0;
        return;
    }
    const int32_t p = sa[midpoint(L, R)];
    key[j] = text_word(text, (uint32_t)p);
    tsa[j] = p;
}

// ------------------------------------------------------------------ per-read record

// The pack kernel's 8-byte record of a read: its length m (-1: not
// searched), then one word holding the length of its ACGT prefix plus one
// (0: a long read, for the long-read kernel) in the low 16 bits and the
// offset of its packed words in its workgroup's region of qw in the high 16.
struct ReadLen {
    int m, mv, wo;
};

__device__ __forceinline__ int2 encode_len(int m, int mv, int wo) {
    return make_int2(m, (int)(((uint32_t)wo << 16) | (uint32_t)(mv + 1)));
}

__device__ __forceinline__ ReadLen decode_len(int2 v) {
    ReadLen r;
    r.m = v.x;
    r.mv = (int)((uint32_t)v.y & 0xFFFFu) - 1;
    r.wo = (int)((uint32_t)v.y >> 16);
    return r;
}

// ------------------------------------------------------------------ pack

// Per-byte flags (0x80 in each byte) of the four bytes of x that are not
// one of a, c, g, t after forcing lower case: a byte is nonzero after
// xor-ing with a letter unless it is that letter.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t v) {
    return (((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
}
__device__ __forceinline__ uint32_t invalid_bytes(uint32_t dw) {
    const uint32_t lc = dw | 0x20202020u;
    return nonzero_bytes(lc ^ 0x61616161u) & nonzero_bytes(lc ^ 0x63636363u) & nonzero_bytes(lc ^ 0x67676767u) &
           nonzero_bytes(lc ^ 0x74747474u);
}

// Four bases (little-endian bytes of dw, the first base in the low byte) to
// 8 bits, first base in the top two bits; `keep` masks the bytes that
// belong to the read.  a->0 c->1 g->2 t->3 for either case, anything else
// becomes 0 and is reported in *bad (0x80 per byte).
__device__ __forceinline__ uint32_t pack4(uint32_t dw, uint32_t keep, uint32_t &bad) {
    bad = invalid_bytes(dw) & keep;
    const uint32_t zero = (bad >> 7) * 0xFFu;  // 0xFF in each flagged byte
    const uint32_t codes = ((dw >> 1) ^ (dw >> 2)) & 0x03030303u & keep & ~zero;
    return ((codes & 3u) << 6) | ((codes >> 4) & 0x30u) | ((codes >> 14) & 0x0Cu) | ((codes >> 24) & 3u);
}

// pack4 with one byte permute instead of four letter tests: the code of a
// byte is ((c >> 1) ^ (c >> 2)) & 3 (a/A -> 0, c/C -> 1, g/G -> 2, t/T ->
// 3), and a byte is a base exactly when, with bit 5 cleared, it equals
// "ACGT"[code] (looked up with v_perm).  Same results as pack4.
__device__ __forceinline__ uint32_t pack4_fast(uint32_t dw, uint32_t keep, uint32_t &bad) {
    uint32_t codes = ((dw >> 1) ^ (dw >> 2)) & 0x03030303u;
    const uint32_t expect = __builtin_amdgcn_perm(0u, 0x54474341u, codes);  // "ACGT"[code] per byte
    bad = nonzero_bytes((dw & 0xDFDFDFDFu) ^ expect) & keep;
    codes &= keep & ~((bad >> 7) * 0xFFu);
    return ((codes & 3u) << 6) | ((codes >> 4) & 0x30u) | ((codes >> 14) & 0x0Cu) | (codes >> 24);
}

// Pack one read from global memory, fetching aligned dwords; an aligned
// dword that holds at least one byte of the read never crosses a page, so
// no fetch can fault.
__device__ __forceinline__ void pack_from_global(const uint8_t *__restrict__ reads, int64_t a, int m,
                                                 uint64_t (&dst)[kWMax + 1], int &mv, uint64_t &w0) {
    mv = m;
    uint64_t word = 0;
    int k = 0;
#pragma unroll
    for (int t = 0; t < kWMax; ++t) dst[t] = 0;
    const uintptr_t start = (uintptr_t)(reads + a);
    const uintptr_t stop = start + (uintptr_t)m;
    for (uintptr_t addr = start & ~(uintptr_t)3; addr < stop; addr += 4) {
        const uint32_t dw = *reinterpret_cast<const uint32_t *>(addr);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uintptr_t at = addr + t;
            if (at < start || at >= stop) continue;
            const int idx = (int)(at - start);
            const uint32_t c = (dw >> (8 * t)) & 0xFFu;
            const uint32_t lc = c | 0x20u;
            const bool ok = lc == 'a' || lc == 'c' || lc == 'g' || lc == 't';
            const uint32_t code = ((c >> 1) ^ (c >> 2)) & 3u;
            if (!ok && idx < mv) mv = idx;
            word |= (uint64_t)(ok ? code : 0u) << (62 - 2 * (idx & 31));
            if ((idx & 31) == 31) {
#pragma unroll
                for (int t = 0; t < kWMax; ++t) dst[t] = (t == k) ? word : dst[t];
                ++k;
                word = 0;
            }
        }
    }
    if ((m & 31) != 0 || m == 0) {
#pragma unroll
        for (int t = 0; t < kWMax; ++t) dst[t] = (t == k) ? word : dst[t];
    }
    w0 = dst[0];
}

// Packing: each workgroup converts the bytes of its 256 consecutive reads
// with coalesced, aligned 16-byte loads into a stream of 2-bit codes in
// LDS (16 bases per word, 12 KB for 48 KB of ASCII) and a flag per byte
// that is not a base; each thread then takes its read's words out of the
// stream with funnel shifts and finds its first non-base from the flags.
// Reads whose bytes are not in the converted span (offsets that are not
// contiguous, or a span larger than 48 KB) take the global path.  The
// packed words go back through LDS so that the workgroup's run of words is
// written with coalesced 16-byte stores.  Read i is reads[offs[i] ..
// offs[i+1]), or reads[offs[i] .. ends[i]) when an end array is given
// (reads scattered over a larger buffer; always the global path).
constexpr int kPackBlock = 256;
constexpr int kPackChunks = 3072;  // 16-byte chunks of ASCII a workgroup converts through LDS (48 KB)
static_assert((kPackChunks + 4) * 6 <= (kPackBlock * kWMax + 8) * 8, "code stream and flags fit the buffer");

// The 0x80 flags of pack4_fast's four bytes as four bits, byte 0 lowest.
__device__ __forceinline__ uint32_t bad_nibble(uint32_t bad) {
    return ((bad >> 7) & 1u) | ((bad >> 14) & 2u) | ((bad >> 21) & 4u) | ((bad >> 28) & 8u);
}

// 16 bytes of ASCII (four little-endian dwords, the first byte lowest) to
// 16 two-bit codes, the first base in the top bits of codes[c], and a flag
// bit per byte that is not a base in badm[c] (bit i for byte i), with the
// code of such a byte 0.  When every byte is a base (either case) -- a
// byte-wise compare with "ACGT"[code] -- the codes of each dword are
// gathered into a byte with two shift-ors and the sixteen pairs are put in
// order by one bit reversal and a swap within each pair; otherwise the
// flags are worked out byte by byte.  Returns whether a byte was not a base.
__device__ __forceinline__ uint32_t gather4(uint32_t cd) {
    const uint32_t x = cd | (cd >> 6);  // bits 0-3: codes of bytes 0, 1; bits 16-19: bytes 2, 3
    return (x | (x >> 12)) & 0xFFu;     // byte i's code at bits 2i, 2i+1
}

__device__ __forceinline__ bool convert_piece(const uint4 &v, uint32_t *codes, uint16_t *badm, int c) {
    const uint32_t k0 = ((v.x >> 1) ^ (v.x >> 2)) & 0x03030303u, k1 = ((v.y >> 1) ^ (v.y >> 2)) & 0x03030303u;
    const uint32_t k2 = ((v.z >> 1) ^ (v.z >> 2)) & 0x03030303u, k3 = ((v.w >> 1) ^ (v.w >> 2)) & 0x03030303u;
    const uint32_t d0 = (v.x & 0xDFDFDFDFu) ^ __builtin_amdgcn_perm(0u, 0x54474341u, k0);
    const uint32_t d1 = (v.y & 0xDFDFDFDFu) ^ __builtin_amdgcn_perm(0u, 0x54474341u, k1);
    const uint32_t d2 = (v.z & 0xDFDFDFDFu) ^ __builtin_amdgcn_perm(0u, 0x54474341u, k2);
    const uint32_t d3 = (v.w & 0xDFDFDFDFu) ^ __builtin_amdgcn_perm(0u, 0x54474341u, k3);
    if ((d0 | d1 | d2 | d3) == 0) {
        uint32_t w = gather4(k0) | (gather4(k1) << 8) | (gather4(k2) << 16) | (gather4(k3) << 24);
        w = __builtin_bitreverse32(w);                          // base i's pair at bits 30-2i, 31-2i, swapped
        w = ((w >> 1) & 0x55555555u) | ((w & 0x55555555u) << 1);  // base 0 in the top two bits
        codes[c] = w;
        badm[c] = 0;
        return false;
    }
    uint32_t bad, code, bits;
    code = pack4_fast(v.x, 0xFFFFFFFFu, bad);
    bits = bad_nibble(bad);
    code = (code << 8) | pack4_fast(v.y, 0xFFFFFFFFu, bad);
    bits |= bad_nibble(bad) << 4;
    code = (code << 8) | pack4_fast(v.z, 0xFFFFFFFFu, bad);
    bits |= bad_nibble(bad) << 8;
    code = (code << 8) | pack4_fast(v.w, 0xFFFFFFFFu, bad);
    bits |= bad_nibble(bad) << 12;
    codes[c] = code;
    badm[c] = (uint16_t)bits;
    return true;
}

__global__ __launch_bounds__(kPackBlock) void pack_kernel(const uint8_t *__restrict__ reads,
                                                          const int64_t *__restrict__ offs,
                                                          const int64_t *__restrict__ ends, int64_t nreads,
                                                          BatchBuffers b, BucketTable bt) {
    // the span's bases as a code stream (16 per word, first in the top bits)
    // and a flag per byte that is not a base; later the packed words
    __shared__ uint64_t lds_buf[kPackBlock * kWMax + 8];
    uint32_t *codes = reinterpret_cast<uint32_t *>(lds_buf);
    uint16_t *badm = reinterpret_cast<uint16_t *>(codes + kPackChunks + 4);
    const int64_t r0 = (int64_t)blockIdx.x * kPackBlock;
    const int64_t r1 = r0 + kPackBlock < nreads ? r0 + kPackBlock : nreads;
    const int64_t i = r0 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < kStatWords) b.stats[threadIdx.x] = 0ull;
    // with an end array, the workgroup's reads still form one span when each
    // ends where the next starts (the usual case for a request's reads)
    bool contiguous = true;
    if (ends) contiguous = __syncthreads_and(i + 1 >= r1 || ends[i] == offs[i + 1]) != 0;
    const int64_t span0 = offs[r0];
    const int64_t span1 = ends ? (contiguous ? ends[r1 - 1] : span0) : offs[r1];
    const uintptr_t A0 = (uintptr_t)(reads + span0) & ~(uintptr_t)15;
    const uintptr_t A1 = ((uintptr_t)(reads + span1) + 15) & ~(uintptr_t)15;
    const bool staged = contiguous && span1 > span0 && A1 - A0 <= (uintptr_t)kPackChunks * 16u;
    if (staged) {
        // every aligned 16-byte chunk here holds a byte of [span0, span1):
        // coalesced loads, converted on the way into LDS
        const int nvec = (int)((A1 - A0) >> 4);
        const uint4 *src = reinterpret_cast<const uint4 *>(A0);
        for (int c = threadIdx.x; c < nvec; c += kPackBlock) convert_piece(src[c], codes, badm, c);
    }
    __syncthreads();
    uint64_t w[kWMax];
#pragma unroll
    for (int t = 0; t < kWMax; ++t) w[t] = 0;
    int m = -1, mv = 0;
    if (i < nreads) {
        const int64_t a = offs[i], e = ends ? ends[i] : offs[i + 1];
        const int64_t m64 = e - a;
        if (m64 > kShortMax && m64 <= SA_MAX_READ) {
            m = (int)m64;  // long read: packed and searched by the long-read kernel
            mv = -1;
        } else if (m64 >= 0 && m64 <= kShortMax) {
            m = (int)m64;
            mv = m;
            if (staged && a >= span0 && e <= span1) {
                // word k: bases s + 32k .. s + 32k + 31 of the code stream
                const uint32_t st0 = (uint32_t)((uintptr_t)(reads + a) - A0);
#pragma unroll
                for (int k = 0; k < kWMax; ++k) {
                    if (32 * k < m) {
                        const uint32_t bpos = st0 + 32u * (uint32_t)k, q = bpos >> 4, r = bpos & 15u;
                        const uint64_t hi = ((uint64_t)codes[q] << 32) | codes[q + 1];
                        uint64_t x = r ? (hi << (2 * r)) | (codes[q + 2] >> (32 - 2 * r)) : hi;
                        const int rem = m - 32 * k;
                        if (rem < 32) x &= ~0ull << (64 - 2 * rem);
                        w[k] = x;
                    }
                }
                if (m > 0) {  // first byte that is not a base
                    const uint32_t q0 = st0 >> 4, q1 = (st0 + (uint32_t)m - 1) >> 4;
                    for (uint32_t q = q0; q <= q1; ++q) {
                        uint32_t bits = badm[q];
                        if (q == q0) bits &= 0xFFFFu << (st0 & 15u);
                        if (q == q1) bits &= (2u << ((st0 + (uint32_t)m - 1) & 15u)) - 1u;
                        if (bits) {
                            mv = (int)(q * 16u + (uint32_t)__builtin_ctz(bits) - st0);
                            break;
                        }
                    }
                }
            } else {
                uint64_t g[kWMax + 1];
                pack_from_global(reads, a, m, g, mv, g[kWMax]);
#pragma unroll
                for (int t = 0; t < kWMax; ++t) w[t] = (32 * t < m || t == 0) ? g[t] : 0;
            }
        }
    }
    // the words of the workgroup's searched reads, back to back from the
    // start of its region of qw (256 * kWMax words): read i's run starts at
    // word `wo` of the region
    __shared__ uint32_t scan_tmp[kPackBlock / 64];
    const int nw = (i < nreads && m >= 0 && mv >= 0) ? (m > 0 ? (m + 31) >> 5 : 1) : 0;
    uint32_t wo;
    const uint32_t run_words = block_exclusive_scan((uint32_t)nw, wo, scan_tmp);
    __syncthreads();  // the code stream is no longer needed
    uint64_t *slots = lds_buf;
    if (i < nreads) {
#pragma unroll
        for (int t = 0; t < kWMax; ++t)
            if (t < nw) slots[wo + t] = w[t];
        b.qlm[i] = encode_len(m, mv, (int)wo);
        if (bt.keys) {  // sort keys, only when the reads are sorted
            if (m >= 0 && mv < 0) {
                b.key[0][i] = long_read_key(bt.count);
            } else if (m >= 0) {
                int bucket = bt.count - 1;
                for (int j = 0; j < bt.count; ++j)
                    if (m <= bt.edge[j]) { bucket = j; break; }
                b.key[0][i] = ((uint32_t)bucket << 24) | (uint32_t)(w[0] >> 40);
            } else {
                b.key[0][i] = 0;
            }
            b.val[0][i] = (uint32_t)i;
        }
    }
    __syncthreads();
    // 16-byte stores of the used words only (an odd count rounds up within
    // the region, whose size is even)
    uint4 *dst = reinterpret_cast<uint4 *>(b.qw + (size_t)r0 * kWMax);
    const uint4 *srcv = reinterpret_cast<const uint4 *>(slots);
    for (uint32_t c = threadIdx.x; c < (run_words + 1) / 2; c += kPackBlock) dst[c] = srcv[c];
}

// First word of read rid's packed words in qw (its workgroup's region plus
// its offset there, as the pack kernel laid them out).
__device__ __forceinline__ const uint64_t *query_words(const uint64_t *qw, int rid, int wo) {
    return qw + (size_t)(rid & ~(kPackBlock - 1)) * kWMax + wo;
}

// ------------------------------------------------------------------ search

template <int W, class Cnt>
__device__ __forceinline__ void tuned_one(const DevIndex &ix, const uint64_t *s_key, const int32_t *s_sa,
                                          int levels, bool use_table, const BatchBuffers &b, int rid, int m, int mv,
                                          int wo, int4 *out, Cnt &cnt) {
    if (m < 0) {
        out[rid] = make_int4(0, 0, 0, (int)kHitTooLong);
        return;
    }
    uint64_t q[W];
    const uint64_t *src = query_words(b.qw, rid, wo);
    const int nw = m > 0 ? (m + 31) >> 5 : 1;
    load_query<W>(src, nw, q);
#pragma unroll
    for (int k = 0; k < W; ++k)
        if (k < nw) cnt.touch(src + k, 8);
    out[rid] = match_read<W>(ix, s_key, s_sa, levels, use_table, q, m, mv, kNoBudget, cnt);
    cnt.touch(out + rid, 16);
}

// tuned_one for a read whose packed words are already in registers, with
// at most `budget` probes: returns true (and writes nothing) when the read
// needs more.
template <int W, int N, class Cnt>
__device__ __forceinline__ bool tuned_regs(const DevIndex &ix, const uint64_t *s_key, const int32_t *s_sa,
                                           int levels, bool use_table, const uint64_t (&w)[N], int rid, int m,
                                           int mv, int budget, int4 *out, Cnt &cnt) {
    if (m < 0) {
        out[rid] = make_int4(0, 0, 0, (int)kHitTooLong);
        return false;
    }
    uint64_t q[W];
#pragma unroll
    for (int k = 0; k < W; ++k) q[k] = w[k];
    const int4 r = match_read<W>(ix, s_key, s_sa, levels, use_table, q, m, mv, budget, cnt);
    if (r.w == (int)kHitDeferred) return true;
    store_stream16(out + rid, r);
    cnt.touch(out + rid, 16);
    return false;
}

// Packing inside the search kernel, for reads in input order with CSR
// offsets: a wave's 64 consecutive reads are one span of the ASCII buffer.
// The wave converts the span with coalesced, aligned 16-byte loads into a
// 2-bit code stream and non-base flags in its own LDS area (as the pack
// kernel does for a workgroup), then each lane takes its read's words out
// of the stream into registers.  A span longer than the area, and a read
// outside its wave's span (offsets that go backwards), take the global
// path.  Saves the pack kernel's writes of the packed words and lengths
// and the search kernel's reads of them.  The loads are pipelined: a wave
// loads the offsets of the chunk after next and the ASCII of the next
// chunk (into registers) before it searches the current one.
// The wave-uniform span of a chunk's reads: the aligned 16-byte pieces
// [A0, A0 + 16 nvec) that hold bytes [s0, s1) of the read buffer; staged
// when it fits the wave's packing area.
struct Span {
    uintptr_t A0;
    int64_t s0, s1;
    int nvec;
    bool staged;
};

// Start and end of each read of chunk (none when chunk < 0): loads issued
// here, used later.  Read j ends at offs[j + 1], or at ends[j] when an end
// array is given (reads gathered from anywhere in the buffer).
__device__ __forceinline__ void chunk_offsets(const int64_t *__restrict__ offs, const int64_t *__restrict__ ends,
                                              int64_t chunk, int64_t nreads, int lane, int64_t &a, int64_t &e) {
    const int64_t j = (chunk << 6) + lane;
    const bool act = chunk >= 0 && j < nreads;
    a = act ? offs[j] : 0;
    e = act ? (ends ? ends[j] : offs[j + 1]) : 0;
}

// With an end array the span is staged only when the chunk's reads follow
// each other (every read ends where the next starts), so that every staged
// byte belongs to one of them; with CSR offsets the span lies between two
// offsets of the one buffer.
__device__ __forceinline__ Span chunk_span(const uint8_t *__restrict__ reads, bool gathered, int64_t chunk,
                                           int64_t nreads, int lane, int64_t a, int64_t e, int max_vec) {
    Span sp{0, 0, 0, 0, false};
    if (chunk < 0) return sp;
    const int last = (int)min_i(63, (int)(nreads - 1 - (chunk << 6)));
    sp.s0 = __shfl(a, 0, 64);
    sp.s1 = __shfl(e, last, 64);
    bool joined = true;
    if (gathered) {
        const int64_t next_a = __shfl_down(a, 1, 64);
        joined = __ballot(lane < last && e != next_a) == 0;
    }
    sp.A0 = (uintptr_t)(reads + sp.s0) & ~(uintptr_t)15;
    const uintptr_t A1 = ((uintptr_t)(reads + sp.s1) + 15) & ~(uintptr_t)15;
    sp.staged = joined && sp.s1 > sp.s0 && A1 - sp.A0 <= (uintptr_t)max_vec * 16u;
    sp.nvec = sp.staged ? (int)((A1 - sp.A0) >> 4) : 0;
    return sp;
}

// Pieces of a staged span a wave holds in registers between chunks (lane l
// holds pieces l, l + 64, ...); the rest of a longer span is loaded when it
// is converted.  Two for the 10-word kernel (on MI355X, 4 and 3 left it
// more registers and a mixed 20-300-base batch 9 % and 5 % slower; 1 was
// 1 % slower), one for the 5-word kernel.
#ifndef SAMATCH_INLINE_AHEAD
#define SAMATCH_INLINE_AHEAD 2
#endif
constexpr int kInlineAhead = SAMATCH_INLINE_AHEAD;

template <int AHEAD, class Cnt>
__device__ __forceinline__ void span_prefetch(const Span &sp, int lane, uint4 (&v)[AHEAD], Cnt &cnt) {
    const uint4 *src = reinterpret_cast<const uint4 *>(sp.A0);
#pragma unroll
    for (int u = 0; u < AHEAD; ++u) {
        const int c = 64 * u + lane;
        if (c < sp.nvec) {
            v[u] = load_stream16(src + c);
            cnt.touch(src + c, 16);
        }
    }
}

// The staged span as codes and flags in the wave's area: the prefetched
// pieces, then the rest (four loads in flight per lane).  Returns, the same
// for every lane, whether any byte of the span was not a base.
template <int AHEAD, class Cnt>
__device__ __forceinline__ bool span_convert(const Span &sp, const uint4 (&v)[AHEAD], uint32_t *codes,
                                             uint16_t *badm, int lane, Cnt &cnt) {
    bool bad = false;
#pragma unroll
    for (int u = 0; u < AHEAD; ++u) {
        const int c = 64 * u + lane;
        if (c < sp.nvec) bad |= convert_piece(v[u], codes, badm, c);
    }
    const uint4 *src = reinterpret_cast<const uint4 *>(sp.A0);
    for (int c0 = 64 * AHEAD; c0 < sp.nvec; c0 += 4 * 64) {
        uint4 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 64 * u + lane;
            if (c < sp.nvec) {
                r[u] = load_stream16(src + c);
                cnt.touch(src + c, 16);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 64 * u + lane;
            if (c < sp.nvec) bad |= convert_piece(r[u], codes, badm, c);
        }
    }
    return __any(bad);
}

// The reads of a chunk of set-aside reads (lane l: m bases at reads[a..];
// m = 0 for a lane without one) as codes and flags in the wave's area:
// lane l's read takes slot l, pieces [l * S, (l + 1) * S) (S =
// inline_slot(WQ)), starting (a & 15) bytes into the slot's first piece.
// The wave loads the slots' pieces with its lanes side by side (pieces of
// one read are neighbours in memory), four loads in flight per lane.
// Returns, the same for every lane, whether any byte loaded was not a base.
template <int WQ, class Cnt>
__device__ __forceinline__ bool gather_convert(const uint8_t *__restrict__ reads, int64_t a, int m, uint32_t *codes,
                                               uint16_t *badm, int lane, Cnt &cnt) {
    constexpr int S = inline_slot(WQ);
    const uintptr_t A0 = (uintptr_t)(reads + a) & ~(uintptr_t)15;
    const int np = m > 0 ? (int)(((((uintptr_t)(reads + a) + (uintptr_t)m + 15) & ~(uintptr_t)15) - A0) >> 4) : 0;
    bool bad = false;
#pragma unroll 1
    for (int c0 = 0; c0 < 64 * S; c0 += 4 * 64) {
        uint4 r[4];
        bool in[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 64 * u + lane;
            const int owner = c / S, k = c - owner * S;
            const uintptr_t base = (uintptr_t)__shfl((unsigned long long)A0, owner & 63, 64);
            const int n_owner = __shfl(np, owner & 63, 64);
            in[u] = c < 64 * S && k < n_owner;
            if (in[u]) {
                r[u] = load_stream16(reinterpret_cast<const uint4 *>(base) + k);
                cnt.touch(reinterpret_cast<const uint4 *>(base) + k, 16);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (in[u]) bad |= convert_piece(r[u], codes, badm, c0 + 64 * u + lane);
    }
    return __any(bad);
}

// LDS written by this wave's lanes is visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Words and first non-base of a read of m bases starting st0 bytes into a
// staged code stream (scan = false: the span has no non-base byte).
template <int N>
__device__ __forceinline__ void inline_extract(const uint32_t *codes, const uint16_t *badm, uint32_t st0, int m,
                                               uint64_t (&w)[N], int &mv, bool scan) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (32 * k < m) {
            const uint32_t bpos = st0 + 32u * (uint32_t)k, q = bpos >> 4, r = bpos & 15u;
            const uint64_t hi = ((uint64_t)codes[q] << 32) | codes[q + 1];
            uint64_t x = r ? (hi << (2 * r)) | (codes[q + 2] >> (32 - 2 * r)) : hi;
            const int rem = m - 32 * k;
            if (rem < 32) x &= ~0ull << (64 - 2 * rem);
            w[k] = x;
        }
    }
    mv = m;
    if (scan && m > 0) {
        const uint32_t q0 = st0 >> 4, q1 = (st0 + (uint32_t)m - 1) >> 4;
        for (uint32_t q = q0; q <= q1; ++q) {
            uint32_t bits = badm[q];
            if (q == q0) bits &= 0xFFFFu << (st0 & 15u);
            if (q == q1) bits &= (2u << ((st0 + (uint32_t)m - 1) & 15u)) - 1u;
            if (bits) {
                mv = (int)(q * 16u + (uint32_t)__builtin_ctz(bits) - st0);
                break;
            }
        }
    }
}

// Sum a per-lane 64-bit count over the wave and add it to a global counter.
__device__ __forceinline__ void wave_add64(unsigned long long *dst, unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

// Sum a per-lane count over the wave and add it to a global counter.
__device__ __forceinline__ void wave_add(unsigned long long *dst, uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// Work split of the persistent kernel, with no global atomics: the reads
// (in input order, or prefix-sorted when the batch is sorted) are cut into
// chunks of 64 (one per lane of a wave) and the chunks into blocks of
// `group` chunks.  Workgroup rank r takes blocks r, r + G, r + 2G, ... (G
// workgroups), so every workgroup sees the same mix of read lengths, and
// all workgroups advance through one window of the order together.  The
// waves of a workgroup share its blocks through a counter in LDS.
// Workgroups are dispatched to the eight XCDs round-robin by id, so ranks
// are assigned XCD by XCD: neighbouring blocks (in a sorted batch, reads
// that visit the same index rows) run in one XCD's L2.
__device__ __forceinline__ int64_t workgroup_rank() {
    const int64_t G = gridDim.x, w = blockIdx.x;
    return (G % 8 == 0) ? (w % 8) * (G / 8) + w / 8 : w;
}

// Persistent kernel: each workgroup stages the top `levels` tree levels in
// LDS once, then its waves take 64-read chunks until the workgroup's blocks
// are done.  Each chunk runs the instantiation for the longest read it
// holds.
//
// INLINE: the kernel packs its reads itself from the ASCII buffer and CSR
// offsets (reads in input order; no pack kernel ran), each wave in its own
// LDS area after the tile.  WQ: query words a read may hold in registers
// (reads of up to 32 * WQ bases; longer ones are the long-read kernel's).
// The 5-word instance keeps fewer registers live (and prefetches one piece
// of the next chunk per lane), so that six waves fit each SIMD (the
// counting instance is not held to that).  Each instance's packing area
// holds the span of 64 reads of its longest length.
template <int BLOCK, bool COUNT, bool INLINE, int WQ>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WQ < kWMax && !COUNT ? 6 : 1))) void search_tuned_kernel(DevIndex ix, int levels, int use_table_i, int group, int defer,
                                                             BatchBuffers b, const uint32_t *__restrict__ order,
                                                             const uint8_t *__restrict__ reads,
                                                             const int64_t *__restrict__ offs,
                                                             const int64_t *__restrict__ ends, int64_t nreads,
                                                             int4 *__restrict__ out) {
    extern __shared__ uint64_t smem[];
    __shared__ unsigned s_next;
    const int nodes = (1 << levels) - 1;
    uint64_t *s_key = smem;
    int32_t *s_sa = reinterpret_cast<int32_t *>(smem + nodes);
    uint32_t *w_codes = nullptr;
    uint16_t *w_badm = nullptr;
    if constexpr (INLINE) {
        uint8_t *area = reinterpret_cast<uint8_t *>(smem) + inline_area_offset(levels) +
                        (size_t)(threadIdx.x >> 6) * inline_wave_bytes(WQ);
        w_codes = reinterpret_cast<uint32_t *>(area);
        w_badm = reinterpret_cast<uint16_t *>(w_codes + inline_vec(WQ) + 4);
    }
    if (threadIdx.x == 0) s_next = 0u;
    for (int i = threadIdx.x; i < nodes; i += BLOCK) {
        s_key[i] = ix.tile_key[i];
        s_sa[i] = ix.tile_sa[i];
    }
    __syncthreads();
    using Cnt = typename std::conditional<COUNT, Count, NoCount>::type;
    Cnt cnt;
    uint32_t nsearched = 0, nqwords = 0;
    const bool use_table = use_table_i != 0;
    const int lane = threadIdx.x & 63;
    const int64_t nchunks = (nreads + 63) >> 6;
    const int64_t G = gridDim.x, rank = workgroup_rank();
    // the next chunk of this wave (-1 when the workgroup's blocks are done;
    // every later one lies further on)
    auto take = [&]() -> int64_t {
        unsigned c = 0;
        if (lane == 0) c = atomicAdd(&s_next, 1u);
        c = __shfl(c, 0, 64);
        const int64_t chunk = ((int64_t)(c / group) * G + rank) * group + (c % group);
        return chunk < nchunks ? chunk : -1;
    };
    if constexpr (INLINE) {
        int64_t c0 = take(), a0, e0;
        chunk_offsets(offs, ends, c0, nreads, lane, a0, e0);
        Span sp0 = chunk_span(reads, ends != nullptr, c0, nreads, lane, a0, e0, inline_vec(WQ));
        constexpr int AHEAD = WQ < kWMax ? 1 : kInlineAhead;
        constexpr int kMaxM = 32 * WQ;  // longest read searched here
        uint4 v[AHEAD];
        span_prefetch(sp0, lane, v, cnt);
        int64_t c1 = c0 >= 0 ? take() : -1, a1, e1;
        chunk_offsets(offs, ends, c1, nreads, lane, a1, e1);
        // reads set aside (their searches ran out of `defer` probes) wait in
        // the wave's queue; when 64 are waiting, or the chunks are done, the
        // wave takes them as a chunk of its own and searches them without a
        // limit, so that one long search does not hold up 63 idle lanes
        uint32_t *w_queue = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(w_codes) + inline_codes_bytes(WQ));
        const int budget = (defer > 0 && !COUNT) ? defer : kNoBudget;
        int queued = 0;  // wave-uniform
        while (c0 >= 0 || queued > 0) {
            const bool drain = queued >= 64 || c0 < 0;
            uint64_t w[WQ];
#pragma unroll
            for (int t = 0; t < WQ; ++t) w[t] = 0;
            int rid, m;
            bool short_read, from_lds, scan, synced;
            uint32_t st0;
            if (drain) {
                const int n = min_i(queued, 64);
                queued -= n;
                short_read = lane < n;
                rid = short_read ? (int)w_queue[queued + lane] : 0;
                const int64_t a = short_read ? offs[rid] : 0;
                const int64_t e = short_read ? (ends ? ends[rid] : offs[rid + 1]) : 0;
                m = (int)(e - a);  // 1 .. kMaxM: the read was searched before
                scan = gather_convert<WQ>(reads, a, m, w_codes, w_badm, lane, cnt);
                wave_lds_sync();
                from_lds = short_read;
                synced = true;
                st0 = (uint32_t)(lane * inline_slot(WQ) * 16) + (uint32_t)(a & 15);
            } else {
                const int64_t j = (c0 << 6) + lane;
                const bool active = j < nreads;
                if (COUNT && active) {
                    cnt.touch(offs + j, ends ? 8 : 16);
                    if (ends) cnt.touch(ends + j, 8);
                }
                const int64_t m64 = e0 - a0;
                // m = -1: length out of range (the too-long result); long reads are the long kernel's
                const bool long_read = active && m64 > kMaxM && m64 <= SA_MAX_READ;
                m = (m64 >= 0 && m64 <= kMaxM) ? (int)m64 : -1;
                if (long_read) b.stats[kLongFlag] = 1ull;
                short_read = active && !long_read;
                rid = (int)j;
                scan = false;
                if (sp0.staged) {
                    scan = span_convert(sp0, v, w_codes, w_badm, lane, cnt);
                    wave_lds_sync();
                }
                synced = sp0.staged;
                from_lds = short_read && m > 0 && sp0.staged && a0 >= sp0.s0 && e0 <= sp0.s1;
                st0 = (uint32_t)((uintptr_t)(reads + a0) - sp0.A0);
            }
            int mv = m;
            if (from_lds) {
                inline_extract(w_codes, w_badm, st0, m, w, mv, scan);
            } else if (short_read && m > 0) {
                uint64_t g[kWMax + 1];
                pack_from_global(reads, a0, m, g, mv, g[kWMax]);
#pragma unroll
                for (int t = 0; t < WQ; ++t) w[t] = (32 * t < m) ? g[t] : 0;
            }
            if (synced) wave_lds_sync();  // every lane has its words before the area is reused
            if (!drain) {
                // loads for the chunks ahead, in flight during this chunk's searches
                const Span sp1 = chunk_span(reads, ends != nullptr, c1, nreads, lane, a1, e1, inline_vec(WQ));
                span_prefetch(sp1, lane, v, cnt);
                const int64_t c2 = c1 >= 0 ? take() : -1;
                int64_t a2, e2;
                chunk_offsets(offs, ends, c2, nreads, lane, a2, e2);
                c0 = c1;
                a0 = a1;
                e0 = e1;
                sp0 = sp1;
                c1 = c2;
                a1 = a2;
                e1 = e2;
            }
            const int wn = max_i(1, (m + 31) >> 5);
            int wc = 1;
#pragma unroll
            for (int t = 2; t <= WQ; ++t)
                if (wave_ballot(short_read && wn >= t)) wc = t;
            const int lim = drain ? kNoBudget : budget;
            bool later = false;
            if (short_read) {
                if (COUNT && m >= 0) { nsearched++; nqwords += wc; }
                switch (wc) {
                    case 1: later = tuned_regs<1>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                    case 2: later = tuned_regs<2>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                    case 3: later = tuned_regs<3>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                    case 4: later = tuned_regs<4>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                    case 5: later = tuned_regs<5>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                    default:
                        if constexpr (WQ >= 10) {
                            switch (wc) {
                                case 6: later = tuned_regs<6>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                                case 7: later = tuned_regs<7>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                                case 8: later = tuned_regs<8>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                                case 9: later = tuned_regs<9>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                                default: later = tuned_regs<10>(ix, s_key, s_sa, levels, use_table, w, rid, m, mv, lim, out, cnt); break;
                            }
                        }
                        break;
                }
            }
            const uint64_t set_aside = wave_ballot(later);
            if (set_aside) {
                if (later) w_queue[queued + __popcll(set_aside & ((1ull << lane) - 1ull))] = (uint32_t)rid;
                queued += __popcll(set_aside);
                wave_lds_sync();
            }
        }
    }
    while (!INLINE) {  // reads packed by the pack kernel
        const int64_t chunk = take();
        if (chunk < 0) break;
        const int64_t j = (chunk << 6) + lane;
        const bool active = j < nreads;
        const int rid = active ? (order ? (int)order[j] : (int)j) : 0;
        const ReadLen lm = decode_len(active ? b.qlm[rid] : encode_len(0, 0, 0));
        if (COUNT && active) {
            if (order) cnt.touch(order + j, 4);
            cnt.touch(b.qlm + rid, 8);
        }
        const int m = lm.m;
        const bool short_read = active && !(m >= 0 && lm.mv < 0);  // long reads are the long kernel's
        const int w = max_i(1, (m + 31) >> 5);
        int wc = 1;
#pragma unroll
        for (int t = 2; t <= kWMax; ++t)
            if (wave_ballot(short_read && w >= t)) wc = t;
        if (active && !short_read && m >= 0) b.stats[kLongFlag] = 1ull;  // a long read: the long kernel runs
        if (!short_read) continue;
        if (COUNT && m >= 0) { nsearched++; nqwords += wc; }
        switch (wc) {
            case 1: tuned_one<1>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 2: tuned_one<2>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 3: tuned_one<3>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 4: tuned_one<4>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 5: tuned_one<5>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 6: tuned_one<6>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 7: tuned_one<7>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 8: tuned_one<8>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            case 9: tuned_one<9>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
            default: tuned_one<10>(ix, s_key, s_sa, levels, use_table, b, rid, m, lm.mv, lm.wo, out, cnt); break;
        }
    }
    if constexpr (COUNT) {
        wave_add(&b.stats[0], cnt.global);
        wave_add(&b.stats[1], cnt.words);
        wave_add(&b.stats[2], cnt.tile);
        wave_add(&b.stats[3], nsearched);
        wave_add(&b.stats[4], nqwords);
        wave_add(&b.stats[5], cnt.keys);
        wave_add(&b.stats[6], cnt.table);
        wave_add64(&b.stats[7], cnt.touched);
        wave_add64(&b.stats[8], cnt.scattered);
        wave_add(&b.stats[9], cnt.index_loads);
    }
}

// Plain kernel, the paper's arrangement (Algorithm 1): one read per
// thread in input order, every search over the whole range (-1, n), every
// probe comparing from the first base, no LDS.  Exact reads take the LB and
// RB searches; other reads add the two neighbour comparisons for l and the
// LB / RB searches of P[0..l).
template <bool UPPER, class Cnt>
__device__ __forceinline__ int plain_search(const DevIndex &ix, const uint64_t (&q)[kWMax], int plen, Cnt &cnt) {
    int L = -1, R = ix.n;
    while (R > L + 1) {
        const int piv = midpoint(L, R);
        int lcp;
        cnt.global_probe();
        cnt.index_touch(ix.sa + piv, 4);
        const int sign = compare_from<kWMax>(ix.text, ix.n, q, plen, ix.sa[piv], 0, lcp, cnt);
        if (UPPER ? (sign < 0) : (sign <= 0)) R = piv; else L = piv;
    }
    return R;
}

template <bool COUNT>
__global__ __launch_bounds__(256) void search_plain_kernel(DevIndex ix, BatchBuffers b, int64_t nreads,
                                                          int4 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    using Cnt = typename std::conditional<COUNT, Count, NoCount>::type;
    Cnt cnt;
    int4 res = make_int4(0, 0, 0, (int)kHitTooLong);
    const ReadLen lm = decode_len(i < nreads ? b.qlm[i] : encode_len(-1, 0, 0));
    if (COUNT && i < nreads) cnt.touch(b.qlm + i, 8);
    const int m = lm.m;
    const bool long_read = m >= 0 && lm.mv < 0;  // the long kernel's
    if (long_read) b.stats[kLongFlag] = 1ull;
    if (m >= 0 && !long_read) {
        const int mv = lm.mv;
        uint64_t q[kWMax];
        const uint64_t *src = query_words(b.qw, (int)i, lm.wo);
#pragma unroll
        for (int k = 0; k < kWMax; ++k) q[k] = (k << 5) < m ? src[k] : 0ull;
#pragma unroll
        for (int k = 0; k < kWMax; ++k)
            if ((k << 5) < m) cnt.touch(src + k, 8);
        const int lo = plain_search<false>(ix, q, mv, cnt);
        int hi = lo;
        if (mv == m) hi = plain_search<true>(ix, q, m, cnt);
        if (mv == m && lo < hi) {
            res = make_int4(lo, hi, m, (int)kHitExact);
        } else {
            int l = 0, lcp;
            if (lo > 0) {
                cnt.global_probe();
                cnt.index_touch(ix.sa + lo - 1, 4);
                compare_from<kWMax>(ix.text, ix.n, q, mv, ix.sa[lo - 1], 0, lcp, cnt);
                l = max_i(l, lcp);
            }
            if (lo < ix.n) {
                cnt.global_probe();
                cnt.index_touch(ix.sa + lo, 4);
                compare_from<kWMax>(ix.text, ix.n, q, mv, ix.sa[lo], 0, lcp, cnt);
                l = max_i(l, lcp);
            }
            res = make_int4(plain_search<false>(ix, q, l, cnt), plain_search<true>(ix, q, l, cnt), l,
                            l == m ? (int)kHitExact : 0);
        }
    }
    if (i < nreads && !long_read) {
        out[i] = res;
        cnt.touch(out + i, 16);
    }
    if constexpr (COUNT) {
        wave_add(&b.stats[0], cnt.global);
        wave_add(&b.stats[1], cnt.words);
        wave_add(&b.stats[3], m >= 0 && !long_read ? 1u : 0u);
        wave_add(&b.stats[4], m >= 0 && !long_read ? (uint32_t)max_i(1, (m + 31) >> 5) : 0u);
        wave_add64(&b.stats[7], cnt.touched);
        wave_add64(&b.stats[8], cnt.scattered);
        wave_add(&b.stats[9], cnt.index_loads);
    }
}

// Dynamic LDS the inline-packing kernels may take (set by prepare_kernels
// from the device's limit per workgroup).
std::atomic<size_t> g_inline_lds{0};

template <int BLOCK, bool COUNT, bool INLINE, int WQ = kWMax>
hipError_t allow_tile_lds(size_t inline_lds) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&search_tuned_kernel<BLOCK, COUNT, INLINE, WQ>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               INLINE ? (int)inline_lds : (int)tile_lds_bytes(kMaxTileLevels));
}

template <int BLOCK, bool COUNT>
hipError_t launch_tuned_block(const DevIndex &ix, int levels, int use_table, int group, int defer, int grid,
                              const BatchBuffers &b,
                              const uint32_t *order, const uint8_t *reads, const int64_t *offs, const int64_t *ends,
                              int64_t nreads, int words, int4 *out, hipStream_t s) {
    if (offs) {
        const size_t lds = tuned_lds_bytes(levels, BLOCK, true, words);
        if (lds > g_inline_lds.load()) return hipErrorInvalidValue;
        if (words == kShortWords)
            hipLaunchKernelGGL((search_tuned_kernel<BLOCK, COUNT, true, kShortWords>), dim3(grid), dim3(BLOCK), lds, s,
                               ix, levels, use_table, group, defer, b, order, reads, offs, ends, nreads, out);
        else
            hipLaunchKernelGGL((search_tuned_kernel<BLOCK, COUNT, true, kWMax>), dim3(grid), dim3(BLOCK), lds, s, ix,
                               levels, use_table, group, defer, b, order, reads, offs, ends, nreads, out);
    } else {
        hipLaunchKernelGGL((search_tuned_kernel<BLOCK, COUNT, false, kWMax>), dim3(grid), dim3(BLOCK),
                           tile_lds_bytes(levels), s, ix, levels, use_table, group, 0, b, order, reads, offs, ends,
                           nreads, out);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ long reads

// Query words in LDS, read on demand by the comparisons.
struct LdsQuery {
    const uint64_t *p;
    __device__ __forceinline__ uint64_t operator[](int k) const { return p[k]; }
};

// The whole wave packs one read of m <= SA_MAX_READ bases at reads[a..a+m)
// into dst[0 .. 32): lane l converts bases 16l .. 16l+15 from aligned dword
// loads (an aligned dword that holds a byte of the read never crosses a
// page) and writes its half word.  Split in two so that a wave can have the
// loads of several reads in flight before it converts them.
struct PackLoad {
    uint32_t dw[5];
    uint32_t sh;
};

template <class Cnt>
__device__ __forceinline__ PackLoad wave_pack_load(const uint8_t *__restrict__ reads, int64_t a, int m, int lane,
                                                   Cnt &cnt) {
    PackLoad pl;
    const int b0 = 16 * lane;
    const uintptr_t x0 = (uintptr_t)(reads + a + b0);
    const uintptr_t base = x0 & ~(uintptr_t)3;
    const uintptr_t stop = (uintptr_t)(reads + a + m);
    pl.sh = (uint32_t)(x0 & 3u);
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const bool in = b0 < m && base + 4u * t < stop;
        pl.dw[t] = in ? *reinterpret_cast<const uint32_t *>(base + 4u * t) : 0u;
        if (in) cnt.touch(reinterpret_cast<const void *>(base + 4u * t), 4);
    }
    return pl;
}

// Returns this lane's first non-ACGT base (0x7FFFFFFF if none); the caller
// takes the minimum over the wave.
__device__ __forceinline__ int wave_pack_store(const PackLoad &pl, int m, uint64_t *dst, int lane) {
    const int b0 = 16 * lane;
    uint32_t half = 0;
    int bad_at = 0x7FFFFFFF;
    if (b0 < m) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int rem = m - b0 - 4 * jj;
            const uint32_t keep = rem >= 4 ? 0xFFFFFFFFu : (rem > 0 ? ((1u << (8 * rem)) - 1u) : 0u);
            uint32_t bad;
            const uint32_t b8 = pack4_fast(__builtin_amdgcn_alignbyte(pl.dw[jj + 1], pl.dw[jj], pl.sh), keep, bad);
            if (bad && bad_at == 0x7FFFFFFF) bad_at = b0 + 4 * jj + (int)(__builtin_ctz(bad) >> 3);
            half = (half << 8) | b8;
        }
    }
    // bases 32k .. 32k+15 (lane 2k) are the high half of word k
    reinterpret_cast<uint32_t *>(dst + (lane >> 1))[(lane & 1) ? 0 : 1] = half;
    return bad_at;
}

// Packs the reads of the lanes in `todo` (a wave-uniform mask; rows `rid`,
// starts `start`, lengths `len` per lane) into their lanes' LDS slots, eight
// reads' loads in flight at a time; *mv of each such lane becomes its
// length up to the first non-ACGT base.
constexpr int kPackInFlight = 8;

template <class Cnt>
__device__ __forceinline__ void wave_pack_reads(const uint8_t *__restrict__ reads, uint64_t todo, int64_t start,
                                                int len, uint64_t (*slot)[kLongWords], int lane, int &mv,
                                                Cnt &cnt) {
    while (todo) {
        int src[kPackInFlight], m[kPackInFlight];
        PackLoad pl[kPackInFlight];
        int nb = 0;
#pragma unroll
        for (int u = 0; u < kPackInFlight; ++u) {
            src[u] = 0;
            m[u] = 0;
            if (todo) {
                src[u] = __ffsll((unsigned long long)todo) - 1;
                todo &= todo - 1;
                m[u] = __shfl(len, src[u], 64);
                pl[u] = wave_pack_load(reads, __shfl(start, src[u], 64), m[u], lane, cnt);
                nb = u + 1;
            }
        }
#pragma unroll
        for (int u = 0; u < kPackInFlight; ++u) {
            if (u < nb) {
                int first_bad = wave_pack_store(pl[u], m[u], slot[src[u]], lane);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) first_bad = min_i(first_bad, __shfl_xor(first_bad, o, 64));
                if (lane == src[u]) mv = min_i(m[u], first_bad);
            }
        }
    }
}

// One wave per workgroup.  In a sorted batch long reads sort last: each
// workgroup finds where they start, then takes 64-row chunks from there (an
// unsorted batch is scanned from its first read).  For every long read of
// a chunk the whole wave packs it into that lane's LDS slot, 16 bases per
// lane from aligned dword loads (an aligned dword holding a byte of the
// read never crosses a page); then each lane searches its own read with
// the query read from LDS.
template <bool COUNT>
__global__ __launch_bounds__(64) void search_long_kernel(DevIndex ix, const uint8_t *__restrict__ reads,
                                                         const int64_t *__restrict__ offs, BatchBuffers b,
                                                         const uint32_t *__restrict__ order,
                                                         const uint32_t *__restrict__ sorted_key, int key_shift,
                                                         uint32_t key_mask, uint32_t long_field, int use_table_i,
                                                         int lengths_from_offs, int long_min,
                                                         const int64_t *__restrict__ ends, int64_t nreads,
                                                         int4 *__restrict__ out) {
    __shared__ uint64_t slot[64][kLongWords];
    __shared__ int64_t s_first;
    const int lane = threadIdx.x;
    // the search kernel before this one flags batches that hold long reads
    if (*reinterpret_cast<volatile const unsigned long long *>(b.stats + kLongFlag) == 0ull) return;
    if (lane == 0) {
        int64_t lo = 0, hi = nreads;  // first sorted row whose key field reaches long_field
        if (sorted_key) {
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (((sorted_key[mid] >> key_shift) & key_mask) >= long_field) hi = mid;
                else lo = mid + 1;
            }
        }
        s_first = lo;
    }
    __syncthreads();
    const int64_t first = s_first;
    const int64_t nchunks = (nreads - first + 63) >> 6;
    using Cnt = typename std::conditional<COUNT, Count, NoCount>::type;
    Cnt cnt;
    uint32_t nsearched = 0, nqwords = 0;
    const bool use_table = use_table_i != 0;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t j = first + (c << 6) + lane;
        const bool act = j < nreads;
        const int rid = act ? (order ? (int)order[j] : (int)j) : 0;
        ReadLen lm;
        if (lengths_from_offs) {  // input order, CSR offsets: a read of long_min+1 .. SA_MAX_READ bases is long
            const int64_t m64 = act ? (ends ? ends[rid] : offs[rid + 1]) - offs[rid] : -1;
            const bool lng = m64 > long_min && m64 <= SA_MAX_READ;
            lm = decode_len(encode_len(lng ? (int)m64 : -1, lng ? -1 : 0, 0));
            if (COUNT && act) cnt.touch(offs + rid, 16);
        } else {
            lm = decode_len(act ? b.qlm[rid] : encode_len(-1, 0, 0));
            if (COUNT && act) {
                if (order) cnt.touch(order + j, 4);
                cnt.touch(b.qlm + rid, 8);
            }
        }
        const bool is_long = act && lm.m >= 0 && lm.mv < 0;
        uint64_t todo = wave_ballot(is_long);
        if (!todo) continue;
        int mv_mine = lm.m;
        wave_pack_reads(reads, todo, is_long ? offs[rid] : 0, lm.m, slot, lane, mv_mine, cnt);
        __syncthreads();  // the slots are written; one wave, so this orders LDS only
        if (is_long) {
            const LdsQuery q{slot[lane]};
            if (COUNT) { nsearched++; nqwords += (uint32_t)((lm.m + 31) >> 5); }
            out[rid] = match_read<kLongWords>(ix, nullptr, nullptr, 0, use_table, q, lm.m, mv_mine, kNoBudget, cnt);
            cnt.touch(out + rid, 16);
        }
        __syncthreads();  // before the next chunk rewrites the slots
    }
    if constexpr (COUNT) {
        wave_add(&b.stats[0], cnt.global);
        wave_add(&b.stats[1], cnt.words);
        wave_add(&b.stats[2], cnt.tile);
        wave_add(&b.stats[3], nsearched);
        wave_add(&b.stats[4], nqwords);
        wave_add(&b.stats[5], cnt.keys);
        wave_add(&b.stats[6], cnt.table);
        wave_add64(&b.stats[7], cnt.touched);
        wave_add64(&b.stats[8], cnt.scattered);
        wave_add(&b.stats[9], cnt.index_loads);
    }
}

// ------------------------------------------------------------------ suffix tree

// Search of the flattened suffix tree: from the root, take the child that
// continues with the read's next base and compare the read with that
// child's first suffix from the depth already matched; stop where the read
// ends, where no child continues, or where the comparison stops inside the
// edge.  The node or leaf reached holds the rows of the matched prefix: the
// same (lo, hi, l, exact) as the suffix-array searches.
template <class Q>
__device__ __forceinline__ int4 st_match(const uint64_t *__restrict__ text, const int32_t *__restrict__ sa,
                                         int32_t n, const StNode *__restrict__ nodes, int32_t root, const Q &q,
                                         int m, int mv) {
    NoCount cnt;
    int lb = 0, rb = n, d = 0, l = 0;
    int node = root;
    const int plen = mv;
    for (;;) {
        if (d >= plen) {
            l = plen;
            break;
        }
        const int c = (int)((q[d >> 5] >> (62 - 2 * (d & 31))) & 3u);
        const int ch = nodes[node].child[c];
        if (ch == -1) {
            l = d;
            break;
        }
        int clb, crb, cdepth;
        if (ch >= 0) {
            const StNode cn = nodes[ch];
            clb = cn.lb;
            crb = cn.rb;
            cdepth = cn.depth;
        } else {
            clb = -2 - ch;
            crb = clb + 1;
            cdepth = 0;
        }
        const int32_t p = sa[clb];
        if (ch < 0) cdepth = n - p;
        int lcp;
        compare_from<kLongWords>(text, n, q, plen, p, d >> 5, lcp, cnt);
        lb = clb;
        rb = crb;
        if (ch < 0 || lcp < cdepth || plen <= cdepth) {
            l = min_i(lcp, plen);
            break;
        }
        node = ch;
        d = cdepth;
    }
    const int flags = l == m ? (int)kHitExact : 0;
    if (l == 0) return make_int4(0, n, 0, flags);
    return make_int4(lb, rb, l, flags);
}

// One wave per workgroup, 64 reads per chunk in input order: the wave packs
// each read of the chunk into LDS, then every lane walks the tree for its own.
__global__ __launch_bounds__(64) void search_st_kernel(const uint64_t *__restrict__ text,
                                                       const int32_t *__restrict__ sa, int32_t n,
                                                       const StNode *__restrict__ nodes, int32_t root,
                                                       const uint8_t *__restrict__ reads,
                                                       const int64_t *__restrict__ offs, int64_t nreads,
                                                       int4 *__restrict__ out) {
    __shared__ uint64_t slot[64][kLongWords];
    const int lane = threadIdx.x;
    NoCount cnt;
    const int64_t nchunks = (nreads + 63) >> 6;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t i = (c << 6) + lane;
        const bool act = i < nreads;
        int64_t a = 0;
        int m = -1;
        if (act) {
            a = offs[i];
            const int64_t m64 = offs[i + 1] - a;
            m = (m64 >= 0 && m64 <= SA_MAX_READ) ? (int)m64 : -1;
        }
        const uint64_t todo = wave_ballot(act && m >= 0);
        int mv = m;
        wave_pack_reads(reads, todo, a, m, slot, lane, mv, cnt);
        __syncthreads();  // one wave: orders the LDS slots
        if (act) {
            if (m < 0) {
                out[i] = make_int4(0, 0, 0, (int)kHitTooLong);
            } else {
                const LdsQuery q{slot[lane]};
                out[i] = st_match(text, sa, n, nodes, root, q, m, mv);
            }
        }
        __syncthreads();  // before the next chunk rewrites the slots
    }
}

__global__ void clear_stats_kernel(BatchBuffers b) {
    if (threadIdx.x < kStatWords) b.stats[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t prepare_kernels() {
    hipError_t e;
    int dev = 0, per_block = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
        return e;
    // room for the kernels' static LDS
    const size_t inline_lds = std::min(kLdsBytes, per_block > 256 ? (size_t)per_block - 256 : (size_t)0);
    if ((e = allow_tile_lds<256, false, false>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<512, false, false>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<1024, false, false>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<256, true, false>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<256, false, true>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<512, false, true>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<1024, false, true>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<256, true, true>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<256, false, true, kShortWords>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<512, false, true, kShortWords>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<1024, false, true, kShortWords>(inline_lds)) != hipSuccess ||
        (e = allow_tile_lds<256, true, true, kShortWords>(inline_lds)) != hipSuccess)
        return e;
    g_inline_lds.store(inline_lds);
    return hipSuccess;
}

size_t inline_lds_limit() { return g_inline_lds.load(); }


hipError_t launch_search_st(const uint64_t *text, const int32_t *sa, int32_t n, const StNode *nodes, int32_t root,
                            const uint8_t *reads, const int64_t *offs, int64_t nreads, void *out, int grid,
                            hipStream_t s) {
    hipLaunchKernelGGL(search_st_kernel, dim3((unsigned)(grid > 0 ? grid : 1)), dim3(64), 0, s, text, sa, n, nodes,
                       root, reads, offs, nreads, static_cast<int4 *>(out));
    return hipGetLastError();
}

hipError_t launch_build_rows(const uint64_t *text, const int32_t *sa, int32_t n, RowRec *rows, hipStream_t s) {
    const int64_t blocks = ((int64_t)n + 255) / 256;
    hipLaunchKernelGGL(build_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, text, sa, n, rows);
    return hipGetLastError();
}

hipError_t launch_build_tile(const uint64_t *text, const int32_t *sa, int32_t n, int levels, uint64_t *key,
                             int32_t *tsa, hipStream_t s) {
    const int nodes = (1 << levels) - 1;
    hipLaunchKernelGGL(build_tile_kernel, dim3((nodes + 255) / 256), dim3(256), 0, s, text, sa, n, levels, key,
                       tsa);
    return hipGetLastError();
}

hipError_t launch_pack(const uint8_t *reads, const int64_t *offs, const int64_t *ends, int64_t nreads,
                       const BatchBuffers &b, const BucketTable &bt, hipStream_t s) {
    const int64_t blocks = (nreads + kPackBlock - 1) / kPackBlock;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kPackBlock), 0, s, reads, offs,
                       ends, nreads, b, bt);
    return hipGetLastError();
}

hipError_t launch_sort(const BatchBuffers &b, int64_t nreads, int lo_bit, int hi_bit, int *which, hipStream_t s) {
    return radix_sort_pairs<uint32_t>(b.key[0], b.val[0], b.key[1], b.val[1], b.hist, b.digit_total, nreads, lo_bit,
                                      hi_bit, which, s);
}

hipError_t launch_search_tuned(const DevIndex &ix, int levels, int use_table, int block, int grid, int group,
                               int defer, const BatchBuffers &b, const uint32_t *order, const uint8_t *reads,
                               const int64_t *offs, const int64_t *ends, int64_t nreads, int words, void *out,
                               bool count, hipStream_t s) {
    int4 *o = static_cast<int4 *>(out);
    if (group < 1 || (offs && order)) return hipErrorInvalidValue;
    if (words != kShortWords && words != kWMax) return hipErrorInvalidValue;
    if (count)  // counts do not depend on the workgroup shape or the work split
        return launch_tuned_block<256, true>(ix, levels, use_table, group, defer, grid * (block / 256), b, order, reads, offs,
                                             ends, nreads, words, o, s);
    switch (block) {
        case 256:
            return launch_tuned_block<256, false>(ix, levels, use_table, group, defer, grid, b, order, reads, offs, ends, nreads,
                                                   words, o, s);
        case 512:
            return launch_tuned_block<512, false>(ix, levels, use_table, group, defer, grid, b, order, reads, offs, ends, nreads,
                                                   words, o, s);
        case 1024:
            return launch_tuned_block<1024, false>(ix, levels, use_table, group, defer, grid, b, order, reads, offs, ends, nreads,
                                                   words, o, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_build_prefix_table(const DevIndex &ix, int k, PrefixEntry *tab, hipStream_t s) {
    // one work-item per entry, in slices of 2^30 entries (a dispatch holds
    // fewer than 2^32 work-items); every T[v] is written before any entry
    // is filled, since the second pass reads T[v + 1]
    const int64_t entries = ((int64_t)1 << (2 * k)) + 1;
    const int64_t slice = (int64_t)1 << 30;
    for (int64_t first = 0; first < entries; first += slice) {
        const int64_t end = std::min(entries, first + slice);
        hipLaunchKernelGGL(build_prefix_table_kernel, dim3((unsigned)((end - first + 255) / 256)), dim3(256), 0, s,
                           ix, k, first, end, tab);
    }
    for (int64_t first = 0; first < entries; first += slice) {
        const int64_t end = std::min(entries, first + slice);
        hipLaunchKernelGGL(fill_prefix_entries_kernel, dim3((unsigned)((end - first + 255) / 256)), dim3(256), 0, s,
                           ix, k, first, end, entries, tab);
    }
    return hipGetLastError();
}

hipError_t launch_search_long(const DevIndex &ix, const uint8_t *reads, const int64_t *offs, const BatchBuffers &b,
                              const uint32_t *order, const uint32_t *sorted_key, int key_shift, uint32_t key_mask,
                              uint32_t long_field, int use_table, bool lengths_from_offs, int long_min,
                              const int64_t *ends, int grid, int64_t nreads, void *out, bool count, hipStream_t s) {
    int4 *o = static_cast<int4 *>(out);
    const dim3 g((unsigned)(grid > 0 ? grid : 1));
    if (lengths_from_offs && order) return hipErrorInvalidValue;
    const int lfo = lengths_from_offs ? 1 : 0;
    if (count)
        hipLaunchKernelGGL(search_long_kernel<true>, g, dim3(64), 0, s, ix, reads, offs, b, order, sorted_key,
                           key_shift, key_mask, long_field, use_table, lfo, long_min, ends, nreads, o);
    else
        hipLaunchKernelGGL(search_long_kernel<false>, g, dim3(64), 0, s, ix, reads, offs, b, order, sorted_key,
                           key_shift, key_mask, long_field, use_table, lfo, long_min, ends, nreads, o);
    return hipGetLastError();
}

hipError_t launch_clear_stats(const BatchBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(clear_stats_kernel, dim3(1), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_search_plain(const DevIndex &ix, const BatchBuffers &b, int64_t nreads, void *out, bool count,
                               hipStream_t s) {
    const int64_t blocks = (nreads + 255) / 256;
    const dim3 grid((unsigned)(blocks > 0 ? blocks : 1));
    if (count)
        hipLaunchKernelGGL(search_plain_kernel<true>, grid, dim3(256), 0, s, ix, b, nreads, static_cast<int4 *>(out));
    else
        hipLaunchKernelGGL(search_plain_kernel<false>, grid, dim3(256), 0, s, ix, b, nreads, static_cast<int4 *>(out));
    return hipGetLastError();
}

}  // namespace samatch
