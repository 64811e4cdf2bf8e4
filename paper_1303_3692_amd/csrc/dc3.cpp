// DC3 (difference cover modulo 3, "skew") suffix array construction of
// Section III: (1) sort the suffixes starting at i mod 3 != 0 by their
// first three symbols, naming the triples and recursing when names repeat;
// (2) sort the suffixes at i mod 3 == 0 by (first symbol, rank of the
// suffix one position later); (3) merge the two lists, comparing a sample
// suffix i with a non-sample suffix j by (t_i, rank(i+1)) against
// (t_j, rank(j+1)) when i mod 3 == 1, and by (t_i, t_{i+1}, rank(i+2))
// against (t_j, t_{j+1}, rank(j+2)) when i mod 3 == 2.  Linear time.
//
// Symbol 0 is the terminator below every base, so a suffix that is a
// proper prefix of another sorts first.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace samatch {
namespace {

// Stable counting sort of the indices src[0..cnt) by key[src[i]] into dst.
void radix_pass(const int32_t *src, int32_t *dst, const int32_t *key, int64_t cnt, int32_t K,
                std::vector<int64_t> &bucket) {
    bucket.assign((size_t)K + 2, 0);
    for (int64_t i = 0; i < cnt; i++) bucket[(size_t)key[src[i]] + 1]++;
    for (int32_t k = 1; k <= K + 1; k++) bucket[k] += bucket[k - 1];
    for (int64_t i = 0; i < cnt; i++) dst[bucket[(size_t)key[src[i]]]++] = src[i];
}

inline bool pair_leq(int32_t a1, int32_t a2, int32_t b1, int32_t b2) {
    return a1 < b1 || (a1 == b1 && a2 <= b2);
}
inline bool triple_leq(int32_t a1, int32_t a2, int32_t a3, int32_t b1, int32_t b2, int32_t b3) {
    return a1 < b1 || (a1 == b1 && pair_leq(a2, a3, b2, b3));
}

void skew(const int32_t *s, int32_t *sa, int64_t n, int32_t K) {
    if (n == 1) { sa[0] = 0; return; }
    // counts of positions with i mod 3 == 0, 1, 2
    const int64_t n0 = (n + 2) / 3, n1 = (n + 1) / 3, n2 = n / 3;
    // When n mod 3 == 1 a dummy sample position n (all-terminator triple) is
    // added to the mod-1 group so that the two groups join correctly.
    const int64_t n02 = n0 + n2;
    std::vector<int32_t> s12((size_t)n02 + 3, 0), sa12((size_t)n02 + 3, 0);
    std::vector<int64_t> bucket;

    int64_t j = 0;
    for (int64_t i = 0; i < n + (n0 - n1); i++)
        if (i % 3 != 0) s12[j++] = (int32_t)i;

    // Step 1: sort sample positions by their triples (least significant first).
    radix_pass(s12.data(), sa12.data(), s + 2, n02, K, bucket);
    radix_pass(sa12.data(), s12.data(), s + 1, n02, K, bucket);
    radix_pass(s12.data(), sa12.data(), s, n02, K, bucket);

    // Name the triples in sorted order; equal triples share a name.
    int32_t name = 0, c0 = -1, c1 = -1, c2 = -1;
    for (int64_t i = 0; i < n02; i++) {
        const int32_t p = sa12[i];
        if (s[p] != c0 || s[p + 1] != c1 || s[p + 2] != c2) {
            name++;
            c0 = s[p]; c1 = s[p + 1]; c2 = s[p + 2];
        }
        // mod-1 names first, then mod-2 names: the reduced string R1 R2
        if (p % 3 == 1) s12[p / 3] = name;
        else s12[p / 3 + n0] = name;
    }

    if (name < n02) {
        // names repeat: sort the reduced string recursively
        skew(s12.data(), sa12.data(), n02, name);
        for (int64_t i = 0; i < n02; i++) s12[sa12[i]] = (int32_t)(i + 1);
    } else {
        for (int64_t i = 0; i < n02; i++) sa12[s12[i] - 1] = (int32_t)i;
    }

    // Step 2: the mod-0 suffixes, ordered by (first symbol, rank of i+1).
    // The sample order already sorts them by the rank of i+1; one stable
    // pass on the first symbol finishes the job.
    std::vector<int32_t> s0((size_t)n0), sa0((size_t)n0);
    j = 0;
    for (int64_t i = 0; i < n02; i++)
        if (sa12[i] < n0) s0[j++] = 3 * sa12[i];
    radix_pass(s0.data(), sa0.data(), s, n0, K, bucket);

    // Step 3: merge.  The rank of sample position i is s12[i/3] when
    // i mod 3 == 1 and s12[i/3 + n0] when i mod 3 == 2 (0 past the end).
    auto pos12 = [&](int64_t t) -> int64_t {
        return sa12[t] < n0 ? (int64_t)sa12[t] * 3 + 1 : ((int64_t)sa12[t] - n0) * 3 + 2;
    };
    int64_t p = 0, t = n0 - n1, k = 0;  // skip the dummy sample suffix
    while (k < n) {
        const int64_t i = pos12(t);
        const int64_t jj = sa0[p];
        bool sample_first;
        if (sa12[t] < n0) {  // i mod 3 == 1
            sample_first = pair_leq(s[i], s12[sa12[t] + n0], s[jj], s12[jj / 3]);
        } else {             // i mod 3 == 2
            sample_first = triple_leq(s[i], s[i + 1], s12[sa12[t] - n0 + 1],
                                      s[jj], s[jj + 1], s12[jj / 3 + n0]);
        }
        if (sample_first) {
            sa[k++] = (int32_t)i;
            if (++t == n02) {
                while (p < n0) sa[k++] = sa0[p++];
            }
        } else {
            sa[k++] = (int32_t)jj;
            if (++p == n0) {
                while (t < n02) sa[k++] = (int32_t)pos12(t++);
            }
        }
    }
}

}  // namespace

void dc3_suffix_array(const int32_t *s, int32_t *sa, int64_t n, int32_t K) {
    if (n <= 0) return;
    skew(s, sa, n, K);
}

}  // namespace samatch
