// Suffix array by difference cover modulo 3 (Section III), in three steps:
//
//   1. the sample suffixes S_i, i mod 3 != 0, are ranked among themselves:
//      radix-sorted by their first three symbols, and where two triples tie,
//      ranked through the suffix array of a reduced string whose symbols are
//      the triples' names (the recursion of the method);
//   2. the other suffixes (i mod 3 == 0) are radix-sorted by the pair
//      (first symbol, rank of S_{i+1});
//   3. the two sorted lists are merged, comparing a sample suffix with a
//      non-sample one by the tuples of Section III: (t_i, rank(S_{i+1})) for
//      i mod 3 == 1, (t_i, t_{i+1}, rank(S_{i+2})) for i mod 3 == 2.
//
// Layout: one array of ranks indexed by text position (0 for the empty
// suffix at and past the end), so that every comparison of steps 2 and 3
// reads a rank by position.  The reduced string of step 1 puts the names of
// the positions i mod 3 == 1 first, then one separator symbol smaller than
// every name, then the names of the positions i mod 3 == 2.  The separator
// ends the first half: a sample suffix whose triples run out before the
// text does (its last triple ends exactly at the end) then sorts below a
// longer one with the same triples, as the text's suffixes do.
//
// Symbols are 1..K; 0 stands for "past the end" and sorts below every
// symbol, so a suffix that is a proper prefix of another sorts first.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace samatch {
namespace {

using Positions = std::vector<int32_t>;

// Stable counting sort of `items` by key(item) in 0..kmax.
template <class Key>
Positions counting_sort(const Positions &items, int64_t kmax, Key key) {
    std::vector<int64_t> start((size_t)kmax + 2, 0);
    for (int32_t it : items) start[(size_t)key(it) + 1]++;
    for (size_t v = 1; v < start.size(); v++) start[v] += start[v - 1];
    Positions out(items.size());
    for (int32_t it : items) out[(size_t)start[(size_t)key(it)]++] = it;
    return out;
}

// Suffix array of a short string by direct comparison of its suffixes.
void sort_directly(const int32_t *s, int64_t n, int32_t *sa) {
    for (int64_t i = 0; i < n; i++) sa[i] = (int32_t)i;
    std::sort(sa, sa + n, [&](int32_t a, int32_t b) {
        return std::lexicographical_compare(s + a, s + n, s + b, s + n);
    });
}

void construct(const int32_t *s, int64_t n, int32_t K, int32_t *sa) {
    if (n < 16) {
        sort_directly(s, n, sa);
        return;
    }
    auto sym = [&](int64_t i) -> int64_t { return i < n ? s[i] : 0; };

    // ---- step 1: rank the sample suffixes
    Positions sample;
    sample.reserve((size_t)(n - (n + 2) / 3));
    for (int64_t i = 1; i < n; i++)
        if (i % 3 != 0) sample.push_back((int32_t)i);
    // by the third symbol, then the second, then the first (stable passes)
    Positions by_triple = counting_sort(sample, K, [&](int32_t i) { return sym(i + 2); });
    by_triple = counting_sort(by_triple, K, [&](int32_t i) { return sym(i + 1); });
    by_triple = counting_sort(by_triple, K, [&](int32_t i) { return sym(i); });

    // names: 2, 3, ... in triple order, equal triples alike (1 is the
    // separator of the reduced string)
    std::vector<int32_t> name((size_t)n + 3, 0);
    int32_t next_name = 1;
    for (size_t r = 0; r < by_triple.size(); r++) {
        const int32_t i = by_triple[r];
        const bool same = r > 0 && sym(i) == sym(by_triple[r - 1]) && sym(i + 1) == sym(by_triple[r - 1] + 1) &&
                          sym(i + 2) == sym(by_triple[r - 1] + 2);
        if (!same) next_name++;
        name[(size_t)i] = next_name;
    }

    // rank[i]: 1-based rank of S_i among the sample suffixes; 0 at and past
    // the end (the empty suffix, below everything)
    std::vector<int32_t> rank((size_t)n + 3, 0);
    Positions sample_sorted;
    if ((size_t)(next_name - 1) == sample.size()) {
        sample_sorted = by_triple;  // all triples distinct: their order is the suffixes' order
    } else {
        std::vector<int32_t> reduced;
        reduced.reserve(sample.size() + 1);
        Positions back;  // text position of each reduced-string position (-1: separator)
        back.reserve(sample.size() + 1);
        for (int64_t i = 1; i < n; i += 3) {
            reduced.push_back(name[(size_t)i]);
            back.push_back((int32_t)i);
        }
        reduced.push_back(1);
        back.push_back(-1);
        for (int64_t i = 2; i < n; i += 3) {
            reduced.push_back(name[(size_t)i]);
            back.push_back((int32_t)i);
        }
        std::vector<int32_t> rsa(reduced.size());
        construct(reduced.data(), (int64_t)reduced.size(), next_name, rsa.data());
        sample_sorted.reserve(sample.size());
        for (int32_t r : rsa)
            if (back[(size_t)r] >= 0) sample_sorted.push_back(back[(size_t)r]);
    }
    for (size_t r = 0; r < sample_sorted.size(); r++) rank[(size_t)sample_sorted[r]] = (int32_t)(r + 1);

    // ---- step 2: the suffixes at i mod 3 == 0 by (t_i, rank(S_{i+1}))
    Positions others;
    others.reserve((size_t)((n + 2) / 3));
    for (int64_t i = 0; i < n; i += 3) others.push_back((int32_t)i);
    const int64_t max_rank = (int64_t)sample_sorted.size();
    others = counting_sort(others, max_rank, [&](int32_t i) { return (int64_t)rank[(size_t)i + 1]; });
    others = counting_sort(others, K, [&](int32_t i) { return sym(i); });

    // ---- step 3: merge, comparing across the lists by Section III's tuples
    auto sample_below = [&](int32_t i, int32_t j) {  // S_i < S_j, i a sample position, j not
        if (sym(i) != sym(j)) return sym(i) < sym(j);
        if (i % 3 == 1) return rank[(size_t)i + 1] < rank[(size_t)j + 1];
        if (sym(i + 1) != sym(j + 1)) return sym(i + 1) < sym(j + 1);
        return rank[(size_t)i + 2] < rank[(size_t)j + 2];
    };
    // std::merge takes from the second list when comp(second, first) holds
    std::merge(sample_sorted.begin(), sample_sorted.end(), others.begin(), others.end(), sa,
               [&](int32_t j_other, int32_t i_sample) { return !sample_below(i_sample, j_other); });
}

}  // namespace

void dc3_suffix_array(const int32_t *s, int32_t *sa, int64_t n, int32_t K) {
    if (n <= 0) return;
    construct(s, n, K, sa);
}

}  // namespace samatch
