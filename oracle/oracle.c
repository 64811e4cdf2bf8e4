/*
 * CPU oracle for suffix-array read matching -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  The product library shares no code with it.
 * It is deliberately plain: bytes compared one by one, a library comparison
 * sort for the suffix array, textbook binary searches.
 *
 * Conventions (readings of the paper, Sections III and IV):
 *   - positions and SA rows are 0-based (Table I is 0-based);
 *   - bases are ordered a < c < g < t, which is byte order of "ACGT";
 *   - a suffix that is a proper prefix of another sorts first (Table I puts
 *     "ac" before "acggtacgtac" and "c" before "cggtacgtac");
 *   - the reference is upper-case ACGT (the caller normalises it).
 *
 * Results per read P[0..m): the longest matched prefix length l (the largest
 * k <= m whose prefix P[0..k) occurs in the text), and the half-open SA row
 * interval [lo, hi) of the occurrences of P[0..l).  The paper's pair of
 * Section IV is LB = lo, RB = hi - 1 when l == m.  Bytes outside ACGT in a
 * read (after upper-casing) occur nowhere, so l never reaches past them.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------ SA
 * Suffix array by the construction the paper calls the most direct one
 * (Section III): list every suffix start and sort the list with a
 * comparison sort.  The comparison is plain lexicographic order in which a
 * shorter string that is a prefix of a longer one comes first.
 */
typedef struct { const uint8_t *t; int64_t n; } sa_ctx;

static int suffix_less_cmp(const void *a, const void *b, void *arg)
{
    const sa_ctx *c = (const sa_ctx *)arg;
    int64_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    int64_t li = c->n - i, lj = c->n - j;
    int64_t k = li < lj ? li : lj;
    int r = memcmp(c->t + i, c->t + j, (size_t)k);
    if (r != 0) return r;
    if (li == lj) return 0;
    return li < lj ? -1 : 1;
}

int oracle_sa_build(const uint8_t *text, int64_t n, int32_t *sa)
{
    if (n < 0 || n > 2147483647LL) return -1;
    for (int64_t i = 0; i < n; i++) sa[i] = (int32_t)i;
    sa_ctx c = { text, n };
    qsort_r(sa, (size_t)n, sizeof(int32_t), suffix_less_cmp, &c);
    return 0;
}

/* Invariants that define a suffix array: a permutation of 0..n-1 whose
 * suffixes are in strictly increasing order.  Returns 0 when both hold, 1
 * when it is not a permutation, 2 when two neighbours are out of order. */
int oracle_sa_check(const uint8_t *text, int64_t n, const int32_t *sa)
{
    uint8_t *seen = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    if (!seen) return -1;
    for (int64_t k = 0; k < n; k++) {
        if (sa[k] < 0 || sa[k] >= n || seen[sa[k]]) { free(seen); return 1; }
        seen[sa[k]] = 1;
    }
    free(seen);
    sa_ctx c = { text, n };
    int bad = 0;
    #pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t k = 1; k < n; k++)
        if (suffix_less_cmp(&sa[k - 1], &sa[k], &c) >= 0) bad = 1;
    return bad ? 2 : 0;
}

/* ------------------------------------------------------------------ search
 * Compare P[0..len) with the suffix at SA row k, the three outcomes of
 * Section IV: 0 when P[0..len) is a prefix of the suffix, negative when P
 * sorts before it, positive when after.  When the suffix runs out first
 * with every compared byte equal, the suffix is the smaller string.
 */
static int cmp_row(const uint8_t *t, int64_t n, const int32_t *sa,
                   const uint8_t *p, int64_t len, int64_t k)
{
    int64_t s = sa[k];
    int64_t avail = n - s;
    int64_t c = len < avail ? len : avail;
    for (int64_t i = 0; i < c; i++) {
        if (p[i] != t[s + i]) return p[i] < t[s + i] ? -1 : 1;
    }
    return c == len ? 0 : 1;
}

/* First SA row whose suffix does not sort before P[0..len): the paper's LB
 * search (Algorithm 1), with open bounds L = -1 and R = n so that LB = R
 * when the loop ends.  A row with P[0..len) as prefix moves R. */
static int64_t lower_row(const uint8_t *t, int64_t n, const int32_t *sa,
                         const uint8_t *p, int64_t len)
{
    int64_t L = -1, R = n;
    while (R > L + 1) {
        int64_t piv = L + (R - L) / 2;
        if (cmp_row(t, n, sa, p, len, piv) <= 0) R = piv; else L = piv;
    }
    return R;
}

/* First SA row whose suffix sorts strictly after every string with prefix
 * P[0..len): the RB search of Algorithm 1, whose result is L = RB, so
 * RB + 1 = R is returned.  A row with P[0..len) as prefix moves L. */
static int64_t upper_row(const uint8_t *t, int64_t n, const int32_t *sa,
                         const uint8_t *p, int64_t len)
{
    int64_t L = -1, R = n;
    while (R > L + 1) {
        int64_t piv = L + (R - L) / 2;
        if (cmp_row(t, n, sa, p, len, piv) < 0) R = piv; else L = piv;
    }
    return R;
}

static int64_t lcp_at(const uint8_t *t, int64_t n, int64_t s, const uint8_t *p, int64_t len)
{
    int64_t i = 0;
    while (i < len && s + i < n && p[i] == t[s + i]) i++;
    return i;
}

/* Index of the first byte outside ACGT (after upper-casing), else m. */
static int64_t valid_prefix(const uint8_t *p, int64_t m)
{
    for (int64_t i = 0; i < m; i++)
        if (p[i] != 'A' && p[i] != 'C' && p[i] != 'G' && p[i] != 'T') return i;
    return m;
}

/* One read.  mode 0: the longest matched prefix comes from the two rows
 * around the insertion point of P (in sorted order the best common prefix
 * with P is found at a neighbour of its insertion point).  mode 1: it
 * comes from a binary search over the prefix length k, since "P[0..k)
 * occurs" holds for every k up to the answer and for none beyond.
 * out = {lo, hi, l, exact}. */
static void match_one(const uint8_t *t, int64_t n, const int32_t *sa,
                      const uint8_t *raw, int64_t m, int mode, uint8_t *buf, int32_t *out)
{
    for (int64_t i = 0; i < m; i++) {
        uint8_t ch = raw[i];
        buf[i] = (ch >= 'a' && ch <= 'z') ? (uint8_t)(ch - 32) : ch;
    }
    int64_t mv = valid_prefix(buf, m);
    int64_t l;
    if (mv == m) {
        int64_t lo = lower_row(t, n, sa, buf, m), hi = upper_row(t, n, sa, buf, m);
        if (lo < hi) {
            out[0] = (int32_t)lo; out[1] = (int32_t)hi; out[2] = (int32_t)m; out[3] = 1;
            return;
        }
    }
    if (mode == 0) {
        int64_t i0 = lower_row(t, n, sa, buf, mv);
        l = 0;
        if (i0 > 0) { int64_t a = lcp_at(t, n, sa[i0 - 1], buf, mv); if (a > l) l = a; }
        if (i0 < n) { int64_t a = lcp_at(t, n, sa[i0], buf, mv); if (a > l) l = a; }
    } else {
        int64_t a = 0, b = mv;             /* occurs(a) holds; find the largest k */
        while (a < b) {
            int64_t k = a + (b - a + 1) / 2;
            if (lower_row(t, n, sa, buf, k) < upper_row(t, n, sa, buf, k)) a = k; else b = k - 1;
        }
        l = a;
    }
    out[0] = (int32_t)lower_row(t, n, sa, buf, l);
    out[1] = (int32_t)upper_row(t, n, sa, buf, l);
    out[2] = (int32_t)l;
    out[3] = (l == m) ? 1 : 0;
}

int oracle_match(const uint8_t *text, int64_t n, const int32_t *sa,
                 const uint8_t *reads, const int64_t *offs, int64_t nreads,
                 int32_t *out, int mode, int nthreads)
{
    if (n < 1 || !text || !sa || !offs || !out) return -1;
    int64_t maxlen = 0;
    for (int64_t r = 0; r < nreads; r++) {
        int64_t m = offs[r + 1] - offs[r];
        if (m < 0) return -1;
        if (m > maxlen) maxlen = m;
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int fail = 0;
    #pragma omp parallel reduction(|:fail)
    {
        uint8_t *buf = (uint8_t *)malloc((size_t)maxlen + 1);
        if (!buf) fail = 1;
        else {
            #pragma omp for schedule(dynamic, 4096)
            for (int64_t r = 0; r < nreads; r++)
                match_one(text, n, sa, reads + offs[r], offs[r + 1] - offs[r], mode, buf, out + 4 * r);
            free(buf);
        }
    }
    return fail ? -2 : 0;
}

/* ------------------------------------------------------------------ scan
 * The same results from the definitions alone, with no suffix array: every
 * text position is visited.  lo counts the suffixes that, cut to l bytes,
 * sort before P[0..l); hi - lo counts the positions where P[0..l) occurs;
 * l is the largest common prefix of P with any suffix.  O(n) per read:
 * for spot checks on references too large for the sorting oracle. */
int oracle_scan_one(const uint8_t *text, int64_t n, const uint8_t *raw, int64_t m, int32_t *out)
{
    if (n < 1 || m < 0) return -1;
    uint8_t *p = (uint8_t *)malloc((size_t)m + 1);
    if (!p) return -2;
    for (int64_t i = 0; i < m; i++) {
        uint8_t ch = raw[i];
        p[i] = (ch >= 'a' && ch <= 'z') ? (uint8_t)(ch - 32) : ch;
    }
    int64_t mv = valid_prefix(p, m);
    int64_t l = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t a = lcp_at(text, n, i, p, mv);
        if (a > l) l = a;
    }
    int64_t below = 0, occ = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t a = lcp_at(text, n, i, p, l);
        if (a == l) occ++;                                  /* P[0..l) occurs at i */
        else if (i + a == n || text[i + a] < p[a]) below++; /* cut suffix sorts first */
    }
    out[0] = (int32_t)below; out[1] = (int32_t)(below + occ); out[2] = (int32_t)l; out[3] = (l == m);
    free(p);
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
