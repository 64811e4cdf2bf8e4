// Suffix tree of the reference as a flat node array (Section III compares
// the suffix array with a suffix tree that is transmitted to the GPU as a
// flattened array; the paper gives no layout, so this one is our own).
//
// The tree is built from the suffix array and its LCP array as the tree of
// lcp-intervals: an internal node is a run of suffix-array rows [lb, rb)
// whose suffixes share `depth` leading bases, with every row just outside
// the run sharing fewer; its children split the run at the rows whose
// common prefix with the row before is exactly `depth`.  Leaves are single
// rows.  Each node stores its run, its depth, and for each base a, c, g, t
// the child that continues with it: a node index, a leaf (-2 - row), or -1.
// A suffix that ends at a node's depth is a leaf without a slot (it sorts
// first in the run and no query base leads to it).
#include <algorithm>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace samatch;

struct st_index {
    int64_t n = 0;
    int32_t root = -1;
    std::vector<StNode> nodes;
};

namespace {

inline int base_at(const std::vector<uint64_t> &packed, int64_t i) {
    return (int)((packed[(size_t)(i >> 5)] >> (62 - 2 * (i & 31))) & 3u);
}

// 32 bases from position b (zero past the text end).
inline uint64_t word_at(const std::vector<uint64_t> &packed, int64_t b) {
    const size_t wi = (size_t)(b >> 5);
    const unsigned sh = (unsigned)(b & 31) * 2u;
    const uint64_t lo = packed[wi], hi = packed[wi + 1];
    return sh ? (lo << sh) | (hi >> (64u - sh)) : lo;
}

// lcp[r] = common prefix length of the suffixes at rows r-1 and r (lcp[0] =
// 0), in linear time from the rank array (each step starts one base below
// the previous value), comparing 32 bases at a time.
void lcp_array(const sa_index &ix, std::vector<int32_t> &lcp) {
    const int64_t n = ix.n;
    std::vector<int32_t> rank((size_t)n);
    for (int64_t r = 0; r < n; r++) rank[(size_t)ix.sa[(size_t)r]] = (int32_t)r;
    lcp.assign((size_t)n, 0);
    int64_t h = 0;
    for (int64_t i = 0; i < n; i++) {
        const int64_t r = rank[(size_t)i];
        if (r == 0) {
            h = 0;
            continue;
        }
        const int64_t j = ix.sa[(size_t)(r - 1)];
        const int64_t lim = std::min(n - i, n - j);
        while (h < lim) {
            const uint64_t x = word_at(ix.packed, i + h) ^ word_at(ix.packed, j + h);
            if (x) {
                h = std::min(lim, h + (int64_t)(__builtin_clzll(x) >> 1));
                break;
            }
            h = std::min(lim, h + 32);
        }
        lcp[(size_t)r] = (int32_t)h;
        if (h > 0) h--;
    }
}

struct Open {
    int32_t depth, lb;
    std::vector<int32_t> children;  // closed child intervals (node ids), ascending lb
};

// Fill the child slots of a closed interval: its child intervals, and the
// rows between them as leaves.
void close_node(const sa_index &ix, std::vector<StNode> &nodes, const Open &o, int32_t rb, int32_t id) {
    StNode &u = nodes[(size_t)id];
    u.lb = o.lb;
    u.rb = rb;
    u.depth = o.depth;
    u.pad = 0;
    for (int c = 0; c < 4; c++) u.child[c] = -1;
    auto slot = [&](int32_t first_row, int32_t code) {
        const int64_t p = ix.sa[(size_t)first_row];
        if (p + o.depth >= ix.n) return;  // the suffix ends at this depth
        u.child[base_at(ix.packed, p + o.depth)] = code;
    };
    int32_t row = o.lb;
    for (int32_t ch : o.children) {
        for (; row < nodes[(size_t)ch].lb; row++) slot(row, -2 - row);
        slot(nodes[(size_t)ch].lb, ch);
        row = nodes[(size_t)ch].rb;
    }
    for (; row < rb; row++) slot(row, -2 - row);
}

}  // namespace

extern "C" int st_build(const sa_index *ix, st_index **out) {
    clear_error();
    if (!ix || !out) return fail(SA_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_ptr<st_index> t(new (std::nothrow) st_index);
    if (!t) return fail(SA_ENOMEM, "suffix tree allocation");
    try {
        const int64_t n = ix->n;
        t->n = n;
        std::vector<int32_t> lcp;
        lcp_array(*ix, lcp);
        // bottom-up pass over the lcp-intervals with a stack; a node's id is
        // reserved when its interval is pushed, filled when it closes
        std::vector<Open> st;
        std::vector<int32_t> ids;
        st.push_back(Open{0, 0, {}});
        ids.push_back(0);
        t->nodes.emplace_back();
        for (int64_t r = 1; r <= n; r++) {
            const int32_t L = r < n ? lcp[(size_t)r] : -1;
            int32_t lb = (int32_t)(r - 1);
            int32_t last = -1;
            while (!st.empty() && L < st.back().depth) {
                Open o = std::move(st.back());
                const int32_t id = ids.back();
                st.pop_back();
                ids.pop_back();
                close_node(*ix, t->nodes, o, (int32_t)r, id);
                lb = o.lb;
                if (st.empty()) {
                    t->root = id;
                    break;
                }
                if (L <= st.back().depth) {
                    st.back().children.push_back(id);
                    last = -1;
                } else {
                    last = id;
                }
            }
            if (!st.empty() && L > st.back().depth) {
                Open o{L, lb, {}};
                if (last >= 0) o.children.push_back(last);
                st.push_back(std::move(o));
                ids.push_back((int32_t)t->nodes.size());
                t->nodes.emplace_back();
            }
        }
        if (t->root < 0) return fail(SA_EDEVICE, "suffix tree construction left intervals open");
    } catch (const std::bad_alloc &) {
        return fail(SA_ENOMEM, "suffix tree construction ran out of host memory");
    }
    *out = t.release();
    return SA_OK;
}

extern "C" void st_free(st_index *t) { delete t; }

extern "C" int64_t st_node_count(const st_index *t) { return t ? (int64_t)t->nodes.size() : -1; }

extern "C" int32_t st_root(const st_index *t) { return t ? t->root : -1; }

extern "C" int st_copy_nodes(const st_index *t, int32_t *out) {
    clear_error();
    if (!t || !out) return fail(SA_EINVAL, "NULL argument");
    std::copy(t->nodes.begin(), t->nodes.end(), reinterpret_cast<StNode *>(out));
    return SA_OK;
}


// ------------------------------------------------------------------ device

#include "device_state.h"

struct st_dindex {
    const sa_dindex *d = nullptr;  // text and suffix array (not owned)
    StNode *d_nodes = nullptr;
    int32_t root = -1;
    int64_t nnodes = 0;
    ~st_dindex() {
        if (d_nodes) {
            DeviceGuard g(d->device);
            (void)hipFree(d_nodes);
        }
    }
};

extern "C" int st_upload(const st_index *t, const sa_dindex *d, st_dindex **out) {
    clear_error();
    if (!t || !d || !out) return fail(SA_EINVAL, "NULL argument");
    *out = nullptr;
    if (t->n != d->n) return fail(SA_EINVAL, "suffix tree and resident index are of different texts");
    DeviceGuard g(d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    std::unique_ptr<st_dindex> s(new st_dindex);
    s->d = d;
    s->root = t->root;
    s->nnodes = (int64_t)t->nodes.size();
    const size_t bytes = sizeof(StNode) * t->nodes.size();
    hipError_t e;
    if ((e = hipMalloc((void **)&s->d_nodes, bytes)) != hipSuccess) return hip_fail(e, "suffix tree allocation");
    if ((e = hipMemcpy(s->d_nodes, t->nodes.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "suffix tree upload");
    *out = s.release();
    return SA_OK;
}

extern "C" void st_dfree(st_dindex *s) { delete s; }

extern "C" int64_t st_index_bytes(const st_index *t) {
    if (!t) return -1;
    // nodes, plus the suffix array (leaves) and the 2-bit text it searches
    return (int64_t)(sizeof(StNode) * t->nodes.size()) + 4 * t->n + 8 * ((t->n + 31) / 32);
}

extern "C" int st_match_batch_dev(const st_dindex *s, const uint8_t *d_reads, const int64_t *d_offs, int64_t nreads,
                                  sa_hit *d_out, void *hip_stream) {
    clear_error();
    if (!s || !d_offs || (nreads > 0 && (!d_reads || !d_out))) return fail(SA_EINVAL, "NULL argument");
    if (nreads < 0 || nreads > INT32_MAX) return fail(SA_EINVAL, "nreads out of range");
    if (nreads == 0) return SA_OK;
    DeviceGuard g(s->d->device);
    if (!g.ok) return fail(SA_EDEVICE, "hipSetDevice failed");
    hipError_t e = launch_search_st(s->d->d_text, s->d->d_sa, (int32_t)s->d->n, s->d_nodes, s->root, d_reads, d_offs,
                                    nreads, d_out,
                                    (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)s->d->cu_count * 8,
                                                                                (nreads + 63) / 64)),
                                    static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? SA_OK : hip_fail(e, "suffix tree search launch");
}
