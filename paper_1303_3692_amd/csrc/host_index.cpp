// Host index: validation, 2-bit packing, DC3 suffix array, save / load.
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

using namespace samatch;

namespace {

constexpr char kMagic[8] = {'S', 'A', 'M', 'A', 'T', 'C', 'H', '1'};
constexpr uint32_t kVersion = 1;

uint64_t fnv1a(uint64_t h, const void *p, size_t len) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < len; i++) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}


}  // namespace

namespace samatch {

int check_text(const char *text, int64_t n) {
    if (!text) return fail(SA_EINVAL, "text is NULL");
    if (n < 1) return fail(SA_EINVAL, "reference length must be at least 1");
    if (n > 2147483647LL) return fail(SA_ETOOBIG, "reference longer than 2^31-1 bases");
    for (int64_t i = 0; i < n; i++)
        if (base_code((unsigned char)text[i]) < 0)
            return fail(SA_EALPHABET, "reference byte " + std::to_string(i) + " is outside ACGT");
    return SA_OK;
}

void pack_text(const char *text, int64_t n, std::vector<uint64_t> &out) {
    const int64_t words = (n + 31) / 32;
    out.assign((size_t)(words + kPadWords), 0);
    for (int64_t w = 0; w < words; w++) {
        uint64_t v = 0;
        const int64_t base = w * 32;
        const int64_t lim = std::min<int64_t>(32, n - base);
        for (int64_t j = 0; j < lim; j++)
            v |= (uint64_t)base_code((unsigned char)text[base + j]) << (62 - 2 * j);
        out[(size_t)w] = v;
    }
}

}  // namespace samatch

extern "C" int sa_build(const char *text, int64_t n, sa_index **out) {
    clear_error();
    if (!out) return fail(SA_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_text(text, n);
    if (rc) return rc;
    sa_index *ix = new (std::nothrow) sa_index;
    if (!ix) return fail(SA_ENOMEM, "index allocation");
    try {
        ix->n = n;
        pack_text(text, n, ix->packed);
        std::vector<int32_t> s((size_t)n + 3, 0);
        for (int64_t i = 0; i < n; i++) s[(size_t)i] = base_code((unsigned char)text[i]) + 1;
        ix->sa.assign((size_t)n, 0);
        dc3_suffix_array(s.data(), ix->sa.data(), n, 4);
    } catch (const std::bad_alloc &) {
        delete ix;
        return fail(SA_ENOMEM, "suffix array construction ran out of host memory");
    }
    *out = ix;
    return SA_OK;
}

extern "C" int sa_build_from_sa(const char *text, int64_t n, const int32_t *sa, sa_index **out) {
    clear_error();
    if (!out || !sa) return fail(SA_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = check_text(text, n);
    if (rc) return rc;
    for (int64_t i = 0; i < n; i++)
        if (sa[i] < 0 || sa[i] >= n) return fail(SA_EINVAL, "suffix array value out of range");
    sa_index *ix = new (std::nothrow) sa_index;
    if (!ix) return fail(SA_ENOMEM, "index allocation");
    try {
        ix->n = n;
        pack_text(text, n, ix->packed);
        ix->sa.assign(sa, sa + n);
    } catch (const std::bad_alloc &) {
        delete ix;
        return fail(SA_ENOMEM, "index allocation");
    }
    *out = ix;
    return SA_OK;
}

extern "C" int64_t sa_index_length(const sa_index *ix) { return ix ? ix->n : -1; }

extern "C" int sa_index_copy_sa(const sa_index *ix, int32_t *sa_out) {
    clear_error();
    if (!ix || !sa_out) return fail(SA_EINVAL, "NULL argument");
    std::memcpy(sa_out, ix->sa.data(), sizeof(int32_t) * (size_t)ix->n);
    return SA_OK;
}

extern "C" void sa_free(sa_index *ix) { delete ix; }

extern "C" int sa_save(const sa_index *ix, const char *path) {
    clear_error();
    if (!ix || !path) return fail(SA_EINVAL, "NULL argument");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(SA_EIO, std::string("cannot open ") + path);
    const int64_t nwords = (int64_t)ix->packed.size();
    uint64_t h = 14695981039346656037ull;
    h = fnv1a(h, &ix->n, sizeof ix->n);
    h = fnv1a(h, ix->packed.data(), sizeof(uint64_t) * (size_t)nwords);
    h = fnv1a(h, ix->sa.data(), sizeof(int32_t) * (size_t)ix->n);
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 &&
              std::fwrite(&kVersion, sizeof kVersion, 1, f) == 1 &&
              std::fwrite(&ix->n, sizeof ix->n, 1, f) == 1 &&
              std::fwrite(&nwords, sizeof nwords, 1, f) == 1 &&
              std::fwrite(ix->packed.data(), sizeof(uint64_t), (size_t)nwords, f) == (size_t)nwords &&
              std::fwrite(ix->sa.data(), sizeof(int32_t), (size_t)ix->n, f) == (size_t)ix->n &&
              std::fwrite(&h, sizeof h, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SA_OK : fail(SA_EIO, std::string("write failed: ") + path);
}

extern "C" int sa_load(const char *path, sa_index **out) {
    clear_error();
    if (!path || !out) return fail(SA_EINVAL, "NULL argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(SA_EIO, std::string("cannot open ") + path);
    char magic[8];
    uint32_t ver = 0;
    int64_t n = 0, nwords = 0;
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, kMagic, 8) != 0 ||
        std::fread(&ver, sizeof ver, 1, f) != 1 || ver != kVersion ||
        std::fread(&n, sizeof n, 1, f) != 1 || std::fread(&nwords, sizeof nwords, 1, f) != 1 ||
        n < 1 || n > 2147483647LL || nwords != (n + 31) / 32 + kPadWords) {
        std::fclose(f);
        return fail(SA_EFORMAT, std::string("not an index file of this version: ") + path);
    }
    sa_index *ix = new (std::nothrow) sa_index;
    if (!ix) { std::fclose(f); return fail(SA_ENOMEM, "index allocation"); }
    try {
        ix->n = n;
        ix->packed.resize((size_t)nwords);
        ix->sa.resize((size_t)n);
    } catch (const std::bad_alloc &) {
        delete ix;
        std::fclose(f);
        return fail(SA_ENOMEM, "index allocation");
    }
    uint64_t h_file = 0;
    bool ok = std::fread(ix->packed.data(), sizeof(uint64_t), (size_t)nwords, f) == (size_t)nwords &&
              std::fread(ix->sa.data(), sizeof(int32_t), (size_t)n, f) == (size_t)n &&
              std::fread(&h_file, sizeof h_file, 1, f) == 1;
    std::fclose(f);
    if (!ok) { delete ix; return fail(SA_EFORMAT, std::string("truncated index file: ") + path); }
    uint64_t h = 14695981039346656037ull;
    h = fnv1a(h, &n, sizeof n);
    h = fnv1a(h, ix->packed.data(), sizeof(uint64_t) * (size_t)nwords);
    h = fnv1a(h, ix->sa.data(), sizeof(int32_t) * (size_t)n);
    if (h != h_file) { delete ix; return fail(SA_EFORMAT, std::string("checksum mismatch: ") + path); }
    *out = ix;
    return SA_OK;
}
