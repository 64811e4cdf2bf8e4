// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <cstddef>
#include <mutex>
#include <string>
#include <vector>
#include <map>
#include <memory>

#include "samatch.h"

namespace samatch {

// Thread-local detail for sa_last_error; returns code for chaining.
int fail(int code, const std::string &msg);
void clear_error();

// ---------------------------------------------------------------- packing
// 2 bits per base, a=0 c=1 g=2 t=3, most significant bits first: base i
// sits in word i/32 at bits [63-2(i%32)-1, 63-2(i%32)].  Integer order of
// words is then lexicographic order of the 32-base blocks.
constexpr int kPadWords = 16;  // zero words after the text (reads never trust them)

inline int base_code(unsigned char c) {
    switch (c | 0x20) {
        case 'a': return 0;
        case 'c': return 1;
        case 'g': return 2;
        case 't': return 3;
        default: return -1;
    }
}

// Validates a reference (1 <= n <= 2^31-1, bytes ACGT in either case).
int check_text(const char *text, int64_t n);
// Packs text[0..n) into ceil(n/32) + kPadWords words.
void pack_text(const char *text, int64_t n, std::vector<uint64_t> &out);

// Suffix array of s[0..n) over integer alphabet 1..K, s padded with three
// zeros (s[n] = s[n+1] = s[n+2] = 0).  DC3 / skew construction.
void dc3_suffix_array(const int32_t *s, int32_t *sa, int64_t n, int32_t K);

}  // namespace samatch

struct sa_index {
    int64_t n = 0;
    std::vector<uint64_t> packed;  // ceil(n/32) + kPadWords words
    std::vector<int32_t> sa;       // n entries
};

// Device-side state lives in device.hip.
struct sa_dindex;
