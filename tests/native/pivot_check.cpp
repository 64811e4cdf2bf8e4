// CPU check of the search kernels' pivot rule (pivot.h) at the ends of the
// supported range of text lengths, built with the undefined-behaviour
// sanitizer so that a signed overflow in the arithmetic fails the run.
#include <climits>
#include <cstdint>
#include <cstdio>

#include "pivot.h"

static int failures = 0;

static void expect(int L, int R) {
    const int got = samatch::midpoint(L, R);
    const int64_t want = (int64_t)L + (((int64_t)R - (int64_t)L) >> 1);  // exact in 64 bits
    if (got != want || got <= L || got >= R) {
        std::printf("midpoint(%d, %d) = %d, want %lld strictly inside\n", L, R, got, (long long)want);
        failures++;
    }
}

int main() {
    const int n = INT32_MAX;  // the largest text the index accepts
    expect(-1, n);            // the first probe of every search from (-1, n)
    expect(-1, 1);
    expect(-1, 2);
    expect(n - 2, n);
    expect(n / 2, n);
    expect(-1, n / 2);
    // every pivot a full search from (-1, n) can take, always going one way
    for (int side = 0; side < 2; side++) {
        int L = -1, R = n;
        while (R > L + 1) {
            expect(L, R);
            const int p = samatch::midpoint(L, R);
            if (side) L = p; else R = p;
        }
    }
    std::printf("%s\n", failures ? "FAIL" : "ok");
    return failures ? 1 : 0;
}
