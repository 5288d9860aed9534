// Test-only pin: PyTorch's open-source header-only Philox4x32-10 engine
// (ATen/core/PhiloxRNGEngine.h), run on the host.  Reads lines
// "seed q c stream" from stdin and prints the four output words of the
// counter (q lo, q hi, c, stream) under key (seed lo, seed hi).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cinttypes>
#include <cstdio>

int main() {
    unsigned long long seed, q, c, stream;
    while (std::scanf("%llu %llu %llu %llu", &seed, &q, &c, &stream) == 4) {
        // engine(seed, subsequence, offset): key = seed, counter words 2,3 =
        // subsequence, counter words 0,1 = offset.
        at::Philox4_32 eng(seed, (stream << 32) | c, q);
        uint32_t r0 = eng(), r1 = eng(), r2 = eng(), r3 = eng();
        std::printf("%u %u %u %u\n", r0, r1, r2, r3);
    }
    return 0;
}
