// Test-only pin: rocRAND's open-source Philox4x32-10 engine
// (rocrand/rocrand_philox4x32_10.h), compiled for and run on the host.
// Reads lines "seed q c stream" from stdin and prints the four output words
// of the counter (q lo, q hi, c, stream) under key (seed lo, seed hi).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Pin : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main() {
    unsigned long long seed, q, c, stream;
    Pin p;
    while (std::scanf("%llu %llu %llu %llu", &seed, &q, &c, &stream) == 4) {
        uint4 ctr;
        ctr.x = (unsigned)q; ctr.y = (unsigned)(q >> 32); ctr.z = (unsigned)c; ctr.w = (unsigned)stream;
        uint2 key;
        key.x = (unsigned)seed; key.y = (unsigned)(seed >> 32);
        uint4 r = p.run(ctr, key);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
