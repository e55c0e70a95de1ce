// Prints Philox4x32-10 blocks computed by PyTorch's independent header-only
// engine (at::philox_engine), for counters and keys read from stdin as
// "c0 c1 c2 c3 k0 k1" lines.  The engine's key is the 64-bit seed and its
// counter is (offset low, offset high, subsequence low, subsequence high).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::philox_engine eng(seed, subseq, offset);
        uint32_t a = eng(), b = eng(), c = eng(), d = eng();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
