// Prints Philox4x32-10 blocks computed by rocRAND's header-only engine (the
// ten rounds of rocrand_device::philox4x32_10_engine, exposed through a
// derived class), for counters and keys read from stdin as
// "c0 c1 c2 c3 k0 k1" lines.  Host code only.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Rounds : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Rounds r;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 out = r.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", out.x, out.y, out.z, out.w);
    }
    return 0;
}
