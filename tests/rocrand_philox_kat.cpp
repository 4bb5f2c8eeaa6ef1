// Host-only helper: Philox4x32-10 outputs from rocRAND's implementation, used to pin the
// oracle's generator.  Reads "seed c0 c1 c2 c3" lines, prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        const unsigned long long subsequence = c2 | (c3 << 32);
        const unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
