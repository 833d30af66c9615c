// Prints rocRAND's Philox-4x32-10 output block for (seed, subsequence, offset) given on
// the command line, one line per triple read from stdin.  Host-only: rocRAND's engine is
// header code usable on the CPU.  Used as a third-party pin for the oracle's generator.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
