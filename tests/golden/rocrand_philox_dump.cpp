// Prints Philox4x32-10 blocks from rocRAND's host-callable generator so the
// oracle's independent implementation can be compared with a library routine.
// Input lines on stdin: seed c0 c1 c2 c3 (decimal).  rocRAND keys the
// generator with (seed lo, seed hi), puts the subsequence in counter words
// 2..3 and advances words 0..1 by offset / 4.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        rocrand_state_philox4x32_10 st;
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ULL * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_init(seed, sub, off, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
