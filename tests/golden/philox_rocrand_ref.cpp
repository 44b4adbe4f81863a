// Independent reference for the oracle's Philox4x32-10: rocRAND's host-callable
// engine.  Reads lines "seed c0 c1 c2 c3" and prints the four output words of
// one block for key = seed and counter = (c0, c1, c2, c3).
// rocRAND's engine(seed, subsequence, 0) starts at counter
// (0, 0, subsequence low, subsequence high); discard(4*n) then advances the
// low 64 counter bits by n (done in steps of at most 2^61 so 4*n never overflows).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long sub = c2 | (c3 << 32);
        unsigned long long n = c0 | (c1 << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        while (n > 0) {
            unsigned long long step = n < (1ull << 61) ? n : (1ull << 61);
            e.discard(4ull * step);
            n -= step;
        }
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
