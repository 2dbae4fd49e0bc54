// Independent Philox4x32-10 for the oracle pin: rocRAND's header implementation, called on the host
// as a black box. Reads lines "seed subsequence offset" (decimal) from stdin and prints the four
// 32-bit words that rocrand4() returns first for that state, in hex.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, subsequence, offset;
    while (std::scanf("%llu %llu %llu", &seed, &subsequence, &offset) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
