// Reference Philox4x32-10 stream from rocRAND's host-callable engine, used only
// to pin the oracle's generator.  Reads lines "seed subsequence offset4" from
// stdin; prints the four words of the engine output at that position.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long seed, subseq, n;
    while (std::scanf("%llu %llu %llu", &seed, &subseq, &n) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, 4ull * n, &st);
        unsigned int w[4];
        for (int k = 0; k < 4; ++k) w[k] = rocrand(&st);
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
