// Prints Philox4x32-10 words computed by rocRAND's open-source engine, used as
// an independent known-answer source for the oracle's Philox.  Host code only.
// Input lines: c0 c1 c2 c3 k0 k1 (decimal); output lines: w0 w1 w2 w3.
// rocRAND's engine maps seed -> key (lo, hi), subsequence -> counter words
// 2..3 and offset/4 -> counter words 0..1.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subseq = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
