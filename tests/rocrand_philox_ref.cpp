// Test helper: Philox4x32-10 blocks from rocRAND's host-callable engine, an
// implementation independent of the oracle's.  Reads n records of
// (key0, key1, c0, c1, c2, c3) as uint32 from stdin and writes n x 4 uint32
// words to stdout.  rocRAND's state maps subsequence -> counter words (2, 3)
// and offset/4 -> counter words (0, 1), so c1 must stay below 2^30.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>

int main() {
    uint32_t rec[6];
    while (std::fread(rec, sizeof(uint32_t), 6, stdin) == 6) {
        unsigned long long seed = (unsigned long long)rec[0] | ((unsigned long long)rec[1] << 32);
        unsigned long long subseq = (unsigned long long)rec[4] | ((unsigned long long)rec[5] << 32);
        unsigned long long offset = 4ull * ((unsigned long long)rec[2] | ((unsigned long long)rec[3] << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        uint32_t out[4];
        for (int i = 0; i < 4; ++i) out[i] = rocrand(&st);
        std::fwrite(out, sizeof(uint32_t), 4, stdout);
    }
    return 0;
}
