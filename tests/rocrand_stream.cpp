// Independent Philox4x32-10 reference for the oracle's tests: AMD's rocRAND
// (open source) run on the host.  Reads requests from stdin, one per line:
//   w <seed> <offset> <count>   -> count consecutive 32-bit words of the stream
//                                  (subsequence 0) starting at word offset
//   b <c0> <c1> <c2> <c3> <k0> <k1> -> the Philox block at that counter and key
// and prints the words in hex, one line per request.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdint>
#include <cstring>

int main()
{
    char kind[8];
    while (std::scanf("%7s", kind) == 1) {
        if (std::strcmp(kind, "w") == 0) {
            unsigned long long seed, offset, count;
            if (std::scanf("%llu %llu %llu", &seed, &offset, &count) != 3) return 2;
            rocrand_state_philox4x32_10 st;
            rocrand_init(seed, 0ull, offset, &st);
            for (unsigned long long i = 0; i < count; ++i) std::printf("%08x ", rocrand(&st));
            std::printf("\n");
        } else if (std::strcmp(kind, "b") == 0) {
            unsigned long long c[4], k[2];
            if (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) != 6)
                return 2;
            unsigned long long seed = (k[1] << 32) | k[0];
            unsigned long long sub = (c[3] << 32) | c[2];
            unsigned long long blk = (c[1] << 32) | c[0];
            rocrand_state_philox4x32_10 st;
            rocrand_init(seed, sub, 0ull, &st);
            // advance the counter by blk blocks in steps that keep 4*step inside 64 bits
            while (blk > 0) {
                unsigned long long step = blk > (1ull << 60) ? (1ull << 60) : blk;
                skipahead(4ull * step, &st);
                blk -= step;
            }
            uint4 r = rocrand4(&st);
            std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
        } else {
            return 3;
        }
        std::fflush(stdout);
    }
    return 0;
}
