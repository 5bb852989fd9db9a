// Prints Philox4x32-10 outputs from rocRAND's engine (run on the host) for the
// (counter, key) pairs read from stdin, one "c0 c1 c2 c3 k0 k1" line (hex) per pair.
// The engine's counter is (offset/4 low, offset/4 high, subsequence low, subsequence high)
// and its key is (seed low, seed high).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
