// Host-only helper: prints rocRAND's Philox4x32-10 output for a given counter and
// key, used as an independent library reference for the oracle's generator.
// rocRAND's engine keys on the 64-bit seed (key word 0 = low half) and places
// the subsequence in counter words 2-3 and offset/4 in counter words 0-1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv)
{
    if (argc != 7) return 2;
    unsigned v[6];
    for (int i = 0; i < 6; ++i) v[i] = (unsigned)strtoul(argv[i + 1], nullptr, 0);
    unsigned long long seed = ((unsigned long long)v[5] << 32) | v[4];
    unsigned long long sub = ((unsigned long long)v[3] << 32) | v[2];
    unsigned long long off = (((unsigned long long)v[1] << 32) | v[0]) * 4ull;
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    for (int i = 0; i < 4; ++i) printf("%u ", e.next());
    printf("\n");
    return 0;
}
