// Independent Philox4x32-10 for cross-checking the oracle: rocRAND's
// open-source header engine, driven through its public seed / subsequence /
// offset interface. Built for the host only by the test that uses it.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void rocrand_philox_block(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    // subsequence s moves counter words (2,3) by s; offset 4*q moves words
    // (0,1) by q. Starting from a zero counter this places the engine at
    // counter (ctr0, ctr1, ctr2, ctr3) with key (key0, key1).
    unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    unsigned long long subsequence = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    unsigned long long q = (unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * q);
    for (int r = 0; r < 4; ++r) out[r] = eng.next();
}
