// Reads lines "k0 k1 c0 c1 c2 c3" (decimal) and prints Philox4x32-10 of that
// key/counter computed by PyTorch's own engine (ATen/core/PhiloxRNGEngine.h),
// an implementation independent of the oracle's.  The engine's state is
// key = seed, counter = (offset, subsequence), so seed = k0 | k1 << 32,
// subsequence = c2 | c3 << 32 and offset = c0 | c1 << 32 select the block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        at::Philox4_32 e(k0 | (k1 << 32), c2 | (c3 << 32), c0 | (c1 << 32));
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
