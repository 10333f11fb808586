// Witness for the oracle's Philox4x32-10: prints rocRAND's open-source
// philox4x32_10 engine output for (key, counter) tuples read from stdin.
// Host code only; no GPU is touched.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    // rocRAND keys the engine with the 64-bit seed (low word = key 0), puts
    // the subsequence in counter words 2..3 and offset/4 in words 0..1.
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = ((unsigned long long)c0 | ((unsigned long long)c1 << 32)) * 4ull;
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
