// Prints Philox4x32-10 blocks computed by rocRAND's host-callable engine, for
// counters and keys read from stdin ("k0 k1 c0 c1 c2 c3" per line, hex).
// rocRAND's engine maps seed -> key, subsequence -> counter words 2..3 and
// offset/4 -> counter words 0..1, so one block is ten_rounds(counter, key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
    unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
