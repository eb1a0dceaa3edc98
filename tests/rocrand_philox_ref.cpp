// Prints rocRAND's Philox4x32-10 output for counters read from stdin, one
// "key_lo key_hi c0 c1 c2 c3" line each, as "x0 x1 x2 x3" in hex.  rocRAND's
// state (seed, subsequence, offset) maps to key = seed and counter words
// (c0, c1) = offset / 4 and (c2, c3) = subsequence.  Used only as an
// independent pin of the oracle's generator; host-only build.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ull;
    rocrand_init(seed, sub, off, &st);
    uint4 v = rocrand4(&st);
    std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
