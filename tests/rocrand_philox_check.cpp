// Test-only cross-check: prints Philox4x32-10 outputs computed by rocRAND's open-source
// header for (counter, key) lines read from stdin.  Never linked into the product.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // reads lines: c0 c1 c2 c3 k0 k1 (hex) and prints 4 words
  unsigned c[4], k[2];
  while (scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    unsigned long long sub = ((unsigned long long)c[3] << 32) | c[2];
    unsigned long long off = (((unsigned long long)c[1] << 32) | c[0]) * 4ull;
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
