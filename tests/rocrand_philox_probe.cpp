// Host-side probe: prints the four Philox4x32-10 words rocRAND produces for
// (seed, subsequence, offset).  Used only by the oracle's pin test to check
// the oracle's own Philox against an independent implementation.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0);
    unsigned long long sub = strtoull(argv[a + 1], 0, 0);
    unsigned long long off = strtoull(argv[a + 2], 0, 0);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    for (int i = 0; i < 4; ++i) printf("%u ", rocrand(&st));
    printf("\n");
  }
  return 0;
}
