// Runs rocRAND's Philox4x32-10 engine on the host (no device needed) and
// prints its first words for a (seed, subsequence, offset) triple; used only
// as an independent implementation to pin the oracle's generator.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  unsigned long long seed = strtoull(argv[1], 0, 0);
  unsigned long long subsequence = strtoull(argv[2], 0, 0);
  unsigned long long offset = strtoull(argv[3], 0, 0);
  int n = atoi(argv[4]);
  rocrand_state_philox4x32_10 state;
  rocrand_init(seed, subsequence, offset, &state);
  for (int i = 0; i < n; ++i) printf("%08x\n", rocrand(&state));
  return 0;
}
