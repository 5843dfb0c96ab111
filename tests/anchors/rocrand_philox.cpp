// External anchor for the oracle's Philox4x32-10 block function: runs the
// rocRAND host-side Philox4x32-10 engine (a third-party implementation of the
// Random123 generator) on the CPU and prints its 32-bit outputs.
// Usage: rocrand_philox <seed> <subsequence> <count>
// The engine's key is (seed low 32, seed high 32); its 128-bit counter starts
// at (0, 0, subsequence low 32, subsequence high 32) and rises by one per
// four outputs.  No GPU call is made.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  if (argc != 4) return 2;
  unsigned long long seed = strtoull(argv[1], 0, 0);
  unsigned long long sub = strtoull(argv[2], 0, 0);
  long n = strtol(argv[3], 0, 0);
  rocrand_device::philox4x32_10_engine eng(seed, sub, 0);
  for (long i = 0; i < n; i++) printf("%u\n", eng());
  return 0;
}
