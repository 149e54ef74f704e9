// Test-only cross-check: prints Philox4x32-10 words from PyTorch's
// header-only engine (ATen/core/PhiloxRNGEngine.h, BSD licence) so the
// oracle's Philox can be compared with an implementation it shares no code
// with.  Usage: philox_torch_ref SEED SUBSEQUENCE OFFSET COUNT
// Prints COUNT lines "w0 w1 w2 w3" (decimal) for counters OFFSET..OFFSET+COUNT-1.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
  unsigned long long subseq = std::strtoull(argv[2], nullptr, 0);
  unsigned long long offset = std::strtoull(argv[3], nullptr, 0);
  long count = std::strtol(argv[4], nullptr, 0);
  at::philox_engine eng(seed, subseq, offset);
  for (long i = 0; i < count; ++i) {
    unsigned w[4];
    for (int j = 0; j < 4; ++j) w[j] = eng();
    std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
  }
  return 0;
}
