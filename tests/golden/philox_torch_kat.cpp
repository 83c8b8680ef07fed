// Known-answer generator built on torch's header-only Philox4x32-10 engine
// (ATen/core/PhiloxRNGEngine.h), an implementation independent of this
// repository.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints the
// four output words of one block for each.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned c[4], k[2];
  while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    // engine mapping: key = seed (lo, hi), counter = (offset lo, offset hi,
    // subsequence lo, subsequence hi)
    uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
    uint64_t offset = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
    uint64_t subseq = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
    at::philox_engine eng(seed, subseq, 0);
    eng.set_offset(offset);
    uint32_t o[4];
    for (int i = 0; i < 4; ++i) o[i] = eng();
    std::printf("%08x %08x %08x %08x\n", o[0], o[1], o[2], o[3]);
  }
  return 0;
}
