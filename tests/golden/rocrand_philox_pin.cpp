// Known-answer source for the Philox4x32-10 pin: rocRAND's own host/device
// engine (header-only, /opt/rocm/include/rocrand), an implementation of the
// same published generator that shares nothing with this repository.
// stdin: lines "c0 c1 c2 c3 key"; stdout: the four output words.
// The engine is seeded so that its counter equals (c0, c1, c2, c3): the
// subsequence fills the upper 64 counter bits, offsets (in words, 4 per
// block) the lower 64; the offset is added in pieces below 2^62 blocks so that
// the word count never overflows.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3;
  unsigned long long key;
  while (std::scanf("%u %u %u %u %llu", &c0, &c1, &c2, &c3, &key) == 5) {
    unsigned long long sub = (static_cast<unsigned long long>(c3) << 32) | c2;
    unsigned long long low = (static_cast<unsigned long long>(c1) << 32) | c0;
    rocrand_device::philox4x32_10_engine e(key, sub, (low & 0x3FFFFFFFFFFFFFFFull) * 4ull);
    for (unsigned long long t = 0; t < 4ull * (low >> 62); ++t) e.discard(1ull << 62);
    unsigned w0 = e.next(), w1 = e.next(), w2 = e.next(), w3 = e.next();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
