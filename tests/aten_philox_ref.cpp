// Reference Philox4x32-10 taken from PyTorch's header-only ATen engine
// (ATen/core/PhiloxRNGEngine.h), used only to pin the oracle's own
// implementation.  The engine's counter is (offset_lo, offset_hi,
// subsequence_lo, subsequence_hi) and its key is the 64-bit seed, so a block
// for an arbitrary (counter, key) is reached through (seed, subsequence,
// offset).
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>

extern "C" void aten_philox_block(const uint32_t ctr[4], const uint32_t key[2],
                                  uint32_t out[4]) {
  uint64_t seed = (uint64_t)key[0] | ((uint64_t)key[1] << 32);
  uint64_t subseq = (uint64_t)ctr[2] | ((uint64_t)ctr[3] << 32);
  uint64_t offset = (uint64_t)ctr[0] | ((uint64_t)ctr[1] << 32);
  at::philox_engine e(seed, subseq, 0);
  e.set_offset(offset);
  for (int i = 0; i < 4; ++i) out[i] = e();
}
