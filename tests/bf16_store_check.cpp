// Host-side check of the FP32 -> BF16 rounding used for stored Jacobian blocks,
// preconditioner factors and network weights: reads FP32 bit patterns (hex, one
// per line) from stdin and prints the BF16 bit pattern of each.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../paper_1204_1533_amd/csrc/ldg_store.hpp"

int main() {
  unsigned int b;
  while (std::scanf("%x", &b) == 1) {
    float f;
    uint32_t u = b;
    std::memcpy(&f, &u, sizeof(f));
    std::printf("%04x\n", (unsigned)ldg::f32_to_bf16(f));
  }
  return 0;
}
