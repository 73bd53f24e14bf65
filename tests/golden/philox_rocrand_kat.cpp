// Known answers of Philox4x32-10 from rocRAND's header-only engine (an
// independent implementation of the generator of Salmon et al., SC'11).
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints "r0 r1 r2 r3".
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct kat_engine : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  kat_engine e;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
