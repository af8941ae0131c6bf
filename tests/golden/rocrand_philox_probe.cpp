// Generator of the "H" rows of philox_kat.txt: rocRAND's PHILOX4_32_10 generator used as a black
// box through its host API on the device (seed s, offset 0, the first 12 uint32 outputs).  rocRAND's
// stream for seed s is block i = Philox4x32-10(counter (i, 0, 0, 0), key (s mod 2^32, s >> 32)), so
// each group of four outputs is one known-answer row.
//
// Build and run (ROCm; prints the rows in the fixture's format):
//   hipcc --offload-arch=gfx950 tests/golden/rocrand_philox_probe.cpp -lrocrand -o rocrand_philox_probe
//   ./rocrand_philox_probe
#include <hip/hip_runtime.h>
#include <rocrand/rocrand.h>

#include <cstdint>
#include <cstdio>

int main() {
  const unsigned long long seeds[] = {0ull, 0xdeadbeef12345678ull, 1ull};
  unsigned int* d = nullptr;
  if (hipMalloc((void**)&d, 12 * sizeof(unsigned int)) != hipSuccess) return 1;
  for (unsigned long long s : seeds) {
    rocrand_generator g;
    if (rocrand_create_generator(&g, ROCRAND_RNG_PSEUDO_PHILOX4_32_10) != ROCRAND_STATUS_SUCCESS) return 2;
    if (rocrand_set_seed(g, s) != ROCRAND_STATUS_SUCCESS || rocrand_set_offset(g, 0) != ROCRAND_STATUS_SUCCESS) return 3;
    if (rocrand_generate(g, d, 12) != ROCRAND_STATUS_SUCCESS) return 4;
    unsigned int h[12];
    if (hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) return 5;
    rocrand_destroy_generator(g);
    for (int i = 0; i < 3; ++i)
      printf("H %08x 00000000 00000000 00000000 %08x %08x %08x %08x %08x %08x\n", i, (unsigned)(s & 0xffffffffu),
             (unsigned)(s >> 32), h[4 * i], h[4 * i + 1], h[4 * i + 2], h[4 * i + 3]);
  }
  (void)hipFree(d);
  return 0;
}
