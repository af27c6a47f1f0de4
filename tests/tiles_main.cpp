// CPU driver that prints the H-kernel tile tables built by the library (thc::h_tiles for the FP64
// kernel, thc::h32_tiles for the FP32 one), one entry per line, for tests/test_host_tiles.py.
// Usage: tiles_main <h|h32> <Pp> <Xb> <slots>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace thc {
std::vector<uint32_t> h_tiles(int64_t Pp, int64_t Xb, int64_t slots);
std::vector<uint32_t> h32_tiles(int64_t Pp, int64_t Xb, int64_t slots);
}  // namespace thc

int main(int argc, char** argv) {
  if (argc != 5) return 64;
  const int64_t Pp = std::atoll(argv[2]), Xb = std::atoll(argv[3]), slots = std::atoll(argv[4]);
  const std::vector<uint32_t> t =
      std::strcmp(argv[1], "h32") == 0 ? thc::h32_tiles(Pp, Xb, slots) : thc::h_tiles(Pp, Xb, slots);
  for (uint32_t v : t) std::printf("%u\n", v);
  return 0;
}
