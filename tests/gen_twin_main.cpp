// CPU build of the library's synthetic-input generator (csrc/synth_core.h), for the test that
// compares it bit for bit with the Python generator.  Usage:
//   gen_twin normal <seed> <stream> <first> <count>    -> count doubles
//   gen_twin uniform <seed> <stream> <first> <count>   -> count doubles
//   gen_twin decay <decay> <count>                     -> e^(-K/decay), K = 0..count-1
// Raw little-endian doubles on stdout.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "synth_core.h"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  std::vector<double> out;
  if (!std::strcmp(argv[1], "normal") || !std::strcmp(argv[1], "uniform")) {
    if (argc != 6) return 2;
    const uint64_t seed = std::strtoull(argv[2], nullptr, 10), stream = std::strtoull(argv[3], nullptr, 10);
    const uint64_t first = std::strtoull(argv[4], nullptr, 10), count = std::strtoull(argv[5], nullptr, 10);
    const uint64_t k = thc_synth::key(seed, stream);
    const bool nrm = argv[1][0] == 'n';
    out.resize(count);
    for (uint64_t i = 0; i < count; ++i) out[i] = nrm ? thc_synth::normal(k, first + i) : thc_synth::uniform(k, first + i);
  } else if (!std::strcmp(argv[1], "decay")) {
    if (argc != 4) return 2;
    const double decay = std::strtod(argv[2], nullptr);
    const int64_t count = std::strtoll(argv[3], nullptr, 10);
    out.resize(count);
    for (int64_t K = 0; K < count; ++K) out[K] = thc_synth::decay_factor(K, decay);
  } else {
    return 2;
  }
  std::fwrite(out.data(), sizeof(double), out.size(), stdout);
  return 0;
}
