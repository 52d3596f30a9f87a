// Test helper: evaluates rocRAND's header-only Philox4x32-10 engine on the
// host for a list of (seed, block k, event id, photon index) tuples read from
// stdin-named binary file, writing 4 words per tuple. It is a third,
// independent implementation used only to check the oracle's Philox.
// Mapping: engine(seed, subsequence = photon index, offset = 4 (k + 2^32 event))
// puts (k, event) into counter words 0-1 and the photon index into words 2-3.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>
#include <vector>

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *in = std::fopen(argv[1], "rb");
  if (!in) return 3;
  std::vector<uint64_t> rec;  // 4 u64 per tuple: seed, k, event, photon index
  uint64_t buf[4];
  while (std::fread(buf, sizeof(uint64_t), 4, in) == 4) rec.insert(rec.end(), buf, buf + 4);
  std::fclose(in);
  const size_t n = rec.size() / 4;
  std::vector<uint32_t> out(4 * n);
  for (size_t i = 0; i < n; ++i) {
    const uint64_t seed = rec[4 * i], k = rec[4 * i + 1], ev = rec[4 * i + 2], idx = rec[4 * i + 3];
    rocrand_device::philox4x32_10_engine eng(seed, idx, 4ull * (k + (ev << 32)));
    const uint4 r = eng.next4();
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
  }
  FILE *o = std::fopen(argv[2], "wb");
  if (!o) return 4;
  std::fwrite(out.data(), sizeof(uint32_t), out.size(), o);
  std::fclose(o);
  return 0;
}
