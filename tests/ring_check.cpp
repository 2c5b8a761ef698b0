// Host check of the descriptor ring's placement arithmetic: over long runs of
// descriptors of one size (sizes that tile a segment exactly, as a solve on
// one mesh produces) and of mixed sizes, every descriptor lies inside one
// segment of the ring, and the segment index stays in range.
#include <cstdio>
#include <cstdlib>

#include "ring_math.h"

int main() {
  const size_t seg_bytes = 2u << 20;
  const int kseg = 8;
  const size_t cap = seg_bytes * kseg;
  const size_t sizes[] = {256, 512, 768, 1024, 4096, 65536, seg_bytes};
  for (int mode = 0; mode < 8; ++mode) {
    size_t end = 0;
    unsigned rng = 12345u + mode;
    for (long k = 0; k < 300000; ++k) {
      size_t need;
      if (mode < 7) {
        need = sizes[mode];
      } else {
        rng = rng * 1664525u + 1013904223u;
        need = 256 * (1 + (rng >> 8) % 64);
      }
      int seg = -1;
      const size_t off = pfem::ring_place(end, need, seg_bytes, kseg, &seg);
      if (seg < 0 || seg >= kseg || off + need > cap || off / seg_bytes != (size_t)seg ||
          (off % seg_bytes) + need > seg_bytes) {
        std::printf("FAIL mode %d put %ld: end %zu need %zu -> off %zu seg %d\n", mode, k, end,
                    need, off, seg);
        return 1;
      }
      end = off + need;
    }
  }
  std::printf("OK\n");
  return 0;
}
