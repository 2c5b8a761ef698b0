// Placement arithmetic of the launch-descriptor ring (host only, no HIP).
#pragma once

#include <cstddef>

namespace pfem {

// Where the next descriptor of `need` bytes goes in a ring of `kseg`
// segments of `seg_bytes` each, the previous descriptor having ended at
// `end` (0 <= end <= kseg * seg_bytes): returns its offset and stores its
// segment in *seg.  A descriptor never straddles two segments; when it does
// not fit in the rest of the current one it starts the next, and a previous
// descriptor that ended exactly at the end of the ring wraps to segment 0.
// Requires need <= seg_bytes.
inline size_t ring_place(size_t end, size_t need, size_t seg_bytes, int kseg, int* seg) {
  size_t off = end >= seg_bytes * (size_t)kseg ? 0 : end;
  int s = (int)(off / seg_bytes);
  if ((off % seg_bytes) + need > seg_bytes) {
    s = (s + 1) % kseg;
    off = (size_t)s * seg_bytes;
  }
  *seg = s;
  return off;
}

}  // namespace pfem
