// Host-side index arithmetic of the device rings (per-step sweep counts, residual
// history).  A ring of `cap` entries holds logical entry i at slot i % cap; reading
// `count` consecutive entries from logical index `first` is at most two contiguous
// copies.  Plain C++ with no HIP dependency, so it is unit-tested on the host.
#pragma once
#include <cstddef>

namespace ehdg {

struct RingSpan {
  size_t off0, n0;  // first copy: slots [off0, off0 + n0)
  size_t off1, n1;  // second copy (wrapped part): slots [off1, off1 + n1); off1 = 0
};

// Valid for first >= 0, 0 <= count <= cap, cap >= 1 (the caller guarantees that the
// entries are still in the ring: at most cap entries were written after `first`).
inline RingSpan ring_span(long long first, long long count, long long cap) {
  RingSpan r{0, 0, 0, 0};
  if (count <= 0 || cap <= 0) return r;
  const long long start = first % cap;
  const long long head = count < cap - start ? count : cap - start;
  r.off0 = (size_t)start;
  r.n0 = (size_t)head;
  r.off1 = 0;
  r.n1 = (size_t)(count - head);
  return r;
}

}  // namespace ehdg
