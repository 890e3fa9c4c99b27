// heat1d_delays.h -- the delay schedules of the emulated asynchronous mode
// (Eq.4 of Section 3 lets a subdomain edge read any of its neighbour's last
// d+1 values; which one is the schedule's choice).
#pragma once

#include "heat1d_device.h"

namespace heat1d {

// Schedule 0: the seeded draw of delay_of.  Schedule 1: every edge read at
// the largest delay d.  Schedule 2: delay d on odd steps, 0 on even ones.
__host__ __device__ __forceinline__ int sched_delay(int sched, uint64_t seed, int64_t k,
                                                    int64_t p, int side, int64_t P, int d) {
  if (sched == 1) return d;
  if (sched == 2) return (k & 1) ? d : 0;
  return delay_of(seed, k, p, side, P, d);
}

}  // namespace heat1d
