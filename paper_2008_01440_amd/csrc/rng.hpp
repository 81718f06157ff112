// Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) on the device.
// Element i of the stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15)
// with the SplitMix64 finaliser; a double in [0, 1) is its top 53 bits times
// 2^-53.  Every element is a pure function of (seed, i), so any grid produces
// the same values as a sequential generator of the same definition.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcheb {

// v[i] = lo + (hi - lo) * U_i, i < n.
void launch_fill_uniform(double* v, int64_t n, uint64_t seed, double lo, double hi, hipStream_t s);

}  // namespace pcheb
