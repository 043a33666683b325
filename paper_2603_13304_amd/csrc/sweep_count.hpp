// Host book-keeping after a message sweep has run on the device.
//
// A sweep writes the new messages into the other of the two message buffers
// whatever their values, so the handle's parity (which buffer is current) and
// its sweep count advance first, for every handle that was swept; only then
// are the per-message convergence distances (Eq. bp:convergenceCriterium)
// reduced to their maximum and checked for non-finite values.  The single,
// batched and asynchronous sweep paths all use this one rule, so a failed
// sweep leaves every handle pointing at the buffer its last sweep wrote.
#pragma once
#include <cmath>
#include <cstdint>

namespace pn {

// Advances (parity, count) and stores the largest of the n distances in
// *max_err; returns false if any distance is NaN or infinite (then *max_err
// is +inf).
inline bool close_sweep(int* parity, int64_t* sweeps_total, const double* dist, int n,
                        double* max_err) {
  *parity ^= 1;
  *sweeps_total += 1;
  double e = 0.0;
  bool finite = true;
  for (int m = 0; m < n; ++m) {
    if (!std::isfinite(dist[m])) finite = false;
    else if (dist[m] > e) e = dist[m];
  }
  *max_err = finite ? e : INFINITY;
  return finite;
}

}  // namespace pn
