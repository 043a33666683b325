// Host check of the sweep book-keeping rule: parity and count advance even
// when a distance is non-finite, and the error is reported.
#include <cmath>
#include <cstdio>
#include "sweep_count.hpp"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

int main() {
  // finite distances: maximum reported, parity flips, count grows
  int parity = 0;
  int64_t count = 7;
  double e = -1.0;
  const double ok[3] = {1e-3, 4e-2, 5e-6};
  CHECK(pn::close_sweep(&parity, &count, ok, 3, &e));
  CHECK(parity == 1 && count == 8 && e == 4e-2);
  // a NaN: still advanced, reported as non-finite with +inf
  const double bad[3] = {1e-3, NAN, 2.0};
  CHECK(!pn::close_sweep(&parity, &count, bad, 3, &e));
  CHECK(parity == 0 && count == 9 && std::isinf(e));
  const double inf[2] = {INFINITY, 0.0};
  CHECK(!pn::close_sweep(&parity, &count, inf, 2, &e));
  CHECK(parity == 1 && count == 10);
  // a batch of handles where the second one fails: all three advance
  int par[3] = {0, 1, 0};
  int64_t cnt[3] = {2, 2, 2};
  double errs[3];
  const double d[3][2] = {{1e-4, 2e-4}, {NAN, 1e-4}, {3e-4, 0.0}};
  bool finite = true;
  for (int i = 0; i < 3; ++i) finite = pn::close_sweep(&par[i], &cnt[i], d[i], 2, &errs[i]) && finite;
  CHECK(!finite);
  CHECK(par[0] == 1 && par[1] == 0 && par[2] == 1);
  CHECK(cnt[0] == 3 && cnt[1] == 3 && cnt[2] == 3);
  CHECK(errs[0] == 2e-4 && std::isinf(errs[1]) && errs[2] == 3e-4);
  // no messages: distance 0
  CHECK(pn::close_sweep(&parity, &count, nullptr, 0, &e) && e == 0.0);
  if (fails == 0) std::printf("ok\n");
  return fails == 0 ? 0 : 1;
}
