// Host-only check of the plan compiler (geometry + plans, no HIP): builds the
// sweep and expectation plans of several problems and options for both
// message parities and checks that every buffer reference starts inside its
// region.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_rules.py.
#include <cstdio>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace pn;

namespace {

int failures = 0;

void fail(const std::string& what) {
  std::printf("FAIL %s\n", what.c_str());
  ++failures;
}

// every reference of a lane's ops starts inside its region
void check_refs(const Compiler& C, const Plan& pl, const std::string& tag) {
  for (int L = 0; L < pl.nlanes; ++L)
    for (const auto& ko : pl.lanes[L].ops) {
      const Op& op = ko.second;
      std::vector<Ref> rs = {op.a, op.b, op.c, op.d};
      rs.insert(rs.end(), op.refs.begin(), op.refs.end());
      for (const Ref& r : rs) {
        if (!r.valid()) continue;
        if (r.off < 0) { fail(tag + ": negative offset"); return; }
        if (r.region >= RG_LANE0) {
          const size_t k = size_t(r.region - RG_LANE0);
          if (k >= C.lane_size.size() || r.off >= C.lane_size[k]) {
            fail(tag + ": lane reference outside its region");
            return;
          }
        } else if ((r.region == RG_MSG0 || r.region == RG_MSG1) && r.off >= C.msg.size) {
          fail(tag + ": message reference outside the message set");
          return;
        }
      }
    }
}

void run(const std::string& tag, const Problem& P, const PlanOptions& o) {
  Compiler C(P, o);
  if (!C.error.empty()) { fail(tag + ": " + C.error); return; }
  const auto bonds = P.kind == 1 ? P.central_bonds() : P.bonds();
  for (int par = 0; par < 2; ++par) {
    Plan sw, ex;
    if (!C.build_sweep(par, &sw)) { fail(tag + " sweep: " + C.error); return; }
    std::vector<std::vector<int>> carry;
    std::vector<int64_t> rho;
    if (!C.build_expect(par, bonds, &ex, &carry, &rho)) { fail(tag + " expect: " + C.error); return; }
    if (sw.nlanes != int(P.msg_keys.size()) || ex.nlanes != int(bonds.size()))
      fail(tag + ": lane counts");
    for (const auto& l : sw.lanes)
      if (l.ops.empty()) fail(tag + ": empty sweep lane");
    check_refs(C, sw, tag + " sweep");
    check_refs(C, ex, tag + " expect");
  }
}

PlanOptions opts(int D, int chi, int trunc, int chi_env, int order = 0, int prec = 0) {
  PlanOptions o;
  o.D = D; o.d = 2; o.chi = chi; o.chi_env = chi_env; o.trunc = trunc;
  o.q = 2; o.p = 8; o.seed = 7; o.order = order; o.precision = prec;
  return o;
}

}  // namespace

int main() {
  for (int N : {2, 3}) {
    Problem P;
    const std::string e = build_hex(&P, N);
    if (!e.empty()) { fail("hex geometry: " + e); continue; }
    for (int order = 0; order < 3; ++order) {
      run("hex N" + std::to_string(N) + " T1 order " + std::to_string(order), P,
          opts(N == 2 ? 2 : 3, N == 2 ? 8 : 16, 0, N == 2 ? 8 : 16, order));
      run("hex N" + std::to_string(N) + " T2 order " + std::to_string(order), P,
          opts(N == 2 ? 2 : 3, N == 2 ? 8 : 16, 1, N == 2 ? 8 : 16, order, 1));
    }
    PlanOptions f2 = opts(2, 8, 0, 8);
    f2.hermitize = 1;
    f2.damping = 0.3;
    run("hex N" + std::to_string(N) + " hermitize + damping", P, f2);
  }
  {
    Problem P;
    const std::string e = build_hex(&P, 4);
    if (!e.empty()) fail("hex geometry: " + e);
    else run("hex N4 D6 chi64 T2", P, opts(6, 64, 1, 64));
  }
  {
    Problem P;
    const std::string e = build_finite(&P, 4, 4, 2, 2);
    if (!e.empty()) {
      fail("patch geometry: " + e);
    } else {
      run("patch T1", P, opts(2, 4, 0, 4));
      run("patch exact", P, opts(2, 4, 0, 0));
      PlanOptions f2 = opts(2, 4, 0, 4);
      f2.hermitize = 1;
      f2.damping = 0.25;
      run("patch hermitize + damping", P, f2);
    }
  }
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
