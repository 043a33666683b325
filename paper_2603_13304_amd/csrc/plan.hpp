// Static execution plans for the BlockBP message update and expectation
// sweeps.  Every tensor shape is fixed by the geometry, chi and D, so the
// complete sweep -- canonical moves, merges, double-layer absorption,
// truncated splits, normalisation, message finalisation and the convergence
// distance -- is compiled once into lists of device operations.  Independent
// message updates ("lanes") are interleaved in "waves" so that one kernel
// launch serves the same operation of every lane: the k-th truncated SVD of
// each lane (the costly, latency-bound step) shares a launch with the k-th of
// every other lane, and the operations between two SVDs are matched by their
// position since the last one.
#pragma once
#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "geometry.hpp"
#include "kernels.hpp"

namespace pn {

// memory regions of the device arena (complex elements) and of the scalar
// array (doubles)
enum RegionId {
  RG_SITE = 0,   // ket tensors as given
  RG_SMAT,       // site tensors permuted for each absorption pattern
  RG_MSG0,       // message set 0
  RG_MSG1,       // message set 1
  RG_CONST,      // constants (the scalar 1)
  RG_RHO,        // carried expectation outputs
  RG_LANE0,      // per lane: chain tensors then scratch (lane L at RG_LANE0 + L)
};

struct Ref {
  int region = -1;
  int64_t off = 0;
  bool valid() const { return region >= 0; }
};

// scalar slots (doubles)
struct SRef {
  int64_t off = -1;
};

enum OpType { OPK_GEMM = 0, OPK_PERM, OPK_QR, OPK_JACOBI, OPK_OMEGA, OPK_NORM, OPK_PAD, OPK_PHASE, OPK_COLPHASE, OPK_CHOL, OPK_SUM, OPK_COUNT };

struct Op {
  int type = -1;
  Ref a, b, c, d;
  // GEMM: M N K lda ldb ldc opA opB prec ; PERM: rank, conj, dims[], perm[]
  // QR: m n lda conjT ; JACOBI: k ; OMEGA: n k ; NORM: len(i[0..1]) ;
  // CHOL: S n shift accumulate m ; SUM: S M N ldc (alpha in x[0..1])
  // PAD: l1 P r1 l2 r2 off_l off_r mode ; PHASE: nsites, then per site l P r D
  int64_t i[72] = {};
  double x[4] = {};   // GEMM alpha (re, im), beta (re, im); PAD sign
  uint64_t key = 0;
  SRef s0, s1;        // NORM: logscale, norm_out ; JACOBI: sigma
  std::vector<Ref> refs;  // PHASE sites
};

struct WaveKey {
  std::vector<int> k;
  bool operator<(const WaveKey& o) const { return k < o.k; }
};

struct LaneOps {
  std::vector<std::pair<WaveKey, Op>> ops;
};

struct PlanOptions {
  int chi = 8;
  int chi_env = 8;     // <= 0: no truncation inside the sweep
  int trunc = 0;       // 0: exact SVD (T1), 1: randomized range finder (T2)
  int q = 2, p = 8;
  int precision = PREC_FP64;
  uint64_t seed = 0;
  int d = 2;
  int D = 2;
  int order = 0;       // swallow order: 0 cost model, 1 merged run, 2 progressive
  int hermitize = 0;   // replace each new message by (A + A^dagger) / 2
  double damping = 0;  // 1 - alpha of the learning step (0: the new message alone)
};

// message storage layout (per slot: sites with cap shapes)
struct MsgLayout {
  std::vector<std::vector<int64_t>> off;   // [slot][site] element offset in the set
  std::vector<std::vector<int>> bl, br, P; // bond left/right, physical dim
  std::vector<std::vector<int>> D;         // ket dimension of each leg
  int64_t size = 0;
};

// pre-permuted site matrices
struct SiteMatKey {
  int tensor;
  std::vector<int> in_slots, out_slots;
  bool open;
  bool operator<(const SiteMatKey& o) const {
    return std::tie(tensor, in_slots, out_slots, open) <
           std::tie(o.tensor, o.in_slots, o.out_slots, o.open);
  }
};

struct Plan {
  std::vector<LaneOps> lanes;
  int nlanes = 0;
};

class Compiler {
 public:
  Compiler(const Problem& P, const PlanOptions& o);
  std::string error;

  // tensor layout
  std::vector<int64_t> tensor_off;                 // element offset of ket tensor t in RG_SITE
  std::vector<std::vector<int>> tensor_dims;       // [d, D0..D3] per tensor
  int64_t site_region_size = 0;
  MsgLayout msg;
  std::map<SiteMatKey, std::pair<Ref, Ref>> smat;  // (ket matrix, bra matrix)
  int64_t smat_size = 0;
  std::vector<Op> prep_ops;                        // builds RG_SMAT from RG_SITE

  // region sizes per lane (max over plans)
  std::vector<int64_t> lane_size;
  int64_t n_scalars = 0;
  int64_t rho_size = 0;

  // scalar layout: [0] sweep counter, [1, 1024) per-lane log-scale,
  // [1024, ...) per-message convergence distance
  static constexpr int64_t kSweepSlot = 0;
  int64_t err_slot(int m) const { return 1024 + m; }
  int64_t logscale_slot(int lane) const { return 1 + lane; }
  // site matrices (ket, bra) for a swallow pattern, created on first use
  std::pair<Ref, Ref> ensure_smat(int tensor, const std::vector<int>& in_slots,
                                  const std::vector<int>& out_slots, bool open);

  // plans
  bool build_sweep(int parity, Plan* out);                         // messages parity -> 1-parity
  bool build_expect(int parity, const std::vector<std::pair<int, int>>& bonds, Plan* out,
                    std::vector<std::vector<int>>* carry_order, std::vector<int64_t>* rho_off);

  const Problem& prob;
  PlanOptions opt;

 private:
  struct CSite {
    Ref buf;
    int l, P, r;
    int D;                       // ket dimension of the leg
    std::vector<int> carries;    // carried open sites
  };
  struct Lane;
  friend struct Lane;
};

}  // namespace pn
