// Executor and C ABI of the BlockBP engine (see include/pepsnet.h).
//
// A compiled plan (plan.hpp) is resolved into batched descriptor tables on
// the device: ops of all lanes are sorted by their wave key, every wave's
// ops are bucketed by kernel, and each bucket becomes one launch whose grid
// spans all its items.  A sweep is therefore a fixed list of launches that
// can be replayed directly or captured once into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pepsnet.h"
#include "geometry.hpp"
#include "kernels.hip"
#include "plan.hpp"
#include "sweep_count.hpp"

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define PN_HIP(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(BBP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

using namespace pn;

struct LaunchRec {
  int type = 0;
  int prec = 0;
  size_t desc_off = 0;   // byte offset into the descriptor blob
  int count = 0;
  dim3 grid;
  size_t lds = 0;
  int variant = 0;       // kernel variant (GEMM: tile shape; QR: 1 = blocked tall kernel, 2 = k_qr_small
                         // (144 x 16), 4 = k_qr_small (288 x 32), 3 =
                         // k_qr_mid (R only); Jacobi: 1 = rows
                         // split between LDS and the work buffer, 2 = top-k SVD through
                         // bidiagonalisation: k_svt_bidiag, k_svd_top, k_svd_back)
  int aux = 0;           // top-k SVD: the largest kept count (k_svd_back's grid)
  double gemm_flops = 0.0, contraction_flops = 0.0;
  double flops = 0.0;    // algorithmic flops of the launch (8 per complex MAC)
  double bytes = 0.0;    // algorithmic bytes moved (operands read once, results written once)
  int64_t shape[3] = {0, 0, 0};   // GEMM: largest M, N, K of the launch; QR / SVD: rows, cols
  int group = 0;         // stream group: launches of different groups share no data
};

struct Compiled {
  // device copy of the blob the launches' desc_off index (set when the blob
  // is uploaded; a list is only ever launched against its own blob)
  const char* desc = nullptr;
  std::vector<LaunchRec> launches;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  double gemm_flops = 0.0, contraction_flops = 0.0;
  int ngroups = 1;
};

// Launch groups of a sweep plan run on up to this many streams.
constexpr int kMaxStreams = 4;

}  // namespace

struct pepsnet_s {
  Problem P;
  PlanOptions opt;
  std::unique_ptr<Compiler> comp;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cplx* arena = nullptr;      // resident: sites, site matrices, messages, constants, rho
  int64_t arena_len = 0;
  cplx* work = nullptr;       // workspace: the lanes' chain and scratch regions
  int64_t work_len = 0;
  int64_t work_epoch = 0;     // bumped whenever the workspace moves
  const void* desc_work = nullptr;   // workspace address the descriptors were resolved against
  double* scal = nullptr;
  std::vector<int64_t> region_base;
  char* desc_dev = nullptr;
  size_t desc_cap = 0;
  std::vector<char> desc_host;
  Compiled prep, sweep[2], expect[2];
  // the plans' ops per lane, kept for batches and for re-resolving
  // descriptors when the workspace moves
  std::vector<std::vector<std::pair<WaveKey, Op>>> sweep_lanes[2], expect_lanes[2], prep_lanes;
  std::vector<std::vector<int>> carry_order[2];
  std::vector<int64_t> rho_off[2];
  std::vector<std::pair<int, int>> bonds;
  RhoDesc* rho_descs[2] = {nullptr, nullptr};
  cplx* rho_mat = nullptr;
  double* ss_dev = nullptr;
  int parity = 0;
  int64_t sweeps_total = 0;
  bool use_graph = false;
  // the lane groups of sweeps and expectations on the handle's stream and
  // the device's shared auxiliary streams (forked from and joined back into
  // the handle's stream by these events); the *_serial plans merge every
  // lane into shared launches for one stream
  int nstreams = kMaxStreams;
  hipEvent_t fork_ev = nullptr, join_ev[kMaxStreams - 1] = {};
  Compiled sweep_serial[2], expect_serial[2];
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double timed_ms = 0.0;
  int64_t timed_sweeps = 0;
  int64_t site_len = 0;
  double* pinned = nullptr;   // host pinned: [0] sweep counter, [1..] distances
  // expectation operators (blockbp_expect): up to kMaxOps 4x4 operators and
  // their values per bond; the default bond selection (identity)
  cplx* ops_dev = nullptr;
  cplx* ops_out = nullptr;
  // rho measures (blockbp_rho_measures): per bond, the (sweeps_total, edits)
  // at which its rho was last computed; edits counts site and message
  // replacements; device staging of bond ids, sigma and the results
  std::vector<std::pair<int64_t, int64_t>> rho_stamp;
  int64_t edits = 0;
  char* meas_dev = nullptr;
  const int32_t* sel_default = nullptr;
  // plans of bond subsets: the default plan's lanes of the chosen bonds
  // (their regions and rho slots are those of the default plan)
  struct Subset {
    Compiled plan[2];
    std::vector<char> blob;
    char* desc_dev = nullptr;
    size_t rho_off[2] = {0, 0};
    size_t sel_off = 0;
    int64_t epoch = -1;
  };
  std::map<std::vector<int>, Subset> subsets;
  // tile shape chosen by pepsnet_autotune per GEMM shape (prec, M, N, K,
  // opA, opB, scatter store); shapes not in it use the fixed rule
  std::map<std::array<int, 7>, int> gemm_tiles;
  // blockbp_sweep_noalloc: the sweep plans resolved against the device's
  // fixed workspace (compiled on its first call) and their descriptors
  int device = 0;
  Compiled sweep_fixed[2];
  char* blob_fixed = nullptr;   // pinned host copy of their descriptors
  size_t blob_fixed_len = 0;
  size_t fixed_need = 0;        // bytes of the array the sweep would use
  bool fixed_ready = false;
};
constexpr int kMaxOps = 64;

// ---- fixed workspace of blockbp_sweep_noalloc: a device array of the code
// object, so that a sweep through it allocates nothing.  It holds one
// sweep's workspace followed by that sweep's launch descriptors.  Each
// device has its own copy at its own address, looked up with
// hipGetSymbolAddress while the device is current: in host code the array's
// name is not a device address and is never passed to a kernel.
constexpr size_t kFixedBytes = size_t(PEPSNET_NOALLOC_MAX_BYTES);
static __device__ __align__(256) char scratch[kFixedBytes];
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
char* g_fixed_ptr[kMaxDevices] = {};

// Once per device, with that device current (called by pepsnet_create).
int32_t resolve_fixed(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BBP_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (g_fixed_ptr[dev]) return BBP_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(BBP_EDEVICE, std::string("fixed workspace address: ") + hipGetErrorString(e));
  g_fixed_ptr[dev] = static_cast<char*>(p);
  return BBP_OK;
}

__global__ void k_fill_zero(uint4* p, int64_t n) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = z;
}


// ---- serving loop
struct SrvReq {
  uint64_t ticket = 0;
  pepsnet_s* h = nullptr;
  std::vector<double> sites;   // new site tensors (empty: unchanged)
  double tol = 0.0;
  int max_sweeps = 0;
  int sweeps = 0;
  double err = INFINITY;
  int phase = 0;               // 0 queued, 1 sweeping, 2 expectation, 3 done (worker only)
  bool ready = false;          // finished and retired (guarded by the server mutex)
  int32_t rc = BBP_OK;
  bool own_work = false;       // a server slot is bound to the state for this request
  std::vector<double> ss;
  double energy = 0.0;
  std::chrono::steady_clock::time_point t_submit, t_done;
  hipEvent_t ev = nullptr;
  struct SrvSlot* slot = nullptr;   // server workspace slot bound for the request
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;   // the request's device-side window
  double window_ms[2] = {NAN, NAN};
};

// A workspace buffer of the serving loop.  Slots are allocated while the
// pool grows (at most max_inflight of them within the HBM budget) and then
// kept: admitting a request binds a free slot to the state, which re-resolves
// the state's launch descriptors only if they point at another address, so
// steady-state admission and completion allocate and free nothing.
struct SrvSlot {
  cplx* ptr = nullptr;
  int64_t bytes = 0;
  bool busy = false;
  const void* last = nullptr;   // state it was last bound to (compared, never dereferenced)
};

struct bbp_server_s {
  int64_t budget = 0;
  int max_inflight = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SrvReq*> queue;
  std::vector<SrvReq*> inflight;
  std::map<uint64_t, SrvReq*> reqs;   // submitted and not yet collected
  uint64_t next_ticket = 1;
  int64_t in_use = 0, peak_in_use = 0;   // bytes of workspace slots held
  int peak_inflight = 0;
  int64_t completed = 0;
  std::atomic<int64_t> slot_allocs{0};
  std::vector<std::unique_ptr<SrvSlot>> slots;   // touched by the worker thread only
  hipEvent_t ev_ref = nullptr;   // origin of the requests' device windows
  bool stop = false;
  std::thread worker;
};

// A batch merges the sweep plans of several handles into one launch
// sequence: ops of every handle at the same wave key share a launch.
// Variant v of the merged plan runs handle i on message set
// base_parity[i] ^ v.
struct pepsnet_batch_s {
  std::vector<pepsnet_s*> hs;
  std::vector<int> base_parity;
  std::vector<int64_t> work_epoch;
  Compiled sweep[2];
  std::vector<char> desc_host[2];
  char* desc_dev[2] = {nullptr, nullptr};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool use_graph = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
};

namespace {

cplx* resolve(pepsnet_s* h, const Ref& r) {
  if (!r.valid()) return nullptr;
  if (r.region >= RG_LANE0) return h->work + h->region_base[r.region] + r.off;
  return h->arena + h->region_base[r.region] + r.off;
}

template <class T>
size_t push_descs(std::vector<char>* blob, const std::vector<T>& v) {
  size_t off = (blob->size() + 255) / 256 * 256;
  blob->resize(off + v.size() * sizeof(T));
  std::memcpy(blob->data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

// kernel variant an op runs with (part of its bucket key, so that an item
// runs the same kernel whether it is launched alone or in a batch)
std::array<int, 7> gemm_key(const Op& op) {
  return {int(op.i[8]), int(op.i[0]), int(op.i[1]), int(op.i[2]), int(op.i[6]), int(op.i[7]),
          op.i[10] > 0 ? 1 : 0};
}

int op_variant(const pepsnet_s* h, const Op& op) {
  if (op.type == OPK_GEMM) {   // k_gemm tile shape: the tuned one, else by M and N
    if (h && !h->gemm_tiles.empty()) {
      auto it = h->gemm_tiles.find(gemm_key(op));
      if (it != h->gemm_tiles.end()) return it->second;
    }
    const int64_t M = op.i[0], N = op.i[1];
    if (M <= 16) return 1;
    if (N <= 16) return 2;
    if (N > 64 && N <= 80) return 3;
    if (M > 64 && M <= 80) return 4;
    return 0;
  }
  if (op.type == OPK_QR) {
    // QRK_CHOL shapes are expanded by the plan compiler; the blocked tall
    // kernel takes any that reach here
    const int v = qr_kernel(op.i[0], op.i[1], op.c.valid());
    return v == QRK_CHOL ? QRK_TALL : v;
  }
  if (op.type == OPK_CHOL) return op.i[1] <= CHB_N ? 1 : 0;   // k_chol_b / k_chol
  if (op.type == OPK_JACOBI) {
    if (op.i[5]) return 2;   // k_svd_top
    const int rows = int(op.i[0]), cols = int(op.i[1]);
    return jacobi_lds_slices(rows, cols) < (rows + 15) / 16 ? 1 : 0;
  }
  return 0;
}

typedef std::vector<std::vector<std::pair<WaveKey, Op>>> LaneList;
struct OpSource {
  pepsnet_s* h;          // resolves the op's references
  const LaneList* lanes;
  const std::vector<int>* groups = nullptr;   // stream group per lane (none: all 0)
};

// Stream groups of a plan whose lanes share no data: the message updates of
// a sweep (each reads the previous sweep's messages and writes its own
// message slot) and the bonds of an expectation (each writes its own rho
// block).  Lanes with the same sequence of (wave key, op kind) form a class
// whose ops merge into shared launches; class c runs in group c mod
// kMaxStreams.  A plan in which a workspace region is referenced by more
// than one lane, or a lane references more than one, stays in one group.
std::vector<int> lane_groups(const LaneList& lanes) {
  std::vector<int> g(lanes.size(), 0);
  std::map<int, size_t> owner;
  for (size_t L = 0; L < lanes.size(); ++L) {
    int mine = -1;
    for (const auto& ko : lanes[L]) {
      const Op& op = ko.second;
      std::vector<Ref> rs = {op.a, op.b, op.c, op.d};
      rs.insert(rs.end(), op.refs.begin(), op.refs.end());
      for (const Ref& r : rs) {
        if (r.region < RG_LANE0) continue;
        if (mine >= 0 && r.region != mine) return g;
        mine = r.region;
      }
    }
    if (mine < 0) continue;
    auto it = owner.find(mine);
    if (it != owner.end() && it->second != L) return g;
    owner[mine] = L;
  }
  std::map<std::vector<std::pair<std::vector<int>, int>>, int> cls;
  for (size_t L = 0; L < lanes.size(); ++L) {
    std::vector<std::pair<std::vector<int>, int>> sig;
    sig.reserve(lanes[L].size());
    for (const auto& ko : lanes[L]) sig.push_back({ko.first.k, int(ko.second.type)});
    auto it = cls.find(sig);
    if (it == cls.end()) it = cls.emplace(std::move(sig), int(cls.size())).first;
    g[L] = it->second % kMaxStreams;
  }
  return g;
}

// Bucket the ops of every source by wave key, then by (kind, precision,
// variant), and emit one launch per bucket with its descriptors in `blob`.
void compile_ops(const std::vector<OpSource>& srcs, std::vector<char>* blob, Compiled* out) {
  // (wave key, source, lane, op index)
  std::vector<std::tuple<WaveKey, int, int, int>> all;
  auto group_of = [&](int S, int L) {
    return srcs[S].groups ? (*srcs[S].groups)[L] : 0;
  };
  for (size_t S = 0; S < srcs.size(); ++S) {
    const LaneList& lanes = *srcs[S].lanes;
    for (size_t L = 0; L < lanes.size(); ++L)
      for (size_t k = 0; k < lanes[L].size(); ++k)
        all.emplace_back(lanes[L][k].first, int(S), int(L), int(k));
  }
  std::stable_sort(all.begin(), all.end(), [](const auto& a, const auto& b) {
    return std::get<0>(a) < std::get<0>(b);
  });
  size_t i = 0;
  while (i < all.size()) {
    size_t j = i;
    while (j < all.size() && !(std::get<0>(all[i]) < std::get<0>(all[j])) &&
           !(std::get<0>(all[j]) < std::get<0>(all[i])))
      ++j;
    std::map<std::tuple<int, int, int, int>, std::vector<std::pair<pepsnet_s*, const Op*>>> buckets;
    for (size_t t = i; t < j; ++t) {
      const OpSource& src = srcs[std::get<1>(all[t])];
      const Op& op = (*src.lanes)[std::get<2>(all[t])][std::get<3>(all[t])].second;
      int prec = op.type == OPK_GEMM ? int(op.i[8]) : 0;
      const int grp = group_of(std::get<1>(all[t]), std::get<2>(all[t]));
      buckets[{grp, op.type, prec, op_variant(src.h, op)}].push_back({src.h, &op});
    }
    for (auto& bk : buckets) {
      LaunchRec rec;
      rec.group = std::get<0>(bk.first);
      rec.type = std::get<1>(bk.first);
      rec.prec = std::get<2>(bk.first);
      rec.variant = std::get<3>(bk.first);
      out->ngroups = std::max(out->ngroups, rec.group + 1);
      rec.count = int(bk.second.size());
      const auto& ops = bk.second;
      switch (rec.type) {
        case OPK_GEMM: {
          std::vector<GemmDesc> v;
          int64_t mM = 1, mN = 1;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            GemmDesc g;
            g.A = resolve(h, op->a); g.B = resolve(h, op->b); g.C = resolve(h, op->c);
            g.M = int(op->i[0]); g.N = int(op->i[1]); g.K = int(op->i[2]);
            g.lda = int(op->i[3]); g.ldb = int(op->i[4]); g.ldc = int(op->i[5]);
            g.opA = int(op->i[6]); g.opB = int(op->i[7]);
            g.alpha = cplx{op->x[0], op->x[1]};
            g.beta = cplx{op->x[2], op->x[3]};
            g.sc_n = int(op->i[10]); g.sc_nr = int(op->i[11]); g.sc_conj = int(op->i[12]);
            for (int k = 0; k < GEMM_SC_MAX; ++k) {
              g.sc_dim[k] = k < g.sc_n ? int(op->i[16 + k]) : 1;
              g.sc_inv[k] = 1.0 / g.sc_dim[k];
              g.sc_ds[k] = k < g.sc_n ? op->i[32 + k] : 0;
            }
            mM = std::max<int64_t>(mM, g.M);
            mN = std::max<int64_t>(mN, g.N);
            rec.shape[0] = mM;
            rec.shape[1] = mN;
            rec.shape[2] = std::max<int64_t>(rec.shape[2], g.K);
            double f = 8.0 * double(g.M) * double(g.N) * double(g.K);
            rec.gemm_flops += f;
            rec.flops += f;
            rec.bytes += 16.0 * (double(g.M) * g.K + double(g.K) * g.N + double(g.M) * g.N);
            if (op->i[9]) rec.contraction_flops += f;
            v.push_back(g);
          }
          rec.desc_off = push_descs(blob, v);
          const int tm = rec.variant == 1 ? 16 : rec.variant == 4 ? 80 : 64;
          const int tn = rec.variant == 2 ? 16 : rec.variant == 3 ? 80 : 64;
          rec.grid = dim3(unsigned((mN + tn - 1) / tn),
                          unsigned(std::min<int64_t>(65535, (mM + tm - 1) / tm)), unsigned(v.size()));
          break;
        }
        case OPK_PERM: {
          std::vector<PermDesc> v;
          int64_t mt = 1;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            PermDesc p;
            std::memset(&p, 0, sizeof p);
            p.src = resolve(h, op->a); p.dst = resolve(h, op->b);
            p.rank = int(op->i[0]); p.conj = int(op->i[1]);
            p.total = 1;
            for (int k = 0; k < p.rank; ++k) {
              p.dims[k] = int(op->i[2 + k]);
              p.stride[k] = op->i[18 + k];
              p.inv[k] = 1.0 / p.dims[k];
              p.total *= p.dims[k];
            }
            mt = std::max(mt, p.total);
            rec.bytes += 32.0 * double(p.total);
            v.push_back(p);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(std::min<int64_t>(4096, (mt + 255) / 256)), unsigned(v.size()));
          break;
        }
        case OPK_QR: {
          std::vector<QrDesc> v;
          int64_t lds_elems = 0;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            QrDesc q;
            q.A = resolve(h, op->a); q.work = resolve(h, op->b);
            q.Q = resolve(h, op->c); q.R = resolve(h, op->d);
            q.m = int(op->i[0]); q.n = int(op->i[1]); q.lda = int(op->i[2]); q.conjT = int(op->i[3]);
            q.qh = int(op->i[4]);
            rec.shape[0] = std::max<int64_t>(rec.shape[0], q.m);
            rec.shape[1] = std::max<int64_t>(rec.shape[1], q.n);
            double m = q.m, n = q.n, k = std::min(q.m, q.n);
            // Householder R (complex: 8 flops per MAC), plus the same again
            // for the explicit Q
            double fr = 8.0 * 2.0 * (m * n * k - (m + n) * k * k / 2.0 + k * k * k / 3.0);
            rec.flops += q.Q ? 2.0 * fr : fr;
            rec.bytes += 16.0 * (m * n + (q.Q ? m * k : 0.0) + k * n);
            int64_t need = int64_t(q.m) * (q.n + (q.Q ? std::min(q.m, q.n) : 0));
            if (need <= QR_LDS_MAX) lds_elems = std::max(lds_elems, need);
            v.push_back(q);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(v.size()));
          // blocked kernel (panel in LDS) for working copies that overflow LDS;
          // k_qr_small and k_qr_mid use static LDS only
          rec.lds = rec.variant == 1 ? size_t(QRT_LDS) * sizeof(cplx)
                  : rec.variant >= 2 ? 0 : size_t(lds_elems) * sizeof(cplx);
          break;
        }
        case OPK_JACOBI: {
          std::vector<JacobiDesc> v;
          int64_t lds_elems = 0;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            JacobiDesc jd;
            jd.A = resolve(h, op->a); jd.work = resolve(h, op->b); jd.U = resolve(h, op->c);
            jd.sigma = reinterpret_cast<double*>(resolve(h, op->d));
            jd.rows = int(op->i[0]); jd.cols = int(op->i[1]); jd.lda = int(op->i[2]);
            jd.conjT = int(op->i[3]); jd.keep = int(op->i[4]); jd.gauge = int(op->i[6]);
            rec.shape[0] = std::max<int64_t>(rec.shape[0], jd.rows);
            rec.shape[1] = std::max<int64_t>(rec.shape[1], jd.cols);
            if (rec.variant == 2) {
              // complex Householder bidiagonalisation, 4 x (4 m n^2 - 4 n^3 / 3)
              const double m = jd.rows, n = jd.cols;
              rec.flops += 16.0 * (m * n * n - n * n * n / 3.0);
            } else {
              const int nl = jacobi_lds_slices(jd.rows, jd.cols);
              lds_elems = std::max<int64_t>(lds_elems, int64_t(nl) * 16 * jd.cols);
              // one sweep of cols(cols-1)/2 rotations, each three length-rows dot
              // products (a, b, g: 2 + 2 + 4 real flops per row) and the update
              // of two columns (2 x 8 per row): the count of one sweep, the
              // minimum any converged run performs
              rec.flops += 0.5 * jd.cols * (jd.cols - 1.0) * 24.0 * jd.rows;
            }
            rec.bytes += 16.0 * (double(jd.rows) * jd.cols + double(jd.rows) * jd.keep);
            rec.aux = std::max(rec.aux, jd.keep);
            v.push_back(jd);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(v.size()));
          rec.lds = size_t(lds_elems) * sizeof(cplx);
          break;
        }
        case OPK_OMEGA: {
          std::vector<OmegaDesc> v;
          int64_t mt = 1;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            OmegaDesc o;
            o.out = resolve(h, op->a);
            o.n = int(op->i[0]); o.k = int(op->i[1]);
            o.prefix = op->key;
            o.last_tag = op->i[2] ? h->scal + Compiler::kSweepSlot : nullptr;
            mt = std::max<int64_t>(mt, int64_t(o.n) * o.k);
            rec.bytes += 16.0 * double(o.n) * o.k;
            v.push_back(o);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(std::min<int64_t>(1024, (mt + 255) / 256)), unsigned(v.size()));
          break;
        }
        case OPK_NORM: {
          std::vector<NormDesc> v;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            NormDesc nd;
            nd.x = resolve(h, op->a);
            nd.len = op->i[0];
            rec.bytes += 32.0 * double(nd.len);
            nd.logscale = op->s0.off >= 0 ? h->scal + op->s0.off : nullptr;
            nd.norm_out = op->s1.off >= 0 ? h->scal + op->s1.off : nullptr;
            nd.part = reinterpret_cast<double*>(resolve(h, op->b));
            v.push_back(nd);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(NORM_CHUNKS), unsigned(v.size()));
          break;
        }
        case OPK_PAD: {
          std::vector<PadDesc> v;
          int64_t mt = 1;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            PadDesc p;
            p.src = resolve(h, op->a); p.dst = resolve(h, op->b);
            p.l1 = int(op->i[0]); p.P = int(op->i[1]); p.r1 = int(op->i[2]);
            p.l2 = int(op->i[3]); p.r2 = int(op->i[4]);
            p.off_l = int(op->i[5]); p.off_r = int(op->i[6]); p.mode = int(op->i[7]);
            p.sign = op->x[0];
            mt = std::max<int64_t>(mt, int64_t(p.l2) * p.P * p.r2);
            rec.bytes += 16.0 * (double(p.l1) * p.P * p.r1 + double(p.l2) * p.P * p.r2);
            v.push_back(p);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(std::min<int64_t>(4096, (mt + 255) / 256)), unsigned(v.size()));
          break;
        }
        case OPK_SUM: {
          std::vector<SumDesc> v;
          int64_t mt = 1;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            SumDesc sd;
            sd.P = resolve(h, op->a); sd.C = resolve(h, op->c);
            sd.S = int(op->i[0]); sd.M = int(op->i[1]); sd.N = int(op->i[2]);
            sd.ldc = int(op->i[3]);
            sd.alpha = cplx{op->x[0], op->x[1]};
            mt = std::max<int64_t>(mt, int64_t(sd.M) * sd.N);
            rec.bytes += 16.0 * double(sd.M) * sd.N * (sd.S + 1.0);
            v.push_back(sd);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(std::min<int64_t>(1024, (mt + 255) / 256)), unsigned(v.size()));
          break;
        }
        case OPK_CHOL: {
          std::vector<CholDesc> v;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            CholDesc c;
            c.G = resolve(h, op->a); c.Rinv = resolve(h, op->b); c.R = resolve(h, op->c);
            c.S = int(op->i[0]); c.n = int(op->i[1]); c.shift = int(op->i[2]);
            c.accumulate = int(op->i[3]); c.m = op->i[4];
            rec.shape[0] = std::max<int64_t>(rec.shape[0], c.m);
            rec.shape[1] = std::max<int64_t>(rec.shape[1], c.n);
            const double n = c.n;
            // Cholesky, triangular inverse, and the running factor's product
            // (n^3 / 3 complex multiply-adds each), 8 flops per complex MAC
            rec.flops += 8.0 * (n * n * n / 3.0) * (c.accumulate ? 3.0 : 2.0);
            rec.bytes += 16.0 * n * n * (double(c.S) + 2.0 + (c.accumulate ? 2.0 : 0.0));
            v.push_back(c);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(v.size()));
          break;
        }
        case OPK_COLPHASE: {
          std::vector<ColPhaseDesc> v;
          int kmax = 1;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            ColPhaseDesc c;
            c.L = resolve(h, op->a); c.R = resolve(h, op->b);
            c.m = int(op->i[0]); c.keep = int(op->i[1]); c.n = int(op->i[2]);
            kmax = std::max(kmax, c.keep);
            v.push_back(c);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(v.size()), unsigned((kmax + 3) / 4));
          break;
        }
        case OPK_PHASE: {
          std::vector<PhaseDesc> v;
          for (const auto& ho : ops) {
            pepsnet_s* h = ho.first;
            const Op* op = ho.second;
            PhaseDesc p;
            std::memset(&p, 0, sizeof p);
            p.nsites = int(op->i[0]);
            for (int s = 0; s < p.nsites; ++s) {
              p.sites[s] = resolve(h, op->refs[s]);
              p.l[s] = int(op->i[1 + 4 * s]);
              p.P[s] = int(op->i[2 + 4 * s]);
              p.r[s] = int(op->i[3 + 4 * s]);
              p.D[s] = int(op->i[4 + 4 * s]);
            }
            v.push_back(p);
          }
          rec.desc_off = push_descs(blob, v);
          rec.grid = dim3(unsigned(v.size()));
          break;
        }
      }
      out->gemm_flops += rec.gemm_flops;
      out->contraction_flops += rec.contraction_flops;
      out->launches.push_back(rec);
    }
    i = j;
  }
}

// part: -1 every kernel of the record; 0 / 1 only the first / second kernel
// of a two-kernel record (the top-k SVD), for per-kernel timing
hipError_t launch(const char* desc_dev, hipStream_t stream, const LaunchRec& r, int part = -1) {
  const void* d = desc_dev + r.desc_off;
  dim3 blk(256);
  switch (r.type) {
    case OPK_GEMM: {
      // variant = tile shape: 0 64x64, 1 16x64 (M <= 16), 2 64x16 (N <= 16),
      // 3 64x80 (64 < N <= 80), 4 80x64 (64 < M <= 80)
      const GemmDesc* gd = (const GemmDesc*)d;
#define PN_GEMM(PP)                                                                         \
  if (r.variant == 1) hipLaunchKernelGGL((k_gemm<PP, 1>), r.grid, blk, 0, stream, gd);      \
  else if (r.variant == 2) hipLaunchKernelGGL((k_gemm<PP, 2>), r.grid, blk, 0, stream, gd); \
  else if (r.variant == 3) hipLaunchKernelGGL((k_gemm<PP, 3>), r.grid, blk, 0, stream, gd); \
  else if (r.variant == 4) hipLaunchKernelGGL((k_gemm<PP, 4>), r.grid, blk, 0, stream, gd); \
  else hipLaunchKernelGGL((k_gemm<PP, 0>), r.grid, blk, 0, stream, gd);
      if (r.prec == PREC_FP64) {
        PN_GEMM(PREC_FP64)
      } else if (r.prec == PREC_FP32) {
        PN_GEMM(PREC_FP32)
      } else {
        PN_GEMM(PREC_BF16X3)
      }
#undef PN_GEMM
      break;
    }
    case OPK_PERM:
      hipLaunchKernelGGL(k_permute, r.grid, blk, 0, stream, (const PermDesc*)d);
      break;
    case OPK_QR:
      if (r.variant == 2)
        hipLaunchKernelGGL((k_qr_small<9, 16>), r.grid, dim3(256), 0, stream, (const QrDesc*)d);
      else if (r.variant == 4)
        hipLaunchKernelGGL((k_qr_small<18, 32>), r.grid, dim3(512), 0, stream, (const QrDesc*)d);
      else if (r.variant == 3)
        hipLaunchKernelGGL(k_qr_mid, r.grid, dim3(QRM_THREADS), 0, stream, (const QrDesc*)d);
      else if (r.variant)
        hipLaunchKernelGGL(k_qr_tall, r.grid, dim3(QRT_THREADS), r.lds, stream,
                           (const QrDesc*)d);
      else
        hipLaunchKernelGGL(k_qr, r.grid, blk, r.lds, stream, (const QrDesc*)d);
      break;
    case OPK_JACOBI:
      if (r.variant == 2) {
        if (part != 1)
          hipLaunchKernelGGL(k_svt_bidiag, r.grid, dim3(SVB_THREADS), 0, stream, (const JacobiDesc*)d);
        if (part != 0) {
          hipLaunchKernelGGL(k_svd_top, r.grid, dim3(SVT_THREADS), 0, stream, (const JacobiDesc*)d);
          const dim3 gb(unsigned((r.aux + SVK_VALS - 1) / SVK_VALS), r.grid.x);
          hipLaunchKernelGGL(k_svd_back, gb, dim3(256), 0, stream, (const JacobiDesc*)d);
        }
      }
      else if (r.variant)
        hipLaunchKernelGGL(k_jacobi<true>, r.grid, dim3(JAC_THREADS), r.lds, stream,
                           (const JacobiDesc*)d);
      else
        hipLaunchKernelGGL(k_jacobi<false>, r.grid, dim3(JAC_THREADS), r.lds, stream,
                           (const JacobiDesc*)d);
      break;
    case OPK_OMEGA:
      hipLaunchKernelGGL(k_omega, r.grid, blk, 0, stream, (const OmegaDesc*)d);
      break;
    case OPK_NORM:
      hipLaunchKernelGGL(k_norm_partial, r.grid, blk, 0, stream, (const NormDesc*)d);
      hipLaunchKernelGGL(k_norm_apply, r.grid, blk, 0, stream, (const NormDesc*)d);
      break;
    case OPK_PAD:
      hipLaunchKernelGGL(k_pad, r.grid, blk, 0, stream, (const PadDesc*)d);
      break;
    case OPK_PHASE:
      hipLaunchKernelGGL(k_phase, r.grid, blk, 0, stream, (const PhaseDesc*)d);
      break;
    case OPK_COLPHASE:
      hipLaunchKernelGGL(k_colphase, r.grid, blk, 0, stream, (const ColPhaseDesc*)d);
      break;
    case OPK_CHOL:
      // blocked form up to 80 columns, packed column-by-column form above
      if (r.variant == 1)
        hipLaunchKernelGGL(k_chol_b, r.grid, dim3(CHOL_THREADS), 0, stream, (const CholDesc*)d);
      else
        hipLaunchKernelGGL(k_chol, r.grid, dim3(CHOL_THREADS), 0, stream, (const CholDesc*)d);
      break;
    case OPK_SUM:
      hipLaunchKernelGGL(k_sum_parts, r.grid, blk, 0, stream, (const SumDesc*)d);
      break;
  }
  return hipGetLastError();
}

// Streams for the launch groups of a plan: group 0 on `main`, group g > 0 on
// aux[g - 1], forked from and joined back into `main` by events.
struct GroupStreams {
  int n = 1;
  const hipStream_t* aux = nullptr;
  hipEvent_t fork = nullptr;
  const hipEvent_t* join = nullptr;
};

// held while a plan's lane groups are enqueued on the shared auxiliary
// streams (directly or into a graph capture), so that the work of two host
// threads never interleaves on them and no capture takes in another
// thread's launches
std::mutex g_aux_issue_mu;

// Enqueue every launch of c in list order; with gs, group g goes to stream
// g mod ns (ns = the streams in use, 0 = `main`), so each lane's ops keep
// their order.
hipError_t issue(const char* desc_dev, hipStream_t main, const Compiled* c,
                 const GroupStreams* gs) {
  const int ns = gs ? std::max(1, std::min(gs->n, c->ngroups)) : 1;
  hipError_t e = hipSuccess;
  if (ns > 1) {
    if ((e = hipEventRecord(gs->fork, main)) != hipSuccess) return e;
    for (int g = 1; g < ns; ++g)
      if ((e = hipStreamWaitEvent(gs->aux[g - 1], gs->fork, 0)) != hipSuccess) return e;
  }
  for (const LaunchRec& r : c->launches) {
    const int q = r.group % ns;
    e = launch(desc_dev, q > 0 ? gs->aux[q - 1] : main, r);
    if (e != hipSuccess) break;
  }
  // join even after a failed launch, so that a capture can end cleanly
  for (int g = 1; g < ns; ++g) {
    hipError_t e2 = hipEventRecord(gs->join[g - 1], gs->aux[g - 1]);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(main, gs->join[g - 1], 0);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

int32_t run_launches(hipStream_t stream, Compiled* c, bool graph,
                     const GroupStreams* gs = nullptr) {
  const char* desc_dev = c->desc;
  if (!desc_dev) return fail(BBP_EDEVICE, "launch list without uploaded descriptors");
  if (graph) {
    if (!c->exec) {
      std::unique_lock<std::mutex> lk(g_aux_issue_mu, std::defer_lock);
      if (gs && c->ngroups > 1 && gs->n > 1) lk.lock();
      PN_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      {
        hipError_t e = issue(desc_dev, stream, c, gs);
        if (e != hipSuccess) {
          // end the capture (the stream must leave capture mode) and drop
          // the partial graph it returns
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(stream, &g);
          if (g) (void)hipGraphDestroy(g);
          return fail(BBP_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
        }
      }
      hipError_t e = hipStreamEndCapture(stream, &c->graph);
      if (e == hipSuccess) e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
        c->exec = nullptr;
        return fail(BBP_EDEVICE, std::string("graph: ") + hipGetErrorString(e));
      }
    }
    PN_HIP(hipGraphLaunch(c->exec, stream));
    return BBP_OK;
  }
  std::unique_lock<std::mutex> lk(g_aux_issue_mu, std::defer_lock);
  if (gs && c->ngroups > 1 && gs->n > 1) lk.lock();
  hipError_t e = issue(desc_dev, stream, c, gs);
  if (e != hipSuccess) return fail(BBP_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  return BBP_OK;
}

// Auxiliary streams for the extra lane groups, shared by every handle on a
// device (one stream per handle keeps the handles' own streams spread over
// the hardware queues), made on first use and kept until the process ends.
struct AuxStreams {
  hipStream_t s[kMaxStreams - 1] = {};
};
std::mutex g_aux_mu;
std::map<int, AuxStreams> g_aux;

const hipStream_t* aux_streams(int dev) {
  std::lock_guard<std::mutex> lk(g_aux_mu);
  auto it = g_aux.find(dev);
  if (it != g_aux.end()) return it->second.s;
  AuxStreams a;
  for (int g = 0; g < kMaxStreams - 1; ++g)
    if (hipStreamCreateWithFlags(&a.s[g], hipStreamNonBlocking) != hipSuccess) {
      for (int k = 0; k < g; ++k) (void)hipStreamDestroy(a.s[k]);
      return nullptr;
    }
  return g_aux.emplace(dev, a).first->second.s;
}

// Run a plan on the handle's stream; a plan with several lane groups (and a
// handle allowed more than one stream) spreads them over the auxiliary
// streams too.
int32_t run_compiled(pepsnet_s* h, Compiled* c, bool allow_graph) {
  GroupStreams gs;
  const GroupStreams* use = nullptr;
  if (h->nstreams > 1 && c->ngroups > 1 && h->fork_ev) {
    gs.aux = aux_streams(h->device);
    if (!gs.aux) return fail(BBP_EDEVICE, "stream creation failed");
    gs.n = h->nstreams;
    gs.fork = h->fork_ev;
    gs.join = h->join_ev;
    use = &gs;
  }
  return run_launches(h->stream, c, allow_graph && h->use_graph, use);
}

std::string build_problem(const pepsnet_desc* d, Problem* P) {
  if (d->lattice == BBP_KAGOME_OPEN) return build_finite(P, d->Lx, d->Ly, d->bLx, d->bLy);
  if (d->lattice == BBP_KAGOME_INF_HEX) return build_hex(P, d->hex_N);
  return "unknown lattice";
}

int32_t check_desc(const pepsnet_desc* d) {
  if (!d) return fail(BBP_EINVAL, "null descriptor");
  if (d->abi_version != PEPSNET_ABI_VERSION) return fail(BBP_EINVAL, "ABI version mismatch");
  if (d->d != 2) return fail(BBP_EINVAL, "physical dimension must be 2 (spin 1/2)");
  if (d->D < 1 || d->D > 16) return fail(BBP_EINVAL, "D must be in [1, 16]");
  if (d->chi < 1 || d->chi > 256) return fail(BBP_EINVAL, "chi must be in [1, 256]");
  if (d->chi_env != d->chi && d->chi_env != 0)
    return fail(BBP_EINVAL, "chi_env must equal chi, or be 0 (exact contraction of the block)");
  if (d->hbm_budget_bytes < 0) return fail(BBP_EINVAL, "negative HBM budget");
  if (d->swallow_order < 0 || d->swallow_order > 2) return fail(BBP_EINVAL, "bad swallow order");
  if (d->hermitize != 0 && d->hermitize != 1) return fail(BBP_EINVAL, "hermitize must be 0 or 1");
  if (!(d->damping >= 0.0 && d->damping < 1.0)) return fail(BBP_EINVAL, "damping must be in [0, 1)");
  if ((d->hermitize || d->damping > 0.0) && d->chi > 72)
    return fail(BBP_EINVAL, "hermitize and damping need chi <= 72 (exact SVDs of 2 chi columns)");
  if (d->precision < 0 || d->precision > 2) return fail(BBP_EINVAL, "bad precision");
  if (d->trunc < 0 || d->trunc > 1) return fail(BBP_EINVAL, "bad truncation mode");
  if (d->rsvd_q < 0 || d->rsvd_q > 8 || d->rsvd_p < 0 || d->rsvd_p > 64)
    return fail(BBP_EINVAL, "bad randomized SVD parameters");
  return BBP_OK;
}

int32_t upload_sites(pepsnet_s* h, const double* sites, int64_t len) {
  if (!sites || len != 2 * h->comp->site_region_size)
    return fail(BBP_EINVAL, "site tensor buffer has the wrong length (expected " +
                                std::to_string(2 * h->comp->site_region_size) + " doubles)");
  for (int64_t i = 0; i < len; ++i)
    if (!std::isfinite(sites[i])) return fail(BBP_ENUMERIC, "non-finite site tensor entry");
  PN_HIP(hipMemcpyAsync(h->arena + h->region_base[RG_SITE], sites, len * sizeof(double),
                        hipMemcpyHostToDevice, h->stream));
  int32_t rc = run_compiled(h, &h->prep, false);
  if (rc) return rc;
  h->edits += 1;
  PN_HIP(hipStreamSynchronize(h->stream));
  return BBP_OK;
}

int32_t reset_messages(pepsnet_s* h) {
  const MsgLayout& M = h->comp->msg;
  std::vector<double> buf(2 * M.size, 0.0);
  for (size_t m = 0; m < M.off.size(); ++m)
    for (size_t j = 0; j < M.off[m].size(); ++j) {
      int D = M.D[m][j], P = M.P[m][j], r = M.br[m][j];
      double v = 1.0 / std::sqrt(double(D));
      for (int k = 0; k < D; ++k) buf[2 * (M.off[m][j] + int64_t(k * D + k) * r)] = v;
      (void)P;
    }
  h->parity = 0;
  h->edits += 1;
  PN_HIP(hipMemcpyAsync(h->arena + h->region_base[RG_MSG0], buf.data(), buf.size() * sizeof(double),
                        hipMemcpyHostToDevice, h->stream));
  PN_HIP(hipStreamSynchronize(h->stream));
  return BBP_OK;
}


// ---- asynchronous sweep / expectation steps (the serving loop's units of
// work): enqueue on the handle's stream, record `ev`, finish once it fired.
int32_t enqueue_sweep(pepsnet_s* h, hipEvent_t ev) {
  const int nm = int(h->P.msg_keys.size());
  h->pinned[0] = double(h->sweeps_total);
  PN_HIP(hipMemcpyAsync(h->scal + Compiler::kSweepSlot, h->pinned, sizeof(double),
                        hipMemcpyHostToDevice, h->stream));
  int32_t rc = run_compiled(h, &h->sweep_serial[h->parity], true);
  if (rc) return rc;
  PN_HIP(hipMemcpyAsync(h->pinned + 1, h->scal + h->comp->err_slot(0), nm * sizeof(double),
                        hipMemcpyDeviceToHost, h->stream));
  PN_HIP(hipEventRecord(ev, h->stream));
  return BBP_OK;
}

int32_t finish_sweep(pepsnet_s* h, double* err) {
  const int nm = int(h->P.msg_keys.size());
  if (!close_sweep(&h->parity, &h->sweeps_total, h->pinned + 1, nm, err))
    return fail(BBP_ENUMERIC, "non-finite message after a sweep");
  return BBP_OK;
}

int32_t enqueue_expect(pepsnet_s* h, hipEvent_t ev) {
  const int nm = int(h->P.msg_keys.size()), nb = int(h->bonds.size());
  int32_t rc = run_compiled(h, &h->expect_serial[h->parity], false);
  if (rc) return rc;
  hipLaunchKernelGGL(k_rho_ss, dim3((nb + 63) / 64), dim3(64), 0, h->stream,
                     h->rho_descs[h->parity], nb);
  PN_HIP(hipGetLastError());
  PN_HIP(hipMemcpyAsync(h->pinned + 1 + nm, h->ss_dev, nb * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
  PN_HIP(hipEventRecord(ev, h->stream));
  return BBP_OK;
}

int32_t finish_expect(pepsnet_s* h, std::vector<double>* ss, double* energy) {
  const int nm = int(h->P.msg_keys.size()), nb = int(h->bonds.size());
  ss->assign(h->pinned + 1 + nm, h->pinned + 1 + nm + nb);
  double e = 0.0;
  for (double x : *ss) {
    if (!std::isfinite(x)) return fail(BBP_ENUMERIC, "non-finite expectation value");
    e += x;
  }
  *energy = h->P.kind == 1 ? e / 3.0 : e / std::max(nb, 1);
  return BBP_OK;
}


// (Re)compile every launch list against the current arena and workspace
// addresses and upload the descriptors; drops captured graphs.
int32_t build_launches(pepsnet_s* h) {
  for (Compiled* c : {&h->sweep[0], &h->sweep[1], &h->expect[0], &h->expect[1], &h->prep,
                      &h->sweep_serial[0], &h->sweep_serial[1], &h->expect_serial[0],
                      &h->expect_serial[1]}) {
    if (c->exec) hipGraphExecDestroy(c->exec);
    if (c->graph) hipGraphDestroy(c->graph);
    *c = Compiled();
  }
  h->desc_host.clear();
  compile_ops({{h, &h->prep_lanes}}, &h->desc_host, &h->prep);
  for (int par = 0; par < 2; ++par) {
    // the message updates of a sweep, and the bonds of an expectation,
    // share no data: their lane groups may run on separate streams
    const std::vector<int> sg = lane_groups(h->sweep_lanes[par]);
    compile_ops({{h, &h->sweep_lanes[par], &sg}}, &h->desc_host, &h->sweep[par]);
    const std::vector<int> eg = lane_groups(h->expect_lanes[par]);
    compile_ops({{h, &h->expect_lanes[par], &eg}}, &h->desc_host, &h->expect[par]);
    compile_ops({{h, &h->sweep_lanes[par]}}, &h->desc_host, &h->sweep_serial[par]);
    compile_ops({{h, &h->expect_lanes[par]}}, &h->desc_host, &h->expect_serial[par]);
  }
  const int nb = int(h->bonds.size());
  size_t rho_off[2];
  for (int par = 0; par < 2; ++par) {
    std::vector<RhoDesc> rd(nb);
    for (int b = 0; b < nb; ++b) {
      rd[b].R = h->arena + h->region_base[RG_RHO] + h->rho_off[par][b];
      rd[b].rho = h->rho_mat + 16 * b;
      rd[b].ss = h->ss_dev + b;
      rd[b].first_is_i = h->carry_order[par][b][0] == h->bonds[b].first ? 1 : 0;
    }
    rho_off[par] = push_descs(&h->desc_host, rd);
  }
  std::vector<int32_t> sel(std::max(nb, 1));
  for (int b = 0; b < nb; ++b) sel[b] = b;
  const size_t sel_off = push_descs(&h->desc_host, sel);
  // the plans' shapes never change, so the descriptor buffer keeps its size
  // after the first build; work still queued may read the old descriptors
  PN_HIP(hipStreamSynchronize(h->stream));
  if (h->desc_cap < h->desc_host.size()) {
    if (h->desc_dev) hipFree(h->desc_dev);
    h->desc_dev = nullptr;
    h->desc_cap = 0;
    if (hipMalloc(&h->desc_dev, std::max<size_t>(h->desc_host.size(), 256)) != hipSuccess)
      return fail(BBP_ENOMEM, "descriptor allocation failed");
    h->desc_cap = std::max<size_t>(h->desc_host.size(), 256);
  }
  PN_HIP(hipMemcpyAsync(h->desc_dev, h->desc_host.data(), h->desc_host.size(),
                        hipMemcpyHostToDevice, h->stream));
  h->desc_work = h->work;
  for (Compiled* c : {&h->sweep[0], &h->sweep[1], &h->expect[0], &h->expect[1], &h->prep,
                      &h->sweep_serial[0], &h->sweep_serial[1], &h->expect_serial[0],
                      &h->expect_serial[1]})
    c->desc = h->desc_dev;
  for (int par = 0; par < 2; ++par)
    h->rho_descs[par] = reinterpret_cast<RhoDesc*>(h->desc_dev + rho_off[par]);
  h->sel_default = reinterpret_cast<const int32_t*>(h->desc_dev + sel_off);
  PN_HIP(hipStreamSynchronize(h->stream));
  return BBP_OK;
}

void free_subsets(pepsnet_s* h) {
  for (auto& kv : h->subsets) {
    for (Compiled& c : kv.second.plan) {
      if (c.exec) hipGraphExecDestroy(c.exec);
      if (c.graph) hipGraphDestroy(c.graph);
    }
    if (kv.second.desc_dev) hipFree(kv.second.desc_dev);
  }
  h->subsets.clear();
}

// Launch list of the expectation of a bond subset (compiled on first use
// and again after the workspace moved): the default plan's lanes of those
// bonds, with their rho descriptors and the selection list.
int32_t subset_plan(pepsnet_s* h, const std::vector<int>& ids, pepsnet_s::Subset** out) {
  auto it = h->subsets.find(ids);
  if (it != h->subsets.end() && it->second.epoch == h->work_epoch) {
    *out = &it->second;
    return BBP_OK;
  }
  if (it != h->subsets.end()) {
    PN_HIP(hipStreamSynchronize(h->stream));
    if (it->second.desc_dev) hipFree(it->second.desc_dev);
    h->subsets.erase(it);
  }
  pepsnet_s::Subset S;
  for (int par = 0; par < 2; ++par) {
    LaneList lanes;
    for (int b : ids) lanes.push_back(h->expect_lanes[par][b]);
    const std::vector<int> eg = lane_groups(lanes);
    compile_ops({{h, &lanes, &eg}}, &S.blob, &S.plan[par]);
    std::vector<RhoDesc> rd;
    for (int b : ids) {
      RhoDesc r;
      r.R = h->arena + h->region_base[RG_RHO] + h->rho_off[par][b];
      r.rho = h->rho_mat + 16 * b;
      r.ss = h->ss_dev + b;
      r.first_is_i = h->carry_order[par][b][0] == h->bonds[b].first ? 1 : 0;
      rd.push_back(r);
    }
    S.rho_off[par] = push_descs(&S.blob, rd);
  }
  std::vector<int32_t> sel(ids.begin(), ids.end());
  S.sel_off = push_descs(&S.blob, sel);
  if (hipMalloc(&S.desc_dev, std::max<size_t>(S.blob.size(), 256)) != hipSuccess)
    return fail(BBP_ENOMEM, "descriptor allocation of a bond subset failed");
  PN_HIP(hipMemcpyAsync(S.desc_dev, S.blob.data(), S.blob.size(), hipMemcpyHostToDevice, h->stream));
  for (Compiled& c : S.plan) c.desc = S.desc_dev;
  PN_HIP(hipStreamSynchronize(h->stream));
  S.epoch = h->work_epoch;
  auto& slot = h->subsets[ids];
  slot = std::move(S);
  *out = &slot;
  return BBP_OK;
}

int32_t need_work(pepsnet_s* h) {
  if (!h->work) return fail(BBP_EINVAL, "the handle's workspace is released");
  return BBP_OK;
}

// Lend a server workspace slot to a handle whose own workspace is released.
// Descriptors already resolved against this address (the state held the
// same slot last time) are kept with their captured graphs.
int32_t bind_slot(pepsnet_s* h, SrvSlot* slot) {
  h->work = slot->ptr;
  slot->last = h;
  if (h->desc_work == h->work) return BBP_OK;
  h->work_epoch += 1;
  return build_launches(h);
}

// Take the slot back once the request's work has drained from the stream.
void unbind_slot(pepsnet_s* h, SrvSlot* slot) {
  hipStreamSynchronize(h->stream);
  h->work = nullptr;
  slot->busy = false;
}


// Start an admitted request: workspace, new sites (messages kept: a warm
// start), then its first sweep (or the expectation when max_sweeps == 0).
void srv_start(bbp_server_s* S, SrvReq* r) {
  pepsnet_s* h = r->h;
  int32_t rc = BBP_OK;
  if (r->slot) {
    SrvSlot* slot = r->slot;
    if (!slot->ptr) {   // the pool grows: the only allocation of the loop
      if (hipMalloc(&slot->ptr, size_t(slot->bytes)) != hipSuccess) {
        slot->ptr = nullptr;
        rc = fail(BBP_ENOMEM, "workspace slot allocation of " + std::to_string(slot->bytes) +
                                  " bytes failed");
      } else {
        S->slot_allocs += 1;
      }
    }
    if (rc == BBP_OK) rc = bind_slot(h, slot);
    if (rc == BBP_OK) {
      r->own_work = true;
    } else {
      if (h->work == slot->ptr) h->work = nullptr;
      slot->busy = false;
    }
  }
  if (rc == BBP_OK && (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreate(&r->ev_begin) != hipSuccess ||
                       hipEventCreate(&r->ev_end) != hipSuccess))
    rc = fail(BBP_EDEVICE, "event creation failed");
  if (rc == BBP_OK && hipEventRecord(r->ev_begin, h->stream) != hipSuccess)
    rc = fail(BBP_EDEVICE, "event record failed");
  if (rc == BBP_OK && !r->sites.empty()) rc = upload_sites(h, r->sites.data(), int64_t(r->sites.size()));
  if (rc == BBP_OK) {
    if (r->max_sweeps > 0) {
      r->phase = 1;
      rc = enqueue_sweep(h, r->ev);
    } else {
      r->phase = 2;
      rc = enqueue_expect(h, r->ev);
      if (rc == BBP_OK) hipEventRecord(r->ev_end, h->stream);
    }
  }
  if (rc != BBP_OK) {
    r->rc = rc;
    r->phase = 3;
  }
}

// Advance a request whose last step finished; false if it is still running.
bool srv_progress(SrvReq* r) {
  if (r->phase == 3) return false;
  if (hipEventQuery(r->ev) == hipErrorNotReady) return false;
  pepsnet_s* h = r->h;
  int32_t rc = BBP_OK;
  if (r->phase == 1) {
    rc = finish_sweep(h, &r->err);
    r->sweeps += 1;
    if (rc == BBP_OK) {
      if (r->err <= r->tol || r->sweeps >= r->max_sweeps) {
        r->phase = 2;
        rc = enqueue_expect(h, r->ev);
        if (rc == BBP_OK) hipEventRecord(r->ev_end, h->stream);
      } else {
        rc = enqueue_sweep(h, r->ev);
      }
    }
  } else {
    rc = finish_expect(h, &r->ss, &r->energy);
    r->phase = 3;
    if (rc == BBP_OK && r->max_sweeps > 0 && !(r->err <= r->tol)) rc = BBP_NOT_CONVERGED;
  }
  if (rc != BBP_OK) {
    r->rc = rc;
    if (rc < 0) r->phase = 3;
  }
  return true;
}

// A free slot for a state whose workspace is released (server mutex held):
// the slot it held last if free, else the smallest free one that fits, else
// a new one while the pool is below max_inflight slots and within the
// budget; as a last resort free slots are given up (queued in *evict, freed
// after the mutex is dropped) until a new one fits.  nullptr: wait.
SrvSlot* srv_pick_slot(bbp_server_s* S, const pepsnet_s* h, std::vector<cplx*>* evict) {
  const int64_t need = h->work_len * int64_t(sizeof(cplx));
  SrvSlot* best = nullptr;
  for (auto& sp : S->slots) {
    SrvSlot* sl = sp.get();
    if (sl->busy || sl->bytes < need) continue;
    if (sl->last == h && sl->ptr && sl->ptr == h->desc_work) {
      best = sl;
      break;
    }
    if (!best || sl->bytes < best->bytes) best = sl;
  }
  if (!best) {
    auto room = [&] {
      return int(S->slots.size()) < S->max_inflight && S->in_use + need <= S->budget;
    };
    while (!room()) {   // give up the smallest free slot, if any
      auto victim = S->slots.end();
      for (auto it = S->slots.begin(); it != S->slots.end(); ++it)
        if (!(*it)->busy && (victim == S->slots.end() || (*it)->bytes < (*victim)->bytes)) victim = it;
      if (victim == S->slots.end()) return nullptr;
      if ((*victim)->ptr) evict->push_back((*victim)->ptr);
      S->in_use -= (*victim)->bytes;
      S->slots.erase(victim);
    }
    S->slots.push_back(std::unique_ptr<SrvSlot>(new SrvSlot()));
    best = S->slots.back().get();
    best->bytes = need;   // allocated by srv_start, outside the mutex
    S->in_use += need;
  }
  best->busy = true;
  return best;
}

void srv_loop(bbp_server_s* S) {
  std::vector<cplx*> evict;
  for (;;) {
    std::vector<SrvReq*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->inflight.empty())
        S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty() && S->inflight.empty()) return;
      // admit in arrival order as slots and memory free up; a request whose
      // state is busy or whose workspace does not fit lets later ones pass
      for (auto it = S->queue.begin();
           it != S->queue.end() && int(S->inflight.size()) < S->max_inflight;) {
        SrvReq* r = *it;
        bool busy = false;
        for (SrvReq* o : S->inflight) busy = busy || o->h == r->h;
        bool ok = !busy;
        if (ok && !r->h->work) {
          r->slot = srv_pick_slot(S, r->h, &evict);
          ok = r->slot != nullptr;
        }
        if (ok) {
          S->inflight.push_back(r);
          admitted.push_back(r);
          it = S->queue.erase(it);
        } else {
          ++it;
        }
      }
      S->peak_in_use = std::max(S->peak_in_use, S->in_use);
      S->peak_inflight = std::max(S->peak_inflight, int(S->inflight.size()));
    }
    // slots given up to make room for a larger one (mixed state sizes only)
    for (cplx* p : evict) hipFree(p);
    evict.clear();
    for (SrvReq* r : admitted) srv_start(S, r);
    bool progressed = !admitted.empty();
    std::vector<SrvReq*> snapshot;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      snapshot = S->inflight;
    }
    for (SrvReq* r : snapshot) progressed = srv_progress(r) || progressed;
    std::vector<SrvReq*> done;
    for (SrvReq* r : snapshot)
      if (r->phase == 3) done.push_back(r);
    for (SrvReq* r : done) {
      if (r->h->stream) hipStreamSynchronize(r->h->stream);
      if (r->ev_begin && r->ev_end && hipEventQuery(r->ev_end) == hipSuccess) {
        float a = 0.0f, b = 0.0f;
        if (hipEventElapsedTime(&a, S->ev_ref, r->ev_begin) == hipSuccess &&
            hipEventElapsedTime(&b, S->ev_ref, r->ev_end) == hipSuccess) {
          r->window_ms[0] = a;
          r->window_ms[1] = b;
        }
      }
      if (r->own_work) unbind_slot(r->h, r->slot);
      for (hipEvent_t* e : {&r->ev, &r->ev_begin, &r->ev_end}) {
        if (*e) hipEventDestroy(*e);
        *e = nullptr;
      }
      r->sites.clear();
      r->t_done = std::chrono::steady_clock::now();
    }
    if (!done.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (SrvReq* r : done) {
        S->inflight.erase(std::find(S->inflight.begin(), S->inflight.end(), r));
        S->completed += 1;
        r->ready = true;
      }
      S->cv_done.notify_all();
    }
    if (!progressed && done.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

// ---- GEMM tile autotuner (pepsnet_autotune)
// Grid of a GEMM launch of `items` descriptors for tile shape v.
dim3 gemm_grid(int v, int64_t M, int64_t N, int items) {
  const int tm = v == 1 ? 16 : v == 4 ? 80 : 64;
  const int tn = v == 2 ? 16 : v == 3 ? 80 : 64;
  return dim3(unsigned((N + tn - 1) / tn), unsigned(std::min<int64_t>(65535, (M + tm - 1) / tm)),
              unsigned(items));
}

// Elements a GEMM descriptor writes past its C pointer (the extent of the
// output, scattered or row-major).
int64_t gemm_out_extent(const GemmDesc& g) {
  if (g.sc_n > 0) {
    int64_t e = 1;
    for (int k = 0; k < g.sc_n; ++k) e += int64_t(g.sc_dim[k] - 1) * g.sc_ds[k];
    return e;
  }
  return int64_t(g.M - 1) * g.ldc + g.N;
}

bool load_tile_cache(const char* path, std::map<std::array<int, 7>, int>* t) {
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    std::array<int, 7> k;
    int v;
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5],
                    &k[6], &v) == 8 && v >= 0 && v <= 4)
      (*t)[k] = v;
  }
  std::fclose(f);
  return true;
}

bool save_tile_cache(const char* path, const std::map<std::array<int, 7>, int>& t) {
  if (!path || !*path) return true;
  std::map<std::array<int, 7>, int> all;
  load_tile_cache(path, &all);
  for (const auto& kv : t) all[kv.first] = kv.second;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "# pepsnet k_gemm tile shapes, gfx950: prec M N K opA opB scatter tile\n");
  for (const auto& kv : all) {
    const auto& k = kv.first;
    std::fprintf(f, "%d %d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], k[4], k[5], k[6], kv.second);
  }
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

// At create: when the workspace and the descriptors fit in the device's
// fixed array, resolve the sweep plans against it (host-side compilation)
// and keep a pinned copy of their descriptors for blockbp_sweep_noalloc.
int32_t prepare_fixed(pepsnet_s* h) {
  h->fixed_need = 0;
  if (h->device < 0 || h->device >= kMaxDevices || !g_fixed_ptr[h->device]) return BBP_OK;
  char* base = g_fixed_ptr[h->device];
  const size_t ws_bytes = (size_t(h->work_len) * sizeof(cplx) + 255) / 256 * 256;
  h->fixed_need = ws_bytes;
  if (ws_bytes > kFixedBytes) return BBP_OK;
  std::vector<char> blob;
  cplx* own = h->work;
  h->work = reinterpret_cast<cplx*>(base);
  for (int par = 0; par < 2; ++par) {
    h->sweep_fixed[par] = Compiled();
    compile_ops({{h, &h->sweep_lanes[par]}}, &blob, &h->sweep_fixed[par]);
    h->sweep_fixed[par].desc = base + ws_bytes;
  }
  h->work = own;
  h->fixed_need = ws_bytes + blob.size();
  if (h->fixed_need > kFixedBytes) return BBP_OK;
  if (hipHostMalloc(&h->blob_fixed, std::max<size_t>(blob.size(), 1), 0) != hipSuccess) {
    h->blob_fixed = nullptr;
    return fail(BBP_ENOMEM, "pinned descriptor buffer");
  }
  std::memcpy(h->blob_fixed, blob.data(), blob.size());
  h->blob_fixed_len = blob.size();
  h->fixed_ready = true;
  return BBP_OK;
}

// Sweeps with plans[parity] until the largest message distance is <= tol
// or max_sweeps ran (graph: replay captured graphs when the handle allows).
int32_t sweep_until(pepsnet_s* h, Compiled* plans, bool graph, int32_t max_sweeps, double tol,
                    int32_t* sweeps_done, double* max_err) {
  const int nm = int(h->P.msg_keys.size());
  double err = INFINITY;
  int s = 0;
  for (; s < max_sweeps;) {
    h->pinned[0] = double(h->sweeps_total);
    PN_HIP(hipMemcpyAsync(h->scal + Compiler::kSweepSlot, h->pinned, sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
    PN_HIP(hipEventRecord(h->ev0, h->stream));
    int32_t rc = run_compiled(h, &plans[h->parity], graph);
    if (rc) return rc;
    PN_HIP(hipEventRecord(h->ev1, h->stream));
    PN_HIP(hipMemcpyAsync(h->pinned + 1, h->scal + h->comp->err_slot(0), nm * sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
    PN_HIP(hipStreamSynchronize(h->stream));
    float ms = 0.0f;
    PN_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->timed_ms += ms;
    h->timed_sweeps += 1;
    ++s;
    if (!close_sweep(&h->parity, &h->sweeps_total, h->pinned + 1, nm, &err)) {
      if (sweeps_done) *sweeps_done = s;
      if (max_err) *max_err = err;
      return fail(BBP_ENUMERIC, "non-finite message after a sweep");
    }
    if (err <= tol) break;
  }
  if (sweeps_done) *sweeps_done = s;
  if (max_err) *max_err = err;
  return err <= tol ? BBP_OK : BBP_NOT_CONVERGED;
}

}  // namespace

extern "C" {

const char* pepsnet_last_error(void) { return g_last_error.c_str(); }

int32_t pepsnet_create(const pepsnet_desc* desc, const double* sites, int64_t sites_len,
                       pepsnet_t* out) {
  if (!out) return fail(BBP_EINVAL, "null output handle");
  *out = nullptr;
  int32_t rc = check_desc(desc);
  if (rc) return rc;
  std::unique_ptr<pepsnet_s> h(new pepsnet_s());
  std::string e = build_problem(desc, &h->P);
  if (!e.empty()) return fail(BBP_EGEOM, e);
  h->opt.chi = desc->chi;
  h->opt.chi_env = desc->chi_env;
  h->opt.trunc = desc->trunc;
  h->opt.q = desc->rsvd_q;
  h->opt.p = desc->rsvd_p;
  h->opt.precision = desc->precision;
  h->opt.seed = desc->seed;
  h->opt.d = desc->d;
  h->opt.D = desc->D;
  h->opt.order = desc->swallow_order;
  h->opt.hermitize = desc->hermitize;
  h->opt.damping = desc->damping;
  h->comp.reset(new Compiler(h->P, h->opt));
  if (!h->comp->error.empty()) return fail(BBP_EGEOM, h->comp->error);
  Plan sp[2], ep[2];
  for (int par = 0; par < 2; ++par)
    if (!h->comp->build_sweep(par, &sp[par])) return fail(BBP_EGEOM, h->comp->error);
  h->bonds = h->P.kind == 1 ? h->P.central_bonds() : h->P.bonds();
  for (int par = 0; par < 2; ++par)
    if (!h->comp->build_expect(par, h->bonds, &ep[par], &h->carry_order[par], &h->rho_off[par]))
      return fail(BBP_EGEOM, h->comp->error);
  // arena layout
  Compiler& C = *h->comp;
  int nl = int(C.lane_size.size());
  std::vector<int64_t> sizes(RG_LANE0 + nl, 0);
  sizes[RG_SITE] = C.site_region_size;
  sizes[RG_SMAT] = C.smat_size;
  sizes[RG_MSG0] = C.msg.size;
  sizes[RG_MSG1] = C.msg.size;
  sizes[RG_CONST] = 8;
  sizes[RG_RHO] = std::max<int64_t>(C.rho_size, 8);
  for (int L = 0; L < nl; ++L) sizes[RG_LANE0 + L] = C.lane_size[L];
  h->region_base.assign(sizes.size(), 0);
  int64_t tot = 0, wtot = 0;
  for (size_t r = 0; r < sizes.size(); ++r) {
    int64_t& t = int(r) >= RG_LANE0 ? wtot : tot;
    h->region_base[r] = t;
    t += (sizes[r] + 31) / 32 * 32;
  }
  h->arena_len = tot;
  h->work_len = std::max<int64_t>(wtot, 32);
  {
    const int64_t nb = int64_t(h->bonds.size());
    const int64_t need = (tot + h->work_len) * int64_t(sizeof(cplx)) +
                         int64_t(C.n_scalars) * int64_t(sizeof(double)) +
                         (17 + kMaxOps) * std::max<int64_t>(nb, 1) * int64_t(sizeof(cplx)) +
                         16 * kMaxOps * int64_t(sizeof(cplx));
    if (desc->hbm_budget_bytes > 0 && need > desc->hbm_budget_bytes)
      return fail(BBP_ENOMEM, "the plans need " + std::to_string(need) +
                                  " bytes of device memory, over the budget of " +
                                  std::to_string(desc->hbm_budget_bytes));
  }
  if (desc->stream) {
    h->stream = (hipStream_t)desc->stream;
  } else {
    PN_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }
  for (int g = 0; g < kMaxStreams - 1; ++g)
    PN_HIP(hipEventCreateWithFlags(&h->join_ev[g], hipEventDisableTiming));
  PN_HIP(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
  PN_HIP(hipGetDevice(&h->device));
  // the no-allocation sweep reports a failure here when it is called
  if (resolve_fixed(h->device) != BBP_OK) g_last_error.clear();
  if (hipMalloc(&h->arena, size_t(tot) * sizeof(cplx)) != hipSuccess)
    return fail(BBP_ENOMEM, "device allocation of " + std::to_string(tot * 16) + " bytes failed");
  if (hipMalloc(&h->work, size_t(h->work_len) * sizeof(cplx)) != hipSuccess)
    return fail(BBP_ENOMEM, "workspace allocation of " + std::to_string(h->work_len * 16) +
                                " bytes failed");
  PN_HIP(hipMemsetAsync(h->work, 0, size_t(h->work_len) * sizeof(cplx), h->stream));
  if (hipMalloc(&h->scal, size_t(C.n_scalars) * sizeof(double)) != hipSuccess)
    return fail(BBP_ENOMEM, "scalar allocation failed");
  PN_HIP(hipMemsetAsync(h->arena, 0, size_t(tot) * sizeof(cplx), h->stream));
  PN_HIP(hipMemsetAsync(h->scal, 0, size_t(C.n_scalars) * sizeof(double), h->stream));
  cplx one = {1.0, 0.0};
  PN_HIP(hipMemcpyAsync(h->arena + h->region_base[RG_CONST], &one, sizeof one,
                        hipMemcpyHostToDevice, h->stream));
  // keep the plans' op lists, then compile and upload descriptors
  h->prep_lanes.resize(1);
  for (size_t k = 0; k < C.prep_ops.size(); ++k) {
    WaveKey wk;
    wk.k = {0};   // prep ops are independent: one wave
    h->prep_lanes[0].push_back({wk, C.prep_ops[k]});
  }
  for (int par = 0; par < 2; ++par) {
    for (auto& L : sp[par].lanes) h->sweep_lanes[par].push_back(L.ops);
    for (auto& L : ep[par].lanes) h->expect_lanes[par].push_back(L.ops);
  }
  int nb = int(h->bonds.size());
  if (hipMalloc(&h->rho_mat, size_t(std::max(nb, 1)) * 16 * sizeof(cplx)) != hipSuccess ||
      hipMalloc(&h->ss_dev, size_t(std::max(nb, 1)) * sizeof(double)) != hipSuccess ||
      hipMalloc(&h->ops_dev, size_t(kMaxOps) * 16 * sizeof(cplx)) != hipSuccess ||
      hipMalloc(&h->ops_out, size_t(std::max(nb, 1)) * kMaxOps * sizeof(cplx)) != hipSuccess ||
      hipMalloc(&h->meas_dev, size_t(std::max(nb, 1)) * (16 * sizeof(cplx) + 2 * sizeof(double) +
                                                         sizeof(int32_t)) + 512) != hipSuccess)
    return fail(BBP_ENOMEM, "expectation buffers");
  for (int par = 0; par < 2; ++par)
    for (int b = 0; b < nb; ++b)
      if (h->carry_order[par][b].size() != 2)
        return fail(BBP_EGEOM, "expectation carries two open sites");
  rc = build_launches(h.get());
  if (rc) return rc;
  rc = prepare_fixed(h.get());
  if (rc) return rc;
  if (hipHostMalloc(&h->pinned, size_t(C.msg.off.size() + h->bonds.size() + 8) * sizeof(double),
                    0) != hipSuccess)
    return fail(BBP_ENOMEM, "pinned host buffer");
  for (const void* f : {(const void*)k_jacobi<false>, (const void*)k_jacobi<true>})
    PN_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(JAC_LDS_MAX * sizeof(cplx))));
  PN_HIP(hipFuncSetAttribute((const void*)k_qr, hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(QR_LDS_MAX * sizeof(cplx))));
  PN_HIP(hipFuncSetAttribute((const void*)k_qr_tall, hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(QRT_LDS * sizeof(cplx))));
  PN_HIP(hipEventCreate(&h->ev0));
  PN_HIP(hipEventCreate(&h->ev1));
  PN_HIP(hipStreamSynchronize(h->stream));
  h->site_len = 2 * C.site_region_size;
  rc = upload_sites(h.get(), sites, sites_len);
  if (rc) return rc;
  rc = reset_messages(h.get());
  if (rc) return rc;
  *out = h.release();
  return BBP_OK;
}

int32_t pepsnet_set_sites(pepsnet_t h, const double* sites, int64_t len, int32_t reset) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  int32_t rc = upload_sites(h, sites, len);
  if (rc) return rc;
  if (reset) return reset_messages(h);
  return BBP_OK;
}

int32_t blockbp_sweep(pepsnet_t h, int32_t max_sweeps, double tol, int32_t* sweeps_done,
                      double* max_err) {
  if (!h || max_sweeps < 0) return fail(BBP_EINVAL, "bad arguments");
  if (int32_t rc = need_work(h)) return rc;
  return sweep_until(h, h->nstreams > 1 ? h->sweep : h->sweep_serial, true, max_sweeps, tol,
                     sweeps_done, max_err);
}

int32_t blockbp_sweep_noalloc(pepsnet_t h, int32_t max_sweeps, double tol, int32_t* sweeps_done,
                              double* max_err) {
  if (!h || max_sweeps < 0) return fail(BBP_EINVAL, "bad arguments");
  if (h->device < 0 || h->device >= kMaxDevices || !g_fixed_ptr[h->device])
    return fail(BBP_EDEVICE, "the fixed workspace is not available on this device");
  if (!h->fixed_ready)
    return fail(BBP_ENOMEM, "the sweep needs " + std::to_string(h->fixed_need) +
                                " bytes of workspace and descriptors; the fixed workspace holds " +
                                std::to_string(kFixedBytes));
  char* base = g_fixed_ptr[h->device];
  const size_t ws_bytes = (size_t(h->work_len) * sizeof(cplx) + 255) / 256 * 256;
  // the array keeps whatever the last call on this device left: put this
  // handle's descriptors back and clear its workspace part
  PN_HIP(hipMemcpyAsync(base + ws_bytes, h->blob_fixed, h->blob_fixed_len, hipMemcpyHostToDevice,
                        h->stream));
  const int64_t n16 = int64_t(ws_bytes / sizeof(uint4));
  hipLaunchKernelGGL(k_fill_zero, dim3(unsigned(std::min<int64_t>((n16 + 255) / 256, 4096))),
                     dim3(256), 0, h->stream, reinterpret_cast<uint4*>(base), n16);
  PN_HIP(hipGetLastError());
  return sweep_until(h, h->sweep_fixed, false, max_sweeps, tol, sweeps_done, max_err);
}

int32_t blockbp_expect(pepsnet_t h, int32_t n_bonds, const int32_t* bond_ids, int32_t n_ops,
                       const double* ops, double* out, double* rho_out, double* energy,
                       int32_t* n_bonds_out) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (int32_t rc = need_work(h)) return rc;
  const int nb = int(h->bonds.size());
  std::vector<int> ids;
  if (bond_ids) {
    if (n_bonds < 1 || n_bonds > nb) return fail(BBP_EINVAL, "bad number of bonds");
    if (energy) return fail(BBP_EINVAL, "the energy needs the whole bond table (bond_ids NULL)");
    std::vector<char> seen(nb, 0);
    for (int b = 0; b < n_bonds; ++b) {
      const int id = bond_ids[b];
      if (id < 0 || id >= nb) return fail(BBP_EINVAL, "bond id out of range");
      if (seen[id]) return fail(BBP_EINVAL, "bond id listed twice");
      seen[id] = 1;
      ids.push_back(id);
    }
  } else {
    for (int b = 0; b < nb; ++b) ids.push_back(b);
  }
  if (ops && (n_ops < 1 || n_ops > kMaxOps)) return fail(BBP_EINVAL, "n_ops must be in [1, 64]");
  const int ns = int(ids.size());
  Compiled* plan = h->nstreams > 1 ? &h->expect[h->parity] : &h->expect_serial[h->parity];
  const RhoDesc* rdesc = h->rho_descs[h->parity];
  const int32_t* sel = h->sel_default;
  if (bond_ids) {
    pepsnet_s::Subset* S = nullptr;
    if (int32_t rc = subset_plan(h, ids, &S)) return rc;
    plan = &S->plan[h->parity];
    rdesc = reinterpret_cast<const RhoDesc*>(S->desc_dev + S->rho_off[h->parity]);
    sel = reinterpret_cast<const int32_t*>(S->desc_dev + S->sel_off);
  }
  int32_t rc = run_compiled(h, plan, false);
  if (rc) return rc;
  hipLaunchKernelGGL(k_rho_ss, dim3((ns + 63) / 64), dim3(64), 0, h->stream, rdesc, ns);
  PN_HIP(hipGetLastError());
  std::vector<cplx> vals;
  if (ops && out) {
    PN_HIP(hipMemcpyAsync(h->ops_dev, ops, size_t(n_ops) * 16 * sizeof(cplx),
                          hipMemcpyHostToDevice, h->stream));
    const int nt = ns * n_ops;
    hipLaunchKernelGGL(k_rho_ops, dim3((nt + 63) / 64), dim3(64), 0, h->stream,
                       (const cplx*)h->rho_mat, sel, ns, (const cplx*)h->ops_dev, n_ops, h->ops_out);
    PN_HIP(hipGetLastError());
    vals.resize(size_t(nt));
    PN_HIP(hipMemcpyAsync(vals.data(), h->ops_out, size_t(nt) * sizeof(cplx),
                          hipMemcpyDeviceToHost, h->stream));
  }
  std::vector<double> ss(nb);
  std::vector<cplx> rho;
  PN_HIP(hipMemcpyAsync(ss.data(), h->ss_dev, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (rho_out) {
    rho.resize(size_t(nb) * 16);
    PN_HIP(hipMemcpyAsync(rho.data(), h->rho_mat, size_t(nb) * 16 * sizeof(cplx),
                          hipMemcpyDeviceToHost, h->stream));
  }
  PN_HIP(hipStreamSynchronize(h->stream));
  double e = 0.0;
  for (int k = 0; k < ns; ++k) {
    const double x = ss[ids[k]];
    if (!std::isfinite(x)) return fail(BBP_ENUMERIC, "non-finite expectation value");
    e += x;
  }
  for (const cplx& v : vals)
    if (!std::isfinite(v.re) || !std::isfinite(v.im))
      return fail(BBP_ENUMERIC, "non-finite expectation value");
  if (out) {
    if (ops) std::memcpy(out, vals.data(), vals.size() * sizeof(cplx));
    else
      for (int k = 0; k < ns; ++k) { out[2 * k] = ss[ids[k]]; out[2 * k + 1] = 0.0; }
  }
  if (rho_out)
    for (int k = 0; k < ns; ++k)
      std::memcpy(rho_out + 32 * int64_t(k), rho.data() + 16 * int64_t(ids[k]), 16 * sizeof(cplx));
  if (energy) *energy = h->P.kind == 1 ? e / 3.0 : e / std::max(nb, 1);
  if (n_bonds_out) *n_bonds_out = ns;
  h->rho_stamp.resize(nb, {-1, -1});
  for (int k = 0; k < ns; ++k) h->rho_stamp[ids[k]] = {h->sweeps_total, h->edits};
  return BBP_OK;
}

int32_t blockbp_rho_measures(pepsnet_t h, int32_t n_bonds, const int32_t* bond_ids,
                             const double* sigma, double* negativity, double* fidelity) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  const int nb = int(h->bonds.size());
  std::vector<int32_t> ids;
  if (bond_ids) {
    if (n_bonds < 1 || n_bonds > nb) return fail(BBP_EINVAL, "bad number of bonds");
    for (int b = 0; b < n_bonds; ++b) {
      if (bond_ids[b] < 0 || bond_ids[b] >= nb) return fail(BBP_EINVAL, "bond id out of range");
      ids.push_back(bond_ids[b]);
    }
  } else {
    if (n_bonds != nb) return fail(BBP_EINVAL, "n_bonds must be the number of default bonds");
    for (int b = 0; b < nb; ++b) ids.push_back(b);
  }
  if (fidelity && !sigma) return fail(BBP_EINVAL, "fidelity needs sigma");
  h->rho_stamp.resize(nb, {-1, -1});
  for (int32_t id : ids)
    if (h->rho_stamp[id] != std::make_pair(h->sweeps_total, h->edits))
      return fail(BBP_EINVAL, "no rho of the current state for bond " + std::to_string(id) +
                                  " (call blockbp_expect first)");
  const int ns = int(ids.size());
  // staging: ids, then sigma (256-byte aligned), then the results
  const size_t off_sg = (size_t(nb) * sizeof(int32_t) + 255) / 256 * 256;
  int32_t* sel = reinterpret_cast<int32_t*>(h->meas_dev);
  cplx* sg = reinterpret_cast<cplx*>(h->meas_dev + off_sg);
  double* res = reinterpret_cast<double*>(h->meas_dev + off_sg + size_t(nb) * 16 * sizeof(cplx));
  PN_HIP(hipMemcpyAsync(sel, ids.data(), size_t(ns) * sizeof(int32_t), hipMemcpyHostToDevice,
                        h->stream));
  if (sigma)
    PN_HIP(hipMemcpyAsync(sg, sigma, size_t(ns) * 16 * sizeof(cplx), hipMemcpyHostToDevice,
                          h->stream));
  hipLaunchKernelGGL(k_rho_measures, dim3((ns + 63) / 64), dim3(64), 0, h->stream,
                     (const cplx*)h->rho_mat, (const int32_t*)sel, ns,
                     sigma ? (const cplx*)sg : nullptr, res);
  PN_HIP(hipGetLastError());
  std::vector<double> r(2 * size_t(ns));
  PN_HIP(hipMemcpyAsync(r.data(), res, r.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  PN_HIP(hipStreamSynchronize(h->stream));
  for (int k = 0; k < ns; ++k) {
    if (!std::isfinite(r[2 * k]) || (sigma && !std::isfinite(r[2 * k + 1])))
      return fail(BBP_ENUMERIC, "non-finite rho measure");
    if (negativity) negativity[k] = r[2 * k];
    if (fidelity) fidelity[k] = r[2 * k + 1];
  }
  return BBP_OK;
}

int32_t pepsnet_bonds(pepsnet_t h, int32_t* pairs, int32_t cap, int32_t* n) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  int nb = int(h->bonds.size());
  if (n) *n = nb;
  if (pairs)
    for (int b = 0; b < nb && 2 * b + 1 < cap; ++b) {
      pairs[2 * b] = h->bonds[b].first;
      pairs[2 * b + 1] = h->bonds[b].second;
    }
  return BBP_OK;
}

int32_t pepsnet_num_messages(pepsnet_t h) { return h ? int32_t(h->P.msg_keys.size()) : 0; }

int32_t pepsnet_message_shape(pepsnet_t h, int32_t m, int32_t j, int32_t* l, int32_t* P,
                              int32_t* r, int32_t* n_sites) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  const MsgLayout& M = h->comp->msg;
  if (m < 0 || m >= int(M.off.size())) return fail(BBP_EINVAL, "bad message index");
  if (n_sites) *n_sites = int(M.off[m].size());
  if (j < 0 || j >= int(M.off[m].size())) return BBP_OK;
  if (l) *l = M.bl[m][j];
  if (P) *P = M.P[m][j];
  if (r) *r = M.br[m][j];
  return BBP_OK;
}

int32_t pepsnet_get_messages(pepsnet_t h, double* buf, int64_t cap, int64_t* len) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  const MsgLayout& M = h->comp->msg;
  int64_t need = 0;
  for (size_t m = 0; m < M.off.size(); ++m)
    for (size_t j = 0; j < M.off[m].size(); ++j) need += 2LL * M.bl[m][j] * M.P[m][j] * M.br[m][j];
  if (len) *len = need;
  if (!buf) return BBP_OK;
  if (cap < need) return fail(BBP_EINVAL, "buffer too small");
  std::vector<cplx> all(M.size);
  PN_HIP(hipMemcpyAsync(all.data(), h->arena + h->region_base[h->parity ? RG_MSG1 : RG_MSG0],
                        M.size * sizeof(cplx), hipMemcpyDeviceToHost, h->stream));
  PN_HIP(hipStreamSynchronize(h->stream));
  int64_t o = 0;
  for (size_t m = 0; m < M.off.size(); ++m)
    for (size_t j = 0; j < M.off[m].size(); ++j) {
      int64_t n = int64_t(M.bl[m][j]) * M.P[m][j] * M.br[m][j];
      std::memcpy(buf + o, all.data() + M.off[m][j], n * sizeof(cplx));
      o += 2 * n;
    }
  return BBP_OK;
}

int32_t pepsnet_set_messages(pepsnet_t h, const double* buf, int64_t len) {
  if (!h || !buf) return fail(BBP_EINVAL, "null argument");
  const MsgLayout& M = h->comp->msg;
  int64_t need = 0;
  for (size_t m = 0; m < M.off.size(); ++m)
    for (size_t j = 0; j < M.off[m].size(); ++j) need += 2LL * M.bl[m][j] * M.P[m][j] * M.br[m][j];
  if (len != need) return fail(BBP_EINVAL, "message buffer has the wrong length");
  std::vector<cplx> all(M.size, cplx{0.0, 0.0});
  int64_t o = 0;
  for (size_t m = 0; m < M.off.size(); ++m)
    for (size_t j = 0; j < M.off[m].size(); ++j) {
      int64_t n = int64_t(M.bl[m][j]) * M.P[m][j] * M.br[m][j];
      std::memcpy(all.data() + M.off[m][j], buf + o, n * sizeof(cplx));
      o += 2 * n;
    }
  PN_HIP(hipMemcpyAsync(h->arena + h->region_base[h->parity ? RG_MSG1 : RG_MSG0], all.data(),
                        M.size * sizeof(cplx), hipMemcpyHostToDevice, h->stream));
  PN_HIP(hipStreamSynchronize(h->stream));
  h->edits += 1;
  return BBP_OK;
}

void* pepsnet_stream(pepsnet_t h) { return h ? (void*)h->stream : nullptr; }

int32_t pepsnet_timing(pepsnet_t h, int32_t reset, double* ms, int64_t* sweeps) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (ms) *ms = h->timed_sweeps ? h->timed_ms / double(h->timed_sweeps) : 0.0;
  if (sweeps) *sweeps = h->timed_sweeps;
  if (reset) { h->timed_ms = 0.0; h->timed_sweeps = 0; }
  return BBP_OK;
}

int32_t pepsnet_use_graph(pepsnet_t h, int32_t on) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  h->use_graph = on != 0;
  return BBP_OK;
}

int32_t pepsnet_use_streams(pepsnet_t h, int32_t n) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (n < 1 || n > kMaxStreams) return fail(BBP_EINVAL, "stream count must be in [1, 4]");
  if (n != h->nstreams) {
    // captured graphs hold the old stream layout
    for (Compiled* c : {&h->sweep[0], &h->sweep[1]}) {
      if (c->exec) hipGraphExecDestroy(c->exec);
      if (c->graph) hipGraphDestroy(c->graph);
      c->exec = nullptr;
      c->graph = nullptr;
    }
  }
  h->nstreams = n;
  return BBP_OK;
}

int32_t pepsnet_sweep_stats(pepsnet_t h, double* cflops, double* gflops, int64_t* launches) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (cflops) *cflops = h->sweep[0].contraction_flops;
  if (gflops) *gflops = h->sweep[0].gemm_flops;
  if (launches) *launches = int64_t(h->sweep[0].launches.size());
  return BBP_OK;
}

int32_t pepsnet_profile_sweeps(pepsnet_t h, int32_t n_sweeps, double* ms, int64_t* launches,
                               double* flops, double* bytes) {
  if (h && !h->work) return fail(BBP_EINVAL, "the handle's workspace is released");
  if (!h || n_sweeps <= 0) return fail(BBP_EINVAL, "bad arguments");
  const int nk = PEPSNET_PROFILE_SLOTS;
  std::vector<double> tms(nk, 0.0), tfl(nk, 0.0), tby(nk, 0.0);
  std::vector<int64_t> tl(nk, 0);
  for (int s = 0; s < n_sweeps; ++s) {
    Compiled& c = h->sweep[h->parity];
    // three events per record: a two-kernel record (top-k SVD) is timed per
    // kernel, the bidiagonalisation in slot 10 and the rest in slot 11
    std::vector<hipEvent_t> ev(3 * c.launches.size());
    for (auto& e : ev) PN_HIP(hipEventCreate(&e));
    h->pinned[0] = double(h->sweeps_total);
    PN_HIP(hipMemcpyAsync(h->scal + Compiler::kSweepSlot, h->pinned, sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
    for (size_t i = 0; i < c.launches.size(); ++i) {
      const LaunchRec& r = c.launches[i];
      const bool two = r.type == OPK_JACOBI && r.variant == 2;
      PN_HIP(hipEventRecord(ev[3 * i], h->stream));
      hipError_t e = launch(c.desc, h->stream, r, two ? 0 : -1);
      if (e != hipSuccess) return fail(BBP_EDEVICE, hipGetErrorString(e));
      PN_HIP(hipEventRecord(ev[3 * i + 1], h->stream));
      if (two) {
        e = launch(c.desc, h->stream, r, 1);
        if (e != hipSuccess) return fail(BBP_EDEVICE, hipGetErrorString(e));
      }
      PN_HIP(hipEventRecord(ev[3 * i + 2], h->stream));
    }
    PN_HIP(hipStreamSynchronize(h->stream));
    for (size_t i = 0; i < c.launches.size(); ++i) {
      float x = 0.0f, y = 0.0f;
      PN_HIP(hipEventElapsedTime(&x, ev[3 * i], ev[3 * i + 1]));
      PN_HIP(hipEventElapsedTime(&y, ev[3 * i + 1], ev[3 * i + 2]));
      const LaunchRec& r = c.launches[i];
      if (r.type == OPK_JACOBI && r.variant == 2) {
        tms[10] += x;
        tl[10] += 1;
        tfl[10] += r.flops;
        tby[10] += r.bytes;
        tms[11] += y;
        tl[11] += 1;
        continue;
      }
      int slot = r.type * 3 + (r.type == OPK_GEMM ? r.prec : 0);
      if (r.type == OPK_QR && r.variant == 1) slot += 1;   // blocked tall QR
      tms[slot] += x;
      tl[slot] += 1;
      tfl[slot] += r.flops;
      tby[slot] += r.bytes;
    }
    for (auto& e : ev) hipEventDestroy(e);
    h->parity ^= 1;
    h->sweeps_total += 1;
  }
  for (int k = 0; k < nk; ++k) {
    if (ms) ms[k] = tms[k];
    if (launches) launches[k] = tl[k];
    if (flops) flops[k] = tfl[k];
    if (bytes) bytes[k] = tby[k];
  }
  return BBP_OK;
}

int32_t pepsnet_profile_launches(pepsnet_t h, double* rec, int64_t cap, int64_t* n) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (int32_t rc = need_work(h)) return rc;
  Compiled& c = h->sweep[h->parity];
  const int64_t nl = int64_t(c.launches.size());
  if (n) *n = nl;
  if (!rec) return BBP_OK;
  if (cap < 10 * nl) return fail(BBP_EINVAL, "buffer too small");
  std::vector<hipEvent_t> ev(nl + 1);
  for (auto& e : ev) PN_HIP(hipEventCreate(&e));
  h->pinned[0] = double(h->sweeps_total);
  PN_HIP(hipMemcpyAsync(h->scal + Compiler::kSweepSlot, h->pinned, sizeof(double),
                        hipMemcpyHostToDevice, h->stream));
  PN_HIP(hipEventRecord(ev[0], h->stream));
  for (int64_t i = 0; i < nl; ++i) {
    hipError_t e = launch(c.desc, h->stream, c.launches[i]);
    if (e != hipSuccess) return fail(BBP_EDEVICE, hipGetErrorString(e));
    PN_HIP(hipEventRecord(ev[i + 1], h->stream));
  }
  PN_HIP(hipStreamSynchronize(h->stream));
  for (int64_t i = 0; i < nl; ++i) {
    const LaunchRec& r = c.launches[i];
    float ms = 0.0f;
    PN_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    double* o = rec + 10 * i;
    o[0] = r.type; o[1] = r.prec; o[2] = r.variant; o[3] = r.count;
    o[4] = double(r.shape[0]); o[5] = double(r.shape[1]); o[6] = double(r.shape[2]);
    o[7] = r.flops; o[8] = r.bytes; o[9] = ms;
  }
  for (auto& e : ev) hipEventDestroy(e);
  h->parity ^= 1;
  h->sweeps_total += 1;
  return BBP_OK;
}

int32_t pepsnet_autotune(pepsnet_t h, const char* cache_path, int32_t* n_timed, int32_t* n_shapes) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (int32_t rc = need_work(h)) return rc;
  std::map<std::array<int, 7>, int> cache;
  load_tile_cache(cache_path, &cache);
  // one representative launch per GEMM shape of the sweep plans
  std::map<std::array<int, 7>, std::pair<const LaunchRec*, const GemmDesc*>> shapes;
  for (int par = 0; par < 2; ++par)
    for (const LaunchRec& r : h->sweep[par].launches) {
      if (r.type != OPK_GEMM) continue;
      const GemmDesc* gd = reinterpret_cast<const GemmDesc*>(h->desc_host.data() + r.desc_off);
      Op probe;
      probe.i[8] = r.prec; probe.i[0] = gd->M; probe.i[1] = gd->N; probe.i[2] = gd->K;
      probe.i[6] = gd->opA; probe.i[7] = gd->opB; probe.i[10] = gd->sc_n;
      shapes.emplace(gemm_key(probe), std::make_pair(&r, gd));
    }
  int timed = 0;
  std::map<std::array<int, 7>, int> chosen;
  cplx* tmp = nullptr;
  size_t tmp_len = 0;
  char* ddev = nullptr;
  size_t ddev_len = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t rc = BBP_OK;
  auto cleanup = [&]() {
    if (tmp) hipFree(tmp);
    if (ddev) hipFree(ddev);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(BBP_EDEVICE, "autotune events");
  }
  for (const auto& kv : shapes) {
    auto hit = cache.find(kv.first);
    if (hit != cache.end()) {
      chosen[kv.first] = hit->second;
      continue;
    }
    const LaunchRec& r = *kv.second.first;
    // the launch's descriptors with every output redirected to a private
    // buffer (operands are only read), so timing leaves the state untouched
    std::vector<GemmDesc> d(kv.second.second, kv.second.second + r.count);
    int64_t ext = 0, mM = 1, mN = 1;
    for (const GemmDesc& g : d) {
      ext = std::max(ext, gemm_out_extent(g));
      mM = std::max<int64_t>(mM, g.M);
      mN = std::max<int64_t>(mN, g.N);
    }
    const size_t need = size_t(ext) * d.size();
    if (need > tmp_len) {
      if (tmp) hipFree(tmp);
      tmp = nullptr;
      if (hipMalloc(&tmp, need * sizeof(cplx)) != hipSuccess) { rc = fail(BBP_ENOMEM, "autotune buffer"); break; }
      tmp_len = need;
    }
    for (size_t i = 0; i < d.size(); ++i) d[i].C = tmp + int64_t(i) * ext;
    if (d.size() * sizeof(GemmDesc) > ddev_len) {
      if (ddev) hipFree(ddev);
      ddev = nullptr;
      if (hipMalloc(&ddev, d.size() * sizeof(GemmDesc)) != hipSuccess) { rc = fail(BBP_ENOMEM, "autotune descriptors"); break; }
      ddev_len = d.size() * sizeof(GemmDesc);
    }
    if (hipMemcpyAsync(ddev, d.data(), d.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
      rc = fail(BBP_EDEVICE, "autotune upload");
      break;
    }
    int best = -1;
    float best_ms = 0.0f;
    for (int v = 0; v <= 4 && rc == BBP_OK; ++v) {
      LaunchRec t = r;
      t.variant = v;
      t.desc_off = 0;
      t.grid = gemm_grid(v, mM, mN, int(d.size()));
      float ms = 0.0f;
      hipError_t e = launch(ddev, h->stream, t);   // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = launch(ddev, h->stream, t);
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) { rc = fail(BBP_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
      if (best < 0 || ms < best_ms) { best = v; best_ms = ms; }
    }
    if (rc != BBP_OK) break;
    chosen[kv.first] = best;
    timed += 1;
  }
  if (rc == BBP_OK) rc = hipStreamSynchronize(h->stream) == hipSuccess ? BBP_OK : fail(BBP_EDEVICE, "autotune sync");
  cleanup();
  if (rc != BBP_OK) return rc;
  h->gemm_tiles = chosen;
  if (!save_tile_cache(cache_path, chosen)) return fail(BBP_EINVAL, "cannot write the tile cache");
  if (n_timed) *n_timed = timed;
  if (n_shapes) *n_shapes = int32_t(chosen.size());
  // recompile every plan with the chosen tiles (results are unchanged: a
  // tile shape does not change any element's sum order)
  free_subsets(h);
  rc = build_launches(h);
  if (rc) return rc;
  if (h->blob_fixed) hipHostFree(h->blob_fixed);
  h->blob_fixed = nullptr;
  h->fixed_ready = false;
  return prepare_fixed(h);
}

int32_t pepsnet_memory(pepsnet_t h, int64_t* resident_bytes, int64_t* workspace_bytes) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (resident_bytes)
    *resident_bytes = h->arena_len * int64_t(sizeof(cplx)) +
                      int64_t(h->comp->n_scalars) * int64_t(sizeof(double)) +
                      int64_t(h->desc_host.size()) +
                      int64_t(h->bonds.size()) * int64_t(17 * sizeof(cplx));
  if (workspace_bytes) *workspace_bytes = h->work_len * int64_t(sizeof(cplx));
  return BBP_OK;
}

int32_t pepsnet_release_workspace(pepsnet_t h) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (!h->work) return BBP_OK;
  PN_HIP(hipStreamSynchronize(h->stream));
  for (Compiled* c : {&h->sweep[0], &h->sweep[1], &h->expect[0], &h->expect[1],
                      &h->sweep_serial[0], &h->sweep_serial[1]}) {
    if (c->exec) hipGraphExecDestroy(c->exec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
  }
  PN_HIP(hipFree(h->work));
  h->work = nullptr;
  h->work_epoch += 1;
  return BBP_OK;
}

int32_t pepsnet_acquire_workspace(pepsnet_t h) {
  if (!h) return fail(BBP_EINVAL, "null handle");
  if (h->work) return BBP_OK;
  if (hipMalloc(&h->work, size_t(h->work_len) * sizeof(cplx)) != hipSuccess) {
    h->work = nullptr;
    return fail(BBP_ENOMEM, "workspace allocation of " + std::to_string(h->work_len * 16) +
                                " bytes failed");
  }
  PN_HIP(hipMemsetAsync(h->work, 0, size_t(h->work_len) * sizeof(cplx), h->stream));
  h->work_epoch += 1;
  return build_launches(h);
}

int32_t pepsnet_batch_create(const pepsnet_t* hs, int32_t n, void* stream, pepsnet_batch_t* out) {
  if (!hs || n < 1 || !out) return fail(BBP_EINVAL, "bad arguments");
  std::unique_ptr<pepsnet_batch_s> b(new pepsnet_batch_s());
  for (int i = 0; i < n; ++i) {
    if (!hs[i]) return fail(BBP_EINVAL, "null handle in batch");
    for (int k = 0; k < i; ++k)
      if (hs[k] == hs[i]) return fail(BBP_EINVAL, "handle listed twice in batch");
    if (!hs[i]->work) return fail(BBP_EINVAL, "a handle of the batch has no workspace");
    b->hs.push_back(hs[i]);
    b->base_parity.push_back(hs[i]->parity);
    b->work_epoch.push_back(hs[i]->work_epoch);
  }
  if (stream) {
    b->stream = static_cast<hipStream_t>(stream);
  } else {
    PN_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->own_stream = true;
  }
  for (int v = 0; v < 2; ++v) {
    std::vector<OpSource> srcs;
    for (int i = 0; i < n; ++i)
      srcs.push_back({b->hs[i], &b->hs[i]->sweep_lanes[b->base_parity[i] ^ v]});
    compile_ops(srcs, &b->desc_host[v], &b->sweep[v]);
    if (hipMalloc(&b->desc_dev[v], std::max<size_t>(b->desc_host[v].size(), 256)) != hipSuccess)
      return fail(BBP_ENOMEM, "batch descriptor allocation failed");
    PN_HIP(hipMemcpyAsync(b->desc_dev[v], b->desc_host[v].data(), b->desc_host[v].size(),
                          hipMemcpyHostToDevice, b->stream));
    b->sweep[v].desc = b->desc_dev[v];
  }
  PN_HIP(hipEventCreate(&b->ev0));
  PN_HIP(hipEventCreate(&b->ev1));
  PN_HIP(hipStreamSynchronize(b->stream));
  *out = b.release();
  return BBP_OK;
}

int32_t pepsnet_batch_use_graph(pepsnet_batch_t b, int32_t on) {
  if (!b) return fail(BBP_EINVAL, "null batch");
  b->use_graph = on != 0;
  return BBP_OK;
}

int32_t blockbp_sweep_batch(pepsnet_batch_t b, int32_t sweeps, double* max_err, double* ms) {
  if (!b || sweeps < 0) return fail(BBP_EINVAL, "bad arguments");
  const int n = int(b->hs.size());
  const int v = b->hs[0]->parity ^ b->base_parity[0];
  for (int i = 0; i < n; ++i) {
    if ((b->hs[i]->parity ^ b->base_parity[i]) != v)
      return fail(BBP_EINVAL, "a handle of the batch was swept on its own; recreate the batch");
    if (b->hs[i]->work_epoch != b->work_epoch[i])
      return fail(BBP_EINVAL, "a handle's workspace moved since the batch was made");
  }
  // work already queued on the handles' own streams comes first
  for (pepsnet_s* h : b->hs) PN_HIP(hipStreamSynchronize(h->stream));
  std::vector<double> errs(n, 0.0);
  double total_ms = 0.0;
  for (int s = 0; s < sweeps; ++s) {
    const int var = b->hs[0]->parity ^ b->base_parity[0];
    for (pepsnet_s* h : b->hs) {
      h->pinned[0] = double(h->sweeps_total);
      PN_HIP(hipMemcpyAsync(h->scal + Compiler::kSweepSlot, h->pinned, sizeof(double),
                            hipMemcpyHostToDevice, b->stream));
    }
    PN_HIP(hipEventRecord(b->ev0, b->stream));
    int32_t rc = run_launches(b->stream, &b->sweep[var], b->use_graph);
    if (rc) return rc;
    PN_HIP(hipEventRecord(b->ev1, b->stream));
    for (pepsnet_s* h : b->hs) {
      const int nm = int(h->P.msg_keys.size());
      PN_HIP(hipMemcpyAsync(h->pinned + 1, h->scal + h->comp->err_slot(0), nm * sizeof(double),
                            hipMemcpyDeviceToHost, b->stream));
    }
    PN_HIP(hipStreamSynchronize(b->stream));
    float e_ms = 0.0f;
    PN_HIP(hipEventElapsedTime(&e_ms, b->ev0, b->ev1));
    total_ms += e_ms;
    // every handle was swept: advance all of them, then report
    bool finite = true;
    for (int i = 0; i < n; ++i) {
      pepsnet_s* h = b->hs[i];
      const int nm = int(h->P.msg_keys.size());
      finite = close_sweep(&h->parity, &h->sweeps_total, h->pinned + 1, nm, &errs[i]) && finite;
    }
    if (!finite) {
      b->last_ms = total_ms;
      if (max_err)
        for (int i = 0; i < n; ++i) max_err[i] = errs[i];
      if (ms) *ms = total_ms;
      return fail(BBP_ENUMERIC, "non-finite message after a sweep");
    }
  }
  b->last_ms = total_ms;
  if (max_err)
    for (int i = 0; i < n; ++i) max_err[i] = errs[i];
  if (ms) *ms = total_ms;
  return BBP_OK;
}

int32_t pepsnet_batch_stats(pepsnet_batch_t b, double* gemm_flops, int64_t* launches) {
  if (!b) return fail(BBP_EINVAL, "null batch");
  const int v = b->hs[0]->parity ^ b->base_parity[0];
  if (gemm_flops) *gemm_flops = b->sweep[v].gemm_flops;
  if (launches) *launches = int64_t(b->sweep[v].launches.size());
  return BBP_OK;
}

void pepsnet_batch_destroy(pepsnet_batch_t b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  for (int v = 0; v < 2; ++v) {
    if (b->sweep[v].exec) hipGraphExecDestroy(b->sweep[v].exec);
    if (b->sweep[v].graph) hipGraphDestroy(b->sweep[v].graph);
    if (b->desc_dev[v]) hipFree(b->desc_dev[v]);
  }
  if (b->ev0) hipEventDestroy(b->ev0);
  if (b->ev1) hipEventDestroy(b->ev1);
  if (b->own_stream && b->stream) hipStreamDestroy(b->stream);
  delete b;
}

int32_t bbp_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, bbp_server_t* out) {
  if (!out || hbm_budget_bytes < 0 || max_inflight < 1) return fail(BBP_EINVAL, "bad arguments");
  bbp_server_s* S = new bbp_server_s();
  S->budget = hbm_budget_bytes;
  S->max_inflight = max_inflight;
  if (hipEventCreate(&S->ev_ref) != hipSuccess || hipEventRecord(S->ev_ref, nullptr) != hipSuccess ||
      hipEventSynchronize(S->ev_ref) != hipSuccess) {
    if (S->ev_ref) hipEventDestroy(S->ev_ref);
    delete S;
    return fail(BBP_EDEVICE, "server clock event failed");
  }
  S->worker = std::thread(srv_loop, S);
  *out = S;
  return BBP_OK;
}

int32_t bbp_server_submit(bbp_server_t S, pepsnet_t state, const double* new_sites,
                          int64_t sites_len, double tol, int32_t max_sweeps, uint64_t* ticket) {
  if (!S || !state || !ticket || max_sweeps < 0) return fail(BBP_EINVAL, "bad arguments");
  if (new_sites && sites_len != state->site_len)
    return fail(BBP_EINVAL, "site tensor buffer has the wrong length");
  if (!state->work && state->work_len * int64_t(sizeof(cplx)) > S->budget)
    return fail(BBP_ENOMEM, "the state's workspace exceeds the server's HBM budget");
  SrvReq* r = new SrvReq();
  r->h = state;
  if (new_sites) r->sites.assign(new_sites, new_sites + sites_len);
  r->tol = tol;
  r->max_sweeps = max_sweeps;
  r->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete r;
      return fail(BBP_EINVAL, "server is shutting down");
    }
    r->ticket = S->next_ticket++;
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
  }
  S->cv_work.notify_one();
  *ticket = r->ticket;
  return BBP_OK;
}

int32_t bbp_server_poll(bbp_server_t S, uint64_t ticket, int32_t wait, double* energy_per_site,
                        double* bond_ss, int32_t cap, int32_t* n_bonds, int32_t* sweeps_done,
                        double* max_err, double* latency_s, double* gpu_window_ms) {
  if (!S) return fail(BBP_EINVAL, "null server");
  SrvReq* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(BBP_EINVAL, "unknown or already collected ticket");
    r = it->second;
    auto finished = [&] { return r->ready; };
    if (!finished()) {
      if (!wait) return BBP_PENDING;
      S->cv_done.wait(lk, finished);
    }
    S->reqs.erase(it);
  }
  std::unique_ptr<SrvReq> own(r);
  const int nb = int(r->ss.size());
  if (n_bonds) *n_bonds = nb;
  if (bond_ss)
    for (int b = 0; b < std::min(nb, int(cap)); ++b) bond_ss[b] = r->ss[b];
  if (energy_per_site) *energy_per_site = r->energy;
  if (sweeps_done) *sweeps_done = r->sweeps;
  if (max_err) *max_err = r->err;
  if (latency_s)
    *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  if (gpu_window_ms) {
    gpu_window_ms[0] = r->window_ms[0];
    gpu_window_ms[1] = r->window_ms[1];
  }
  if (r->rc < 0) return fail(r->rc, "request failed");
  return r->rc;
}

int32_t bbp_server_stats(bbp_server_t S, int64_t* peak_bytes, int32_t* peak_inflight,
                         int64_t* completed, int32_t* queued, int64_t* slot_allocations) {
  if (!S) return fail(BBP_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (slot_allocations) *slot_allocations = S->slot_allocs.load();
  if (peak_bytes) *peak_bytes = S->peak_in_use;
  if (peak_inflight) *peak_inflight = S->peak_inflight;
  if (completed) *completed = S->completed;
  if (queued) *queued = int32_t(S->queue.size());
  return BBP_OK;
}

void bbp_server_destroy(bbp_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& kv : S->reqs) delete kv.second;
  for (auto& sl : S->slots)
    if (sl->ptr) hipFree(sl->ptr);
  if (S->ev_ref) hipEventDestroy(S->ev_ref);
  delete S;
}

void pepsnet_destroy(pepsnet_t h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  for (Compiled* c : {&h->sweep[0], &h->sweep[1], &h->expect[0], &h->expect[1], &h->prep,
                      &h->sweep_serial[0], &h->sweep_serial[1]}) {
    if (c->exec) hipGraphExecDestroy(c->exec);
    if (c->graph) hipGraphDestroy(c->graph);
  }
  if (h->arena) hipFree(h->arena);
  if (h->work) hipFree(h->work);
  if (h->scal) hipFree(h->scal);
  if (h->desc_dev) hipFree(h->desc_dev);
  free_subsets(h);
  if (h->rho_mat) hipFree(h->rho_mat);
  if (h->ss_dev) hipFree(h->ss_dev);
  if (h->ops_dev) hipFree(h->ops_dev);
  if (h->ops_out) hipFree(h->ops_out);
  if (h->meas_dev) hipFree(h->meas_dev);
  if (h->pinned) hipHostFree(h->pinned);
  if (h->blob_fixed) hipHostFree(h->blob_fixed);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  for (int g = 0; g < kMaxStreams - 1; ++g)
    if (h->join_ev[g]) hipEventDestroy(h->join_ev[g]);
  if (h->fork_ev) hipEventDestroy(h->fork_ev);
  if (h->own_stream && h->stream) hipStreamDestroy(h->stream);
  delete h;
}

int32_t pepsnet_describe(const pepsnet_desc* desc, int32_t what, int32_t a, int32_t b,
                         int32_t n_open, const int32_t* open_sites, int32_t* buf, int64_t cap,
                         int64_t* len) {
  if (!desc) return fail(BBP_EINVAL, "null descriptor");
  Problem P;
  std::string e = build_problem(desc, &P);
  if (!e.empty()) return fail(BBP_EGEOM, e);
  std::vector<int32_t> out;
  if (what == 0) {
    if (a < 0 || a >= int(P.blocks.size())) return fail(BBP_EINVAL, "bad block");
    out.push_back(int32_t(P.faces[a].size()));
    for (auto& f : P.faces[a]) {
      out.push_back(f.keytype);
      out.push_back(f.key);
      out.push_back(int32_t(f.legs.size()));
      for (auto& sl : f.legs) { out.push_back(sl.first); out.push_back(sl.second); }
    }
  } else if (what == 1) {
    if (a < 0 || a >= int(P.blocks.size())) return fail(BBP_EINVAL, "bad block");
    std::vector<int> opens;
    for (int k = 0; k < n_open; ++k) opens.push_back(open_sites[k]);
    Schedule sc;
    e = sweep_schedule(P, a, b, opens, &sc);
    if (!e.empty()) return fail(BBP_EGEOM, e);
    out.push_back(int32_t(sc.steps.size()));
    for (auto& st : sc.steps) {
      out.push_back(st.site);
      out.push_back(st.pos);
      out.push_back(int32_t(st.in_slots.size()));
      out.push_back(int32_t(st.out_slots.size()));
      for (int x : st.in_slots) out.push_back(x);
      for (int x : st.out_slots) out.push_back(x);
      out.push_back(st.open ? 1 : 0);
      out.push_back(st.absorb);
    }
    out.push_back(int32_t(sc.final_legs.size()));
    for (auto& sl : sc.final_legs) { out.push_back(sl.first); out.push_back(sl.second); }
  } else if (what == 2) {
    out = {int32_t(P.sites.size()), int32_t(P.blocks.size()), int32_t(P.msg_keys.size()),
           int32_t(P.kind == 1 ? 6 : P.bonds().size())};
  } else {
    return fail(BBP_EINVAL, "unknown query");
  }
  if (len) *len = int64_t(out.size());
  if (buf) {
    if (cap < int64_t(out.size())) return fail(BBP_EINVAL, "buffer too small");
    std::memcpy(buf, out.data(), out.size() * sizeof(int32_t));
  }
  return BBP_OK;
}

}  // extern "C"
