// Plan compiler: turns the geometry's sweep orders into static device
// operations (see plan.hpp).
//
// Boundary chain (Sec. "The boundary-MPS method"): a chain site is a tensor
// A[l, P, r] whose leg P fuses (ket, bra, carried pairs...) row-major, ket and
// bra of the leg's bond dimension D (double leg I = k*D + b), each carried
// pair of an open site d*d (p*d + p').  Bond dimensions are static: a
// factorisation of an m x n matrix keeps min(m, n) columns, a truncated
// split keeps min(chi_env, m, n); stored messages are zero-padded to the MPS
// caps min(chi, prod of leg dims on each side).
//
// Per swallowed site (ket tensor t[p, slots]) with in-legs at chain
// positions pos..pos+r-1 and out-legs o_1..o_s:
//   1. canonical moves: QR steps to the right / LQ steps to the left bring
//      the orthogonality centre into the run (Sec. "Canonical MPS");
//   2. merge the run: Theta[a, L_1 .. L_r, b] by r-1 GEMMs;
//   3. absorb the ket (GEMM over the in-legs' ket indices) and the bra
//      (GEMM over p and the in-legs' bra indices; p kept open for an open
//      site), with three tensor transposes around the two GEMMs;
//   4. split Theta'[a, O_1 .. O_s, b] left to right into s sites with
//      truncated SVDs: T1 exact (Householder QR + one-sided Jacobi), or T2
//      randomized range finder with q power iterations and p oversampling
//      (Halko, Martinsson & Tropp 2011, Alg. 4.4) on a SplitMix64 sign
//      sketch, then the same exact small SVD;
//   5. normalise the centre and accumulate log10 of its norm (Sec.
//      "Mantissa and Exponent").
// A site with no out-leg leaves a bond matrix that is absorbed into the
// chain neighbour.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <functional>

namespace pn {
namespace {

// largest fully merged in-leg run (complex elements) before the swallow
// switches to the progressive contraction order
constexpr int64_t kMergedPeakElems = int64_t(1) << 25;
// narrowest truncated SVD block that goes through bidiagonalisation instead
// of one-sided Jacobi (measured crossover on 144-row blocks)
constexpr int64_t kSvdTopMinCols = 72;
constexpr int64_t kSvdTopWideCols = 112;   // from here also when most columns are kept

uint64_t mix_out0(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t key_prefix(uint64_t seed, const std::vector<uint64_t>& tags) {
  uint64_t k = seed;
  for (uint64_t t : tags) k = mix_out0(k ^ t);
  return k;
}

int64_t prod(const std::vector<int>& v) {
  int64_t p = 1;
  for (int x : v) p *= x;
  return p;
}

int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

}  // namespace

// ----------------------------------------------------------------- lane
struct Compiler::Lane {
  Compiler* C;
  int id;
  LaneOps* out;
  // Every buffer of the lane gets a fresh offset in one virtual space while
  // the plan is built (so each reference names exactly one buffer); once
  // the lane's ops are final, pack_lane() places the buffers by liveness.
  int64_t vtop = 0;
  std::vector<std::pair<int64_t, int64_t>> vallocs;   // (virtual offset, size)
  int stage = 0, step = 0, phase = 0, counter = 0;
  // launch keys: within a stage the lanes are independent, so each lane's
  // ops are keyed by (stage, SVDs emitted so far in the stage, index since
  // the last SVD) and every SVD by (stage, its index): the k-th truncated
  // SVDs of all lanes share one launch, whatever their swallow schedules
  int key_stage = -1, svd_seq = 0, seg_idx = 0;
  std::string err;

  Lane(Compiler* c, int lane, LaneOps* o) : C(c), id(lane), out(o) {}

  int rg_chain() const { return RG_LANE0 + 2 * id; }
  Ref valloc(int64_t n) {
    const int64_t sz = std::max<int64_t>((n + 7) / 8 * 8, 8);
    Ref r{rg_chain(), vtop};
    vallocs.push_back({vtop, sz});
    vtop += sz;
    return r;
  }
  // chain tensors and per-swallow temporaries differ only in lifetime,
  // which the packing reads from the ops
  Ref chain_alloc(int64_t n) { return valloc(n); }
  Ref scratch(int64_t n) { return valloc(n); }
  void reset_scratch() {}
  void at(int st, int sp, int ph) {
    if (st != stage || sp != step || ph != phase) counter = 0;
    stage = st; step = sp; phase = ph;
  }
  // the next op shares the launch of the previous one (independent ops of
  // one step, e.g. the chunks of a split Gram product)
  bool join_next = false;
  void push(const Op& op) {
    if (join_next && !out->ops.empty() && stage == key_stage) {
      join_next = false;
      ++counter;
      out->ops.push_back({out->ops.back().first, op});
      return;
    }
    join_next = false;
    if (stage != key_stage) {
      key_stage = stage;
      svd_seq = 0;
      seg_idx = 0;
    }
    WaveKey k;
    if (op.type == OPK_JACOBI) {
      k.k = {stage, svd_seq++, 1 << 30};
      seg_idx = 0;
    } else {
      k.k = {stage, svd_seq, seg_idx++};
    }
    ++counter;
    out->ops.push_back({k, op});
  }

  // ------------------------------------------------------------ emitters
  // A product with a long K and few output tiles is split over K: S partial
  // products (one launch, S times the workgroups) into scratch, then their
  // sum in a fixed order (deterministic).  Output tiles as the executor's
  // tile choice: 64 x 64, 64 x 80 for 64 < N <= 80, 80 x 64 for 64 < M <= 80.
  static int64_t gemm_tiles(int64_t M, int64_t N) {
    const int64_t tm = (M > 64 && M <= 80) ? 80 : M <= 16 ? 16 : 64;
    const int64_t tn = (N > 64 && N <= 80) ? 80 : N <= 16 ? 16 : 64;
    return ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
  }
  static int gemm_split(int64_t M, int64_t N, int64_t K) {
    if (K < 1024 || M <= 16 || N <= 16 || gemm_tiles(M, N) > 64) return 1;
    return int(std::min<int64_t>(8, K / 512));
  }
  void gemm(Ref A, Ref B, Ref Cc, int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb,
            int64_t ldc, int opA, int opB, int prec, int contraction = 0, double ar = 1.0,
            double ai = 0.0, double br = 0.0, double bi = 0.0) {
    const int S = (br == 0.0 && bi == 0.0) ? gemm_split(M, N, K) : 1;
    if (S > 1) {
      const int64_t kc = (K + S - 1) / S;
      Ref Pp = scratch(int64_t(S) * M * N);
      for (int s = 0; s < S; ++s) {
        const int64_t k0 = s * kc, ks = std::min(kc, K - k0);
        const Ref As{A.region, A.off + (opA == OP_N ? k0 : k0 * lda)};
        const Ref Bs{B.region, B.off + (opB == OP_N ? k0 * ldb : k0)};
        const Ref Ps{Pp.region, Pp.off + s * M * N};
        join_next = s > 0;
        gemm(As, Bs, Ps, M, N, ks, lda, ldb, N, opA, opB, prec, contraction);
      }
      Op op;
      op.type = OPK_SUM;
      op.a = Pp; op.c = Cc;
      op.i[0] = S; op.i[1] = M; op.i[2] = N; op.i[3] = ldc;
      op.x[0] = ar; op.x[1] = ai;
      push(op);
      return;
    }
    Op op;
    op.type = OPK_GEMM;
    op.a = A; op.b = B; op.c = Cc;
    op.i[0] = M; op.i[1] = N; op.i[2] = K;
    op.i[3] = lda; op.i[4] = ldb; op.i[5] = ldc;
    op.i[6] = opA; op.i[7] = opB; op.i[8] = prec; op.i[9] = contraction;
    op.x[0] = ar; op.x[1] = ai; op.x[2] = br; op.x[3] = bi;
    push(op);
  }
  // dst = transpose(src) with output axis k = input axis perm[k]
  void perm(Ref src, Ref dst, const std::vector<int>& dims, const std::vector<int>& pm,
            int conj = 0) {
    int n = int(dims.size());
    std::vector<int64_t> st(n, 1);
    for (int k = n - 2; k >= 0; --k) st[k] = st[k + 1] * dims[k + 1];
    std::vector<int> od;
    std::vector<int64_t> os;
    for (int k = 0; k < n; ++k) {
      int ax = pm[k];
      if (dims[ax] == 1) continue;
      if (!od.empty() && os.back() == st[ax] * dims[ax]) {  // merge contiguous axes
        od.back() *= dims[ax];
        os.back() = st[ax];
        continue;
      }
      od.push_back(dims[ax]);
      os.push_back(st[ax]);
    }
    if (od.empty()) { od.push_back(1); os.push_back(1); }
    if (od.size() > 16) { err = "tensor rank too large for the transpose kernel"; return; }
    Op op;
    op.type = OPK_PERM;
    op.a = src; op.b = dst;
    op.i[0] = int64_t(od.size());
    op.i[1] = conj;
    for (size_t k = 0; k < od.size(); ++k) { op.i[2 + k] = od[k]; op.i[18 + k] = os[k]; }
    push(op);
  }
  // Q may be an invalid Ref: only R is produced; with qh, Q^H (k x m) is
  // written in place of Q
  // R may be invalid when only Q is wanted (the Cholesky QR then skips it)
  void qr(Ref A, int64_t m, int64_t n, int64_t lda, int conjT, Ref Q, Ref R, bool qh = false) {
    if (std::min(m, n) > 256) { err = "QR width above 256"; return; }
    const int kq = qr_kernel(m, n, Q.valid());
    if (kq == QRK_CHOL) {
      cholqr(A, m, n, lda, conjT, Q, R, qh);
      return;
    }
    if (kq == QRK_TALL && m >= n && n <= 2 * CHOLQR_MAXN) {
      cholqr_panels(A, m, n, lda, conjT, Q, R, qh);
      return;
    }
    if (!R.valid()) R = scratch(std::min(m, n) * n);
    Op op;
    op.type = OPK_QR;
    op.a = A; op.b = scratch(m * (n + (Q.valid() ? std::min(m, n) : 0))); op.c = Q; op.d = R;
    op.i[0] = m; op.i[1] = n; op.i[2] = lda; op.i[3] = conjT; op.i[4] = qh ? 1 : 0;
    push(op);
  }
  // Tall QR (m >= n, n <= CHOLQR_MAXN) on many workgroups: Cholesky QR in
  // three passes, the first with the shift of Fukaya et al. (2020), which
  // keeps it stable for condition numbers up to about 1e12, the other two
  // restoring orthogonality to rounding (CholeskyQR2).  Each pass: the Gram
  // matrix Y^H Y as partial products over row chunks (one launch) and their
  // sum, k_chol (Cholesky, R^-1, running R), then Y R^-1 (a GEMM).  The last pass's
  // product is skipped when Q is not wanted, and writes Q^H with qh.
  void cholqr(Ref A, int64_t m, int64_t n, int64_t lda, int conjT, Ref Q, Ref R, bool qh,
              int64_t ldq = 0) {
    if (ldq <= 0) ldq = n;
    int64_t rb = std::max<int64_t>(144, (m + 31) / 32);
    rb = (rb + 15) / 16 * 16;
    const int64_t S = (m + rb - 1) / rb;
    Ref Gp = scratch(S * n * n), G1 = scratch(n * n), Rinv = scratch(n * n);
    Ref cur = A;
    int64_t cld = lda;
    int cT = conjT;
    for (int pass = 0; pass < 3; ++pass) {
      for (int64_t s = 0; s < S; ++s) {
        const int64_t r0 = s * rb, rows = std::min(rb, m - r0);
        const Ref G{Gp.region, Gp.off + s * n * n};
        join_next = s > 0;
        if (!cT) {
          const Ref X{cur.region, cur.off + r0 * cld};
          gemm(X, X, G, n, n, rows, cld, cld, n, OP_C, OP_N, PREC_FP64);
        } else {
          const Ref X{cur.region, cur.off + r0};
          gemm(X, X, G, n, n, rows, cld, cld, n, OP_N, OP_C, PREC_FP64);
        }
      }
      // the partials summed in order over many workgroups, so that the
      // one-workgroup Cholesky reads a single matrix
      Op sum;
      sum.type = OPK_SUM;
      sum.a = Gp; sum.c = G1;
      sum.i[0] = S; sum.i[1] = n; sum.i[2] = n; sum.i[3] = n;
      sum.x[0] = 1.0; sum.x[1] = 0.0;
      push(sum);
      Op op;
      op.type = OPK_CHOL;
      op.a = G1; op.b = Rinv; op.c = R;
      op.i[0] = 1; op.i[1] = n; op.i[2] = pass == 0; op.i[3] = pass > 0; op.i[4] = m;
      push(op);
      const bool last = pass == 2;
      if (last && !Q.valid()) break;
      Ref out = last ? Q : scratch(m * n);
      if (last && qh)   // Q^H = R^-H Y^H (n x m)
        gemm(Rinv, cur, out, n, m, n, n, cld, m, OP_C, cT ? OP_N : OP_C, PREC_FP64);
      else
        gemm(cur, Rinv, out, m, n, n, cld, n, last ? ldq : n, cT ? OP_C : OP_N, OP_N, PREC_FP64);
      cur = out;
      cld = n;
      cT = 0;
    }
  }
  // Strided copy: dst (contiguous, shape dims) <- src at element offsets
  // sum_k idx_k * strides[k], conjugated with conj.
  void gather(Ref src, Ref dst, const std::vector<int64_t>& dims,
              const std::vector<int64_t>& strides, int conj) {
    Op op;
    op.type = OPK_PERM;
    op.a = src; op.b = dst;
    op.i[0] = int64_t(dims.size());
    op.i[1] = conj;
    for (size_t k = 0; k < dims.size(); ++k) { op.i[2 + k] = dims[k]; op.i[18 + k] = strides[k]; }
    push(op);
  }
  // Tall QR with CHOLQR_MAXN < n <= 2 CHOLQR_MAXN: two column panels, each
  // factorised by Cholesky QR; the second panel is projected off the first
  // panel's Q twice (block classical Gram-Schmidt with reorthogonalisation)
  // before its factorisation.  R = [[R11, R12], [0, R22]] with R12 the sum
  // of the two projections' coefficients; diag(R) stays real non-negative.
  void cholqr_panels(Ref A, int64_t m, int64_t n, int64_t lda, int conjT, Ref Q, Ref R, bool qh) {
    const int64_t n1 = (n / 2 + 15) / 16 * 16, n2 = n - n1;
    const Ref Qn = (Q.valid() && !qh) ? Q : scratch(m * n);
    const bool want_r = R.valid();
    Ref R11 = want_r ? scratch(n1 * n1) : Ref(), R22 = want_r ? scratch(n2 * n2) : Ref();
    // panel 1: columns [0, n1) of op(A)
    cholqr(A, m, n1, lda, conjT, Qn, R11, false, n);
    // panel 2 as a dense m x n2 copy, then X -= Q1 (Q1^H X) twice
    Ref X = scratch(m * n2);
    if (!conjT)
      gather(Ref{A.region, A.off + n1}, X, {m, n2}, {lda, 1}, 0);
    else
      gather(Ref{A.region, A.off + n1 * lda}, X, {m, n2}, {1, lda}, 1);
    Ref Sc = scratch(2 * n1 * n2);
    for (int pass = 0; pass < 2; ++pass) {
      const Ref Sp{Sc.region, Sc.off + pass * n1 * n2};
      gemm(Qn, X, Sp, n1, n2, m, n, n2, n2, OP_C, OP_N, PREC_FP64);
      gemm(Qn, Sp, X, m, n2, n1, n, n2, n2, OP_N, OP_N, PREC_FP64, 0, -1.0, 0.0, 1.0, 0.0);
    }
    const Ref Q2{Qn.region, Qn.off + n1};
    cholqr(X, m, n2, n2, 0, Q2, R22, false, n);
    if (want_r) {
      Ref R12 = scratch(n1 * n2);
      Op sum;
      sum.type = OPK_SUM;
      sum.a = Sc; sum.c = R12;
      sum.i[0] = 2; sum.i[1] = n1; sum.i[2] = n2; sum.i[3] = n2;
      sum.x[0] = 1.0; sum.x[1] = 0.0;
      push(sum);
      pad(R11, R, int(n1), 1, int(n1), int(n), int(n), 0, 0, 0);
      pad(R12, R, int(n1), 1, int(n2), int(n), int(n), 0, int(n1), 1);
      pad(R22, R, int(n2), 1, int(n2), int(n), int(n), int(n1), int(n1), 1);
    }
    if (Q.valid() && qh)   // Q^H (n x m) from Qn (m x n)
      gather(Qn, Q, {n, m}, {1, n}, 1);
  }
  // leading `keep` left singular vectors U (rows x keep) and values of the
  // rows x cols matrix A (element (i, c) at A[i*lda + c], conj(A[c*lda + i])
  // with conjT)
  // with gauge, the top-k kernel also fixes the columns' gauge (as colphase
  // does); returns whether it did
  bool jacobi(Ref A, int64_t rows, int64_t cols, int64_t lda, int conjT, int64_t keep, Ref U,
              Ref sig, bool gauge = false) {
    if (rows > kJacobiMaxRows) { err = "Jacobi SVD with more than 144 rows"; return false; }
    if (cols > rows || cols > kJacobiMaxCols) { err = "Jacobi SVD needs cols <= rows"; return false; }
    Op op;
    op.type = OPK_JACOBI;
    // wide blocks with a truncated rank go through bidiagonalisation: its
    // cost grows like cols^3 once plus cols^2 per kept value, the Jacobi
    // sweeps' like cols^3 per sweep; below 112 columns Jacobi stays ahead
    // when most columns are kept (72x72 keeping 64: 1.8 against 2.1 ms)
    const bool top = keep < cols && cols >= kSvdTopMinCols &&
                     (2 * keep <= cols || cols >= kSvdTopWideCols);
    op.a = A; op.c = U; op.d = sig;
    op.b = scratch(top ? svd_top_work_elems(rows, cols, keep) : jacobi_work_elems(rows, cols));
    op.i[0] = rows; op.i[1] = cols; op.i[2] = lda; op.i[3] = conjT; op.i[4] = keep;
    op.i[5] = top ? 1 : 0;
    op.i[6] = top && gauge ? 1 : 0;
    push(op);
    return top && gauge;
  }
  void omega(Ref dst, int64_t n, int64_t k, uint64_t prefix, bool sweep_tag) {
    Op op;
    op.type = OPK_OMEGA;
    op.a = dst;
    op.i[0] = n; op.i[1] = k; op.i[2] = sweep_tag ? 1 : 0;
    op.key = prefix;
    push(op);
  }
  void norm(Ref x, int64_t len, int64_t logslot, int64_t normslot) {
    Op op;
    op.type = OPK_NORM;
    op.a = x;
    op.b = scratch(NORM_CHUNKS / 2);   // partial sums (doubles)
    op.i[0] = len;
    op.s0.off = logslot;
    op.s1.off = normslot;
    push(op);
  }
  void pad(Ref src, Ref dst, int l1, int P, int r1, int l2, int r2, int offl, int offr,
           int mode, double sign = 1.0) {
    Op op;
    op.type = OPK_PAD;
    op.a = src; op.b = dst;
    op.i[0] = l1; op.i[1] = P; op.i[2] = r1; op.i[3] = l2; op.i[4] = r2;
    op.i[5] = offl; op.i[6] = offr; op.i[7] = mode;
    op.x[0] = sign;
    push(op);
  }
  void phase_fix(const std::vector<CSite>& sites) {
    if (sites.size() > 16) { err = "message longer than 16 legs"; return; }
    Op op;
    op.type = OPK_PHASE;
    op.i[0] = int64_t(sites.size());
    for (size_t j = 0; j < sites.size(); ++j) {
      op.refs.push_back(sites[j].buf);
      op.i[1 + 4 * j] = sites[j].l;
      op.i[2 + 4 * j] = sites[j].P;
      op.i[3 + 4 * j] = sites[j].r;
      op.i[4 + 4 * j] = sites[j].D;
    }
    push(op);
  }

  void colphase(Ref L, Ref R, int64_t m, int64_t keep, int64_t n) {
    Op op;
    op.type = OPK_COLPHASE;
    op.a = L; op.b = R;
    op.i[0] = m; op.i[1] = keep; op.i[2] = n;
    push(op);
  }

  // ------------------------------------------------------ chain operations
  // left-canonicalise site j, push R into j+1
  void move_right(std::vector<CSite>& ch, int j) {
    CSite& A = ch[j];
    CSite& B = ch[j + 1];
    int64_t m = int64_t(A.l) * A.P, n = A.r, k = std::min(m, n);
    Ref Q = chain_alloc(m * k), R = scratch(k * n);
    qr(A.buf, m, n, n, 0, Q, R);
    Ref NB = chain_alloc(k * B.P * B.r);
    gemm(R, B.buf, NB, k, int64_t(B.P) * B.r, n, n, int64_t(B.P) * B.r, int64_t(B.P) * B.r,
         OP_N, OP_N, PREC_FP64);
    A.buf = Q; A.r = int(k);
    B.buf = NB; B.l = int(k);
  }
  // right-canonicalise site j, push L into j-1
  void move_left(std::vector<CSite>& ch, int j) {
    CSite& A = ch[j];
    CSite& B = ch[j - 1];
    int64_t m = int64_t(A.P) * A.r, n = A.l, k = std::min(m, n);
    // A^H (m x n) = Q' R'  ->  A = R'^H Q'^H; the QR writes Q'^H directly
    Ref NA = chain_alloc(k * m), Rp = scratch(k * n);
    qr(A.buf, m, n, m, 1, NA, Rp, true);
    Ref NB = chain_alloc(int64_t(B.l) * B.P * k);
    gemm(B.buf, Rp, NB, int64_t(B.l) * B.P, k, n, n, n, k, OP_N, OP_C, PREC_FP64);
    A.buf = NA; A.l = int(k);
    B.buf = NB; B.r = int(k);
  }
  void move_center(std::vector<CSite>& ch, int& center, int lo, int hi) {
    while (center < lo) { move_right(ch, center); ++center; }
    while (center > hi) { move_left(ch, center); --center; }
  }

  // truncated split of the m x n matrix M: writes L (m x keep) and R (keep x n)
  // (chi_keep > 0: keep min(chi_keep, m, n) values by the exact SVD, the
  // compression of an exactly contracted message)
  int split(Ref M, int64_t m, int64_t n, Ref Lout, Ref Rout, uint64_t prefix, bool sweep_tag,
            int* keep_out, int64_t chi_keep = 0) {
    const PlanOptions& o = C->opt;
    int64_t full = std::min(m, n);
    int64_t keep = chi_keep > 0 ? std::min(chi_keep, full)
                 : o.chi_env > 0 ? std::min<int64_t>(o.chi_env, full) : full;
    *keep_out = int(keep);
    bool t2 = chi_keep <= 0 && o.trunc == 1 && o.chi_env > 0 && o.chi_env + o.p < full;
    if (t2) {
      int64_t k = o.chi_env + o.p;
      Ref Om = scratch(n * k);
      omega(Om, n, k, prefix, sweep_tag);
      Ref Y = scratch(m * k);
      gemm(M, Om, Y, m, k, n, n, k, k, OP_N, OP_N, o.precision, 1);
      for (int it = 0; it < o.q; ++it) {
        Ref Qy = scratch(m * k);
        qr(Y, m, k, k, 0, Qy, Ref());
        Ref Z = scratch(n * k);
        gemm(M, Qy, Z, n, k, m, n, k, k, OP_C, OP_N, o.precision, 1);
        Ref Qz = scratch(n * k);
        qr(Z, n, k, k, 0, Qz, Ref());
        Y = scratch(m * k);
        gemm(M, Qz, Y, m, k, n, n, k, k, OP_N, OP_N, o.precision, 1);
      }
      Ref Q = scratch(m * k);
      qr(Y, m, k, k, 0, Q, Ref());
      // B = Q^H M (k x n) = R3^H Q3^H with B^H = Q3 R3; the columns of R3^H
      // rotated to orthogonality are U Sigma of B, so M ~ (Q U) Sigma (...)^H
      Ref B = scratch(k * n);
      gemm(Q, M, B, k, n, m, k, n, n, OP_C, OP_N, o.precision, 1);
      Ref R3 = scratch(k * k);
      qr(B, n, k, n, 1, Ref(), R3);
      Ref U = scratch(k * keep), sig = scratch(keep);
      jacobi(R3, k, k, k, 1, keep, U, sig);
      gemm(Q, U, Lout, m, keep, k, k, keep, keep, OP_N, OP_N, PREC_FP64);
      gemm(U, B, Rout, keep, n, k, keep, n, n, OP_C, OP_N, PREC_FP64);
      colphase(Lout, Rout, m, keep, n);
      return 0;
    }
    // where L is the SVD's U itself, the top-k kernel fixes the gauge before
    // R = L^H M is formed, so R follows without the colphase pass
    bool gauged = false;
    if (m >= n && m <= kJacobiMaxRows) {
      // M W = U Sigma directly on the columns of M
      Ref sig = scratch(keep);
      gauged = jacobi(M, m, n, n, 0, keep, Lout, sig, true);
      gemm(Lout, M, Rout, keep, n, m, keep, n, n, OP_C, OP_N, PREC_FP64);
    } else if (m < n) {
      // M^H = Q3 R3, M = R3^H Q3^H: the left singular vectors of M are those
      // of R3^H (m x m, the conjugated rows of R3); Q3 is not needed
      Ref R3 = scratch(m * m);
      qr(M, n, m, n, 1, Ref(), R3);
      Ref sig = scratch(keep);
      gauged = jacobi(R3, m, m, m, 1, keep, Lout, sig, true);
      gemm(Lout, M, Rout, keep, n, m, keep, n, n, OP_C, OP_N, PREC_FP64);
    } else {
      // tall: M = Q R, left singular vectors Q U with U those of R (n x n)
      Ref Q = scratch(m * n), R = scratch(n * n);
      qr(M, m, n, n, 0, Q, R);
      Ref U = scratch(n * keep), sig = scratch(keep);
      jacobi(R, n, n, n, 0, keep, U, sig);
      gemm(Q, U, Lout, m, keep, n, n, keep, keep, OP_N, OP_N, PREC_FP64);
      gemm(U, R, Rout, keep, n, n, keep, n, n, OP_C, OP_N, PREC_FP64);
    }
    if (!gauged) colphase(Lout, Rout, m, keep, n);
    return 0;
  }

  // swallow one site; stepno used for wave alignment and the sketch tags
  void swallow(std::vector<CSite>& ch, int& center, const Step& st, int stepno,
               const std::vector<uint64_t>& tag_head, bool sweep_tag) {
    const Problem& P = C->prob;
    const PlanOptions& o = C->opt;
    const int pos = st.pos, r = int(st.in_slots.size()), s = int(st.out_slots.size());
    const int t = P.sites[st.site].tensor;
    const std::vector<int>& td = C->tensor_dims[t];
    const int d = td[0];
    reset_scratch();
    at(stage, stepno, 0);
    move_center(ch, center, pos, pos + r - 1);
    // --- merge the in-leg run and absorb the ket tensor.  Two orders give
    // the same Y[a, (b_j, Q_j)..., b, p, ko...]:
    //   merged:      multiply the run into Theta[a, (k_j b_j Q_j)..., b]
    //                (a D^(2r) b elements), then one GEMM over all k_j;
    //   progressive: contract the ket tensor with the first chain site over
    //                k_1, then each further site over its left bond and k_j
    //                together (intermediates of a D^r d Kout chi elements).
    // The merged order is used when its Theta is small and it is not more
    // expensive; the progressive one otherwise (many in-legs, large D).
    at(stage, stepno, 1);
    const int64_t a = ch[pos].l, b = ch[pos + r - 1].r;
    std::vector<int> Din(r), Qin(r), carry_ids;
    for (int j = 0; j < r; ++j) {
      Din[j] = ch[pos + j].D;
      Qin[j] = ipow(d * d, int(ch[pos + j].carries.size()));
      for (int c : ch[pos + j].carries) carry_ids.push_back(c);
      if (Din[j] != td[1 + st.in_slots[j]]) { err = "leg dimension mismatch"; return; }
    }
    std::vector<int> Dout(s);
    for (int j = 0; j < s; ++j) Dout[j] = td[1 + st.out_slots[j]];
    if (st.open) carry_ids.push_back(st.site);
    auto sm = C->ensure_smat(t, st.in_slots, st.out_slots, st.open);
    const int64_t Kin = prod(Din), Qtot_in = prod(Qin), Kout = prod(Dout);
    int64_t M1 = a * b * Kin * Qtot_in;     // rows (a, b_j, Q_j, b)
    int64_t N1 = d * Kout;
    // cost model (complex multiply-adds) and peak intermediate of each order
    double merged_cma = 0.0, prog_cma = 0.0;
    double merged_peak = double(a) * ch[pos].P * ch[pos].r, prog_peak = 0.0;
    {
      double rows = double(a) * ch[pos].P;
      for (int j = 1; j < r; ++j) {
        const CSite& A = ch[pos + j];
        merged_cma += rows * double(A.P) * A.r * A.l;
        rows *= A.P;
        merged_peak = std::max(merged_peak, rows * A.r);
      }
      merged_cma += double(M1) * Kin * N1;
      merged_peak = std::max(merged_peak, double(M1) * N1);
      double rest = double(a) * Din[0] * Qin[0] * (double(Kin) / Din[0]) * d * Kout;
      prog_cma += rest * ch[pos].r * Din[0];
      prog_peak = rest * ch[pos].r;
      for (int j = 1; j < r; ++j) {
        const CSite& A = ch[pos + j];
        rest = rest / Din[j] * Din[j] * Qin[j];   // kk_j out, (b_j, Q_j) in
        prog_cma += rest * A.l * Din[j] * A.r;
        prog_peak = std::max(prog_peak, rest * A.r);
      }
    }
    const bool progressive =
        r > 1 && (o.order == 2 || (o.order == 0 && (merged_peak > double(kMergedPeakElems) ||
                                                    prog_cma < merged_cma)));
    Ref Y;
    if (!progressive) {
      Ref th = ch[pos].buf;
      int64_t rows = int64_t(ch[pos].l) * ch[pos].P, bb = ch[pos].r;
      for (int j = 1; j < r; ++j) {
        const CSite& A = ch[pos + j];
        Ref dst = scratch(rows * A.P * A.r);
        gemm(th, A.buf, dst, rows, int64_t(A.P) * A.r, bb, bb, int64_t(A.P) * A.r,
             int64_t(A.P) * A.r, OP_N, OP_N, o.precision, 1);
        th = dst;
        rows *= A.P;
        bb = A.r;
      }
      at(stage, stepno, 2);
      // theta axes: 0 = a, 1+3j = k_j, 2+3j = b_j, 3+3j = Q_j, 1+3r = b
      std::vector<int> thd = {int(a)};
      for (int j = 0; j < r; ++j) { thd.push_back(Din[j]); thd.push_back(Din[j]); thd.push_back(Qin[j]); }
      thd.push_back(int(b));
      std::vector<int> p1 = {0};
      for (int j = 0; j < r; ++j) { p1.push_back(2 + 3 * j); p1.push_back(3 + 3 * j); }
      p1.push_back(1 + 3 * r);
      for (int j = 0; j < r; ++j) p1.push_back(1 + 3 * j);
      Ref X = scratch(M1 * Kin);
      perm(th, X, thd, p1);
      Y = scratch(M1 * N1);
      gemm(X, sm.first, Y, M1, N1, Kin, Kin, N1, N1, OP_N, OP_N, o.precision, 1);
    } else {
      // axis ids: a, bond x, p, chain ket k_j, bra b_j, carry Q_j, pending
      // ket-tensor leg kk_j, ket out-leg ko_m
      enum { AX_A = 0, AX_X = 1, AX_P = 2 };
      auto AX_K = [](int j) { return 100 + j; };
      auto AX_B = [](int j) { return 200 + j; };
      auto AX_Q = [](int j) { return 300 + j; };
      auto AX_KK = [](int j) { return 400 + j; };
      auto AX_KO = [](int m) { return 500 + m; };
      struct Axes { std::vector<int> id, dim; };
      auto reorder = [&](Ref src, const Axes& in, const std::vector<int>& order, Axes* out) {
        std::vector<int> pm;
        out->id = order;
        out->dim.clear();
        for (int id : order) {
          int k = int(std::find(in.id.begin(), in.id.end(), id) - in.id.begin());
          pm.push_back(k);
          out->dim.push_back(in.dim[k]);
        }
        Ref dst = scratch(prod(out->dim));
        perm(src, dst, in.dim, pm);
        return dst;
      };
      // chain site [a, (k_0 b_0 Q_0), x] -> rows (a, b_0, Q_0, x), cols k_0
      Axes c0{{AX_A, AX_K(0), AX_B(0), AX_Q(0), AX_X},
              {int(a), Din[0], Din[0], Qin[0], ch[pos].r}};
      Axes xm;
      Ref Xm = reorder(ch[pos].buf, c0, {AX_A, AX_B(0), AX_Q(0), AX_X, AX_K(0)}, &xm);
      const int64_t M0 = a * Din[0] * Qin[0] * ch[pos].r;
      const int64_t N0 = (Kin / Din[0]) * d * Kout;
      Y = scratch(M0 * N0);
      gemm(Xm, sm.first, Y, M0, N0, Din[0], Din[0], N0, N0, OP_N, OP_N, o.precision, 1);
      Axes ya{{AX_A, AX_B(0), AX_Q(0), AX_X}, {int(a), Din[0], Qin[0], ch[pos].r}};
      for (int j = 1; j < r; ++j) { ya.id.push_back(AX_KK(j)); ya.dim.push_back(Din[j]); }
      ya.id.push_back(AX_P);
      ya.dim.push_back(d);
      for (int m = 0; m < s; ++m) { ya.id.push_back(AX_KO(m)); ya.dim.push_back(Dout[m]); }
      for (int j = 1; j < r; ++j) {
        // contract (x, kk_j) of Y with (x, k_j) of chain site j [x, (k_j b_j Q_j), x']
        const CSite& A = ch[pos + j];
        std::vector<int> order;
        for (int id : ya.id)
          if (id != AX_X && id != AX_KK(j)) order.push_back(id);
        const int64_t Mj = prod(ya.dim) / (int64_t(A.l) * Din[j]);
        order.push_back(AX_X);
        order.push_back(AX_KK(j));
        Axes ym;
        Ref Ym = reorder(Y, ya, order, &ym);
        const int64_t Kj = int64_t(A.l) * Din[j], Nj = int64_t(Din[j]) * Qin[j] * A.r;
        Ref Yn = scratch(Mj * Nj);
        gemm(Ym, A.buf, Yn, Mj, Nj, Kj, Kj, Nj, Nj, OP_N, OP_N, o.precision, 1);
        ya.id.assign(order.begin(), order.end() - 2);
        ya.dim.assign(ym.dim.begin(), ym.dim.end() - 2);
        ya.id.push_back(AX_B(j)); ya.dim.push_back(Din[j]);
        ya.id.push_back(AX_Q(j)); ya.dim.push_back(Qin[j]);
        ya.id.push_back(AX_X); ya.dim.push_back(A.r);
        Y = Yn;
      }
      at(stage, stepno, 2);
      // to the layout [a, (b_j, Q_j)..., b, p, ko...]
      std::vector<int> order = {AX_A};
      for (int j = 0; j < r; ++j) { order.push_back(AX_B(j)); order.push_back(AX_Q(j)); }
      order.push_back(AX_X);
      order.push_back(AX_P);
      for (int m = 0; m < s; ++m) order.push_back(AX_KO(m));
      if (order != ya.id) {
        Axes yo;
        Y = reorder(Y, ya, order, &yo);
      }
    }
    // Y axes: 0 = a, 1+2j = b_j, 2+2j = Q_j, 1+2r = b, 2+2r = p, 3+2r+m = ko_m
    std::vector<int> yd = {int(a)};
    for (int j = 0; j < r; ++j) { yd.push_back(Din[j]); yd.push_back(Qin[j]); }
    yd.push_back(int(b));
    yd.push_back(d);
    for (int m = 0; m < s; ++m) yd.push_back(Dout[m]);
    std::vector<int> p2 = {0, 1 + 2 * r};
    for (int j = 0; j < r; ++j) p2.push_back(2 + 2 * j);
    if (st.open) p2.push_back(2 + 2 * r);
    for (int m = 0; m < s; ++m) p2.push_back(3 + 2 * r + m);
    if (!st.open) p2.push_back(2 + 2 * r);
    for (int j = 0; j < r; ++j) p2.push_back(1 + 2 * j);
    Ref Z = scratch(M1 * N1);
    perm(Y, Z, yd, p2);
    int64_t K2 = (st.open ? 1 : d) * Kin;
    int64_t N2 = (st.open ? d : 1) * Kout;
    int64_t M2 = M1 * N1 / K2;
    Ref W = scratch(M2 * N2);
    gemm(Z, sm.second, W, M2, N2, K2, K2, N2, N2, OP_N, OP_N, o.precision, 1);
    // W axes (not open): 0 = a, 1 = b, 2+j = Q_j, 2+r+m = ko_m, 2+r+s+m = bo_m
    // W axes (open):     0 = a, 1 = b, 2+j = Q_j, 2+r = p, 3+r+m = ko_m,
    //                    3+r+s = p', 4+r+s+m = bo_m
    std::vector<int> wd = {int(a), int(b)};
    for (int j = 0; j < r; ++j) wd.push_back(Qin[j]);
    if (st.open) wd.push_back(d);
    for (int m = 0; m < s; ++m) wd.push_back(Dout[m]);
    if (st.open) wd.push_back(d);
    for (int m = 0; m < s; ++m) wd.push_back(Dout[m]);
    const int ko0 = st.open ? 3 + r : 2 + r;
    const int bo0 = st.open ? 4 + r + s : 2 + r + s;
    std::vector<int> p3 = {0};
    if (s > 0) { p3.push_back(ko0); p3.push_back(bo0); }
    for (int j = 0; j < r; ++j) p3.push_back(2 + j);
    if (st.open) { p3.push_back(2 + r); p3.push_back(3 + r + s); }
    for (int m = 1; m < s; ++m) { p3.push_back(ko0 + m); p3.push_back(bo0 + m); }
    p3.push_back(1);
    int64_t Qtot = ipow(d * d, int(carry_ids.size()));
    std::vector<int> phys(s);
    for (int m = 0; m < s; ++m) phys[m] = Dout[m] * Dout[m];
    if (s > 0) phys[0] *= int(Qtot);
    const int64_t thp_len = M2 * N2;
    if (s == 0) {
      Ref Tp = scratch(thp_len);
      perm(W, Tp, wd, p3);
      // Theta'[a, Q, b] absorbed into a neighbour
      if (st.absorb == 0) {
        CSite& Nb = ch[pos + r];
        Ref G = scratch(a * Qtot * Nb.P * Nb.r);
        gemm(Tp, Nb.buf, G, a * Qtot, int64_t(Nb.P) * Nb.r, b, b, int64_t(Nb.P) * Nb.r,
             int64_t(Nb.P) * Nb.r, OP_N, OP_N, PREC_FP64);
        Ref NS = chain_alloc(a * Qtot * Nb.P * Nb.r);
        perm(G, NS, {int(a), int(Qtot), Nb.P, Nb.r}, {0, 2, 1, 3});
        Nb.buf = NS;
        Nb.l = int(a);
        Nb.P = int(Nb.P * Qtot);
        for (int c : carry_ids) Nb.carries.push_back(c);
        at(stage, stepno, 4);
        norm(NS, int64_t(Nb.l) * Nb.P * Nb.r, C->logscale_slot(id), -1);
        ch.erase(ch.begin() + pos, ch.begin() + pos + r);
        center = pos;
      } else {
        CSite& Nb = ch[pos - 1];
        Ref NS = chain_alloc(int64_t(Nb.l) * Nb.P * Qtot * b);
        gemm(Nb.buf, Tp, NS, int64_t(Nb.l) * Nb.P, Qtot * b, a, a, Qtot * b, Qtot * b, OP_N,
             OP_N, PREC_FP64);
        Nb.buf = NS;
        Nb.r = int(b);
        Nb.P = int(Nb.P * Qtot);
        for (int c : carry_ids) Nb.carries.push_back(c);
        at(stage, stepno, 4);
        norm(NS, int64_t(Nb.l) * Nb.P * Nb.r, C->logscale_slot(id), -1);
        ch.erase(ch.begin() + pos, ch.begin() + pos + r);
        center = pos - 1;
      }
      return;
    }
    Ref Tp = (s == 1) ? chain_alloc(thp_len) : scratch(thp_len);
    perm(W, Tp, wd, p3);
    // --- split left to right
    at(stage, stepno, 3);
    std::vector<CSite> news;
    int64_t left = a;
    Ref rest = Tp;
    for (int m = 0; m < s - 1; ++m) {
      int64_t rws = left * phys[m];
      int64_t cols = b;
      for (int u = m + 1; u < s; ++u) cols *= phys[u];
      int64_t full = std::min(rws, cols);
      int64_t keep = o.chi_env > 0 ? std::min<int64_t>(o.chi_env, full) : full;
      Ref L = chain_alloc(rws * keep);
      Ref R = (m == s - 2) ? chain_alloc(keep * cols) : scratch(keep * cols);
      std::vector<uint64_t> tags = tag_head;
      tags.push_back(uint64_t(stepno));
      tags.push_back(uint64_t(m));
      int kk = 0;
      split(rest, rws, cols, L, R, key_prefix(o.seed, tags), sweep_tag, &kk);
      CSite ns;
      ns.buf = L; ns.l = int(left); ns.P = phys[m]; ns.r = kk; ns.D = Dout[m];
      if (m == 0) ns.carries = carry_ids;
      news.push_back(ns);
      rest = R;
      left = kk;
    }
    CSite last;
    last.buf = rest; last.l = int(left); last.P = phys[s - 1]; last.r = int(b); last.D = Dout[s - 1];
    if (s == 1) last.carries = carry_ids;
    news.push_back(last);
    at(stage, stepno, 4);
    norm(last.buf, int64_t(last.l) * last.P * last.r, C->logscale_slot(id), -1);
    ch.erase(ch.begin() + pos, ch.begin() + pos + r);
    ch.insert(ch.begin() + pos, news.begin(), news.end());
    center = pos + s - 1;
  }

  // chain from face legs of block b: faces after ``target`` counter-clockwise;
  // ``override_face`` replaces one face's message by the given sites
  std::vector<CSite> initial_chain(int blk, int target, int msg_region,
                                   int override_face, const std::vector<CSite>* ovr) {
    const Problem& P = C->prob;
    const std::vector<Face>& F = P.faces[blk];
    int nf = int(F.size());
    std::vector<CSite> ch;
    for (int k = 1; k < nf; ++k) {
      int f = (target + k) % nf;
      if (f == override_face && ovr) {
        for (auto& x : *ovr) ch.push_back(x);
        continue;
      }
      int slot = P.incoming_msg(blk, f);
      for (size_t j = 0; j < F[f].legs.size(); ++j) {
        const auto& sl = F[f].legs[j];
        int D = C->tensor_dims[P.sites[sl.first].tensor][1 + sl.second];
        CSite cs;
        cs.D = D;
        if (slot < 0) {
          cs.buf = Ref{RG_CONST, 0};   // trivial message: [1] on a dimension-1 leg
          cs.l = 1; cs.P = 1; cs.r = 1;
          if (D != 1) { err = "trivial face with a non-trivial leg"; }
        } else {
          cs.buf = Ref{msg_region, C->msg.off[slot][j]};
          cs.l = C->msg.bl[slot][j];
          cs.P = C->msg.P[slot][j];
          cs.r = C->msg.br[slot][j];
        }
        ch.push_back(cs);
      }
    }
    return ch;
  }

  std::vector<CSite> run_sweep(int blk, int target, const std::vector<int>& open_sites,
                               int msg_region, const std::vector<uint64_t>& tag_head,
                               bool sweep_tag, int override_face,
                               const std::vector<CSite>* ovr,
                               std::vector<std::pair<int, int>>* final_legs, int* center_out) {
    Schedule sc;
    std::string e = sweep_schedule(C->prob, blk, target, open_sites, &sc);
    if (!e.empty()) { err = e; return {}; }
    std::vector<CSite> ch = initial_chain(blk, target, msg_region, override_face, ovr);
    int center = 0;
    for (size_t n = 0; n < sc.steps.size() && err.empty(); ++n)
      swallow(ch, center, sc.steps[n], int(n), tag_head, sweep_tag);
    *final_legs = sc.final_legs;
    *center_out = center;
    return ch;
  }

  void reverse_chain(std::vector<CSite>& ch, int& center) {
    std::vector<CSite> rv;
    for (int j = int(ch.size()) - 1; j >= 0; --j) {
      CSite x = ch[j];
      Ref nb = chain_alloc(int64_t(x.l) * x.P * x.r);
      perm(x.buf, nb, {x.l, x.P, x.r}, {2, 1, 0});
      x.buf = nb;
      std::swap(x.l, x.r);
      rv.push_back(x);
    }
    center = int(ch.size()) - 1 - center;
    ch = rv;
  }

  void right_canonical(std::vector<CSite>& ch, int& center) {
    move_center(ch, center, int(ch.size()) - 1, int(ch.size()) - 1);
    move_center(ch, center, 0, 0);
    norm(ch[0].buf, int64_t(ch[0].l) * ch[0].P * ch[0].r, C->logscale_slot(id), -1);
  }

  // Message of an exactly contracted block (no truncation inside the
  // update), right-canonical with the centre at site 0: truncated to bond
  // chi left to right by exact SVDs, then brought back to right-canonical
  // form with unit norm.
  void compress(std::vector<CSite>& ch, int& center) {
    const int n = int(ch.size());
    for (int j = 0; j + 1 < n; ++j) {
      CSite& A = ch[j];
      CSite& B = ch[j + 1];
      const int64_t m = int64_t(A.l) * A.P, cols = A.r;
      const int64_t keep = std::min<int64_t>(C->opt.chi, std::min(m, cols));
      Ref Lq = chain_alloc(m * keep), Rq = scratch(keep * cols);
      int kk = 0;
      split(A.buf, m, cols, Lq, Rq, 0, false, &kk, C->opt.chi);
      const int64_t bn = int64_t(B.P) * B.r;
      Ref NB = chain_alloc(int64_t(kk) * bn);
      gemm(Rq, B.buf, NB, kk, bn, cols, cols, bn, bn, OP_N, OP_N, PREC_FP64);
      A.buf = Lq; A.r = kk;
      B.buf = NB; B.l = kk;
    }
    center = n - 1;
    right_canonical(ch, center);
  }

  // a A + b B for two open MPS on the same legs (Sec. "BlockBP Learning-step":
  // MPS addition after Schollwoeck 2011): the bond spaces are the direct sums of
  // the two, with the first site [a A, b B] along its right bond, inner
  // sites block diagonal and the last site stacked along its left bond.
  // The sum is brought to right-canonical form with unit norm and, where a
  // bond exceeds chi, compressed to chi by exact truncated SVDs.
  std::vector<CSite> compressed_sum(const std::vector<CSite>& A, const std::vector<CSite>& B,
                                    double a, double b, int& center) {
    const int n = int(A.size());
    std::vector<CSite> S(n);
    for (int j = 0; j < n; ++j) {
      const CSite& x = A[j];
      const CSite& y = B[j];
      CSite z = x;
      z.l = (j == 0) ? 1 : x.l + y.l;
      z.r = (j == n - 1) ? 1 : x.r + y.r;
      z.buf = chain_alloc(int64_t(z.l) * z.P * z.r);
      const double sa = (j == 0) ? a : 1.0, sb = (j == 0) ? b : 1.0;
      const int offl = (j == 0) ? 0 : x.l, offr = (j == n - 1) ? 0 : x.r;
      pad(x.buf, z.buf, x.l, x.P, x.r, z.l, z.r, 0, 0, 0, sa);
      // one site: both terms land on the same elements, so add
      pad(y.buf, z.buf, y.l, y.P, y.r, z.l, z.r, offl, offr, n == 1 ? 2 : 1, sb);
      S[j] = z;
    }
    center = 0;
    right_canonical(S, center);
    bool over = false;
    for (const CSite& x : S) over = over || x.r > C->opt.chi;
    if (over) compress(S, center);
    return S;
  }
};

// ------------------------------------------------------------- compiler
Compiler::Compiler(const Problem& P, const PlanOptions& o) : prob(P), opt(o) {
  // tensor dims: legs to outside a finite patch have dimension 1
  int nt = P.n_tensors();
  tensor_dims.assign(nt, {});
  tensor_off.assign(nt, 0);
  for (size_t s = 0; s < P.sites.size(); ++s) {
    int t = P.sites[s].tensor;
    if (!tensor_dims[t].empty()) continue;
    std::vector<int> dims = {opt.d};
    for (int l = 0; l < P.sites[s].nslot; ++l)
      dims.push_back(P.links[s][l].type == LINK_OUTSIDE ? 1 : opt.D);
    tensor_dims[t] = dims;
  }
  int64_t off = 0;
  for (int t = 0; t < nt; ++t) {
    tensor_off[t] = off;
    off += prod(tensor_dims[t]);
  }
  site_region_size = off;
  // message layout: caps min(chi, prod of leg dims on each side)
  int nm = int(P.msg_keys.size());
  msg.off.resize(nm); msg.bl.resize(nm); msg.br.resize(nm); msg.P.resize(nm); msg.D.resize(nm);
  int64_t moff = 0;
  for (int m = 0; m < nm; ++m) {
    const auto& legs = P.stored_legs(m);
    int n = int(legs.size());
    std::vector<int> pd(n), Ds(n);
    for (int j = 0; j < n; ++j) {
      Ds[j] = tensor_dims[P.sites[legs[j].first].tensor][1 + legs[j].second];
      pd[j] = Ds[j] * Ds[j];
    }
    std::vector<int64_t> capb(n + 1, 1);
    for (int j = 1; j < n; ++j) {
      int64_t lp = 1, rp = 1;
      for (int u = 0; u < j; ++u) lp = std::min<int64_t>(lp * pd[u], 1 << 30);
      for (int u = j; u < n; ++u) rp = std::min<int64_t>(rp * pd[u], 1 << 30);
      capb[j] = std::min<int64_t>(std::min<int64_t>(opt.chi, lp), rp);
    }
    for (int j = 0; j < n; ++j) {
      msg.off[m].push_back(moff);
      msg.bl[m].push_back(int(capb[j]));
      msg.br[m].push_back(int(capb[j + 1]));
      msg.P[m].push_back(pd[j]);
      msg.D[m].push_back(Ds[j]);
      moff += (capb[j] * pd[j] * capb[j + 1] + 7) / 8 * 8;
    }
  }
  msg.size = moff;
  n_scalars = 1024 + nm + 8;
}

std::pair<Ref, Ref> Compiler::ensure_smat(int tensor, const std::vector<int>& in_slots,
                                          const std::vector<int>& out_slots, bool open) {
  SiteMatKey k{tensor, in_slots, out_slots, open};
  auto it = smat.find(k);
  if (it != smat.end()) return it->second;
  const std::vector<int>& td = tensor_dims[tensor];
  int64_t len = prod(td);
  Ref ket{RG_SMAT, smat_size};
  smat_size += (len + 7) / 8 * 8;
  Ref bra{RG_SMAT, smat_size};
  smat_size += (len + 7) / 8 * 8;
  smat[k] = {ket, bra};
  // ket: [k_in..., p, k_out...]; bra: [p, b_in..., b_out...] or, for an open
  // site, [b_in..., p', b_out...] (complex conjugated)
  std::vector<int> pk, pb;
  for (int l : in_slots) pk.push_back(1 + l);
  pk.push_back(0);
  for (int l : out_slots) pk.push_back(1 + l);
  if (!open) pb.push_back(0);
  for (int l : in_slots) pb.push_back(1 + l);
  if (open) pb.push_back(0);
  for (int l : out_slots) pb.push_back(1 + l);
  Ref src{RG_SITE, tensor_off[tensor]};
  auto mk = [&](Ref dst, const std::vector<int>& pm, int conj) {
    Op op;
    op.type = OPK_PERM;
    op.a = src; op.b = dst;
    int n = int(td.size());
    std::vector<int64_t> stv(n, 1);
    for (int q = n - 2; q >= 0; --q) stv[q] = stv[q + 1] * td[q + 1];
    op.i[0] = n; op.i[1] = conj;
    for (int q = 0; q < n; ++q) { op.i[2 + q] = td[pm[q]]; op.i[18 + q] = stv[pm[q]]; }
    prep_ops.push_back(op);
  };
  mk(ket, pk, 0);
  mk(bra, pb, 1);
  return smat[k];
}

namespace {

bool same_ref(const Ref& x, const Ref& y) { return x.region == y.region && x.off == y.off; }

// Does op q touch buffer r, and only as an output (so that the contents it
// held before are dead)?  Every reference in a plan names a whole buffer.
// Returns 0: not touched, 1: written only, 2: read.
int touches(const Op& q, const Ref& r) {
  const bool a = same_ref(q.a, r), b = same_ref(q.b, r), c = same_ref(q.c, r),
             d = same_ref(q.d, r);
  bool ref = false;
  for (const Ref& x : q.refs) ref = ref || same_ref(x, r);
  if (!(a || b || c || d || ref)) return 0;
  if (ref) return 2;
  switch (q.type) {
    case OPK_GEMM: return (a || b || (c && (q.x[2] != 0.0 || q.x[3] != 0.0))) ? 2 : 1;
    case OPK_PERM: return a ? 2 : 1;
    case OPK_PAD: return (a || q.i[7] != 0) ? 2 : 1;   // modes 1, 2 keep the rest of dst
    case OPK_QR: case OPK_JACOBI: return a ? 2 : 1;
    case OPK_OMEGA: return 1;
    default: return 2;
  }
}

// [lo, hi) element range of a GEMM operand stored rows x cols with leading
// dimension ld, or transposed
void operand_range(const Ref& x, bool trans, int64_t rows, int64_t cols, int64_t ld,
                   int64_t* lo, int64_t* hi) {
  *lo = x.off;
  *hi = x.off + (trans ? (cols - 1) * ld + rows : (rows - 1) * ld + cols);
}

// A transpose that only reads the output of the GEMM just before it is
// folded into that GEMM's store: the GEMM writes the transposed layout
// directly (one launch and one pass over the data fewer).  Applies when the
// GEMM writes a dense lane buffer without accumulating, the destination
// does not overlap the GEMM's operands, and no later op of the lane reads
// the untransposed buffer.
void fuse_gemm_perm(LaneOps& L) {
  auto& ops = L.ops;
  std::vector<bool> drop(ops.size(), false);
  for (size_t p = 1; p < ops.size(); ++p) {
    Op& g = ops[p - 1].second;
    const Op& t = ops[p].second;
    if (t.type != OPK_PERM || g.type != OPK_GEMM || drop[p - 1] || g.i[10] != 0) continue;
    if (!same_ref(g.c, t.a) || g.c.region < RG_LANE0) continue;
    if (g.x[2] != 0.0 || g.x[3] != 0.0) continue;
    const int64_t M = g.i[0], N = g.i[1], K = g.i[2];
    if (g.i[5] != N || M < 1 || N < 1) continue;
    // the transpose: output axis k has extent od[k] and source stride os[k]
    const int n = int(t.i[0]);
    struct Ax { int64_t dim, src, dst; };
    std::vector<Ax> ax(n);
    int64_t total = 1;
    for (int k = n - 1; k >= 0; --k) {
      ax[k] = Ax{t.i[2 + k], t.i[18 + k], total};
      total *= ax[k].dim;
    }
    if (total != M * N) continue;
    // source order (slowest first) must be a dense mixed radix
    std::sort(ax.begin(), ax.end(), [](const Ax& x, const Ax& y) { return x.src > y.src; });
    bool ok = true;
    for (int k = 0; k < n; ++k)
      ok = ok && ax[k].src == (k + 1 < n ? ax[k + 1].src * ax[k + 1].dim : 1);
    if (!ok) continue;
    // split at the column extent N: axes below it index the GEMM column
    std::vector<Ax> rows, cols;
    int64_t prod = 1;
    for (int k = n - 1; k >= 0; --k) {
      const Ax& x = ax[k];
      if (prod == N) { rows.insert(rows.begin(), x); continue; }
      if (prod * x.dim <= N) { cols.insert(cols.begin(), x); prod *= x.dim; continue; }
      if (N % prod != 0 || x.dim % (N / prod) != 0) { ok = false; break; }
      const int64_t f = N / prod;
      cols.insert(cols.begin(), Ax{f, x.src, x.dst});
      rows.insert(rows.begin(), Ax{x.dim / f, x.src * f, x.dst * f});
      prod = N;
    }
    if (!ok || prod != N) continue;
    if (int(rows.size() + cols.size()) > GEMM_SC_MAX) continue;
    for (const Ax& x : rows) ok = ok && x.dim <= 65536;
    for (const Ax& x : cols) ok = ok && x.dim <= 65536;
    if (!ok) continue;
    // destination apart from the operands
    if (t.b.region == g.a.region || t.b.region == g.b.region) {
      int64_t lo, hi;
      const int64_t dlo = t.b.off, dhi = t.b.off + M * N;
      if (t.b.region == g.a.region) {
        operand_range(g.a, g.i[6] != OP_N, M, K, g.i[3], &lo, &hi);
        if (lo < dhi && dlo < hi) continue;
      }
      if (t.b.region == g.b.region) {
        operand_range(g.b, g.i[7] != OP_N, K, N, g.i[4], &lo, &hi);
        if (lo < dhi && dlo < hi) continue;
      }
    }
    // the untransposed buffer must be dead after the transpose
    int use = 0;
    for (size_t q = p + 1; q < ops.size() && use == 0; ++q) use = touches(ops[q].second, t.a);
    if (use == 2) continue;
    int k = 0;
    for (const Ax& x : rows) { g.i[16 + k] = x.dim; g.i[32 + k] = x.dst; ++k; }
    for (const Ax& x : cols) { g.i[16 + k] = x.dim; g.i[32 + k] = x.dst; ++k; }
    g.i[10] = k;
    g.i[11] = int64_t(rows.size());
    g.i[12] = t.i[1];
    g.c = t.b;
    drop[p] = true;
  }
  // compact in place (an element is never moved onto itself: a self-moved
  // vector comes out empty)
  size_t w = 0;
  for (size_t p = 0; p < ops.size(); ++p) {
    if (drop[p]) continue;
    if (w != p) ops[w] = std::move(ops[p]);
    ++w;
  }
  ops.resize(w);
}

// Place the lane's buffers (virtual offsets in `region`, allocations
// `va` in increasing order) by liveness and rewrite every reference;
// returns the region size.  Time runs over the lane's ops in order, ops of a
// joined group (same wave key, launched together) sharing one time step; a
// buffer's memory is reused by a buffer first touched strictly after the
// last op touching it (best fit from the freed blocks, else the top); the
// region size is the high-water mark of the placement.
int64_t pack_lane(LaneOps& L, const std::vector<std::pair<int64_t, int64_t>>& va, int region) {
  const size_t na = va.size();
  if (na == 0) return 0;
  std::vector<int64_t> first(na, -1), last(na, -1);
  auto find = [&](int64_t off) {
    size_t lo = 0, hi = na;
    while (hi - lo > 1) {
      const size_t mid = (lo + hi) / 2;
      if (va[mid].first <= off) lo = mid; else hi = mid;
    }
    return lo;
  };
  std::vector<int64_t> tstep(L.ops.size());
  int64_t t = -1;
  for (size_t p = 0; p < L.ops.size(); ++p) {
    if (p == 0 || L.ops[p].first < L.ops[p - 1].first || L.ops[p - 1].first < L.ops[p].first) ++t;
    tstep[p] = t;
    const Op& op = L.ops[p].second;
    auto touch = [&](const Ref& r) {
      if (r.region != region) return;
      const size_t a = find(r.off);
      if (first[a] < 0) first[a] = t;
      last[a] = t;
    };
    touch(op.a); touch(op.b); touch(op.c); touch(op.d);
    for (const Ref& r : op.refs) touch(r);
  }
  std::vector<size_t> order;
  for (size_t a = 0; a < na; ++a)
    if (first[a] >= 0) order.push_back(a);
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return first[x] < first[y]; });
  std::vector<int64_t> real(na, 0);
  std::map<int64_t, int64_t> freeb;                     // offset -> size
  std::multimap<int64_t, size_t> active;               // last time -> allocation
  int64_t top = 0, high = 0;   // current top of the used space, its high-water mark
  for (size_t a : order) {
    while (!active.empty() && active.begin()->first < first[a]) {
      const size_t b = active.begin()->second;
      active.erase(active.begin());
      int64_t off = real[b], sz = va[b].second;
      auto nx = freeb.lower_bound(off);
      if (nx != freeb.end() && nx->first == off + sz) { sz += nx->second; freeb.erase(nx); }
      auto pv = freeb.lower_bound(off);
      if (pv != freeb.begin()) {
        --pv;
        if (pv->first + pv->second == off) { off = pv->first; sz += pv->second; freeb.erase(pv); }
      }
      if (off + sz == top) top = off;   // a freed block at the top lowers it
      else freeb[off] = sz;
    }
    const int64_t sz = va[a].second;
    auto best = freeb.end();
    for (auto it = freeb.begin(); it != freeb.end(); ++it)
      if (it->second >= sz && (best == freeb.end() || it->second < best->second)) best = it;
    if (best != freeb.end()) {
      const int64_t off = best->first, bsz = best->second;
      freeb.erase(best);
      if (bsz > sz) freeb[off + sz] = bsz - sz;
      real[a] = off;
    } else {
      real[a] = top;
      top += sz;
      high = std::max(high, top);
    }
    active.insert({last[a], a});
  }
  // self-check: buffers sharing memory never share a time step
  {
    std::vector<size_t> byoff(order);
    std::sort(byoff.begin(), byoff.end(), [&](size_t x, size_t y) { return real[x] < real[y]; });
    for (size_t i = 0; i < byoff.size(); ++i) {
      const size_t a = byoff[i];
      for (size_t j = i + 1; j < byoff.size() && real[byoff[j]] < real[a] + va[a].second; ++j) {
        const size_t b = byoff[j];
        if (!(last[a] < first[b] || last[b] < first[a])) return -1;
      }
    }
  }
  for (auto& pr : L.ops) {
    Op& op = pr.second;
    auto moved = [&](Ref& r) {
      if (r.region != region) return;
      const size_t a = find(r.off);
      r.off = real[a] + (r.off - va[a].first);
    };
    moved(op.a); moved(op.b); moved(op.c); moved(op.d);
    for (Ref& r : op.refs) moved(r);
  }
  return high;
}

}  // namespace

bool Compiler::build_sweep(int parity, Plan* out) {
  const Problem& P = prob;
  int nm = int(P.msg_keys.size());
  int rin = parity ? RG_MSG1 : RG_MSG0;
  int rout = parity ? RG_MSG0 : RG_MSG1;
  out->lanes.assign(nm, {});
  out->nlanes = nm;
  if (int(lane_size.size()) < 2 * nm) lane_size.resize(2 * nm, 0);
  for (int m = 0; m < nm; ++m) {
    Lane L(this, m, &out->lanes[m]);
    int blk, face;
    std::vector<std::pair<int, int>> recv;
    P.update_target(m, &blk, &face, &recv);
    std::vector<std::pair<int, int>> fin;
    int center = 0;
    L.stage = 0;
    // the sketch keys do not depend on the sweep: the truncated map is the
    // same at every sweep, so BlockBP can reach its fixed point
    std::vector<CSite> ch = L.run_sweep(blk, face, {}, rin, {1, uint64_t(m), 0}, false, -1, nullptr,
                                        &fin, &center);
    if (!L.err.empty()) { error = L.err; return false; }
    // order the result like the receiving face
    L.stage = 1;
    L.reset_scratch();
    L.at(1, 0, 0);
    if (fin == recv) {
    } else {
      std::vector<std::pair<int, int>> rv(fin.rbegin(), fin.rend());
      if (rv != recv) { error = "final chain does not match the receiving face"; return false; }
      L.reverse_chain(ch, center);
    }
    L.at(1, 1, 0);
    L.right_canonical(ch, center);
    bool over = false;
    for (const CSite& x : ch) over = over || x.r > opt.chi;
    if (over) {
      L.at(1, 5, 0);
      L.compress(ch, center);
    }
    for (size_t j = 0; j < ch.size(); ++j) {
      if (ch[j].r > msg.br[L.C->prob.stored_slot_of_update(m)][j] && opt.chi_env > 0) {
        error = "bond above the message cap (chi_env > chi is not supported)";
        return false;
      }
    }
    int slot = P.stored_slot_of_update(m);
    if (opt.hermitize || opt.damping > 0.0) {
      // both act on the finished message: unit norm, trace real and positive
      L.at(1, 6, 0);
      L.phase_fix(ch);
      if (opt.hermitize) {
        // Sec. "'Hermitize' MPSs": each double leg unfused to (ket, bra),
        // the two exchanged and conjugated, then (A + A^dagger) / 2
        L.at(1, 7, 0);
        std::vector<CSite> hc = ch;
        for (size_t j = 0; j < hc.size(); ++j) {
          CSite& x = hc[j];
          x.buf = L.chain_alloc(int64_t(x.l) * x.P * x.r);
          L.perm(ch[j].buf, x.buf, {x.l, x.D, x.D, x.r}, {0, 2, 1, 3}, 1);
        }
        ch = L.compressed_sum(ch, hc, 0.5, 0.5, center);
      }
      if (opt.damping > 0.0) {
        // Eq. blockBP:kagome:numerics:learning_step1 with alpha = 1 - damping:
        // alpha new + (1 - alpha) old, the old message as stored (caps)
        L.at(1, 8, 0);
        std::vector<CSite> old = ch;
        for (size_t j = 0; j < old.size(); ++j) {
          old[j].buf = Ref{rin, msg.off[slot][j]};
          old[j].l = msg.bl[slot][j];
          old[j].r = msg.br[slot][j];
        }
        ch = L.compressed_sum(ch, old, 1.0 - opt.damping, opt.damping, center);
      }
      if (!L.err.empty()) { error = L.err; return false; }
    }
    // pad into the stored message (caps), fix the phase, then the distance
    L.at(1, 2, 0);
    std::vector<CSite> stored;
    for (size_t j = 0; j < ch.size(); ++j) {
      if (ch[j].l > msg.bl[slot][j] || ch[j].r > msg.br[slot][j]) {
        error = "message bond above its cap";
        return false;
      }
      Ref dst{rout, msg.off[slot][j]};
      L.pad(ch[j].buf, dst, ch[j].l, ch[j].P, ch[j].r, msg.bl[slot][j], msg.br[slot][j], 0, 0, 0);
      CSite cs = ch[j];
      cs.buf = dst; cs.l = msg.bl[slot][j]; cs.r = msg.br[slot][j];
      stored.push_back(cs);
    }
    L.at(1, 3, 0);
    L.phase_fix(stored);
    // convergence distance ||new - old|| from the direct-sum MPS and a QR sweep
    L.at(1, 4, 0);
    int n = int(stored.size());
    if (n == 1) {
      Ref X = L.scratch(int64_t(stored[0].l) * stored[0].P * stored[0].r);
      L.pad(stored[0].buf, X, 1, stored[0].P, 1, 1, 1, 0, 0, 0);
      L.pad(Ref{rin, msg.off[slot][0]}, X, 1, stored[0].P, 1, 1, 1, 0, 0, 2, -1.0);
      L.norm(X, stored[0].P, -1, err_slot(slot));
    } else {
      Ref Rm;
      int64_t rl = 1;
      for (int j = 0; j < n; ++j) {
        int lN = msg.bl[slot][j], rN = msg.br[slot][j], Pj = msg.P[slot][j];
        int l2 = (j == 0) ? 1 : 2 * lN, r2 = (j == n - 1) ? 1 : 2 * rN;
        Ref X = L.scratch(int64_t(l2) * Pj * r2);
        Ref newb = stored[j].buf, oldb{rin, msg.off[slot][j]};
        L.pad(newb, X, lN, Pj, rN, l2, r2, 0, 0, 0);
        L.pad(oldb, X, lN, Pj, rN, l2, r2, (j == 0) ? 0 : lN, (j == n - 1) ? 0 : rN, 1,
              j == 0 ? -1.0 : 1.0);
        Ref Mx;
        int64_t ml;
        if (j == 0) { Mx = X; ml = l2; }
        else {
          Mx = L.scratch(rl * Pj * r2);
          L.gemm(Rm, X, Mx, rl, int64_t(Pj) * r2, l2, l2, int64_t(Pj) * r2, int64_t(Pj) * r2,
                 OP_N, OP_N, PREC_FP64);
          ml = rl;
        }
        if (j == n - 1) {
          L.norm(Mx, ml * Pj * r2, -1, err_slot(slot));
        } else {
          int64_t mm = ml * Pj, nn = r2, k = std::min(mm, nn);
          Ref Qx = L.scratch(mm * k);
          Rm = L.scratch(k * nn);
          L.qr(Mx, mm, nn, nn, 0, Qx, Rm);
          rl = k;
        }
      }
    }
    if (!L.err.empty()) { error = L.err; return false; }
    fuse_gemm_perm(out->lanes[m]);
    const int64_t sz = pack_lane(out->lanes[m], L.vallocs, L.rg_chain());
    if (sz < 0) { error = "internal error: overlapping workspace buffers"; return false; }
    lane_size[2 * m] = std::max(lane_size[2 * m], sz);
  }
  return true;
}

bool Compiler::build_expect(int parity, const std::vector<std::pair<int, int>>& bonds,
                            Plan* out, std::vector<std::vector<int>>* carry_order,
                            std::vector<int64_t>* rho_off) {
  const Problem& P = prob;
  int rin = parity ? RG_MSG1 : RG_MSG0;
  int nb = int(bonds.size());
  out->lanes.assign(nb, {});
  out->nlanes = nb;
  if (int(lane_size.size()) < 2 * nb) lane_size.resize(2 * nb, 0);
  carry_order->assign(nb, {});
  rho_off->assign(nb, 0);
  for (int bi = 0; bi < nb; ++bi) {
    int i = bonds[bi].first, j = bonds[bi].second;
    Lane L(this, bi, &out->lanes[bi]);
    int a = P.block_of[i], b = P.block_of[j];
    // closing face: first face carrying a real message, else the first face
    auto expect_face = [&](int blk, int skip) {
      const std::vector<Face>& F = P.faces[blk];
      for (size_t n = 0; n < F.size(); ++n)
        if (int(n) != skip && F[n].keytype != FACE_OUTSIDE) return int(n);
      for (size_t n = 0; n < F.size(); ++n)
        if (int(n) != skip) return int(n);
      return 0;
    };
    std::vector<std::pair<int, int>> fin;
    int center = 0, cblk, cface;
    std::vector<CSite> ch;
    L.stage = 0;
    if (a == b) {
      cblk = a;
      cface = expect_face(a, -1);
      ch = L.run_sweep(a, cface, {i, j}, rin, {2, uint64_t(bi), 0}, false, -1, nullptr, &fin,
                       &center);
    } else {
      int fa = P.face_index(a, FACE_BLOCK, b), fb = P.face_index(b, FACE_BLOCK, a);
      std::vector<CSite> c1 = L.run_sweep(a, fa, {i}, rin, {2, uint64_t(bi), 0}, false, -1,
                                          nullptr, &fin, &center);
      if (!L.err.empty()) { error = L.err; return false; }
      std::vector<std::pair<int, int>> recv;
      for (auto& sl : P.faces[b][fb].legs) {
        const Link& k = P.links[sl.first][sl.second];
        recv.push_back({k.s2, k.l2});
      }
      L.stage = 1;
      L.reset_scratch();
      L.at(1, 0, 0);
      if (fin != recv) {
        std::vector<std::pair<int, int>> rv(fin.rbegin(), fin.rend());
        if (rv != recv) { error = "carried message does not match the receiving face"; return false; }
        L.reverse_chain(c1, center);
      }
      L.right_canonical(c1, center);
      cblk = b;
      cface = expect_face(b, fb);
      L.stage = 2;
      ch = L.run_sweep(b, cface, {j}, rin, {2, uint64_t(bi), 1}, false, fb, &c1, &fin, &center);
    }
    if (!L.err.empty()) { error = L.err; return false; }
    // close with the incoming message of the closing face
    L.stage = 3;
    L.reset_scratch();
    L.at(3, 0, 0);
    const std::vector<Face>& F = P.faces[cblk];
    std::vector<std::pair<int, int>> legs = F[cface].legs;
    bool rev;
    if (fin == legs) rev = false;
    else {
      std::vector<std::pair<int, int>> rv(legs.rbegin(), legs.rend());
      if (fin != rv) { error = "final chain does not match the closing face"; return false; }
      rev = true;
    }
    int slot = P.incoming_msg(cblk, cface);
    int nl = int(legs.size());
    std::vector<CSite> msgs(nl);
    for (int q = 0; q < nl; ++q) {
      CSite cs;
      int D = tensor_dims[P.sites[legs[q].first].tensor][1 + legs[q].second];
      cs.D = D;
      if (slot < 0) { cs.buf = Ref{RG_CONST, 0}; cs.l = cs.P = cs.r = 1; }
      else {
        cs.buf = Ref{rin, msg.off[slot][q]};
        cs.l = msg.bl[slot][q]; cs.P = msg.P[slot][q]; cs.r = msg.br[slot][q];
      }
      msgs[q] = cs;
    }
    if (rev) {
      int dummy = 0;
      L.reverse_chain(msgs, dummy);
    }
    // L[c, d, X]: start from the scalar 1
    Ref Lb{RG_CONST, 0};
    int64_t Lc = 1, Ld = 1, LX = 1;
    std::vector<int> order;
    for (size_t q = 0; q < ch.size(); ++q) {
      const CSite& A = ch[q];
      const CSite& M = msgs[q];
      int64_t Qd = ipow(opt.d * opt.d, int(A.carries.size()));
      int64_t I = A.P / Qd;
      if (I != M.P || A.l != Lc || M.l != Ld) { error = "closing shapes mismatch"; return false; }
      // S1[(d X), (I q e)] = L^T[(d X), c] A[c, (I q e)]
      Ref S1 = L.scratch(Ld * LX * A.P * A.r);
      L.gemm(Lb, A.buf, S1, Ld * LX, int64_t(A.P) * A.r, Lc, Ld * LX, int64_t(A.P) * A.r,
             int64_t(A.P) * A.r, OP_T, OP_N, PREC_FP64);
      Ref S1p = L.scratch(Ld * LX * A.P * A.r);
      L.perm(S1, S1p, {int(Ld), int(LX), int(I), int(Qd), A.r}, {1, 3, 4, 0, 2});
      Ref S2 = L.scratch(LX * Qd * A.r * M.r);
      L.gemm(S1p, M.buf, S2, LX * Qd * A.r, M.r, Ld * I, Ld * I, M.r, M.r, OP_N, OP_N,
             PREC_FP64);
      Ref Ln = L.scratch(LX * Qd * A.r * M.r);
      L.perm(S2, Ln, {int(LX), int(Qd), A.r, M.r}, {2, 3, 0, 1});
      Lb = Ln;
      Lc = A.r; Ld = M.r; LX *= Qd;
      for (int c : A.carries) order.push_back(c);
    }
    if (Lc != 1 || Ld != 1) { error = "closing contraction left open bonds"; return false; }
    int64_t roff = rho_size;
    rho_size += (LX + 7) / 8 * 8;
    L.pad(Lb, Ref{RG_RHO, roff}, 1, int(LX), 1, 1, 1, 0, 0, 0);
    (*carry_order)[bi] = order;
    (*rho_off)[bi] = roff;
    if (!L.err.empty()) { error = L.err; return false; }
    fuse_gemm_perm(out->lanes[bi]);
    const int64_t sz = pack_lane(out->lanes[bi], L.vallocs, L.rg_chain());
    if (sz < 0) { error = "internal error: overlapping workspace buffers"; return false; }
    lane_size[2 * bi] = std::max(lane_size[2 * bi], sz);
  }
  return true;
}

}  // namespace pn
