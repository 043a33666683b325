// Device-side operation descriptors shared by the plan compiler and the
// HIP kernels.  Every kernel is batched: it receives an array of descriptors
// (one per independent work item, e.g. one per message update running side
// by side) and blockIdx.z / blockIdx.y selects the item.
//
// Complex numbers are stored as interleaved double pairs (re, im), C order.
#pragma once
#include <cstdint>

namespace pn {

struct cplx {
  double re, im;
};

enum GemmOp { OP_N = 0, OP_T = 1, OP_C = 2 };        // op(X) = X, X^T, X^H
enum Precision { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2 };

constexpr int GEMM_SC_MAX = 12;   // scatter-store axes

// C = alpha * op(A) * op(B) + beta * C, row-major, op(A) is M x K, op(B) K x N.
struct GemmDesc {
  const cplx* A;
  const cplx* B;
  cplx* C;
  int M, N, K;
  int lda, ldb, ldc;
  int opA, opB;
  cplx alpha, beta;
  // Scatter store (sc_n > 0, beta = 0): the output is written already
  // transposed.  Element (r, c) goes to C + off_r(r) + off_c(c); the first
  // sc_nr axes split r, the other sc_n - sc_nr split c (row-major, last axis
  // fastest), axis k adding idx_k * sc_ds[k] (sc_inv[k] = 1 / sc_dim[k]);
  // sc_conj stores the conjugate.
  int sc_n, sc_nr, sc_conj;
  int sc_dim[GEMM_SC_MAX];
  double sc_inv[GEMM_SC_MAX];
  int64_t sc_ds[GEMM_SC_MAX];
};

// dst[o] = src[sum_k idx_k(o) * stride[k]] for o over the row-major output
// shape dims[0..rank).
struct PermDesc {
  const cplx* src;
  cplx* dst;
  int rank;
  int conj;       // 1: complex-conjugate while copying
  int64_t total;
  int dims[16];
  int64_t stride[16];
  double inv[16];   // 1 / dims[k]: the index split without integer division
};

// Householder QR of the m x n matrix A (row-major, lda) or, with conjT, of
// A^H where A is n x m.  Work is an m x (n + k) scratch (used when the working
// copies do not fit in LDS); R (k x n, ldr = n) with k = min(m, n) and, unless
// Q is null, Q (m x k, ldq = k) are written explicitly, diag(R) real
// non-negative.
struct QrDesc {
  const cplx* A;
  cplx* work;
  cplx* Q;
  cplx* R;
  int m, n, lda, conjT;
  int qh;       // Q written as Q^H (k x m, row-major) instead of Q (m x k)
};

// Which QR kernel factorises an m x n matrix (the plan compiler and the
// executor take the same decision):
//   QRK_SMALL   k_qr_small<9, 16>, m <= 144, n <= 16 (registers)
//   QRK_MID     k_qr_mid, R only, m <= 144, n <= 128 (registers)
//   QRK_SMALL2  k_qr_small<18, 32>, m <= 288, n <= 32 (registers)
//   QRK_LDS     k_qr, working copy m (n + k) <= QR_LDS_MAX in LDS
//   QRK_CHOL    tall blocks with n <= CHOLQR_MAXN, n <= m: Cholesky QR on several
//               workgroups (Gram GEMMs, k_chol, Q GEMMs; three passes, the
//               first shifted), expanded into those ops by the plan compiler
//   QRK_TALL    k_qr_tall, one workgroup, blocked panels (everything else)
constexpr int QR_LDS_MAX = 8192;   // complex elements (128 KB)
constexpr int QRS_MAXM = 144, QRS_MAXN = 16;
constexpr int QRM_MAXN = 128;
constexpr int CHOLQR_MAXN = 128;
enum QrKernel { QRK_LDS = 0, QRK_TALL = 1, QRK_SMALL = 2, QRK_MID = 3, QRK_SMALL2 = 4, QRK_CHOL = 5 };
inline int qr_kernel(int64_t m, int64_t n, bool with_q) {
  const int64_t k = m < n ? m : n;
  if (m <= QRS_MAXM && n <= QRS_MAXN) return QRK_SMALL;
  if (!with_q && m <= QRS_MAXM && n <= QRM_MAXN) return QRK_MID;
  if (m <= 2 * QRS_MAXM && n <= 2 * QRS_MAXN) return QRK_SMALL2;
  if (m * (n + (with_q ? k : 0)) <= QR_LDS_MAX) return QRK_LDS;
  if (n <= CHOLQR_MAXN && m >= n) return QRK_CHOL;
  return QRK_TALL;
}

// Split-K GEMM: C (M x N, ldc) = alpha * sum_s P_s, P_s the S partial
// products (M x N each, consecutive, row-major), summed in order.
struct SumDesc {
  const cplx* P;
  cplx* C;
  int S, M, N, ldc;
  cplx alpha;
};

// Cholesky step of the tall QR (k_chol, one workgroup per item): the S
// partial Gram matrices G_s (n x n each, consecutive, row-major; only their
// upper triangles are read) are summed in order, shifted when `shift` is set
// (sigma = 11 (m n + n (n + 1)) 2^-53 tr G, the shifted Cholesky QR of
// Fukaya et al. 2020), and factorised G = R^H R with R upper triangular and
// real positive diagonal.  A pivot at or below 1e-24 max_i G_ii marks a
// column inside the span of the previous ones: its row of R and its column of
// R^-1 are zero (the matching column of Q comes out zero).  Writes R^-1 and,
// when `accumulate`, R <- R_new R (the running factor of the passes, updated
// in place), else R <- R_new.  n <= CHOLQR_MAXN.
struct CholDesc {
  const cplx* G;
  cplx* Rinv;
  cplx* R;
  int S, n, shift, accumulate;
  int64_t m;
};

// One-sided Jacobi SVD of the rows x cols matrix A with element (i, c) at
// A[i * lda + c], or conj(A[c * lda + i]) with conjT.  Rotating the columns to
// mutual orthogonality gives A W = U Sigma; the `keep` columns of largest norm
// are written normalised, in decreasing order, as U (rows x keep, ld keep) and
// their norms into sigma.  Singular values at or below 1e-15 ||A||_F are
// rounding noise: they are returned as 0 with a zero column of U.
constexpr int kJacobiMaxRows = 144;
inline int64_t jacobi_work_elems(int64_t rows, int64_t cols) { return (rows + 15) / 16 * 16 * cols; }
constexpr int kJacobiMaxCols = 144;   // and cols <= rows
struct JacobiDesc {
  const cplx* A;
  cplx* work;   // cols x roundup(rows, 16) scratch (used when it does not fit in LDS)
  cplx* U;
  double* sigma;
  int rows, cols, lda, conjT, keep;
  int gauge;    // top-k SVD only (k_svd_back): each kept column's entry of largest modulus
                // (first row on ties) made real and positive
};
// k_svt_bidiag followed by k_svd_top take the same descriptor and write the
// same outputs for keep <= cols <= rows <= 144 through Householder
// bidiagonalisation, bisection on the Golub-Kahan tridiagonal and inverse
// iteration, with the larger scratch below (the left reflectors, rows padded
// to 16; the bidiagonal, 3 cols + 2; per value 2 cols + 2 rows doubles; the
// unit phases of the real bidiagonal, cols).  k_svd_back then forms the
// singular vectors from what k_svd_top leaves there.
inline int64_t svd_top_work_elems(int64_t rows, int64_t cols, int64_t keep) {
  return (rows + 15) / 16 * 16 * cols + 3 * cols + 2 + ((2 * cols + 2 * rows) * keep + 1) / 2 + cols + 16;
}

// Random sign sketch: out[i, j] = (+-1 +- 1j)/sqrt(2) from SplitMix64 output
// number i*k + j of the generator seeded with key (n x k, row-major).  The
// key is out0(prefix ^ tag) where tag is read from *last_tag (the sweep
// counter, kept on the device so captured launches stay valid).
struct OmegaDesc {
  cplx* out;
  int n, k;
  uint64_t prefix;
  const double* last_tag;
};

// x /= ||x||_F, logscale += log10 ||x||_F
// (two launches over NORM_CHUNKS workgroups per item: partial sums of
// |x|^2 per chunk into part[], then every chunk sums the partials in order
// and scales its elements; the first chunk updates the log-scale)
constexpr int NORM_CHUNKS = 64;
struct NormDesc {
  cplx* x;
  int64_t len;
  double* logscale;
  double* norm_out;   // optional: stores ||x||
  double* part;       // NORM_CHUNKS doubles of scratch
};

// Block copy between [l, P, r] tensors: dst[l, p, r] <- sign * src[l - off_l,
// p, r - off_r] where the source index is in range.  mode 0 writes every
// destination element (zero outside the block), mode 1 writes the block only,
// mode 2 adds the block to the destination.  Also used to crop (r2 < r1).
struct PadDesc {
  const cplx* src;
  cplx* dst;
  int l1, P, r1, l2, r2, off_l, off_r;
  int mode;
  double sign;
};

// Message trace (ket = bra on every leg) and phase fix of site 0.
struct PhaseDesc {
  cplx* sites[16];
  int l[16], P[16], r[16], D[16];
  int nsites;
};

}  // namespace pn

namespace pn {
// Canonical gauge of a split bond: for each column j of L (m x keep, ld keep)
// the entry of largest modulus (first on ties) becomes real positive; row j of
// R (keep x n, ld n) takes the inverse phase.
struct ColPhaseDesc {
  cplx* L;
  cplx* R;
  int m, keep, n;
};

// rho and <S_i.S_j> from the carried expectation vectors: R[q_a * d^2 + q_b]
// with q = p * d + p' for the two carried open sites in carry order (first
// is site i when first_is_i).  rho is written as [(p_i p_j), (p_i' p_j')].
struct RhoDesc {
  const cplx* R;
  cplx* rho;
  double* ss;
  int first_is_i;
};
}  // namespace pn
