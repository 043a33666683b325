// HIP kernels for the BlockBP boundary-chain engine (gfx950 / CDNA4).
//
// * k_gemm<P>: batched complex GEMM on the matrix cores.  One 64x64 output
//   tile per 256-thread workgroup, four wave64s each owning a 32x32 quadrant
//   (2x2 MFMA 16x16 tiles).  A complex product is four real MFMA products
//   (re*re - im*im, re*im + im*re).  P selects the arithmetic:
//     PREC_FP64   v_mfma_f64_16x16x4   (complex128 in, FP64 accumulate)
//     PREC_FP32   v_mfma_f32_16x16x4   (operands rounded to FP32, FP32 acc)
//     PREC_BF16X3 v_mfma_f32_16x16x32_bf16, every FP32 operand split as
//                 hi + lo (bf16 each), product hi*hi + hi*lo + lo*hi, FP32 acc
//   Operands are staged through LDS; storage stays complex128.
// * k_permute: batched tensor transpose (rank <= 16).
// * k_qr: Householder QR with explicit thin Q and R, one workgroup per item.
// * k_jacobi: one-sided (Hestenes) Jacobi SVD of a small square matrix, one
//   workgroup per item, LDS-resident when it fits, parallel round-robin pairs.
// * small kernels: sketch generation (SplitMix64), normalisation with
//   log-scale, zero-padded copies, message trace phase fix.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels.hpp"

namespace pn {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ cplx ld_op(const cplx* X, int ld, int op, int r, int c) {
  if (op == OP_N) return X[(int64_t)r * ld + c];
  cplx v = X[(int64_t)c * ld + r];
  if (op == OP_C) v.im = -v.im;
  return v;
}

// ------------------------------------------------------------------ GEMM
constexpr int GT_M = 64, GT_N = 64;

template <int P>
struct GemmCfg;
template <>
struct GemmCfg<PREC_FP64> { typedef double T; static constexpr int TK = 16; };
template <>
struct GemmCfg<PREC_FP32> { typedef float T; static constexpr int TK = 16; };
template <>
struct GemmCfg<PREC_BF16X3> { typedef float T; static constexpr int TK = 32; };

__device__ __forceinline__ void split_bf16(float x, __bf16* hi, __bf16* lo) {
  __bf16 h = (__bf16)x;
  *hi = h;
  *lo = (__bf16)(x - (float)h);
}

template <int P>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ descs) {
  typedef typename GemmCfg<P>::T T;
  constexpr int TK = GemmCfg<P>::TK;
  constexpr int PAD = (sizeof(T) == 8) ? 2 : 4;
  const GemmDesc g = descs[blockIdx.z];
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  if (m0 >= g.M || n0 >= g.N) return;
  __shared__ T As_r[TK][GT_M + PAD], As_i[TK][GT_M + PAD];
  __shared__ T Bs_r[TK][GT_N + PAD], Bs_i[TK][GT_N + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  typedef typename std::conditional<P == PREC_FP64, d4, f4>::type acc_t;
  acc_t accr[2][2], acci[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      accr[i][j] = acc_t{0, 0, 0, 0};
      acci[i][j] = acc_t{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    // stage op(A)[m0:m0+64, k0:k0+TK] and op(B)[k0:k0+TK, n0:n0+64]
    for (int e = tid; e < GT_M * TK; e += 256) {
      int mm, kk;
      if (g.opA == OP_N) { mm = e / TK; kk = e % TK; } else { mm = e % GT_M; kk = e / GT_M; }
      int r = m0 + mm, c = k0 + kk;
      cplx v = {0.0, 0.0};
      if (r < g.M && c < g.K) v = ld_op(g.A, g.lda, g.opA, r, c);
      As_r[kk][mm] = (T)v.re;
      As_i[kk][mm] = (T)v.im;
    }
    for (int e = tid; e < GT_N * TK; e += 256) {
      int nn, kk;
      if (g.opB == OP_N) { nn = e % GT_N; kk = e / GT_N; } else { kk = e % TK; nn = e / TK; }
      int r = k0 + kk, c = n0 + nn;
      cplx v = {0.0, 0.0};
      if (r < g.K && c < g.N) v = ld_op(g.B, g.ldb, g.opB, r, c);
      Bs_r[kk][nn] = (T)v.re;
      Bs_i[kk][nn] = (T)v.im;
    }
    __syncthreads();
    if constexpr (P == PREC_FP64 || P == PREC_FP32) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        const int kq = kk + (lane >> 4);
        T ar[2], ai[2], br[2], bi[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ar[i] = As_r[kq][wm + i * 16 + (lane & 15)];
          ai[i] = As_i[kq][wm + i * 16 + (lane & 15)];
          br[i] = Bs_r[kq][wn + i * 16 + (lane & 15)];
          bi[i] = Bs_i[kq][wn + i * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if constexpr (P == PREC_FP64) {
              accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accr[i][j], 0, 0, 0);
              accr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], accr[i][j], 0, 0, 0);
              acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acci[i][j], 0, 0, 0);
              acci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acci[i][j], 0, 0, 0);
            } else {
              accr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], accr[i][j], 0, 0, 0);
              accr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[i], bi[j], accr[i][j], 0, 0, 0);
              acci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi[j], acci[i][j], 0, 0, 0);
              acci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], br[j], acci[i][j], 0, 0, 0);
            }
          }
      }
    } else {
      // split-BF16, three-term products, K = 32 per MFMA
      const int kb = 8 * (lane >> 4);
      bf8 arh[2], arl[2], aih[2], ail[2], anh[2], anl[2];
      bf8 brh[2], brl[2], bih[2], bil[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          __bf16 h, l;
          split_bf16(As_r[kb + t][wm + i * 16 + (lane & 15)], &h, &l);
          arh[i][t] = h; arl[i][t] = l;
          split_bf16(As_i[kb + t][wm + i * 16 + (lane & 15)], &h, &l);
          aih[i][t] = h; ail[i][t] = l;
          anh[i][t] = -h; anl[i][t] = -l;
          split_bf16(Bs_r[kb + t][wn + i * 16 + (lane & 15)], &h, &l);
          brh[i][t] = h; brl[i][t] = l;
          split_bf16(Bs_i[kb + t][wn + i * 16 + (lane & 15)], &h, &l);
          bih[i][t] = h; bil[i][t] = l;
        }
      }
#define PN_MFMA3(acc, xh, xl, yh, yl)                                      \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);     \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0);     \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          PN_MFMA3(accr[i][j], arh[i], arl[i], brh[j], brl[j]);
          PN_MFMA3(accr[i][j], anh[i], anl[i], bih[j], bil[j]);
          PN_MFMA3(acci[i][j], arh[i], arl[i], bih[j], bil[j]);
          PN_MFMA3(acci[i][j], aih[i], ail[i], brh[j], brl[j]);
        }
#undef PN_MFMA3
    }
    __syncthreads();
  }
  // epilogue: f64 layout row = lane/16 + 4t, f32 layout row = 4(lane/16) + t
  const bool beta0 = (g.beta.re == 0.0 && g.beta.im == 0.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        int rr = (P == PREC_FP64) ? ((lane >> 4) + 4 * t) : (4 * (lane >> 4) + t);
        int r = m0 + wm + i * 16 + rr;
        int c = n0 + wn + j * 16 + (lane & 15);
        if (r < g.M && c < g.N) {
          double vr = (double)accr[i][j][t], vi = (double)acci[i][j][t];
          cplx out;
          out.re = g.alpha.re * vr - g.alpha.im * vi;
          out.im = g.alpha.re * vi + g.alpha.im * vr;
          cplx* cp = g.C + (int64_t)r * g.ldc + c;
          if (!beta0) {
            cplx o = *cp;
            out.re += g.beta.re * o.re - g.beta.im * o.im;
            out.im += g.beta.re * o.im + g.beta.im * o.re;
          }
          *cp = out;
        }
      }
}

template __global__ void k_gemm<PREC_FP64>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP32>(const GemmDesc*);
template __global__ void k_gemm<PREC_BF16X3>(const GemmDesc*);

// --------------------------------------------------------------- permute
__global__ __launch_bounds__(256) void k_permute(const PermDesc* __restrict__ descs) {
  const PermDesc& p = descs[blockIdx.y];
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < p.total; o += step) {
    int64_t rem = o, off = 0;
    for (int k = p.rank - 1; k >= 0; --k) {
      int64_t idx = rem % p.dims[k];
      rem /= p.dims[k];
      off += idx * p.stride[k];
    }
    cplx v = p.src[off];
    if (p.conj) v.im = -v.im;
    p.dst[o] = v;
  }
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int NT>
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// --------------------------------------------------------------------- QR
// Householder reflections H = I - tau v v^H with v[j] = x[j] - alpha,
// alpha = -e^{i arg x_j} ||x||.  Working copies are column-major (W[c*m+i],
// Qt[c*m+i]) in LDS when m*(n+k) <= QR_LDS_MAX, else in the work buffer
// (W) and a column-major staging area behind it (Qt).  Column operations use
// one 16-lane group per column, 16 columns at a time.
constexpr int QR_LDS_MAX = 8192;   // complex elements (128 KB)

// Sum over the 16 lanes of a DPP row, result in every lane: xor-1 and xor-2
// quad permutations, then half-row and row mirrors (VALU moves, no LDS).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double group16_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// W and Qt point into LDS (INLDS) or into the work buffer; keeping the two
// cases apart lets the compiler use ds_read/ds_write for LDS data.
template <bool INLDS>
__device__ __forceinline__ void qr_body(const QrDesc& d, cplx* W, cplx* Qt, double* tau_s,
                                        cplx* phs, cplx* alpha_s, double (*part_s)[4]) {
  const int m = d.m, n = d.n, k = m < n ? m : n;
  const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
  for (int64_t e = tid; e < (int64_t)m * n; e += 256) {
    int r = (int)(e / n), c = (int)(e % n);
    cplx v;
    if (d.conjT) { v = d.A[(int64_t)c * d.lda + r]; v.im = -v.im; }
    else v = d.A[(int64_t)r * d.lda + c];
    W[(int64_t)c * m + r] = v;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < k; ++j) {
    cplx* wj = W + (int64_t)j * m;
    // column norm: wave sums, one barrier, every thread finishes the sum
    double part = 0.0;
    for (int i = j + tid; i < m; i += 256) part += wj[i].re * wj[i].re + wj[i].im * wj[i].im;
    part = wave_sum(part);
    if (lane == 0) part_s[j & 1][wave] = part;
    __syncthreads();
    const double nx2 = part_s[j & 1][0] + part_s[j & 1][1] + part_s[j & 1][2] + part_s[j & 1][3];
    const cplx x0 = wj[j];
    const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im), nx = sqrt(nx2);
    double tau = 0.0;
    cplx alpha = {0.0, 0.0}, v0 = x0;
    if (nx > 0.0) {
      cplx ph = ax0 > 0.0 ? cplx{x0.re / ax0, x0.im / ax0} : cplx{1.0, 0.0};
      alpha = cplx{-ph.re * nx, -ph.im * nx};
      v0 = cplx{x0.re - alpha.re, x0.im - alpha.im};
      double nv2 = nx2 - ax0 * ax0 + v0.re * v0.re + v0.im * v0.im;
      tau = nv2 > 0.0 ? 2.0 / nv2 : 0.0;
    }
    if (tid == 0) tau_s[j] = tau;
    if (tau != 0.0) {
      for (int c = j + 1 + grp; c < n; c += 16) {
        cplx* wc = W + (int64_t)c * m;
        double wr = 0.0, wi = 0.0;
        for (int i = j + gl; i < m; i += 16) {
          cplx v = (i == j) ? v0 : wj[i], a = wc[i];
          wr += v.re * a.re + v.im * a.im;   // conj(v) * a
          wi += v.re * a.im - v.im * a.re;
        }
        wr = group16_sum(wr);
        wi = group16_sum(wi);
        for (int i = j + gl; i < m; i += 16) {
          cplx v = (i == j) ? v0 : wj[i];
          wc[i].re -= tau * (v.re * wr - v.im * wi);
          wc[i].im -= tau * (v.re * wi + v.im * wr);
        }
      }
    }
    // diag(R) is alpha; the rest of row j of R stays in W (rows above the
    // diagonal are final once their step is done) and is written at the end
    if (tid == 0) {
      double a = sqrt(alpha.re * alpha.re + alpha.im * alpha.im);
      phs[j] = a > 0.0 ? cplx{alpha.re / a, alpha.im / a} : cplx{1.0, 0.0};
      alpha_s[j] = cplx{a, 0.0};
    }
    __syncthreads();
    // the reflector's head replaces x0 only after every column used x0
    if (tid == 0 && tau != 0.0) wj[j] = v0;
  }
  __syncthreads();
  // R with the canonical gauge: diag(R) real non-negative, row j * conj(phase_j)
  for (int64_t e = tid; e < (int64_t)k * n; e += 256) {
    int j = (int)(e / n), c = (int)(e % n);
    cplx x = {0.0, 0.0};
    if (c == j) x = alpha_s[j];
    else if (c > j) {
      cplx w = W[(int64_t)c * m + j], ph = phs[j];
      x = cplx{w.re * ph.re + w.im * ph.im, w.im * ph.re - w.re * ph.im};
    }
    d.R[e] = x;
  }
  // Q = H_0 ... H_{k-1} [I; 0], built backwards (column-major Qt)
  for (int64_t e = tid; e < (int64_t)m * k; e += 256) {
    int c = (int)(e / m), r = (int)(e % m);
    Qt[e] = cplx{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau != 0.0) {
      const cplx* wj = W + (int64_t)j * m;
      for (int c = j + grp; c < k; c += 16) {
        cplx* qc = Qt + (int64_t)c * m;
        double wr = 0.0, wi = 0.0;
        for (int i = j + gl; i < m; i += 16) {
          cplx v = wj[i], a = qc[i];
          wr += v.re * a.re + v.im * a.im;
          wi += v.re * a.im - v.im * a.re;
        }
        wr = group16_sum(wr);
        wi = group16_sum(wi);
        for (int i = j + gl; i < m; i += 16) {
          cplx v = wj[i];
          qc[i].re -= tau * (v.re * wr - v.im * wi);
          qc[i].im -= tau * (v.re * wi + v.im * wr);
        }
      }
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < (int64_t)m * k; e += 256) {
    int r = (int)(e / k), c = (int)(e % k);
    cplx ph = phs[c], x = Qt[(int64_t)c * m + r];
    d.Q[e] = cplx{x.re * ph.re - x.im * ph.im, x.re * ph.im + x.im * ph.re};
  }
}

__global__ __launch_bounds__(256) void k_qr(const QrDesc* __restrict__ descs) {
  const QrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n, k = m < n ? m : n;
  extern __shared__ cplx qlds[];
  __shared__ double tau_s[256];
  __shared__ cplx phs[256];
  __shared__ cplx alpha_s[256];
  __shared__ double part_s[2][4];
  if ((int64_t)m * (n + k) <= QR_LDS_MAX)
    qr_body<true>(d, qlds, qlds + (int64_t)m * n, tau_s, phs, alpha_s, part_s);
  else
    qr_body<false>(d, d.work, d.work + (int64_t)m * n, tau_s, phs, alpha_s, part_s);
}

// ----------------------------------------------------------------- Jacobi
// One-sided Jacobi on the columns of A (k x k): for a pair (p, q) with
// a = ||a_p||^2, b = ||a_q||^2, g = a_p^H a_q = |g| e^{i phi}, the rotation
// [a_p, a_q] <- [a_p, a_q] [[c, s], [-s e^{-i phi}, c e^{-i phi}]] with the
// symmetric Schur pair (c, s) of [[a, |g|], [|g|, b]] makes the columns
// orthogonal; the same rotation is applied to J (initially I).  Columns are
// kept contiguous (column-major working copies At, Jt); every pair of a
// round-robin round is handled by its own 16-lane group.
constexpr int JAC_LDS_MAX = 64;

__device__ __forceinline__ void jac_pair(cplx* At, cplx* Jt, int k, int p, int q, int gl,
                                         int* rotated) {
  cplx* x_ = At + (int64_t)p * k;
  cplx* y_ = At + (int64_t)q * k;
  double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
  for (int i = gl; i < k; i += 16) {
    cplx x = x_[i], y = y_[i];
    a += x.re * x.re + x.im * x.im;
    b += y.re * y.re + y.im * y.im;
    gr += x.re * y.re + x.im * y.im;
    gi += x.re * y.im - x.im * y.re;
  }
  a = group16_sum(a);
  b = group16_sum(b);
  gr = group16_sum(gr);
  gi = group16_sum(gi);
  double ag = sqrt(gr * gr + gi * gi);
  // orthogonal to working precision: |g| <= k eps sqrt(a b) (rounding of a
  // length-k dot product); a stricter test is never met and wastes sweeps
  if (ag == 0.0 || ag <= 2.220446049250313e-16 * (k > 16 ? k : 16) * sqrt(a * b)) return;
  double zeta = (b - a) / (2.0 * ag);
  double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  double er = gr / ag, ei = -gi / ag;  // e^{-i phi}
  cplx* u_ = Jt + (int64_t)p * k;
  cplx* v_ = Jt + (int64_t)q * k;
  for (int i = gl; i < k; i += 16) {
    cplx x = x_[i], y = y_[i];
    cplx ye = {y.re * er - y.im * ei, y.re * ei + y.im * er};  // y e^{-i phi}
    x_[i] = cplx{c * x.re - s * ye.re, c * x.im - s * ye.im};
    y_[i] = cplx{s * x.re + c * ye.re, s * x.im + c * ye.im};
    cplx u = u_[i], v = v_[i];
    cplx ve = {v.re * er - v.im * ei, v.re * ei + v.im * er};
    u_[i] = cplx{c * u.re - s * ve.re, c * u.im - s * ve.im};
    v_[i] = cplx{s * u.re + c * ve.re, s * u.im + c * ve.im};
  }
  if (gl == 0) *rotated = 1;
}

template <bool INLDS>
__device__ __forceinline__ void jacobi_body(const JacobiDesc& d, cplx* At, cplx* Jt, int* rotated_p,
                                            double* sig, int* order) {
  const int k = d.k;
  const bool in_lds = INLDS;
  int& rotated = *rotated_p;
  const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
  for (int e = tid; e < k * k; e += 256) {
    int i = e / k, c = e % k;
    At[(int64_t)c * k + i] = d.R[e];
    Jt[e] = cplx{i == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int n = (k % 2) ? k + 1 : k;   // round-robin needs an even count
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      for (int pi = grp; pi < n / 2; pi += 16) {
        int p, q;
        if (pi == 0) { p = r; q = n - 1; }
        else { p = (r + pi) % (n - 1); q = (r - pi + n - 1) % (n - 1); }
        if (p > q) { int t = p; p = q; q = t; }
        if (q < k) jac_pair(At, Jt, k, p, q, gl, &rotated);
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  for (int c = tid; c < k; c += 256) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) {
      cplx x = At[(int64_t)c * k + i];
      s += x.re * x.re + x.im * x.im;
    }
    sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < k; c += 256) {
    int rank = 0;
    for (int o = 0; o < k; ++o)
      if (sig[o] > sig[c] || (sig[o] == sig[c] && o < c)) ++rank;
    order[rank] = c;
  }
  __syncthreads();
  const cplx* Jsrc = Jt;
  if (!in_lds) {
    // Jt lives in d.V: move it to the (now free) work buffer first
    for (int e = tid; e < k * k; e += 256) d.work[e] = Jt[e];
    __syncthreads();
    Jsrc = d.work;
  }
  for (int e = tid; e < k * k; e += 256) {
    int i = e / k, c = e % k;
    d.V[e] = Jsrc[(int64_t)order[c] * k + i];
  }
  for (int c = tid; c < k; c += 256) d.sigma[c] = sig[order[c]];
}

__global__ __launch_bounds__(256) void k_jacobi(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc d = descs[blockIdx.x];
  extern __shared__ cplx jlds[];
  __shared__ int rotated;
  __shared__ double sig[256];
  __shared__ int order[256];
  if (d.k <= JAC_LDS_MAX)
    jacobi_body<true>(d, jlds, jlds + d.k * d.k, &rotated, sig, order);
  else
    jacobi_body<false>(d, d.work, d.V, &rotated, sig, order);
}

__global__ __launch_bounds__(256) void k_colphase(const ColPhaseDesc* __restrict__ descs) {
  const ColPhaseDesc d = descs[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = wave; j < d.keep; j += 4) {
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < d.m; i += 64) {
      cplx x = d.L[(int64_t)i * d.keep + j];
      double v = x.re * x.re + x.im * x.im;
      if (v > best) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o);
      int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    cplx x = d.L[(int64_t)bi * d.keep + j];
    double a = sqrt(x.re * x.re + x.im * x.im);
    if (a > 0.0) {
      cplx ph = {x.re / a, x.im / a};
      for (int i = lane; i < d.m; i += 64) {
        cplx y = d.L[(int64_t)i * d.keep + j];
        d.L[(int64_t)i * d.keep + j] = cplx{y.re * ph.re + y.im * ph.im, y.im * ph.re - y.re * ph.im};
      }
      for (int c = lane; c < d.n; c += 64) {
        cplx y = d.R[(int64_t)j * d.n + c];
        d.R[(int64_t)j * d.n + c] = cplx{y.re * ph.re - y.im * ph.im, y.re * ph.im + y.im * ph.re};
      }
    }
  }
}

// ------------------------------------------------------------ small kernels
__device__ __forceinline__ uint64_t splitmix_out(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_omega(const OmegaDesc* __restrict__ descs) {
  const OmegaDesc d = descs[blockIdx.y];
  const uint64_t tag = d.last_tag ? (uint64_t)(*d.last_tag) : 0ull;
  const uint64_t key = splitmix_out(d.prefix ^ tag, 0);
  const int64_t total = (int64_t)d.n * d.k;
  const double s = 0.70710678118654752440;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    uint64_t z = splitmix_out(key, (uint64_t)e);
    d.out[e] = cplx{((z >> 63) & 1) ? -s : s, ((z >> 62) & 1) ? -s : s};
  }
}

__global__ __launch_bounds__(256) void k_normalize(const NormDesc* __restrict__ descs) {
  const NormDesc d = descs[blockIdx.x];
  __shared__ double sh[8];
  double part = 0.0;
  for (int64_t e = threadIdx.x; e < d.len; e += 256) {
    cplx x = d.x[e];
    part += x.re * x.re + x.im * x.im;
  }
  double nrm = sqrt(block_sum<256>(part, sh));
  double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t e = threadIdx.x; e < d.len; e += 256) {
    cplx x = d.x[e];
    d.x[e] = cplx{x.re * inv, x.im * inv};
  }
  if (threadIdx.x == 0) {
    if (d.logscale && nrm > 0.0) *d.logscale += log10(nrm);
    if (d.norm_out) *d.norm_out = nrm;
  }
}

__global__ __launch_bounds__(256) void k_pad(const PadDesc* __restrict__ descs) {
  const PadDesc d = descs[blockIdx.y];
  const int64_t total = (int64_t)d.l2 * d.P * d.r2;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    int r = (int)(e % d.r2);
    int64_t t = e / d.r2;
    int p = (int)(t % d.P);
    int l = (int)(t / d.P);
    int ls = l - d.off_l, rs = r - d.off_r;
    bool in = ls >= 0 && ls < d.l1 && rs >= 0 && rs < d.r1;
    cplx v = {0.0, 0.0};
    if (in) {
      v = d.src[((int64_t)ls * d.P + p) * d.r1 + rs];
      v.re *= d.sign;
      v.im *= d.sign;
    }
    if (d.mode == 0) d.dst[e] = v;
    else if (in && d.mode == 1) d.dst[e] = v;
    else if (in) { cplx o = d.dst[e]; d.dst[e] = cplx{o.re + v.re, o.im + v.im}; }
  }
}

// trace of a message MPS read as an operator, then site 0 *= conj(tr)/|tr|
__global__ __launch_bounds__(256) void k_phase(const PhaseDesc* __restrict__ descs) {
  const PhaseDesc& d = descs[blockIdx.x];
  __shared__ cplx v[256], w[256];
  const int tid = threadIdx.x;
  if (tid == 0) v[0] = cplx{1.0, 0.0};
  __syncthreads();
  for (int s = 0; s < d.nsites; ++s) {
    const cplx* A = d.sites[s];
    const int l = d.l[s], P = d.P[s], r = d.r[s], D = d.D[s];
    for (int c = tid; c < r; c += 256) {
      double ar = 0.0, ai = 0.0;
      for (int a = 0; a < l; ++a) {
        double sr = 0.0, si = 0.0;
        for (int kk = 0; kk < D; ++kk) {
          cplx x = A[((int64_t)a * P + kk * D + kk) * r + c];
          sr += x.re;
          si += x.im;
        }
        ar += v[a].re * sr - v[a].im * si;
        ai += v[a].re * si + v[a].im * sr;
      }
      w[c] = cplx{ar, ai};
    }
    __syncthreads();
    for (int c = tid; c < r; c += 256) v[c] = w[c];
    __syncthreads();
  }
  cplx tr = v[0];
  double at = sqrt(tr.re * tr.re + tr.im * tr.im);
  if (at > 0.0) {
    cplx ph = {tr.re / at, -tr.im / at};
    cplx* A0 = d.sites[0];
    const int64_t len = (int64_t)d.l[0] * d.P[0] * d.r[0];
    for (int64_t e = tid; e < len; e += 256) {
      cplx x = A0[e];
      A0[e] = cplx{x.re * ph.re - x.im * ph.im, x.re * ph.im + x.im * ph.re};
    }
  }
}

}  // namespace pn

namespace pn {
__global__ void k_rho_ss(const RhoDesc* __restrict__ descs, int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const RhoDesc d = descs[b];
  cplx rho[16];
  for (int pi = 0; pi < 2; ++pi)
    for (int pj = 0; pj < 2; ++pj)
      for (int qi = 0; qi < 2; ++qi)
        for (int qj = 0; qj < 2; ++qj) {
          int ci = pi * 2 + qi, cj = pj * 2 + qj;
          cplx x = d.first_is_i ? d.R[ci * 4 + cj] : d.R[cj * 4 + ci];
          rho[(pi * 2 + pj) * 4 + (qi * 2 + qj)] = x;
        }
  // h = S.S = (1/4)(XX + YY + ZZ) in the basis (p_i p_j)
  const double h[4][4] = {{0.25, 0, 0, 0}, {0, -0.25, 0.5, 0}, {0, 0.5, -0.25, 0}, {0, 0, 0, 0.25}};
  double tr = 0.0, trh = 0.0;
  for (int a = 0; a < 4; ++a) {
    tr += rho[a * 4 + a].re;
    for (int c = 0; c < 4; ++c) trh += rho[a * 4 + c].re * h[c][a];
  }
  for (int e = 0; e < 16; ++e) d.rho[e] = rho[e];
  *d.ss = trh / tr;
}
}  // namespace pn
