// HIP kernels for the BlockBP boundary-chain engine (gfx950 / CDNA4).
//
// * k_gemm<P, SH>: batched complex GEMM on the matrix cores.  One 64x64
//   output tile per 256-thread workgroup, four wave64s each owning a 32x32
//   quadrant (2x2 MFMA 16x16 tiles); 16x64 or 64x16 tiles for products with
//   at most 16 rows or columns.  A complex product is four real MFMA products
//   (re*re - im*im, re*im + im*re).  P selects the arithmetic:
//     PREC_FP64   v_mfma_f64_16x16x4   (complex128 in, FP64 accumulate)
//     PREC_FP32   v_mfma_f32_16x16x4   (operands rounded to FP32, FP32 acc)
//     PREC_BF16X3 v_mfma_f32_16x16x32_bf16, every FP32 operand split as
//                 hi + lo (bf16 each), product hi*hi + hi*lo + lo*hi, FP32 acc
//   Operands are staged through LDS; storage stays complex128.
// * k_permute: batched tensor transpose (rank <= 16).
// * k_qr: Householder QR with R and (optionally) the explicit thin Q, one
//   workgroup per item, working copy in LDS; k_qr_tall: the same
//   factorisation blocked in panels (compact WY) for working copies that do
//   not fit in LDS.
// * k_jacobi: one-sided (Hestenes) Jacobi SVD, one workgroup per item, one
//   16-lane group per column pair of a round-robin round, working copy in
//   LDS (the leading rows when the matrix does not fit) and the work buffer;
//   returns the leading left singular vectors and singular values.
// * small kernels: sketch generation (SplitMix64), normalisation with
//   log-scale, zero-padded copies, message trace phase fix.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels.hpp"

namespace pn {

// Descriptor pointers are generic, and accesses through generic pointers
// compile to FLAT instructions, which count against the LDS wait counter as
// well as the memory one: every wait for an LDS result would then also wait
// for outstanding global loads and stores.  Kernels that mix the two convert
// their device-memory pointers to global ones first.
// (The host pass only parses device code; it keeps plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;
#endif
template <class T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ cplx ld_op(gptr<const cplx> X, int ld, int op, int r, int c) {
  if (op == OP_N) return X[(int64_t)r * ld + c];
  cplx v = X[(int64_t)c * ld + r];
  if (op == OP_C) v.im = -v.im;
  return v;
}

// ------------------------------------------------------------------ GEMM
// Tile shapes (SH): 0 = 64x64 output tile, four waves of 2x2 16x16 MFMA
// blocks; 1 = 16x64 for M <= 16, four waves side by side along N, one block
// each; 2 = 64x16 for N <= 16, four waves along M.  The narrow shapes stop
// the matrix cores from multiplying padding on products with 16 or fewer rows
// or columns.
// 3 = 64x80 for 64 < N <= 80, four waves along M, each 16 x 80 (five
// blocks); 4 = 80x64 for 64 < M <= 80, four waves along N, each 80 x 16.
// They cover the sketch width chi + p = 72 with 11 % padding instead of 78 %.
template <int SH>
struct GemmTile {
  static constexpr int TM = SH == 1 ? 16 : SH == 4 ? 80 : 64;
  static constexpr int TN = SH == 2 ? 16 : SH == 3 ? 80 : 64;
  static constexpr int IB = SH == 0 ? 2 : SH == 4 ? 5 : 1;   // 16x16 blocks per wave
  static constexpr int JB = SH == 0 ? 2 : SH == 3 ? 5 : 1;
};
// workgroups per CU the register budget is set for (two waves per SIMD
// for FP64 / FP32; the split-BF16 tiles keep the full budget)
template <int P>
struct GemmOcc { static constexpr int value = P == PREC_BF16X3 ? 1 : 2; };

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

// Offset contributed by index x of a scatter store, split over axes
// [k0, k1) (last fastest).  The quotients come from the double reciprocal:
// for dims up to 2^16 and x < 2^31, x + 1/2 keeps every floor exact.
__device__ __forceinline__ int64_t gemm_sc_offset(const GemmDesc* __restrict__ g, int k0, int k1,
                                                  int x) {
  int64_t off = 0;
  if (k1 <= k0) return 0;
  for (int k = k1 - 1; k > k0; --k) {
    const int q = (int)floor(((double)x + 0.5) * g->sc_inv[k]);
    off += (int64_t)(x - q * g->sc_dim[k]) * g->sc_ds[k];
    x = q;
  }
  return off + (int64_t)x * g->sc_ds[k0];
}

// The descriptor's scalar fields are read into a small struct (the
// scatter-store tables stay behind the pointer and are read only by the
// tiles that use them).
struct GemmArgs {
  const cplx* A;
  const cplx* B;
  cplx* C;
  int M, N, K, lda, ldb, ldc, opA, opB, sc_n, sc_nr, sc_conj;
  cplx alpha, beta;
};

template <int P, int SH>
__global__ __launch_bounds__(256, GemmOcc<P>::value) void k_gemm(const GemmDesc* __restrict__ descs) {
  constexpr int GT_M = GemmTile<SH>::TM, GT_N = GemmTile<SH>::TN;
  constexpr int IB = GemmTile<SH>::IB, JB = GemmTile<SH>::JB;
  typedef typename GemmCfg<P>::T T;
  constexpr int TK = GemmCfg<P>::TK;
  constexpr int PAD = (sizeof(T) == 8) ? 2 : 4;
  // XCD-aware order: the hardware hands consecutive workgroups round-robin
  // to the chip's 8 XCDs, each with its own L2; renumber them so that every
  // XCD works through one contiguous range of tiles, whose operand rows and
  // output lines then meet in the same L2 (partial lines of a scattered
  // store fill up there before they go to HBM)
  const unsigned gx = gridDim.x, gy = gridDim.y, nwg = gx * gy * gridDim.z;
  const unsigned wid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned xcd = wid % 8u, per = nwg / 8u, extra = nwg % 8u;
  const unsigned vid = xcd * per + (xcd < extra ? xcd : extra) + wid / 8u;
  const unsigned bx = vid % gx, by = (vid / gx) % gy, bz = vid / (gx * gy);
  const GemmDesc* const gp0 = descs + bz;
  GemmArgs g;
  g.A = gp0->A; g.B = gp0->B; g.C = gp0->C;
  g.M = gp0->M; g.N = gp0->N; g.K = gp0->K;
  g.lda = gp0->lda; g.ldb = gp0->ldb; g.ldc = gp0->ldc;
  g.opA = gp0->opA; g.opB = gp0->opB;
  g.sc_n = gp0->sc_n; g.sc_nr = gp0->sc_nr; g.sc_conj = gp0->sc_conj;
  g.alpha = gp0->alpha; g.beta = gp0->beta;
  const int n0 = bx * GT_N;
  if (n0 >= g.N) return;
  const gptr<const cplx> Ag = to_global(g.A), Bg = to_global(g.B);
  const gptr<cplx> Cg = to_global(g.C);
  __shared__ T As_r[TK][GT_M + PAD], As_i[TK][GT_M + PAD];
  __shared__ T Bs_r[TK][GT_N + PAD], Bs_i[TK][GT_N + PAD];
  // M tiles are grid-strided (the grid's y extent is capped at 65535)
  for (int m0 = by * GT_M; m0 < g.M; m0 += gy * GT_M) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = SH == 0 ? (wave >> 1) * 32 : (SH == 2 || SH == 3) ? wave * 16 : 0;
  const int wn = SH == 0 ? (wave & 1) * 32 : (SH == 1 || SH == 4) ? wave * 16 : 0;
  typedef typename std::conditional<P == PREC_FP64, d4, f4>::type acc_t;
  acc_t accr[IB][JB], acci[IB][JB];
  for (int i = 0; i < IB; ++i)
    for (int j = 0; j < JB; ++j) {
      accr[i][j] = acc_t{0, 0, 0, 0};
      acci[i][j] = acc_t{0, 0, 0, 0};
    }
  // op(A)[m0:m0+TM, k0:k0+TK] and op(B)[k0:k0+TK, n0:n0+TN] pass through
  // registers: with 16-deep slices the next one is loaded while the current
  // one is used (the 32-deep split-BF16 slices would need too many
  // registers).  Each thread's elements keep their operand pointer (advanced
  // by one slice per load), their K index, their row / column test and
  // their LDS slot, set once per output tile.
  constexpr int EA = GT_M * TK / 256, EB = GT_N * TK / 256;
  constexpr bool PF = P != PREC_BF16X3;
  const bool conjA = g.opA == OP_C, conjB = g.opB == OP_C;
  const int64_t stA = g.opA == OP_N ? TK : (int64_t)TK * g.lda;
  const int64_t stB = g.opB == OP_N ? (int64_t)TK * g.ldb : TK;
  gptr<const cplx> pA[EA], pB[EB];
  int kA[EA], kB[EB], lA[EA], lB[EB];
  bool okA[EA], okB[EB];
#pragma unroll
  for (int q = 0; q < EA; ++q) {
    const int e = tid + 256 * q;
    int mm, kk;
    if (g.opA == OP_N) { mm = e / TK; kk = e % TK; } else { mm = e % GT_M; kk = e / GT_M; }
    const int r = m0 + mm;
    okA[q] = r < g.M;
    kA[q] = kk;
    lA[q] = kk * (GT_M + PAD) + mm;
    pA[q] = Ag + (okA[q] ? (g.opA == OP_N ? (int64_t)r * g.lda + kk : (int64_t)kk * g.lda + r) : 0);
  }
#pragma unroll
  for (int q = 0; q < EB; ++q) {
    const int e = tid + 256 * q;
    int nn, kk;
    if (g.opB == OP_N) { nn = e % GT_N; kk = e / GT_N; } else { kk = e % TK; nn = e / TK; }
    const int c = n0 + nn;
    okB[q] = c < g.N;
    kB[q] = kk;
    lB[q] = kk * (GT_N + PAD) + nn;
    pB[q] = Bg + (okB[q] ? (g.opB == OP_N ? (int64_t)kk * g.ldb + c : (int64_t)c * g.ldb + kk) : 0);
  }
  // Every element is loaded unconditionally (from the operand's first
  // element when it lies outside), so that all loads of a slice are in
  // flight together; validity and conjugation are applied when the slice is
  // written to LDS, after the loads have landed.
  cplx pa[EA], pb[EB];
  bool va[EA], vb[EB];
  int kload = 0;   // K offset of the next slice to load
  auto fetch = [&]() {
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      va[q] = okA[q] && kload + kA[q] < g.K;
      pa[q] = *(va[q] ? pA[q] : Ag);
      pA[q] += stA;
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      vb[q] = okB[q] && kload + kB[q] < g.K;
      pb[q] = *(vb[q] ? pB[q] : Bg);
      pB[q] += stB;
    }
    kload += TK;
  };
  T* const Asr = &As_r[0][0];
  T* const Asi = &As_i[0][0];
  T* const Bsr = &Bs_r[0][0];
  T* const Bsi = &Bs_i[0][0];
  if constexpr (PF) fetch();
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    if constexpr (!PF) fetch();
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      const double re = pa[q].re, im = conjA ? -pa[q].im : pa[q].im;
      Asr[lA[q]] = va[q] ? (T)re : (T)0;
      Asi[lA[q]] = va[q] ? (T)im : (T)0;
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      const double re = pb[q].re, im = conjB ? -pb[q].im : pb[q].im;
      Bsr[lB[q]] = vb[q] ? (T)re : (T)0;
      Bsi[lB[q]] = vb[q] ? (T)im : (T)0;
    }
    if constexpr (PF) {
      if (k0 + TK < g.K) fetch();
    }
    __syncthreads();
    if constexpr (P == PREC_FP64 || P == PREC_FP32) {
#pragma unroll 2
      for (int kk = 0; kk < TK; kk += 4) {
        if (k0 + kk >= g.K) break;   // past K the slice holds zeros only
        const int kq = kk + (lane >> 4);
        T ar[IB], ai[IB], br[JB], bi[JB];
#pragma unroll
        for (int i = 0; i < IB; ++i) {
          ar[i] = As_r[kq][wm + i * 16 + (lane & 15)];
          ai[i] = As_i[kq][wm + i * 16 + (lane & 15)];
        }
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          br[j] = Bs_r[kq][wn + j * 16 + (lane & 15)];
          bi[j] = Bs_i[kq][wn + j * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < IB; ++i)
#pragma unroll
          for (int j = 0; j < JB; ++j) {
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
      bf8 arh[IB], arl[IB], aih[IB], ail[IB], anh[IB], anl[IB];
      bf8 brh[JB], brl[JB], bih[JB], bil[JB];
#pragma unroll
      for (int i = 0; i < IB; ++i) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          __bf16 h, l;
          split_bf16(As_r[kb + t][wm + i * 16 + (lane & 15)], &h, &l);
          arh[i][t] = h; arl[i][t] = l;
          split_bf16(As_i[kb + t][wm + i * 16 + (lane & 15)], &h, &l);
          aih[i][t] = h; ail[i][t] = l;
          anh[i][t] = -h; anl[i][t] = -l;
        }
      }
#pragma unroll
      for (int j = 0; j < JB; ++j) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          __bf16 h, l;
          split_bf16(Bs_r[kb + t][wn + j * 16 + (lane & 15)], &h, &l);
          brh[j][t] = h; brl[j][t] = l;
          split_bf16(Bs_i[kb + t][wn + j * 16 + (lane & 15)], &h, &l);
          bih[j][t] = h; bil[j][t] = l;
        }
      }
#define PN_MFMA3(acc, xh, xl, yh, yl)                                      \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);     \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0);     \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) {
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
  if (g.sc_n > 0) {
    // transposed store: the tile's row and column offsets are formed once,
    // one per thread, and shared through LDS
    __shared__ int64_t sc_ro[GT_M], sc_co[GT_N];
    const GemmDesc* const gp = descs + bz;
    if (tid < GT_M) {
      const int r = m0 + tid;
      sc_ro[tid] = r < g.M ? gemm_sc_offset(gp, 0, g.sc_nr, r) : 0;
    } else if (tid >= 128 && tid < 128 + GT_N) {
      const int c = n0 + tid - 128;
      sc_co[tid - 128] = c < g.N ? gemm_sc_offset(gp, g.sc_nr, g.sc_n, c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IB; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int rr = (P == PREC_FP64) ? ((lane >> 4) + 4 * t) : (4 * (lane >> 4) + t);
        const int rl = wm + i * 16 + rr;
        if (m0 + rl >= g.M) continue;
        const int64_t ro = sc_ro[rl];
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          const int cl = wn + j * 16 + (lane & 15);
          if (n0 + cl >= g.N) continue;
          const double vr = (double)accr[i][j][t], vi = (double)acci[i][j][t];
          cplx out = {g.alpha.re * vr - g.alpha.im * vi, g.alpha.re * vi + g.alpha.im * vr};
          if (g.sc_conj) out.im = -out.im;
          Cg[ro + sc_co[cl]] = out;
        }
      }
    __syncthreads();   // the offsets are rewritten by the next M tile
    continue;
  }
  const bool beta0 = (g.beta.re == 0.0 && g.beta.im == 0.0);
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j)
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
          const gptr<cplx> cp = Cg + (int64_t)r * g.ldc + c;
          if (!beta0) {
            const cplx o = *cp;
            out.re += g.beta.re * o.re - g.beta.im * o.im;
            out.im += g.beta.re * o.im + g.beta.im * o.re;
          }
          *cp = out;
        }
      }
  }
}

template __global__ void k_gemm<PREC_FP64, 0>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP32, 0>(const GemmDesc*);
template __global__ void k_gemm<PREC_BF16X3, 0>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP64, 1>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP32, 1>(const GemmDesc*);
template __global__ void k_gemm<PREC_BF16X3, 1>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP64, 2>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP32, 2>(const GemmDesc*);
template __global__ void k_gemm<PREC_BF16X3, 2>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP64, 3>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP32, 3>(const GemmDesc*);
template __global__ void k_gemm<PREC_BF16X3, 3>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP64, 4>(const GemmDesc*);
template __global__ void k_gemm<PREC_FP32, 4>(const GemmDesc*);
template __global__ void k_gemm<PREC_BF16X3, 4>(const GemmDesc*);

// --------------------------------------------------------------- permute
__global__ __launch_bounds__(256) void k_permute(const PermDesc* __restrict__ descs) {
  const PermDesc& p = descs[blockIdx.y];
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < p.total; o += step) {
    // mixed-radix split of o by the double reciprocal (exact: o < 2^51, so
    // (rem + 1/2) / dims[k] stays far enough from an integer for the two
    // roundings), with no 64-bit integer division
    int64_t rem = o, off = 0;
    for (int k = p.rank - 1; k > 0; --k) {
      const int64_t q = (int64_t)floor(((double)rem + 0.5) * p.inv[k]);
      off += (rem - q * p.dims[k]) * p.stride[k];
      rem = q;
    }
    off += rem * p.stride[0];
    cplx v = p.src[off];
    if (p.conj) v.im = -v.im;
    p.dst[o] = v;
  }
}

// ---------------------------------------------------------------- reductions
// Sum over the 16 lanes of a DPP row, result in every lane: xor-1 and xor-2
// quad permutations, then half-row and row mirrors (VALU moves, no LDS).
// Every lane reads a valid source lane under these controls, so the moves
// need no old value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double group16_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// sum over lanes l, l ^ 16, l ^ 32, l ^ 48 (the four 16-lane rows of the
// wave), every lane active
__device__ __forceinline__ double rows4_sum(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  v = __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
  lo = __double2loint(v);
  hi = __double2hiint(v);
  a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}

// sum over the 64 lanes (16-lane DPP sums, then the four rows); every lane
// must be active
__device__ __forceinline__ double wave_sum_all(double v) { return rows4_sum(group16_sum(v)); }

// Reduce-scatter steps over the wave's 16-lane rows (r = lane / 16): p's sum
// over rows r and r ^ 2 lands in rows 0-1, q's in rows 2-3 (swap32_sum); p's
// sum over rows r and r ^ 1 in rows 0 and 2, q's in rows 1 and 3 (swap16_sum).
// Every lane active.
__device__ __forceinline__ double swap32_sum(double p, double q) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(p), __double2loint(q), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(p), __double2hiint(q), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double swap16_sum(double p, double q) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(p), __double2loint(q), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(p), __double2hiint(q), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// sum over the wave, result in every lane (all lanes active)
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_all(v); }

// 1/q from the hardware estimate and two Newton steps: full precision for
// normal q well inside the double range (the pivots of the scaled
// tridiagonal, |q| >= eps, and Householder norms), at a fraction of the cost
// of the IEEE division sequence
__device__ __forceinline__ double svt_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// 1/sqrt(g) for normal g > 0 from the hardware estimate and two
// Newton-Raphson steps y <- y + y (1 - g y^2) / 2 (each squares the
// estimate's relative error): full precision at a fraction of the cost of
// sqrt followed by an IEEE division
__device__ __forceinline__ double rsqrt_nr(double g) {
  double y = __builtin_amdgcn_rsq(g);
  y = fma(0.5 * y, fma(-g * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-g * y, y, 1.0), y);
  return y;
}

// v of lane l (l uniform over the wave)
__device__ __forceinline__ double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
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

// Householder columns whose squared norm is positive but below 1e-200 are
// rescaled by this power of two (exact) before the reflector is formed:
// tau = 2 / ||v||^2 would otherwise overflow once ||x||^2 nears the bottom of
// the double range.  Returns 1 when no rescaling is needed.
__device__ __forceinline__ double house_rescale(double nx2) {
  if (!(nx2 > 0.0 && nx2 < 1e-200)) return 1.0;
  return ldexp(1.0, -ilogb(sqrt(nx2)));
}

// W and Qt point into LDS (INLDS) or into the work buffer; keeping the two
// cases apart lets the compiler use ds_read/ds_write for LDS data.
template <bool INLDS, class PW>
__device__ __forceinline__ void qr_body(const QrDesc& d, PW W, PW Qt, double* tau_s,
                                        cplx* phs, cplx* alpha_s, double (*part_s)[4]) {
  const int m = d.m, n = d.n, k = m < n ? m : n;
  const gptr<const cplx> Ain = to_global(d.A);
  const gptr<cplx> Rout = to_global(d.R), Qout = to_global(d.Q);
  const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
  for (int64_t e = tid; e < (int64_t)m * n; e += 256) {
    int r = (int)(e / n), c = (int)(e % n);
    cplx v;
    if (d.conjT) { v = Ain[(int64_t)c * d.lda + r]; v.im = -v.im; }
    else v = Ain[(int64_t)r * d.lda + c];
    W[(int64_t)c * m + r] = v;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < k; ++j) {
    const PW wj = W + (int64_t)j * m;
    // column norm: wave sums, one barrier, every thread finishes the sum
    double part = 0.0;
    for (int i = j + tid; i < m; i += 256) part += wj[i].re * wj[i].re + wj[i].im * wj[i].im;
    part = wave_sum(part);
    if (lane == 0) part_s[j & 1][wave] = part;
    __syncthreads();
    double nx2 = part_s[j & 1][0] + part_s[j & 1][1] + part_s[j & 1][2] + part_s[j & 1][3];
    const double sc = house_rescale(nx2);   // uniform
    if (sc != 1.0) {
      for (int i = j + tid; i < m; i += 256) wj[i] = cplx{wj[i].re * sc, wj[i].im * sc};
      __syncthreads();                        // also: every thread has read nx2
      part = 0.0;
      for (int i = j + tid; i < m; i += 256) part += wj[i].re * wj[i].re + wj[i].im * wj[i].im;
      part = wave_sum(part);
      if (lane == 0) part_s[j & 1][wave] = part;
      __syncthreads();
      nx2 = part_s[j & 1][0] + part_s[j & 1][1] + part_s[j & 1][2] + part_s[j & 1][3];
    }
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
        const PW wc = W + (int64_t)c * m;
        double wr = 0.0, wi = 0.0;
        for (int i = j + gl; i < m; i += 16) {
          const cplx v = (i == j) ? v0 : cplx(wj[i]), a = wc[i];
          wr += v.re * a.re + v.im * a.im;   // conj(v) * a
          wi += v.re * a.im - v.im * a.re;
        }
        wr = group16_sum(wr);
        wi = group16_sum(wi);
        for (int i = j + gl; i < m; i += 16) {
          const cplx v = (i == j) ? v0 : cplx(wj[i]);
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
      alpha_s[j] = cplx{a / sc, 0.0};
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
    Rout[e] = x;
  }
  if (d.Q == nullptr) return;
  // Q = H_0 ... H_{k-1} [I; 0], built backwards (column-major Qt)
  for (int64_t e = tid; e < (int64_t)m * k; e += 256) {
    int c = (int)(e / m), r = (int)(e % m);
    Qt[e] = cplx{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau != 0.0) {
      const PW wj = W + (int64_t)j * m;
      for (int c = j + grp; c < k; c += 16) {
        const PW qc = Qt + (int64_t)c * m;
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
  if (d.qh) {
    // Q^H shares the column-major order of Qt: contiguous on both sides
    for (int64_t e = tid; e < (int64_t)m * k; e += 256) {
      const cplx ph = phs[e / m], x = Qt[e];
      Qout[e] = cplx{x.re * ph.re - x.im * ph.im, -(x.re * ph.im + x.im * ph.re)};
    }
    return;
  }
  for (int64_t e = tid; e < (int64_t)m * k; e += 256) {
    int r = (int)(e / k), c = (int)(e % k);
    cplx ph = phs[c], x = Qt[(int64_t)c * m + r];
    Qout[e] = cplx{x.re * ph.re - x.im * ph.im, x.re * ph.im + x.im * ph.re};
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
  if ((int64_t)m * (n + (d.Q ? k : 0)) <= QR_LDS_MAX)
    qr_body<true>(d, qlds, qlds + (int64_t)m * n, tau_s, phs, alpha_s, part_s);
  else
    qr_body<false>(d, to_global(d.work), to_global(d.work) + (int64_t)m * n, tau_s, phs, alpha_s, part_s);
}

// x -= tau v (v^H x) for a vector held as rows gl + 16 t (t < T) of a
// 16-lane group; the dot product is a 16-lane DPP sum
template <int T>
__device__ __forceinline__ void house_apply(cplx (&x)[T], const cplx (&v)[T], double tau) {
  double wr0 = 0.0, wi0 = 0.0, wr1 = 0.0, wi1 = 0.0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    double& wr = t & 1 ? wr1 : wr0;
    double& wi = t & 1 ? wi1 : wi0;
    wr = fma(v[t].re, x[t].re, wr);
    wr = fma(v[t].im, x[t].im, wr);
    wi = fma(v[t].re, x[t].im, wi);
    wi = fma(-v[t].im, x[t].re, wi);
  }
  const double wr = tau * group16_sum(wr0 + wr1), wi = tau * group16_sum(wi0 + wi1);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    x[t].re = fma(-v[t].re, wr, x[t].re);
    x[t].re = fma(v[t].im, wi, x[t].re);
    x[t].im = fma(-v[t].re, wi, x[t].im);
    x[t].im = fma(-v[t].im, wr, x[t].im);
  }
}


// Householder step j on a column held by one 16-lane group as rows gl + 16 t
// (only that group active): the reflector (zero above row j, its head at row
// j) goes to Vr[0 .. 143]; lane gl == 0 stores tau, the unit phase of alpha
// and |alpha| (rescaled back when the column was tiny).  The column's rows
// from j on may be left rescaled.
template <int T>
__device__ __forceinline__ void qr_group_reflector(cplx (&a)[T], int j, int gl, int lane, cplx* Vr,
                                                   double* tau_o, cplx* phs_o, cplx* alpha_o) {
  // three partial sums keep the dependent chain short
  double p3[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (gl + 16 * t >= j) p3[t % 3] = fma(a[t].re, a[t].re, fma(a[t].im, a[t].im, p3[t % 3]));
  double part = p3[0] + p3[1] + p3[2];
  double nx2 = group16_sum(part);
  // a tiny column is rescaled by the power of two 2^es that brings its
  // squared norm into [1/2, 2) (exact; es = 0 when no rescaling is needed),
  // taken from the exponent of nx2 alone
  const int es = (nx2 > 0.0 && nx2 < 1e-200) ? -(__builtin_amdgcn_frexp_exp(nx2) >> 1) : 0;
  const double sc = ldexp(1.0, es);
  if (sc != 1.0) {
    part = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t)
      if (gl + 16 * t >= j) {
        a[t] = cplx{a[t].re * sc, a[t].im * sc};
        part += a[t].re * a[t].re + a[t].im * a[t].im;
      }
    nx2 = group16_sum(part);
  }
  cplx mine = a[0];
#pragma unroll
  for (int t = 1; t < T; ++t)
    if (t == (j >> 4)) mine = a[t];
  // only the owner group is active here: its lanes share lane & 48
  const int src = __builtin_amdgcn_readfirstlane(lane & 48) | (j & 15);
  const cplx x0 = {readlane_d(mine.re, src), readlane_d(mine.im, src)};
  const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im), nx = sqrt(nx2);
  double tau = 0.0;
  cplx ph = {1.0, 0.0}, v0 = x0;
  if (nx > 0.0) {
    // alpha = -ph nx; ||v||^2 = 2 nx (nx + |x0|), so tau does not wait for v0
    const double iax = ax0 > 0.0 ? svt_rcp(ax0) : 0.0;
    if (ax0 > 0.0) ph = cplx{x0.re * iax, x0.im * iax};
    tau = svt_rcp(nx * (nx + ax0));
    v0 = cplx{x0.re + ph.re * nx, x0.im + ph.im * nx};
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int r = gl + 16 * t;
    if (r < 16 * T) Vr[r] = r < j ? cplx{0.0, 0.0} : r == j ? v0 : a[t];
  }
  if (gl == 0) {
    // |alpha| = nx and its unit phase is -ph (1 for a zero column)
    *tau_o = tau;
    *phs_o = nx > 0.0 ? cplx{-ph.re, -ph.im} : cplx{1.0, 0.0};
    *alpha_o = cplx{ldexp(nx, -es), 0.0};
  }
}

// QR of a block with n <= G columns and m <= 16 T rows (the reflectors,
// phases and outputs of k_qr): 16-lane group g holds column g in registers
// (rows lane + 16 t, t < T).  Step j: group j forms the reflector with DPP sums and
// stores it in LDS, one barrier, every later group applies it to its column
// with a 16-lane DPP dot product.  The reflectors stay in LDS, so forming Q
// (group c applies H_{k-1} .. H_0 to e_c) needs no barrier at all.
template <int T, int G>
__global__ __launch_bounds__(16 * G) void k_qr_small(const QrDesc* __restrict__ descs) {
  const QrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n, k = m < n ? m : n;
  if (m > 16 * T || n > G) return;            // excluded by the plan compiler
  const int tid = threadIdx.x, g = tid >> 4, gl = tid & 15, lane = tid & 63;
  const gptr<const cplx> Ain = to_global(d.A);
  const gptr<cplx> Rout = to_global(d.R), Qout = to_global(d.Q);
  __shared__ cplx V[G][16 * T];
  __shared__ double tau_s[G];
  __shared__ cplx phs[G], alpha_s[G];
  cplx a[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int r = gl + 16 * t;
    const bool ok = r < m && g < n;
    const int64_t o = !ok ? 0 : d.conjT ? (int64_t)g * d.lda + r : (int64_t)r * d.lda + g;
    cplx v = Ain[o];
    if (d.conjT) v.im = -v.im;
    a[t] = ok ? v : cplx{0.0, 0.0};
  }
  for (int j = 0; j < k; ++j) {
    if (g == j) qr_group_reflector(a, j, gl, lane, V[j], tau_s + j, phs + j, alpha_s + j);
    __syncthreads();
    const double tau = tau_s[j];
    if (g > j && g < n) {                                   // tau = 0 changes nothing
      cplx v[T];                                            // zero above row j
#pragma unroll
      for (int t = 0; t < T; ++t) v[t] = V[j][gl + 16 * t];
      house_apply(a, v, tau);
    }
  }
  __syncthreads();
  // R (k x n) with the canonical gauge: diag real non-negative, row r times
  // conj(phase_r); group g writes column g
  if (g < n) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int r = gl + 16 * t;
      if (r >= k) continue;
      cplx x = {0.0, 0.0};
      if (r == g) {
        x = alpha_s[r];
      } else if (r < g) {
        const cplx ph = phs[r];
        x = cplx{a[t].re * ph.re + a[t].im * ph.im, a[t].im * ph.re - a[t].re * ph.im};
      }
      Rout[(int64_t)r * n + g] = x;
    }
  }
  if (d.Q == nullptr || g >= k) return;
  // Q = H_0 ... H_{k-1} [I; 0] times the phases, column g
  cplx q[T];
#pragma unroll
  for (int t = 0; t < T; ++t) q[t] = cplx{gl + 16 * t == g ? 1.0 : 0.0, 0.0};
  // two reflectors per pass, both read before the first is applied (tau = 0
  // changes nothing)
  for (int j = g; j >= 0; j -= 2) {
    const int j1 = j > 0 ? j - 1 : 0;
    const double tau = tau_s[j], tau1 = j > 0 ? tau_s[j1] : 0.0;
    cplx v[T], w[T];
#pragma unroll
    for (int t = 0; t < T; ++t) v[t] = V[j][gl + 16 * t];
#pragma unroll
    for (int t = 0; t < T; ++t) w[t] = V[j1][gl + 16 * t];
    house_apply(q, v, tau);
    house_apply(q, w, tau1);
  }
  const cplx ph = phs[g];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int r = gl + 16 * t;
    if (r >= m) continue;
    const cplx x = {q[t].re * ph.re - q[t].im * ph.im, q[t].re * ph.im + q[t].im * ph.re};
    if (d.qh) Qout[(int64_t)g * m + r] = cplx{x.re, -x.im};
    else Qout[(int64_t)r * k + g] = x;
  }
}

// R-only QR of a block with 16 < n <= 128 columns and m <= 144 rows (the same
// R as k_qr): 16-lane group g of 32 holds columns g + 32 s (s < 4) in
// registers (rows lane + 16 t).  Step j: the group holding column j forms the
// reflector into one of two LDS buffers, one barrier, every later column
// applies it with a 16-lane DPP dot product.  Step j + 1 writes the other
// buffer, so one barrier per step is enough.
constexpr int QRM_THREADS = 512;
__global__ __launch_bounds__(QRM_THREADS) void k_qr_mid(const QrDesc* __restrict__ descs) {
  const QrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n, k = m < n ? m : n;
  if (m > QRS_MAXM || n > QRM_MAXN || d.Q != nullptr) return;   // excluded by the plan compiler
  const int tid = threadIdx.x, g = tid >> 4, gl = tid & 15, lane = tid & 63;
  const gptr<const cplx> Ain = to_global(d.A);
  const gptr<cplx> Rout = to_global(d.R);
  __shared__ cplx V[2][QRS_MAXM];
  __shared__ double tau_s[QRM_MAXN];
  __shared__ cplx phs[QRM_MAXN], alpha_s[QRM_MAXN];
  cplx a[4][9];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = g + 32 * q;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int r = gl + 16 * t;
      const bool ok = r < m && c < n;
      const int64_t o = !ok ? 0 : d.conjT ? (int64_t)c * d.lda + r : (int64_t)r * d.lda + c;
      cplx v = Ain[o];
      if (d.conjT) v.im = -v.im;
      a[q][t] = ok ? v : cplx{0.0, 0.0};
    }
  }
  for (int j = 0; j < k; ++j) {
    if (g == (j & 31)) {
      const int so = j >> 5;                         // slot of column j
      cplx col[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) col[t] = a[0][t];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (q == so) {
#pragma unroll
          for (int t = 0; t < 9; ++t) col[t] = a[q][t];
        }
      // the finished column's rows from j on are not read again
      qr_group_reflector(col, j, gl, lane, V[j & 1], tau_s + j, phs + j, alpha_s + j);
    }
    __syncthreads();
    const double tau = tau_s[j];                     // tau = 0 changes nothing
    if (g + 96 > j) {                                // some column of this group is trailing
      cplx v[9];                                     // zero above row j
#pragma unroll
      for (int t = 0; t < 9; ++t) v[t] = V[j & 1][gl + 16 * t];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = g + 32 * q;
        if (c > j && c < n) house_apply(a[q], v, tau);
      }
    }
  }
  __syncthreads();
  // R (k x n) with the canonical gauge, as k_qr_small; group g writes its columns
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = g + 32 * q;
    if (c >= n) continue;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int r = gl + 16 * t;
      if (r >= k) continue;
      cplx x = {0.0, 0.0};
      if (r == c) {
        x = alpha_s[r];
      } else if (r < c) {
        const cplx ph = phs[r];
        x = cplx{a[q][t].re * ph.re + a[q][t].im * ph.im, a[q][t].im * ph.re - a[q][t].re * ph.im};
      }
      Rout[(int64_t)r * n + c] = x;
    }
  }
}

// --------------------------------------------------------------- tall QR
// Blocked Householder QR for matrices whose working copy does not fit in LDS
// (same reflectors, phases and outputs as k_qr).  Panels of pb <= 8 columns
// are factorised in LDS (in place in the work buffer when the panel does not
// fit); the panel's reflectors H_1 .. H_pb = I - V T V^H
// (compact WY, T upper triangular) are then applied to every trailing column
// in two passes over its rows (s = V^H a, a -= V T^H s), one wave per
// column.  The explicit Q is formed backwards with the same block reflectors.
constexpr int QRT_THREADS = 1024;
constexpr int QRT_PB = 8;
constexpr int QRT_LDS = 9216;   // complex elements of the LDS panel (144 KB)

// sum over the 64 lanes of a wave, result in every lane (all lanes active)
__device__ __forceinline__ double wave_sum64(double v) { return wave_sum_all(v); }

// sum over the workgroup (QRT_THREADS), result in every thread
__device__ __forceinline__ double qrt_block_sum(double v, double* sh) {
  v = wave_sum64(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < QRT_THREADS / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// V[i][j] of the panel (column-major, leading dimension ldp): unit structure
// with the reflector head v0 stored on the diagonal
__device__ __forceinline__ cplx qrt_v(const cplx* P, int64_t ldp, int i, int j) {
  return i < j ? cplx{0.0, 0.0} : P[j * ldp + i];
}

// a[p0 + i] -= sum_j V[i][j] w[j] after s = V^H a (w = T^H s for the
// factorisation, w = T s for forming Q); one wave per column
// (kept out of line: inlining both instantiations exhausts the registers)
template <bool TRANS>
__device__ __noinline__ void qrt_apply(cplx* col, const cplx* P, int64_t ldp, const cplx* T, int mr,
                                       int pb, int lane) {
  double sr[QRT_PB], si[QRT_PB];
#pragma unroll
  for (int j = 0; j < QRT_PB; ++j) { sr[j] = 0.0; si[j] = 0.0; }
  for (int i = lane; i < mr; i += 64) {
    const cplx a = col[i];
#pragma unroll
    for (int j = 0; j < QRT_PB; ++j)
      if (j < pb) {
        const cplx v = qrt_v(P, ldp, i, j);
        sr[j] += v.re * a.re + v.im * a.im;   // conj(v) a
        si[j] += v.re * a.im - v.im * a.re;
      }
  }
  double wr[QRT_PB], wi[QRT_PB];
#pragma unroll
  for (int j = 0; j < QRT_PB; ++j) {
    sr[j] = wave_sum64(sr[j]);
    si[j] = wave_sum64(si[j]);
  }
  // w = T^H s (TRANS) or T s
#pragma unroll
  for (int r = 0; r < QRT_PB; ++r) {
    double xr = 0.0, xi = 0.0;
#pragma unroll
    for (int c = 0; c < QRT_PB; ++c)
      if (r < pb && c < pb) {
        cplx t;
        if (TRANS) { t = T[c * QRT_PB + r]; t.im = -t.im; }   // (T^H)[r][c]
        else t = T[r * QRT_PB + c];
        xr += t.re * sr[c] - t.im * si[c];
        xi += t.re * si[c] + t.im * sr[c];
      }
    wr[r] = xr;
    wi[r] = xi;
  }
  for (int i = lane; i < mr; i += 64) {
    cplx a = col[i];
#pragma unroll
    for (int j = 0; j < QRT_PB; ++j)
      if (j < pb) {
        const cplx v = qrt_v(P, ldp, i, j);
        a.re -= v.re * wr[j] - v.im * wi[j];
        a.im -= v.re * wi[j] + v.im * wr[j];
      }
    col[i] = a;
  }
}

// T (pb x pb, row-major in LDS) of the panel: T[j][j] = tau_j,
// T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^H v_j)
__device__ void qrt_form_t(const cplx* P, int64_t ldp, const double* tau, cplx* T, cplx* G, int mr,
                           int pb) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // G[a][b] = V[:, a]^H V[:, b] for a < b: one wave per entry
  for (int e = wave; e < pb * pb; e += QRT_THREADS / 64) {
    const int a = e / pb, b = e % pb;
    if (a >= b) continue;
    double gr = 0.0, gi = 0.0;
    for (int i = lane; i < mr; i += 64) {
      const cplx x = qrt_v(P, ldp, i, a), y = qrt_v(P, ldp, i, b);
      gr += x.re * y.re + x.im * y.im;
      gi += x.re * y.im - x.im * y.re;
    }
    gr = wave_sum64(gr);
    gi = wave_sum64(gi);
    if (lane == 0) G[a * QRT_PB + b] = cplx{gr, gi};
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < pb; ++j) {
      for (int r = 0; r < QRT_PB; ++r) if (r >= j) T[r * QRT_PB + j] = cplx{0.0, 0.0};
      T[j * QRT_PB + j] = cplx{tau[j], 0.0};
      for (int r = 0; r < j; ++r) {
        double xr = 0.0, xi = 0.0;
        for (int c = r; c < j; ++c) {
          const cplx t = T[r * QRT_PB + c], g = G[c * QRT_PB + j];
          xr += t.re * g.re - t.im * g.im;
          xi += t.re * g.im + t.im * g.re;
        }
        T[r * QRT_PB + j] = cplx{-tau[j] * xr, -tau[j] * xi};
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(QRT_THREADS) void k_qr_tall(const QrDesc* __restrict__ descs) {
  const QrDesc d = descs[blockIdx.x];
  const int m = d.m, n = d.n, k = m < n ? m : n;
  extern __shared__ cplx Pn[];            // panel, column-major
  __shared__ cplx T[QRT_PB * QRT_PB], G[QRT_PB * QRT_PB];
  __shared__ double tau_s[256];
  __shared__ cplx phs[256];
  __shared__ double alpha_s[256];
  __shared__ double red[QRT_THREADS / 64];
  __shared__ int pstart[257];             // panel starts (for forming Q)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = QRT_THREADS / 64;
  cplx* W = d.work;                       // m x n column-major
  cplx* Qt = d.work + (int64_t)m * n;     // m x k column-major
  for (int64_t e = tid; e < (int64_t)m * n; e += QRT_THREADS) {
    const int r = (int)(e % m), c = (int)(e / m);
    cplx v;
    if (d.conjT) { v = d.A[(int64_t)c * d.lda + r]; v.im = -v.im; }
    else v = d.A[(int64_t)r * d.lda + c];
    W[e] = v;
  }
  __syncthreads();
  int np = 0;
  for (int p0 = 0; p0 < k; ) {
    const int mr = m - p0;
    const int pb = k - p0 < QRT_PB ? k - p0 : QRT_PB;
    const bool inl = (int64_t)pb * mr <= QRT_LDS;
    cplx* P = inl ? Pn : W + (int64_t)p0 * m + p0;
    const int64_t ldp = inl ? mr : m;
    if (tid == 0) pstart[np] = p0;
    ++np;
    if (inl) {
      for (int e = tid; e < pb * mr; e += QRT_THREADS) {
        const int c = e / mr, i = e % mr;
        Pn[e] = W[(int64_t)(p0 + c) * m + p0 + i];
      }
    }
    __syncthreads();
    // factor the panel
    for (int j = 0; j < pb; ++j) {
      cplx* xj = P + j * ldp;
      double part = 0.0;
      for (int i = j + tid; i < mr; i += QRT_THREADS) part += xj[i].re * xj[i].re + xj[i].im * xj[i].im;
      double nx2 = qrt_block_sum(part, red);
      const double sc = house_rescale(nx2);   // uniform
      if (sc != 1.0) {
        for (int i = j + tid; i < mr; i += QRT_THREADS) xj[i] = cplx{xj[i].re * sc, xj[i].im * sc};
        __syncthreads();
        part = 0.0;
        for (int i = j + tid; i < mr; i += QRT_THREADS) part += xj[i].re * xj[i].re + xj[i].im * xj[i].im;
        nx2 = qrt_block_sum(part, red);
      }
      const cplx x0 = xj[j];
      const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im), nx = sqrt(nx2);
      double tau = 0.0;
      cplx alpha = {0.0, 0.0}, v0 = x0;
      if (nx > 0.0) {
        const cplx ph = ax0 > 0.0 ? cplx{x0.re / ax0, x0.im / ax0} : cplx{1.0, 0.0};
        alpha = cplx{-ph.re * nx, -ph.im * nx};
        v0 = cplx{x0.re - alpha.re, x0.im - alpha.im};
        const double nv2 = nx2 - ax0 * ax0 + v0.re * v0.re + v0.im * v0.im;
        tau = nv2 > 0.0 ? 2.0 / nv2 : 0.0;
      }
      // remaining panel columns, one wave each
      if (tau != 0.0) {
        for (int c = j + 1 + wave; c < pb; c += NW) {
          cplx* xc = P + c * ldp;
          double wr = 0.0, wi = 0.0;
          for (int i = j + lane; i < mr; i += 64) {
            const cplx v = (i == j) ? v0 : xj[i], a = xc[i];
            wr += v.re * a.re + v.im * a.im;
            wi += v.re * a.im - v.im * a.re;
          }
          wr = wave_sum64(wr);
          wi = wave_sum64(wi);
          for (int i = j + lane; i < mr; i += 64) {
            const cplx v = (i == j) ? v0 : xj[i];
            xc[i].re -= tau * (v.re * wr - v.im * wi);
            xc[i].im -= tau * (v.re * wi + v.im * wr);
          }
        }
      }
      if (tid == 0) {
        tau_s[p0 + j] = tau;
        const double a = sqrt(alpha.re * alpha.re + alpha.im * alpha.im);
        phs[p0 + j] = a > 0.0 ? cplx{alpha.re / a, alpha.im / a} : cplx{1.0, 0.0};
        alpha_s[p0 + j] = a / sc;
      }
      __syncthreads();
      // the reflector head replaces x0 once every column used x0
      if (tid == 0 && tau != 0.0) xj[j] = v0;
      __syncthreads();
    }
    qrt_form_t(P, ldp, tau_s + p0, T, G, mr, pb);
    if (inl) {
      // write the panel back (R rows above, reflectors below / on the diagonal)
      for (int e = tid; e < pb * mr; e += QRT_THREADS) {
        const int c = e / mr, i = e % mr;
        W[(int64_t)(p0 + c) * m + p0 + i] = Pn[e];
      }
    }
    // trailing columns: A <- (I - V T V^H)^H A
    for (int c = p0 + pb + wave; c < n; c += NW)
      qrt_apply<true>(W + (int64_t)c * m + p0, P, ldp, T, mr, pb, lane);
    __syncthreads();
    p0 += pb;
  }
  // R with the canonical gauge: diag(R) real non-negative, row j * conj(phase_j)
  for (int64_t e = tid; e < (int64_t)k * n; e += QRT_THREADS) {
    const int j = (int)(e / n), c = (int)(e % n);
    cplx x = {0.0, 0.0};
    if (c == j) x = cplx{alpha_s[j], 0.0};
    else if (c > j) {
      const cplx w = W[(int64_t)c * m + j], ph = phs[j];
      x = cplx{w.re * ph.re + w.im * ph.im, w.im * ph.re - w.re * ph.im};
    }
    d.R[e] = x;
  }
  if (d.Q == nullptr) return;
  // Q = H_0 ... H_{k-1} [I; 0], panels applied backwards
  for (int64_t e = tid; e < (int64_t)m * k; e += QRT_THREADS) {
    const int c = (int)(e / m), r = (int)(e % m);
    Qt[e] = cplx{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  if (tid == 0) pstart[np] = k;
  __syncthreads();
  for (int q = np - 1; q >= 0; --q) {
    const int p0 = pstart[q], mr = m - p0;
    const int pb = pstart[q + 1] - p0;
    const bool inl = (int64_t)pb * mr <= QRT_LDS;
    const cplx* P = inl ? Pn : W + (int64_t)p0 * m + p0;
    const int64_t ldp = inl ? mr : m;
    if (inl) {
      for (int e = tid; e < pb * mr; e += QRT_THREADS) {
        const int c = e / mr, i = e % mr;
        Pn[e] = W[(int64_t)(p0 + c) * m + p0 + i];
      }
    }
    __syncthreads();
    qrt_form_t(P, ldp, tau_s + p0, T, G, mr, pb);
    for (int c = p0 + wave; c < k; c += NW)
      qrt_apply<false>(Qt + (int64_t)c * m + p0, P, ldp, T, mr, pb, lane);
    __syncthreads();
  }
  if (d.qh) {
    for (int64_t e = tid; e < (int64_t)m * k; e += QRT_THREADS) {
      const cplx ph = phs[e / m], x = Qt[e];
      d.Q[e] = cplx{x.re * ph.re - x.im * ph.im, -(x.re * ph.im + x.im * ph.re)};
    }
    return;
  }
  for (int64_t e = tid; e < (int64_t)m * k; e += QRT_THREADS) {
    const int r = (int)(e / k), c = (int)(e % k);
    const cplx ph = phs[c], x = Qt[(int64_t)c * m + r];
    d.Q[e] = cplx{x.re * ph.re - x.im * ph.im, x.re * ph.im + x.im * ph.re};
  }
}

// ------------------------------------------------------------ Cholesky QR
// k_chol: the Cholesky step of the tall QR (see CholDesc), one workgroup of
// 16 waves per item (fewer waves cost more in serial updates per step than
// they save in barriers: 214 against 137 us at n = 72).  The upper triangle is kept packed in LDS (row i
// from i (2n - i + 1) / 2; n <= 128: 129 KB); when the running factor is
// updated and the two triangles fit (n <= 92), the previous factor is staged
// in LDS behind it.  The partial Gram matrices are summed eight elements at
// a time with their loads in flight together.  The right-looking
// factorisation takes one barrier per step: every thread reads the finished
// row j and updates its elements of the trailing triangle with the unscaled
// row and the factor 1 / G_jj; the rows of R are scaled afterwards.  R^-1 is
// then formed in place column by column (column j of R^-1 needs R^-1 of the
// leading block, stored over the finished columns, and column j of R), a
// 16-lane group per row.
constexpr int CHOL_THREADS = 1024;
constexpr int CHOL_PACKED = CHOLQR_MAXN * (CHOLQR_MAXN + 1) / 2;
constexpr int CHOL_ROUND = 4;   // packed elements per thread per load round

__device__ __forceinline__ int chol_off(int n, int i, int j) { return i * (2 * n - i + 1) / 2 + (j - i); }

// (row, column) of packed index e (row: the largest i with chol_off(i, i) <= e)
__device__ __forceinline__ void chol_ij(int n, int e, int* i, int* j) {
  const double b = 2.0 * n + 1.0;
  int r = (int)((b - sqrt(b * b - 8.0 * e)) * 0.5);
  r = r < 0 ? 0 : (r > n - 1 ? n - 1 : r);
  while (r > 0 && chol_off(n, r, r) > e) --r;
  while (r + 1 < n && chol_off(n, r + 1, r + 1) <= e) ++r;
  *i = r;
  *j = r + (e - chol_off(n, r, r));
}

__global__ __launch_bounds__(CHOL_THREADS) void k_chol(const CholDesc* __restrict__ descs) {
  const CholDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x, nn = n * n, np = n * (n + 1) / 2;
  __shared__ cplx A[CHOL_PACKED];
  __shared__ double rd[CHOLQR_MAXN], ird[CHOLQR_MAXN];
  __shared__ cplx tcol[CHOLQR_MAXN];
  __shared__ double sc[2];
  if (n > CHOLQR_MAXN) return;   // excluded by the plan compiler
  const gptr<const cplx> G = to_global(d.G);
  const bool want_r = d.R != nullptr;
  const bool acc_r = want_r && d.accumulate;
  const bool stage = acc_r && 2 * np <= CHOL_PACKED;   // previous R behind A
  cplx* const Rs = A + np;
  const gptr<cplx> Rg = to_global(d.R);
  // sum of the partials in order (deterministic); the previous R when staged
  for (int e0 = tid; e0 < np; e0 += CHOL_THREADS * CHOL_ROUND) {
    int full[CHOL_ROUND];
    cplx acc[CHOL_ROUND];
#pragma unroll
    for (int q = 0; q < CHOL_ROUND; ++q) {
      const int e = e0 + q * CHOL_THREADS;
      full[q] = -1;
      acc[q] = cplx{0.0, 0.0};
      if (e < np) {
        int i, j;
        chol_ij(n, e, &i, &j);
        full[q] = i * n + j;
      }
    }
    for (int p = 0; p < d.S; ++p) {
      cplx v[CHOL_ROUND];
#pragma unroll
      for (int q = 0; q < CHOL_ROUND; ++q)
        v[q] = full[q] >= 0 ? cplx(G[(int64_t)p * nn + full[q]]) : cplx{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < CHOL_ROUND; ++q) {
        acc[q].re += v[q].re;
        acc[q].im += v[q].im;
      }
    }
#pragma unroll
    for (int q = 0; q < CHOL_ROUND; ++q) {
      if (full[q] < 0) continue;
      A[e0 + q * CHOL_THREADS] = acc[q];
      if (stage) Rs[e0 + q * CHOL_THREADS] = Rg[full[q]];
    }
  }
  __syncthreads();
  if (tid < 64) {
    // trace and largest diagonal entry, one wave
    double t = 0.0, mx = 0.0;
    for (int i = tid; i < n; i += 64) {
      const double g = A[chol_off(n, i, i)].re;
      t += g;
      mx = fmax(mx, g);
    }
    t = wave_sum(t);
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (tid == 0) {
      sc[0] = d.shift ? 11.0 * ((double)d.m * n + (double)n * (n + 1)) * 0x1p-53 * t : 0.0;
      sc[1] = 1e-24 * mx;
    }
  }
  __syncthreads();
  const double thr = sc[1];
  if (tid < n) A[chol_off(n, tid, tid)].re += sc[0];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int dj = chol_off(n, j, j);
    const double gjj = A[dj].re;
    // a NaN pivot is kept (it propagates to the outputs)
    const bool ok = !(gjj <= thr);
    if (tid == 0) {
      rd[j] = ok ? sqrt(gjj) : 0.0;
      ird[j] = ok ? 1.0 / sqrt(gjj) : 0.0;
    }
    const int t = n - 1 - j;
    if (ok && t > 0) {
      const double inv = 1.0 / gjj;
      // trailing triangle row by row: row a (i = j + 1 + a) holds t - a
      // elements starting at packed offset chol_off(n, i, i)
      for (int e = tid; e < t * t; e += CHOL_THREADS) {
        const int a = e / t, b = e - a * t;
        if (a > b) continue;
        const int i = j + 1 + a;
        const cplx gi = A[dj + 1 + a], gk = A[dj + 1 + b];
        cplx& x = A[chol_off(n, i, i) + (b - a)];
        x.re -= (gi.re * gk.re + gi.im * gk.im) * inv;   // conj(g_ji) g_jk / g_jj
        x.im -= (gi.re * gk.im - gi.im * gk.re) * inv;
      }
    }
    __syncthreads();
  }
  // R_new in place: row i scaled by 1 / r_ii, real diagonal
  for (int e = tid; e < np; e += CHOL_THREADS) {
    int i, k;
    chol_ij(n, e, &i, &k);
    A[e] = k == i ? cplx{rd[i], 0.0} : cplx{A[e].re * ird[i], A[e].im * ird[i]};
  }
  __syncthreads();
  if (acc_r) {
    // R <- R_new R_prev (both upper triangular).  R_prev comes from LDS when
    // staged; otherwise from global memory, and the products go to the R^-1
    // buffer first (R^-1 is written last) and are copied over R once every
    // thread has read its terms.
    const gptr<cplx> Tg = stage ? Rg : to_global(d.Rinv);
    for (int base = 0; base < np; base += CHOL_THREADS * CHOL_ROUND) {
      cplx acc[CHOL_ROUND];
      int full[CHOL_ROUND];
#pragma unroll
      for (int q = 0; q < CHOL_ROUND; ++q) {
        const int e = base + tid + q * CHOL_THREADS;
        cplx s = {0.0, 0.0};
        full[q] = -1;
        if (e < np) {
          int i, k;
          chol_ij(n, e, &i, &k);
          full[q] = i * n + k;
          const int row = chol_off(n, i, i) - i;   // A[row + l] = R_new[i][l]
          for (int l = i; l <= k; ++l) {
            const cplx a = A[row + l];
            const cplx b = stage ? Rs[chol_off(n, l, k)] : cplx(Rg[(int64_t)l * n + k]);
            s.re += a.re * b.re - a.im * b.im;
            s.im += a.re * b.im + a.im * b.re;
          }
        }
        acc[q] = s;
      }
#pragma unroll
      for (int q = 0; q < CHOL_ROUND; ++q)
        if (full[q] >= 0) Tg[full[q]] = acc[q];
    }
    if (!stage) {
      __syncthreads();
      for (int e = tid; e < np; e += CHOL_THREADS) {
        int i, k;
        chol_ij(n, e, &i, &k);
        Rg[i * n + k] = Tg[i * n + k];
      }
    }
  } else if (want_r) {
    for (int e = tid; e < np; e += CHOL_THREADS) {
      int i, k;
      chol_ij(n, e, &i, &k);
      Rg[i * n + k] = A[e];
    }
  }
  if (want_r)
    for (int e = tid; e < nn; e += CHOL_THREADS) {
      const int i = e / n, k = e - i * n;
      if (k < i) Rg[e] = cplx{0.0, 0.0};
    }
  // R^-1 in place: X[j][j] = 1 / r_jj, X[i][j] = -(sum_{i <= l < j} X[i][l] R[l][j]) / r_jj
  const int grp = tid >> 4, gl = tid & 15;
  for (int j = 0; j < n; ++j) {
    for (int i = grp; i < j; i += CHOL_THREADS / 16) {
      const int row = chol_off(n, i, i) - i;
      double sr = 0.0, si = 0.0;
      for (int l = i + gl; l < j; l += 16) {
        const cplx x = A[row + l], r = A[chol_off(n, l, j)];
        sr += x.re * r.re - x.im * r.im;
        si += x.re * r.im + x.im * r.re;
      }
      sr = group16_sum(sr);
      si = group16_sum(si);
      if (gl == 0) tcol[i] = cplx{-sr * ird[j], -si * ird[j]};
    }
    __syncthreads();
    for (int i = tid; i <= j; i += CHOL_THREADS)
      A[chol_off(n, i, j)] = i < j ? tcol[i] : cplx{ird[j], 0.0};
    __syncthreads();
  }
  const gptr<cplx> Xg = to_global(d.Rinv);
  for (int e = tid; e < nn; e += CHOL_THREADS) {
    const int i = e / n, k = e - i * n;
    Xg[e] = k >= i ? A[chol_off(n, i, k)] : cplx{0.0, 0.0};
  }
}

// k_chol_b: the same step for n <= 80 by 16-wide blocks (far fewer barriers
// than the column-by-column form).  Full storage in LDS (row stride 80).
// The Cholesky factorisation is carried out as row operations on [G | I]:
// the operations that turn G into R turn I into R^-H (lower triangular), so
// R^-1 = (R^-H)^H comes out of the same pass.  R fills the upper triangle,
// R^-H the strictly lower one, its diagonal (1 / R_jj) a separate array.
// Per 16-row block: (1) the block row is finished by its 16 pivot steps,
// one column per lane, the pivot and the multipliers R[j][i] broadcast from
// the lanes holding the diagonal block (readlane); (2) the rows below get
// the rank-16 update on the matrix cores, in G's upper part and in R^-H.
// The previous running factor is staged packed in W.
constexpr int CHB_N = 80, CHB_LD = 80;

// Complex 16 x 16 tile product on the matrix cores, acc += A B over
// k in [kb, ke) (stepping by 4 from kb; loaders return 0 outside): four real
// FP64 MFMAs per step.  MFMA operand layout: lane supplies A[lane % 16][k]
// and B[k][lane % 16] with k = k0 + lane / 16; the accumulator holds rows
// lane / 16 + 4 t, column lane % 16.  All 64 lanes must be active.
template <class LA, class LB>
__device__ __forceinline__ void cmma16(int kb, int ke, int lane, LA la, LB lb, d4& accr, d4& acci) {
  for (int k0 = kb; k0 < ke; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const cplx a = la(lane & 15, k), b = lb(k, lane & 15);
    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, accr, 0, 0, 0);
    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.im, accr, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, acci, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.re, acci, 0, 0, 0);
  }
}

__global__ __launch_bounds__(CHOL_THREADS) void k_chol_b(const CholDesc* __restrict__ descs) {
  const CholDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x, nn = n * n;
  const int lane = tid & 63, wave = tid >> 6;
  __shared__ cplx A[CHB_N * CHB_LD];
  __shared__ cplx W[CHB_N * (CHB_N + 1) / 2];
  __shared__ double ird[CHB_N];
  __shared__ double sc[2];
  if (n > CHB_N) return;   // excluded by the executor
  const gptr<const cplx> G = to_global(d.G);
  const bool want_r = d.R != nullptr;
  const bool acc_r = want_r && d.accumulate;
  const gptr<cplx> Rg = to_global(d.R);
  // sum of the partials in order (deterministic), upper triangle; the
  // previous factor staged packed
  for (int base = 0; base < nn; base += CHOL_THREADS * CHOL_ROUND) {
    cplx acc[CHOL_ROUND];
    bool up[CHOL_ROUND];
#pragma unroll
    for (int q = 0; q < CHOL_ROUND; ++q) {
      const int e = base + tid + q * CHOL_THREADS;
      up[q] = e < nn && (e / n) <= (e % n);
      acc[q] = cplx{0.0, 0.0};
    }
    for (int p = 0; p < d.S; ++p) {
      cplx v[CHOL_ROUND];
#pragma unroll
      for (int q = 0; q < CHOL_ROUND; ++q)
        v[q] = up[q] ? cplx(G[(int64_t)p * nn + base + tid + q * CHOL_THREADS]) : cplx{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < CHOL_ROUND; ++q) {
        acc[q].re += v[q].re;
        acc[q].im += v[q].im;
      }
    }
#pragma unroll
    for (int q = 0; q < CHOL_ROUND; ++q) {
      const int e = base + tid + q * CHOL_THREADS;
      if (e >= nn) continue;
      const int i = e / n, j = e - i * n;
      A[i * CHB_LD + j] = acc[q];   // zero below the diagonal
      if (acc_r && up[q]) W[chol_off(n, i, j)] = Rg[e];
    }
  }
  __syncthreads();
  if (tid < 64) {
    double t = 0.0, mx = 0.0;
    for (int i = tid; i < n; i += 64) {
      const double g = A[i * CHB_LD + i].re;
      t += g;
      mx = fmax(mx, g);
    }
    t = wave_sum(t);
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (tid == 0) {
      sc[0] = d.shift ? 11.0 * ((double)d.m * n + (double)n * (n + 1)) * 0x1p-53 * t : 0.0;
      sc[1] = 1e-24 * mx;
    }
  }
  __syncthreads();
  const double thr = sc[1];
  if (tid < n) A[tid * CHB_LD + tid].re += sc[0];
  __syncthreads();
  const int nb = (n + 15) / 16;
  for (int kb = 0; kb < nb; ++kb) {
    const int k0 = 16 * kb, kw = n - k0 < 16 ? n - k0 : 16, c1 = k0 + kw;
    // (1) rows k0 .. c1 - 1 of [G | I] by row operations.  Lanes 0-15 of
    // every working wave hold the diagonal block's columns of G (the pivots
    // and multipliers, the same in every wave); lanes 16-63 hold the other
    // columns of the block row: the identity's diagonal block, R^-H left of
    // it, then G right of it (n columns in all, 48 per wave).
    const int nwork = (n + 47) / 48;
    if (wave < nwork) {
      const int c = lane & 15;
      int kind = -1, col = 0;   // 0 G diagonal, 1 identity diagonal, 2 R^-H left, 3 G right
      if (lane < 16) {
        if (c < kw) { kind = 0; col = k0 + c; }
      } else {
        const int q = wave * 48 + lane - 16;
        if (q < kw) { kind = 1; col = k0 + q; }
        else if (q < c1) { kind = 2; col = q - kw; }
        else if (q < n) { kind = 3; col = q; }
      }
      cplx a[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cplx v = {0.0, 0.0};
        if (r < kw) {
          if (kind == 0) {
            if (r <= c) v = A[(k0 + r) * CHB_LD + col];
          } else if (kind == 1) {
            if (r == col - k0) v.re = 1.0;
          } else if (kind > 1) {
            v = A[(k0 + r) * CHB_LD + col];
          }
        }
        a[r] = v;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (j < kw) {
          const double g = readlane_d(a[j].re, j);   // pivot, diagonal lane j
          const bool ok = !(g <= thr);
          // taken before the test, which only selects (a rejected pivot's
          // non-finite 1/sqrt is discarded), to keep the test off the chain
          const double y = rsqrt_nr(g);
          const double ir = ok ? y : 0.0, r = ok ? g * y : 0.0;
          a[j].re *= ir;
          a[j].im *= ir;
          if (lane == j) a[j] = cplx{r, 0.0};   // R's diagonal is the root itself
          if (tid == 0) ird[k0 + j] = ir;
          // row i -= conj(R[j][i]) row j, R[j][i] from diagonal lane i
#pragma unroll
          for (int i = j + 1; i < 16; ++i) {
            const double rr = readlane_d(a[j].re, i), ri = readlane_d(a[j].im, i);
            a[i].re = fma(-rr, a[j].re, fma(-ri, a[j].im, a[i].re));
            a[i].im = fma(-rr, a[j].im, fma(ri, a[j].re, a[i].im));
          }
        }
      }
      // R in the upper triangle, R^-H below it (its diagonal is ird)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const bool st = r < kw && ((kind == 0 && wave == 0 && r <= c) ||
                                   (kind == 1 && r > col - k0) || kind > 1);
        if (st) A[(k0 + r) * CHB_LD + col] = a[r];
      }
    }
    __syncthreads();
    // (2) rows c1 .. n - 1 of [G | I] -= (block row multipliers) x (block
    // row): G's upper tiles right of c1 and R^-H's tiles left of c1, one
    // wave per 16 x 16 tile on the matrix cores
    const int t = n - c1, tt = (t + 15) / 16, tw = tt + kb + 1;
    for (int p = wave; p < tt * tw; p += CHOL_THREADS / 64) {
      const int ta = p / tw, tb = p - ta * tw;
      const bool gpart = tb < tt;
      if (gpart && ta > tb) continue;
      const int i0 = c1 + 16 * ta, j0 = gpart ? c1 + 16 * tb : 16 * (tb - tt);
      const int jend = gpart ? n : c1;
      d4 accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
      cmma16(0, 16, lane,
             [&](int r, int l) {   // conj(R[k0 + l][i0 + r])
               cplx v = {0.0, 0.0};
               if (l < kw && i0 + r < n) {
                 v = A[(k0 + l) * CHB_LD + i0 + r];
                 v.im = -v.im;
               }
               return v;
             },
             [&](int l, int cc) {   // block row, column j0 + cc
               const int col = j0 + cc;
               cplx v = {0.0, 0.0};
               if (l < kw && col < jend) {
                 if (gpart || col < k0 + l) v = A[(k0 + l) * CHB_LD + col];
                 else if (col == k0 + l) v.re = ird[k0 + l];
               }
               return v;
             },
             accr, acci);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + (lane >> 4) + 4 * q, col = j0 + (lane & 15);
        if (i < n && col < jend && (!gpart || i <= col)) {
          cplx v = A[i * CHB_LD + col];
          v.re -= accr[q];
          v.im -= acci[q];
          A[i * CHB_LD + col] = v;
        }
      }
    }
    __syncthreads();
  }
  // running factor R <- R_new R_prev (R_prev staged packed in W) on the
  // matrix cores: one wave per 16 x 16 output tile; tiles below the
  // diagonal are zero
  if (acc_r) {
    const int nt = (n + 15) / 16;
    for (int p = wave; p < nt * nt; p += CHOL_THREADS / 64) {
      const int ta = p / nt, tb = p - ta * nt;
      d4 accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
      if (ta <= tb) {
        const int i0 = 16 * ta, j0 = 16 * tb;
        cmma16(i0, j0 + 16 < n ? j0 + 16 : n, lane,
               [&](int r, int k) {   // R_new[i0 + r][k], upper
                 cplx v = {0.0, 0.0};
                 if (i0 + r < n && i0 + r <= k && k < n) v = A[(i0 + r) * CHB_LD + k];
                 return v;
               },
               [&](int k, int c) {   // R_prev[k][j0 + c], upper, packed
                 cplx v = {0.0, 0.0};
                 if (j0 + c < n && k <= j0 + c) v = W[chol_off(n, k, j0 + c)];
                 return v;
               },
               accr, acci);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * ta + (lane >> 4) + 4 * q, c = 16 * tb + (lane & 15);
        if (r < n && c < n) Rg[r * n + c] = r <= c ? cplx{accr[q], acci[q]} : cplx{0.0, 0.0};
      }
    }
  } else if (want_r) {
    for (int e = tid; e < nn; e += CHOL_THREADS) {
      const int i = e / n, k = e - i * n;
      Rg[e] = k >= i ? A[i * CHB_LD + k] : cplx{0.0, 0.0};
    }
  }
  // R^-1 = (R^-H)^H
  const gptr<cplx> Xg = to_global(d.Rinv);
  for (int e = tid; e < nn; e += CHOL_THREADS) {
    const int i = e / n, kk = e - i * n;
    cplx v = {0.0, 0.0};
    if (kk == i) {
      v.re = ird[i];
    } else if (kk > i) {
      v = A[kk * CHB_LD + i];
      v.im = -v.im;
    }
    Xg[e] = v;
  }
}

// ----------------------------------------------------------------- Jacobi
// One-sided (Hestenes) Jacobi on the columns of A (rows x cols).  For a pair
// (p, q) with a = ||a_p||^2, b = ||a_q||^2 and g = a_p^H a_q = |g| e^{i phi},
// the rotation [a_p, a_q] <- [a_p, a_q] [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
// with the symmetric Schur pair (c, s) of [[a, |g|], [|g|, b]] makes the two
// columns orthogonal.  At convergence A W = U Sigma: the column norms are the
// singular values and the normalised columns the left singular vectors, so
// the rotations W are never accumulated.
//
// Every pair of a round-robin round is handled by one 16-lane group that
// loads its two columns into registers (up to JAC_RC rows per lane, all loads
// in flight together), reduces the three dot products over the group with
// DPP and writes the rotated columns back.
constexpr int JAC_G = 16;                      // lanes per column pair
constexpr int JAC_RC = 9;                      // rows per lane (max)
constexpr int JAC_THREADS = 1024;              // 64 pairs per pass
constexpr int JAC_MAX_ROWS = JAC_G * JAC_RC;   // 144
constexpr int JAC_MAX_COLS = JAC_MAX_ROWS;   // the plan keeps cols <= rows
constexpr int JAC_LDS_MAX = 9216;              // complex elements (144 KB)
constexpr int JAC_MAX_SWEEPS = 60;
static_assert(JAC_MAX_ROWS == kJacobiMaxRows && JAC_MAX_COLS == kJacobiMaxCols,
              "Jacobi limits of the plan compiler and the kernel differ");

// (re, im) pairs as a vector type so that address-space qualified pointers
// (global: global_load/store, LDS: ds_read/write) can be used directly
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) d2v gd2;   // global memory
typedef __attribute__((address_space(3))) d2v ld2;   // LDS

// The working copy of column c is split by rows: its first NL 16-row slices
// live in LDS (L[c * NL * 16 + ...]) and the remaining NT - NL slices in the
// work buffer (G[c * (NT - NL) * 16 + ...]).  Columns are padded with zero
// rows to rows_pad = 16 NT, so every lane owns NT rows and no row needs a
// bounds test (rotations keep zero rows zero).
template <int NT, int NL>
struct JacStore {
  ld2* L;
  gd2* G;
  __device__ __forceinline__ d2v ld(int c, int t, int gl) const {
    if (t < NL) return L[(c * NL + t) * JAC_G + gl];
    return G[(c * (NT - NL) + (t - NL)) * JAC_G + gl];
  }
  __device__ __forceinline__ void st(int c, int t, int gl, d2v v) const {
    if (t < NL) L[(c * NL + t) * JAC_G + gl] = v;
    else G[(c * (NT - NL) + (t - NL)) * JAC_G + gl] = v;
  }
};

template <int NT, int NL>
__device__ __forceinline__ void jac_pair(const JacStore<NT, NL>& S, int p, int q, int gl,
                                         double tol, double floor2, int* rotated) {
  d2v x[NT], y[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    x[t] = S.ld(p, t, gl);
    y[t] = S.ld(q, t, gl);
  }
  double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    a += x[t].x * x[t].x + x[t].y * x[t].y;
    b += y[t].x * y[t].x + y[t].y * y[t].y;
    gr += x[t].x * y[t].x + x[t].y * y[t].y;
    gi += x[t].x * y[t].y - x[t].y * y[t].x;
  }
  a = group16_sum(a);
  b = group16_sum(b);
  gr = group16_sum(gr);
  gi = group16_sum(gi);
  // columns at the rounding floor of the matrix are left alone (their
  // direction is noise, and their squares may be denormal)
  if (a <= floor2 || b <= floor2) return;
  // |g|^2 <= tol^2 a b: orthogonal to working precision (|g|^2, a and b are
  // above the floor, so nothing here under- or overflows)
  const double g2 = gr * gr + gi * gi;
  if (g2 == 0.0 || g2 <= (tol * tol) * (a * b)) return;
  const double rg = rsqrt_nr(g2);               // 1 / |g|
  const double zeta = (b - a) * (0.5 * rg);
  const double t1 = fma(zeta, zeta, 1.0);
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) * svt_rcp(fabs(zeta) + t1 * rsqrt_nr(t1));
  const double c = rsqrt_nr(fma(tt, tt, 1.0)), s = c * tt;
  const double er = gr * rg, ei = -gi * rg;     // e^{-i phi}
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double yr = y[t].x * er - y[t].y * ei, yi = y[t].x * ei + y[t].y * er;
    S.st(p, t, gl, d2v{c * x[t].x - s * yr, c * x[t].y - s * yi});
    S.st(q, t, gl, d2v{s * x[t].x + c * yr, s * x[t].y + c * yi});
  }
  if (gl == 0) *rotated = 1;
}

template <int NT, int NL>
__device__ __forceinline__ void jacobi_body(const JacobiDesc& d, const JacStore<NT, NL>& S,
                                            int* rotated_p, double* sig, int* order,
                                            double* fro_s) {
  constexpr int rows_pad = NT * JAC_G;
  const int rows = d.rows, cols = d.cols;
  const int tid = threadIdx.x, grp = tid / JAC_G, gl = tid % JAC_G;
  constexpr int NG = JAC_THREADS / JAC_G;
  int& rotated = *rotated_p;
  for (int e = tid; e < rows_pad * cols; e += JAC_THREADS) {
    const int c = e / rows_pad, i = e % rows_pad;
    cplx v = {0.0, 0.0};
    if (i < rows) {
      if (d.conjT) { v = d.A[(int64_t)c * d.lda + i]; v.im = -v.im; }
      else v = d.A[(int64_t)i * d.lda + c];
    }
    const int t = i / JAC_G;
    if (t < NL) S.L[(c * NL + t) * JAC_G + i % JAC_G] = d2v{v.re, v.im};
    else S.G[(c * (NT - NL) + (t - NL)) * JAC_G + i % JAC_G] = d2v{v.re, v.im};
  }
  __syncthreads();
  // squared Frobenius norm of A, summed by the lane groups
  double f2 = 0.0;
  for (int c = grp; c < cols; c += NG) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const d2v x = S.ld(c, t, gl);
      f2 += x.x * x.x + x.y * x.y;
    }
  }
  f2 = block_sum<JAC_THREADS>(f2, fro_s);
  // singular values below 1e-15 ||A||_F are rounding noise: not rotated, and
  // returned as zero columns of U
  const double floor2 = 1e-30 * f2;
  // orthogonal to working precision: |g| <= rows eps sqrt(a b), the rounding
  // level of a length-rows dot product; a stricter test is never met
  const double tol = 2.220446049250313e-16 * (rows > 16 ? rows : 16);
  const int n = cols + (cols & 1);   // round-robin needs an even count
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      for (int pi = grp; pi < n / 2; pi += NG) {
        int p, q;
        if (pi == 0) { p = r; q = n - 1; }
        else {
          p = r + pi;
          if (p >= n - 1) p -= n - 1;
          q = r - pi;
          if (q < 0) q += n - 1;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        if (q < cols) jac_pair<NT, NL>(S, p, q, gl, tol, floor2, &rotated);
      }
      __syncthreads();
    }
    const bool again = rotated != 0;
    __syncthreads();
    if (!again) break;
  }
  for (int c = grp; c < cols; c += NG) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const d2v x = S.ld(c, t, gl);
      s += x.x * x.x + x.y * x.y;
    }
    s = group16_sum(s);
    if (gl == 0) sig[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < cols; c += JAC_THREADS) {
    int rank = 0;
    const double sc = sig[c];
    for (int o = 0; o < cols; ++o)
      if (sig[o] > sc || (sig[o] == sc && o < c)) ++rank;
    order[rank] = c;
  }
  __syncthreads();
  const int keep = d.keep;
  for (int e = tid; e < rows * keep; e += JAC_THREADS) {
    const int i = e / keep, j = e % keep;
    const int c = order[j];
    const double s = sig[c];
    cplx v = {0.0, 0.0};
    if (s * s > floor2) {
      const d2v x = S.ld(c, i / JAC_G, i % JAC_G);
      v = cplx{x.x / s, x.y / s};
    }
    d.U[e] = v;
  }
  for (int j = tid; j < keep; j += JAC_THREADS) {
    const double s = sig[order[j]];
    d.sigma[j] = s * s > floor2 ? s : 0.0;
  }
}

// slices kept in LDS for an item: all of them when the padded matrix fits,
// else as many leading slices as fit (the kernels dispatch on the result)
__host__ __device__ inline int jacobi_lds_slices(int rows, int cols) {
  const int nt = (rows + JAC_G - 1) / JAC_G;
  if (nt * JAC_G * cols <= JAC_LDS_MAX) return nt;
  const int nl = JAC_LDS_MAX / (JAC_G * cols);
  return nl < nt ? nl : nt;
}

template <int NT, int NL>
__device__ __forceinline__ void jac_run(const JacobiDesc& d, ld2* L, int* rotated, double* sig,
                                        int* order, double* fro_s) {
  JacStore<NT, NL> S{L, (gd2*)d.work};
  jacobi_body<NT, NL>(d, S, rotated, sig, order, fro_s);
}

template <int NT>
__device__ __forceinline__ void jac_dispatch_nl(const JacobiDesc& d, int nl, ld2* L, int* rotated,
                                                double* sig, int* order, double* fro_s) {
  if (nl >= NT) { jac_run<NT, NT>(d, L, rotated, sig, order, fro_s); return; }
  // a partial split only occurs for rows > 96 (NT >= 7) with cols <= rows <=
  // 144, where at least 4 of the NT slices fit: JAC_LDS_MAX / (16 * 144) = 4
  if constexpr (NT >= 7) {
    switch (nl) {
      case 4: jac_run<NT, 4>(d, L, rotated, sig, order, fro_s); return;
      case 5: jac_run<NT, 5>(d, L, rotated, sig, order, fro_s); return;
      case 6: jac_run<NT, 6>(d, L, rotated, sig, order, fro_s); return;
      case 7: jac_run<NT, (NT > 7 ? 7 : 4)>(d, L, rotated, sig, order, fro_s); return;
      case 8: jac_run<NT, (NT > 8 ? 8 : 4)>(d, L, rotated, sig, order, fro_s); return;
      default: return;   // excluded by the plan compiler (cols <= rows <= 144)
    }
  }
}

// SPLIT = false: every slice in LDS; true: the leading slices in LDS and
// the rest in the work buffer (separate kernels keep the register budget of
// the common all-LDS case apart)
template <bool SPLIT>
__device__ __forceinline__ void jacobi_dispatch(const JacobiDesc& d, ld2* L, int* rotated,
                                                double* sig, int* order, double* fro_s) {
  const int nl = SPLIT ? jacobi_lds_slices(d.rows, d.cols) : 99;
  switch ((d.rows + JAC_G - 1) / JAC_G) {
    case 1: jac_dispatch_nl<1>(d, nl, L, rotated, sig, order, fro_s); break;
    case 2: jac_dispatch_nl<2>(d, nl, L, rotated, sig, order, fro_s); break;
    case 3: jac_dispatch_nl<3>(d, nl, L, rotated, sig, order, fro_s); break;
    case 4: jac_dispatch_nl<4>(d, nl, L, rotated, sig, order, fro_s); break;
    case 5: jac_dispatch_nl<5>(d, nl, L, rotated, sig, order, fro_s); break;
    case 6: jac_dispatch_nl<6>(d, nl, L, rotated, sig, order, fro_s); break;
    case 7: jac_dispatch_nl<7>(d, nl, L, rotated, sig, order, fro_s); break;
    case 8: jac_dispatch_nl<8>(d, nl, L, rotated, sig, order, fro_s); break;
    default: jac_dispatch_nl<9>(d, nl, L, rotated, sig, order, fro_s); break;
  }
}

// one workgroup per item; dynamic LDS holds the leading row slices
template <bool SPLIT>
__global__ __launch_bounds__(JAC_THREADS) void k_jacobi(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc d = descs[blockIdx.x];
  extern __shared__ d2v jlds[];   // 16-byte aligned for ds_read/write_b128
  __shared__ int rotated;
  __shared__ double sig[JAC_MAX_COLS];
  __shared__ int order[JAC_MAX_COLS];
  __shared__ double fro_s[JAC_THREADS / 64];
  jacobi_dispatch<SPLIT>(d, (ld2*)jlds, &rotated, sig, order, fro_s);
}
template __global__ void k_jacobi<false>(const JacobiDesc*);
template __global__ void k_jacobi<true>(const JacobiDesc*);

// ------------------------------------------------------------ top-k SVD
// Exact leading k singular values and left singular vectors of A (rows x
// cols, cols <= rows <= 144), for truncated splits that keep k << cols:
//   1. Householder bidiagonalisation A = Q_L B Q_R^H (left reflectors kept in
//      the working copy, right ones applied and dropped), then diagonal
//      phases making B real: B = D_L B' D_R^H with d_j, e_j >= 0;
//   2. the singular values of B' are the positive eigenvalues of the
//      Golub-Kahan tridiagonal T (zero diagonal, off-diagonal d_0, e_0,
//      d_1, ...): each of the k largest is found by multisection on Sturm
//      counts, 16 shifts per step (one per lane of a 16-lane group);
//   3. inverse iteration on T - sigma I (Gaussian elimination with partial
//      pivoting, once; tiny pivots raised to eps ||T||; then a forward and a
//      back substitution per step), eigenvectors of close values
//      re-orthogonalised; the odd entries of the eigenvector are the left
//      singular vector u of B';
//   4. U = Q_L D_L u through the stored reflectors.
// Singular values at or below 1e-15 ||A||_F give zero columns, as k_jacobi.
// Step 1 is its own kernel (k_svt_bidiag, the matrix held on chip); steps 2
// and 3 run in k_svd_top on what it leaves in the work buffer, and step 4 in
// k_svd_back (several workgroups per block).
constexpr int SVT_THREADS = 1024;
constexpr int SVT_MAXN = 144;          // rows and cols limit, as k_jacobi
constexpr int SVT_ITERS = 3;           // inverse iteration steps
constexpr int SVT_BATCH = 16;          // values per inverse-iteration batch (LDS)

// work buffer: the left reflectors (rows padded to 16, column-major), the
// bidiagonal (3 cols + 2 complex), then per value the eigenvector of T (2n
// doubles) and the complex output vector (rows)
__host__ __device__ inline int64_t svt_stride(int64_t rows, int64_t cols) {
  return 2 * cols + 2 * rows;
}

// number of eigenvalues below x of the symmetric tridiagonal T with zero
// diagonal and squared off-diagonal c2[0 .. N-2], scaled by a power of two so
// that ||T|| < 2, with c2 >= 2^-300 and x >= 2^-64 (changes far below the
// noise floor).  Sturm: the leading minors p_i of T - x I (p_0 = 1, p_1 = -x,
// p_{i+2} = -x p_{i+1} - c2[i] p_i) change sign once per eigenvalue below x.
// A step rounds as the pivot recurrence q_{i+1} = p_{i+1} / p_i does (one
// relative error on c2[i] q_i^-1 and one on the sum), without its division;
// a zero minor counts by its sign bit and the next step settles the pair.
// Every four steps both minors are scaled by the power of two that brings the
// newer one into [1/2, 1) (the older one when the newer is zero): no sign or
// rounding changes, and over four steps the magnitudes stay within 2^+-500.
__device__ __forceinline__ int svt_count(const double* c2, int N, double x) {
  double P = 1.0, Q = -x;
  int cnt = 1;
  auto step = [&](double c) {
    const double R = fma(-x, Q, -(c * P));
    cnt += int((unsigned(__double2hiint(R)) ^ unsigned(__double2hiint(Q))) >> 31);
    P = Q;
    Q = R;
  };
  auto group = [&](double a0, double a1, double a2, double a3) {
    step(a0);
    step(a1);
    step(a2);
    step(a3);
    const int e = __builtin_amdgcn_frexp_exp(Q != 0.0 ? Q : P);
    Q = ldexp(Q, -e);
    P = ldexp(P, -e);
  };
  int i = 0;
  for (const int r = (N - 1) & 3; i < r; ++i) step(c2[i]);
  for (int g = ((N - 1 - i) >> 2) & 3; g > 0; --g, i += 4) group(c2[i], c2[i + 1], c2[i + 2], c2[i + 3]);
  // blocks of 16 steps: the block's coefficients are all read first, so the
  // LDS latency is paid once per block
  for (; i < N - 1; i += 16) {
    double c[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) c[q] = c2[i + q];
    group(c[0], c[1], c[2], c[3]);
    group(c[4], c[5], c[6], c[7]);
    group(c[8], c[9], c[10], c[11]);
    group(c[12], c[13], c[14], c[15]);
  }
  return cnt;
}

// Householder reflector H = I - tau v v^H with H x = alpha e_0 for the
// vector x of norm^2 nx2 and head x0: alpha = -phase(x0) |x|, v = x - alpha
// e_0 (only the head changes); returns the head of v.  A vector with
// nx2 <= thr is left alone (tau = 0, alpha = x0): its tail is far below the
// rounding of the factorisation, and 2 / ||v||^2 could overflow.
__device__ __forceinline__ cplx svt_house(cplx x0, double nx2, double thr, double* tau,
                                          cplx* alpha) {
  const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im), nx = sqrt(nx2);
  *tau = 0.0;
  *alpha = x0;
  if (!(nx2 > thr) || !(nx > 0.0)) return x0;
  // ||v||^2 = |x0 - alpha|^2 + (nx2 - |x0|^2) = 2 nx (nx + |x0|): tau does
  // not wait for alpha
  const double r = ax0 > 0.0 ? nx / ax0 : 0.0;
  const double hv = nx * (nx + ax0);
  *tau = hv > 0.0 ? 1.0 / hv : 0.0;
  *alpha = ax0 > 0.0 ? cplx{-x0.re * r, -x0.im * r} : cplx{-nx, 0.0};
  return cplx{x0.re - alpha->re, x0.im - alpha->im};
}

// Stage 1 (k_svt_bidiag, 512 threads): the matrix stays on chip.  Thread
// (r, g) = (tid % 16, tid / 16) holds rows r + 16 a (a < 9) of five column
// slots: columns g (slot 0, in LDS: finished after 32 steps), g + 32, g + 64,
// g + 96 (slots 1-3, registers) and, for g < 16, g + 128 (slot 4, LDS until it
// moves into registers).  A column reduction is a 16-lane DPP sum; a row
// reduction sums the four 16-lane rows of a wave (lane swaps), then the 8
// waves (LDS).  Writes the left reflectors (column j, rows j.., head at row j)
// and, after them, the bidiagonal: d_j, conj(e_j), tau_j (real part) and
// ||A||_F^2.
constexpr int SVB_THREADS = 512;
__host__ __device__ inline int64_t svt_bd_off(int64_t rows, int64_t cols) {
  return (rows + 15) / 16 * 16 * cols;
}
__host__ __device__ inline int64_t svt_pv_off(int64_t rows, int64_t cols) {
  return svt_bd_off(rows, cols) + 3 * cols + 2;
}
// the unit phases D_L of the real bidiagonal (cols complex), after the
// per-value vectors
__host__ __device__ inline int64_t svt_ph_off(int64_t rows, int64_t cols, int64_t keep) {
  return svt_pv_off(rows, cols) + ((2 * cols + 2 * rows) * keep + 1) / 2;
}
constexpr int SVK_VALS = 4;     // k_svd_back: values per workgroup (one wave each)
constexpr int SVK_CH = 16;      // k_svd_back: reflectors per LDS chunk

// One block of 16 bidiagonalisation steps (steps j0 .. j0+15) after r row
// shifts, with NA = nt - r live row slots: every row-slot loop has a
// compile-time bound (the slots past the matrix are zero and skipped).
struct SvbCtx {
  gptr<cplx> W, bd;
  cplx *xl, *xa, *uL, *yR, *xs;
  double *xpr, *xpi;
  double *red, *tau_s;
  int m, n, mp, tid, lane, wave, rl, cg, q4;
  bool has4;
  double hthr;
};
constexpr int SVB_NW = SVB_THREADS / 64, SVB_NS = 5;
constexpr int SVB_NR = SVT_MAXN + 16 * 8;   // row index range of the shifted slots

template <int NA>
__device__ __forceinline__ void svb_block(cplx (&A)[9][3], const SvbCtx& c, int j0, int r) {
  constexpr int NW = SVB_NW, NS = SVB_NS, NR = SVB_NR;
  const gptr<cplx> W = c.W;
  const gptr<cplx> bd = c.bd;
  cplx* const xl = c.xl;
  cplx* const xa = c.xa;
  double* const xpr = c.xpr;
  double* const xpi = c.xpi;
  cplx* const uL = c.uL;
  cplx* const yR = c.yR;
  cplx* const xs = c.xs;
  double* const red = c.red;
  double* const tau_s = c.tau_s;
  const int m = c.m, n = c.n, mp = c.mp, tid = c.tid, lane = c.lane, wave = c.wave;
  const int rl = c.rl, cg = c.cg, q4 = c.q4;
  const bool has4 = c.has4;
  const double hthr = c.hthr;
    const int s = r >> 1;                          // 32-column blocks done
    const int t = s > 1 ? s - 1 : 0;               // register column shifts
    const int rb = rl + 16 * r;                    // row of row slot a: rb + 16 a
    // slot b: 0 = LDS columns g, 1..3 = A[.][b-1], 4 = LDS columns g + 128
    auto col = [&](int b) { return b == 0 ? cg : b < 4 ? cg + 32 * (b + t) : cg + 128; };
    auto live = [&](int b) {
      return b == 0 ? s == 0 : b < 4 ? (b + t <= 3 || (b + t == 4 && has4)) : (t == 0 && has4);
    };
    // LDS element of row slot a (index clamped in range for every lane;
    // padded row slots read 0)
    // one index form for reads and writes, so that the compiler can tell
    // the rows of a slot apart
    auto lds_idx = [&](int gmask, int a) {
      return (cg & gmask) * SVT_MAXN + (a + r < 9 ? rb + 16 * a : 0);
    };
    auto lds_at = [&](const cplx* base, int gmask, int a) -> cplx {
      cplx x = base[lds_idx(gmask, a)];
      if (a + r >= 9) x = cplx{0.0, 0.0};
      return x;
    };
    auto get = [&](int a, int b) -> cplx {
      if (b == 0) return lds_at(xl, 31, a);
      if (b == 4) return lds_at(xa, 15, a);
      cplx x = A[a][0];
      if (b == 2) x = A[a][1];
      if (b == 3) x = A[a][2];
      return x;
    };
    auto put = [&](int a, int b, cplx x) {
      if (b == 0) { if (a + r < 9) xl[lds_idx(31, a)] = x; }
      else if (b == 4) { if (a + r < 9) xa[lds_idx(15, a)] = x; }
      else if (b == 1) A[a][0] = x;
      else if (b == 2) A[a][1] = x;
      else A[a][2] = x;
    };
    const int jend = j0 + 16 < n ? j0 + 16 : n;
    for (int j = j0; j < jend; ++j) {
      const int jj = j - j0;                       // row j: row slot 0 of lane rl == jj
      const int bj = s == 0 ? 0 : 1;               // column slot of column j
      // ---- left reflector from column j (lanes cg == j % 32), rows j..m-1
      if (cg == (j & 31)) {
        double p3[3] = {0.0, 0.0, 0.0};   // three partial sums: a short chain
        cplx head = {0.0, 0.0};
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const int i = rb + 16 * a;
          cplx v = bj == 0 ? lds_at(xl, 31, a) : A[a][0];
          if (a == 0) head = v;
          if (i < j || i >= m) v = cplx{0.0, 0.0};
          uL[i] = v;
          if (i > j && i < m) W[(int64_t)j * mp + i] = v;
          p3[a % 3] = fma(v.re, v.re, fma(v.im, v.im, p3[a % 3]));
        }
        const double nx2 = group16_sum(p3[0] + p3[1] + p3[2]);
        // only the group of column j is active here: its lanes share lane & 48
        const int src = __builtin_amdgcn_readfirstlane(lane & 48) | jj;
        const cplx x0 = {readlane_d(head.re, src), readlane_d(head.im, src)};
        double tau;
        cplx alpha;
        const cplx v0 = svt_house(x0, nx2, hthr, &tau, &alpha);
        if (rl == jj) {
          uL[j] = v0;
          W[(int64_t)j * mp + j] = v0;
        }
        if (rl == 0) {
          *tau_s = tau;
          bd[j] = alpha;
          bd[2 * n + j] = cplx{tau, 0.0};
        }
      }
      __syncthreads();
      // ---- trailing columns c > j: a -= tau u (u^H a)
      const double tau = *tau_s;
      if (tau != 0.0) {
        cplx u[9];
#pragma unroll
        for (int a = 0; a < NA; ++a) u[a] = uL[rb + 16 * a];
#pragma unroll
        for (int b = 0; b < NS; ++b) {
          if (!live(b)) continue;                  // scalar
          cplx x[9];
          double wr = 0.0, wi = 0.0;
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            x[a] = get(a, b);
            wr = fma(u[a].re, x[a].re, fma(u[a].im, x[a].im, wr));
            wi = fma(u[a].re, x[a].im, fma(-u[a].im, x[a].re, wi));
          }
          wr = group16_sum(wr);
          wi = group16_sum(wi);
          const bool cl = col(b) > j;              // this lane's column is trailing
          wr = cl ? tau * wr : 0.0;
          wi = cl ? tau * wi : 0.0;
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            x[a].re = fma(-u[a].re, wr, fma(u[a].im, wi, x[a].re));
            x[a].im = fma(-u[a].re, wi, fma(-u[a].im, wr, x[a].im));
            put(a, b, x[a]);
          }
        }
      }
      if (j == n - 1) break;
      // ---- right reflector from row j (row slot 0 of lane rl == jj), columns
      // j+1..: y = conj(row j) into yR, its norm summed per wave.  The row
      // sums the right update needs, x_i = sum_c a_ic v2_c with v2_c = y_c
      // past the head, are taken here too (row j broadcast in each 16-lane
      // group); only the head term a_{i,j+1} u0 waits for the reflector, so
      // the right reflector costs one barrier less.  Column j+1 goes to xs
      // (each entry is read and then overwritten by the same thread below).
      {
        double part = 0.0;
        double xr[9], xi[9];
#pragma unroll
        for (int a = 0; a < NA; ++a) xr[a] = xi[a] = 0.0;
        const int src = (lane & 48) | jj;
#pragma unroll
        for (int b = 0; b < NS; ++b) {
          if (!live(b)) continue;                  // scalar
          const int c = col(b);
          const cplx x0 = get(0, b);
          const cplx xj = {__shfl(x0.re, src), __shfl(x0.im, src)};   // a_jc
          cplx y = {0.0, 0.0};
          if (c > j && c < n) y = cplx{xj.re, -xj.im};
          if (rl == jj) {
            yR[c] = y;
            part = fma(y.re, y.re, fma(y.im, y.im, part));
          }
          if (c == j + 1) {                        // the group holding column j+1
#pragma unroll
            for (int a = 0; a < NA; ++a) xs[rb + 16 * a] = get(a, b);
          }
          const cplx yh = c > j + 1 ? y : cplx{0.0, 0.0};
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            const cplx x = get(a, b);
            xr[a] = fma(x.re, yh.re, fma(-x.im, yh.im, xr[a]));
            xi[a] = fma(x.re, yh.im, fma(x.im, yh.re, xi[a]));
          }
        }
        part = rows4_sum(part);
        if (lane == jj) red[wave] = part;
        // sums over the wave's four 16-lane rows as a reduce-scatter: the
        // first swaps leave re(a) in rows 0-1 and im(a) in rows 2-3, the
        // second ones rows a < H in the even 16-lane rows and a >= H in the
        // odd ones (an odd NA's last row is summed in every lane)
        constexpr int H = NA / 2;
        double s1[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) s1[a] = swap32_sum(xr[a], xi[a]);
        double* const xo = (q4 >= 2 ? xpi : xpr) + wave * NR + rb;
        const int ah = (q4 & 1) ? H : 0;
#pragma unroll
        for (int i = 0; i < H; ++i) xo[16 * (i + ah)] = swap16_sum(s1[i], s1[i + H]);
        if constexpr ((NA & 1) != 0) {
          const double t = swap16_sum(s1[NA - 1], s1[NA - 1]);
          if (!(q4 & 1)) xo[16 * (NA - 1)] = t;
        }
      }
      __syncthreads();
      // the waves' partial row sums are read while the reflector is formed
      const bool xrow = tid < mp && tid > j;
      double pr = 0.0, pi = 0.0;
      cplx aj1 = {0.0, 0.0};
      if (xrow) {
        // all 17 loads are issued before the first add (under register
        // pressure the scheduler would otherwise wait on each in turn)
        double a[NW], b[NW];
        aj1 = xs[tid];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          a[w] = xpr[w * NR + tid];
          b[w] = xpi[w * NR + tid];
        }
        __builtin_amdgcn_sched_group_barrier(0x0100, 2 * NW + 1, 0);   // DS reads
        __builtin_amdgcn_sched_group_barrier(0x0002, 2 * NW - 2, 0);   // VALU adds
#pragma unroll
        for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
          for (int w = 0; w < h; ++w) {
            a[w] += a[w + h];
            b[w] += b[w + h];
          }
        pr = a[0];
        pi = b[0];
      }
      const double ny2 = group16_sum(rl < NW ? red[rl] : 0.0);
      double tau2;
      cplx beta;
      const cplx u0 = svt_house(yR[j + 1], ny2, hthr, &tau2, &beta);
      if (tid == 0) bd[n + j] = cplx{beta.re, -beta.im};
      // ---- rows i > j: a -= tau2 x_i conj(v2), x_i = partial sums + a_{i,j+1} u0
      if (tau2 != 0.0 && xrow) {
        const double sr = fma(aj1.re, u0.re, fma(-aj1.im, u0.im, pr));
        const double si = fma(aj1.re, u0.im, fma(aj1.im, u0.re, pi));
        xs[tid] = cplx{tau2 * sr, tau2 * si};
      }
      cplx v2[NS];
#pragma unroll
      for (int b = 0; b < NS; ++b) {
        const int c = col(b);
        v2[b] = cplx{0.0, 0.0};
        if (live(b) && c > j + 1) v2[b] = yR[c];
        if (c == j + 1) v2[b] = u0;
      }
      __syncthreads();
      if (tau2 != 0.0) {
        cplx x[9];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const int i = rb + 16 * a;
          x[a] = xs[i];
          if (i <= j || i >= mp) x[a] = cplx{0.0, 0.0};
        }
#pragma unroll
        for (int b = 0; b < NS; ++b) {
          if (!live(b)) continue;
          // every row of the slot is read before the first write back (the
          // LDS slots' reads and writes use different index forms, so they
          // would otherwise be kept in order, one round trip per row)
          cplx y[9];
#pragma unroll
          for (int a = 0; a < NA; ++a) y[a] = get(a, b);
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            y[a].re = fma(-x[a].re, v2[b].re, fma(-x[a].im, v2[b].im, y[a].re));   // x conj(v2)
            y[a].im = fma(-x[a].im, v2[b].re, fma(x[a].re, v2[b].im, y[a].im));
            put(a, b, y[a]);
          }
        }
      }
    }
}

__global__ __launch_bounds__(SVB_THREADS) void k_svt_bidiag(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc dsc = descs[blockIdx.x];
  const int m = dsc.rows, n = dsc.cols, k = dsc.keep;
  if (n > SVT_MAXN || m > SVT_MAXN || n > m || k > n || n < 1) return;   // excluded by the plan
  const int nt = (m + 15) / 16, mp = nt * 16;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rl = tid & 15, cg = tid >> 4, q4 = (tid >> 4) & 3;
  constexpr int NW = SVB_THREADS / 64, NS = 5;
  constexpr int NR = SVT_MAXN + 16 * 8;  // row index range of the shifted slots
  static_assert(NW == 8 && SVT_MAXN == 144, "thread layout");
  __shared__ cplx xl[32 * SVT_MAXN];     // slot 0: [g][row], column g
  __shared__ cplx xa[16 * SVT_MAXN];     // slot 4 before it moves: [g][row], column g + 128
  __shared__ double xpr[NW * NR], xpi[NW * NR];   // [wave][row]: partial row sums
  __shared__ cplx uL[NR], yR[SVT_MAXN], xs[NR];
  __shared__ double red[NW], tau_s;
  const gptr<cplx> W = to_global(dsc.work);
  const gptr<cplx> bd = W + svt_bd_off(m, n);
  const gptr<const cplx> Ain = to_global(dsc.A);
  if (tid == 0) bd[2 * n - 1] = cplx{0.0, 0.0};   // e_{n-1} does not exist
  for (int i = tid; i < NR; i += SVB_THREADS) uL[i] = xs[i] = cplx{0.0, 0.0};
  const bool has4 = wave < 4;                      // column g + 128 exists (g < 16)
  // Register slot A[a][q] (slot q + 1) holds row rl + 16 (a + r) of column
  // cg + 32 (q + 1 + t), after r row shifts and t column shifts: every 16
  // steps the finished row slot drops off the front (a zero row slot enters
  // at the back); from step 64 on, every 32 steps the finished register
  // column slot does, column g + 128 entering from LDS at the first of them.
  // So row j is always row slot 0 and, from step 32 on, column j is register
  // slot 0 (before, LDS slot 0).  Rows past the matrix stay exactly zero (their
  // u and x are zero): every pass runs all 9 row slots without a test.  A is
  // only indexed with constants, so it stays in registers.
  cplx A[9][3];
  double f = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const int i = rl + 16 * a;
#pragma unroll
    for (int b = 0; b < NS; ++b) {
      if (b == 4 && !has4) continue;
      const int c = cg + 32 * b;
      const bool ok = i < m && c < n;
      const int64_t o = !ok ? 0 : dsc.conjT ? (int64_t)c * dsc.lda + i : (int64_t)i * dsc.lda + c;
      cplx v = Ain[o];
      if (dsc.conjT) v.im = -v.im;
      if (!ok) v = cplx{0.0, 0.0};
      f += v.re * v.re + v.im * v.im;
      if (b == 0) xl[cg * SVT_MAXN + i] = v;
      else if (b < 4) A[a][b - 1] = v;
      else xa[cg * SVT_MAXN + i] = v;
    }
  }
  f = wave_sum_all(f);
  if (lane == 0) red[wave] = f;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < NW; ++w) fro2 += red[w];
  if (tid == 0) bd[3 * n] = cplx{fro2, 0.0};
  // columns and rows below 1e-100 ||A||_F get no reflector
  const double hthr = 1e-200 * fro2;
  const SvbCtx ctx{W, bd, xl, xa, uL, yR, xs, xpr, xpi, red, &tau_s, m, n, mp, tid, lane, wave,
                   rl, cg, q4, has4, hthr};
  // blocks of 16 steps with nt, nt-1, .. 1 live row slots, in sequence (a
  // loop or a switch over the templates would merge the register tile from
  // many paths); a block's templates for more slots than nt are skipped
  int j0 = 0, r = 0;
  auto block_shift = [&]() {
    // drop the finished row slot; from the block at step 64 on, every other
    // block also the finished register column slot (column g + 128 moving in
    // from LDS the first time)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
#pragma unroll
      for (int a = 0; a < 8; ++a) A[a][q] = A[a + 1][q];
      A[8][q] = cplx{0.0, 0.0};
    }
    const int s = r >> 1, s1 = (r + 1) >> 1;
    if (s1 != s && s1 >= 2) {
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        A[a][0] = A[a][1];
        A[a][1] = A[a][2];
        const int ra = a + r + 1;                    // row slot index after the row shift
        const cplx x = xa[(cg & 15) * SVT_MAXN + (ra < 9 ? rl + 16 * ra : 0)];
        A[a][2] = (s1 == 2 && has4 && ra < 9) ? x : cplx{0.0, 0.0};
      }
    }
  };
#define SVB_BLOCK(NAV)                                  \
  if (nt >= NAV && j0 < n) {                            \
    svb_block<NAV>(A, ctx, j0, r);                      \
    if (j0 + 16 < n) block_shift();                     \
    j0 += 16;                                           \
    ++r;                                                \
  }
  SVB_BLOCK(9) SVB_BLOCK(8) SVB_BLOCK(7) SVB_BLOCK(6) SVB_BLOCK(5)
  SVB_BLOCK(4) SVB_BLOCK(3) SVB_BLOCK(2) SVB_BLOCK(1)
#undef SVB_BLOCK
}

// Stages 2 and 3 on the bidiagonal written by k_svt_bidiag.
__global__ __launch_bounds__(SVT_THREADS) void k_svd_top(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc dsc = descs[blockIdx.x];
  const int m = dsc.rows, n = dsc.cols, k = dsc.keep, N = 2 * n;
  const int nt = (m + 15) / 16, mp = nt * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = SVT_THREADS / 64;
  __shared__ double tauL[SVT_MAXN];
  __shared__ cplx dcx[SVT_MAXN], ecx[SVT_MAXN], pL[SVT_MAXN];
  __shared__ double off[2 * SVT_MAXN], b2[2 * SVT_MAXN], sig[SVT_MAXN];
  __shared__ double fro2_s, bmax[NW];
  // inverse iteration: per value and step i the record (1/pivot, u1, u2, x)
  // at iib[v * pstr + 4 i]; pstr = 4 N + 2 keeps the records 16-byte aligned
  // and the 16 values' records in different LDS banks
  __shared__ __align__(16) double iib[SVT_BATCH * (4 * 2 * SVT_MAXN + 2)];
  if (n > SVT_MAXN || m > SVT_MAXN || n > m || k > n || n < 1) return;   // excluded by the plan
  const gptr<const cplx> W = to_global(dsc.work);    // reflectors, mp x n column-major
  const gptr<const cplx> bd = W + svt_bd_off(m, n);
  const gptr<double> pv = to_global(reinterpret_cast<double*>(dsc.work + svt_pv_off(m, n)));
  const gptr<cplx> Uout = to_global(dsc.U);
  const gptr<double> sgout = to_global(dsc.sigma);
  for (int j = tid; j < n; j += SVT_THREADS) {
    dcx[j] = bd[j];
    ecx[j] = bd[n + j];
    tauL[j] = bd[2 * n + j].re;
  }
  if (tid == 0) fro2_s = bd[3 * n].re;
  __syncthreads();
  // ---- real bidiagonal: B = D_L B' D_R^H.  |d_j| and |e_j| need no phases;
  // with the unit phases ph(d_j), ph(e_j) (1 for zero), the running phase is
  // p_j = ph(d_j) q_j, q_{j+1} = p_j conj(ph(e_j)), q_0 = 1
  for (int j = tid; j < n; j += SVT_THREADS) {
    const cplx d = dcx[j];
    const double ad = sqrt(d.re * d.re + d.im * d.im);
    off[2 * j] = ad;
    pL[j] = ad > 0.0 ? cplx{d.re / ad, d.im / ad} : cplx{1.0, 0.0};
    if (j < n - 1) {
      const cplx e = ecx[j];
      const double ae = sqrt(e.re * e.re + e.im * e.im);
      off[2 * j + 1] = ae;
      ecx[j] = ae > 0.0 ? cplx{e.re / ae, e.im / ae} : cplx{1.0, 0.0};
    }
  }
  __syncthreads();
  // the running phases by a scan over one wave: step j maps q_j to q_{j+1} =
  // A_j q_j + B_j with A = ph(d_j) conj(ph(e_j)), B = 0 when both are nonzero,
  // A = 0, B = conj(ph(e_j)) when d_j = 0, and A = 0, B = 1 when e_j = 0;
  // lane l composes steps 3l .. 3l+2, the lanes' maps are scanned, and each
  // lane then walks its own steps from q_{3l}
  if (wave == 0) {
    auto mul = [](cplx a, cplx b) { return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; };
    cplx A = {1.0, 0.0}, B = {0.0, 0.0};
    for (int t = 0; t < 3; ++t) {
      const int j = 3 * lane + t;
      if (j >= n - 1) break;
      const cplx pe = {ecx[j].re, -ecx[j].im};
      cplx a = {0.0, 0.0}, b = {1.0, 0.0};
      if (off[2 * j + 1] > 0.0) {
        if (off[2 * j] > 0.0) {
          a = mul(pL[j], pe);
          b = cplx{0.0, 0.0};
        } else {
          b = pe;
        }
      }
      const cplx aB = mul(a, B);
      B = cplx{aB.re + b.re, aB.im + b.im};
      A = mul(a, A);
    }
    for (int o = 1; o < 64; o <<= 1) {   // inclusive scan, later lanes applied last
      const cplx Ao = {__shfl_up(A.re, o), __shfl_up(A.im, o)};
      const cplx Bo = {__shfl_up(B.re, o), __shfl_up(B.im, o)};
      if (lane >= o) {
        const cplx aB = mul(A, Bo);
        B = cplx{aB.re + B.re, aB.im + B.im};
        A = mul(A, Ao);
      }
    }
    cplx q = {__shfl_up(A.re, 1) + __shfl_up(B.re, 1), __shfl_up(A.im, 1) + __shfl_up(B.im, 1)};
    if (lane == 0) q = cplx{1.0, 0.0};
    for (int t = 0; t < 3; ++t) {
      const int j = 3 * lane + t;
      if (j >= n) break;
      const cplx p = off[2 * j] > 0.0 ? mul(pL[j], q) : cplx{1.0, 0.0};
      pL[j] = p;
      if (j < n - 1) {
        const cplx pe = {ecx[j].re, -ecx[j].im};
        q = off[2 * j + 1] > 0.0 ? mul(p, pe) : cplx{1.0, 0.0};
      }
    }
  }
  // the Gershgorin bound max_i (off_{i-1} + off_i); then off is scaled in
  // place by the power of two 2^-bexp that brings the bound into [1, 2)
  // (exact: counts and eigenvectors are those of the unscaled matrix)
  double bl = 0.0;
  for (int i = tid; i < N; i += SVT_THREADS) {
    const double l = i > 0 ? off[i - 1] : 0.0, r = i < N - 1 ? off[i] : 0.0;
    bl = fmax(bl, l + r);
  }
  for (int o = 32; o > 0; o >>= 1) bl = fmax(bl, __shfl_xor(bl, o));
  if (lane == 0) bmax[wave] = bl;
  __syncthreads();
  double bound = 0.0;
  for (int w = 0; w < NW; ++w) bound = fmax(bound, bmax[w]);
  bound = bound * (1.0 + 1e-14) + 1e-300;
  const int bexp = ilogb(bound);
  const double bs = ldexp(bound, -bexp);
  for (int i = tid; i < N; i += SVT_THREADS) {
    const double o = i < N - 1 ? ldexp(off[i], -bexp) : 0.0;   // off[N-1] = 0 pads
    off[i] = o;
    b2[i] = fmax(o * o, 0x1p-300);
  }
  __syncthreads();
  // ---- 2. multisection: 16 shifts (lanes) per value, 4 values per wave on
  // waves 0..3 (one per SIMD: each count is a dependent chain)
  {
    const int g16 = lane >> 4, gl = lane & 15;
    for (int v0 = 0; v0 < k; v0 += 16) {
      if (wave < 4 && v0 + 4 * wave < k) {
        const int v = v0 + 4 * wave + g16;
        const int target = N - 1 - (v < k ? v : k - 1);   // ascending index of the value
        double lo = 0.0, hi = bs;
        for (int it = 0; it < 96; ++it) {
          const double x = lo + (hi - lo) * double(gl + 1) / 17.0;
          const int c = svt_count(b2, N, fmax(x, 0x1p-64));
          const unsigned long long above = __ballot(c > target);
          const unsigned ag = unsigned(above >> (16 * g16)) & 0xFFFFu;
          const int first = ag ? __ffs(ag) - 1 : 16;
          const double nlo = __shfl(x, 16 * g16 + (first > 0 ? first - 1 : 0));
          const double nhi = __shfl(x, 16 * g16 + (first < 16 ? first : 15));
          lo = first == 0 ? lo : nlo;
          hi = first == 16 ? hi : nhi;
          // a bracket of at most two ulps (its midpoint is within one ulp; one
          // ulp can exceed 2.2e-16 |x| just above a power of two, so a 1-ulp
          // test would never end there), or below 1e-18 ||T|| (values under
          // the noise floor of 1e-15 ||A||_F are returned as zero anyway)
          const bool done = (hi - lo) <= 4.5e-16 * fmax(fabs(lo), fabs(hi)) + 1e-18 * bs;
          if (__ballot(!done) == 0) break;
        }
        if (gl == 0 && v < k) sig[v] = ldexp(0.5 * (lo + hi), bexp);
      }
    }
  }
  __syncthreads();
  // ---- 3. inverse iteration on the scaled matrix, one thread per value:
  // T - sigma I = P L U by elimination with partial pivoting (once), then per
  // step a forward and a back substitution in LDS.  Wave w normalises value w
  // of the batch; a value with a close predecessor is re-orthogonalised
  // against the earlier close values in order (wave 0) and normalised there.
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * bs;
  const double ortol = 1e-3 * bound;
  const int pstr = 4 * N + 2;
  // values at or below the noise floor get zero columns: no vector is solved
  // for them (their cluster makes the solve singular)
  const double floor2 = 1e-30 * fro2_s;
  const double ctol = 1.0 / (sqrt(double(N)) * eps * bs);
  for (int v0b = 0; v0b < k; v0b += SVT_BATCH) {
    const int kb = k - v0b < SVT_BATCH ? k - v0b : SVT_BATCH;
    bool zv = true;
    double bfw = 0.0;   // the first solve's forward substitution, carried value
    if (tid < kb) {
      const int v = v0b + tid;
      double* rec = iib + (int64_t)tid * pstr;
      const double lam = sig[v];
      zv = lam * lam <= floor2;
      // deterministic start vector (golden-ratio sequence); zero for a value
      // under the floor, which then stays zero
      for (int i = 0; i < N; ++i) {
        const double fr = double(i + 1) * 0.6180339887498949 + 0.1 * v;
        rec[4 * i + 3] = zv ? 0.0 : 0.5 + (fr - floor(fr));
      }
      if (!zv) {
        // step i pivots on row i or i+1 (the larger entry in column i); record
        // i keeps 1/pivot, the pivot row's entry in column i+1 (its entry in
        // column i+2 is off[i+1] after a swap, else zero) and the multiplier,
        // whose last bit is replaced by the swap flag (a change within its
        // rounding, used in every solve)
        const double ls = ldexp(lam, -bexp);
        double di = -ls, ui = off[0], li = off[0];
        // the first solve's forward substitution runs along (same steps and
        // order as the later ones): its right side, the start vector, is
        // already in slot 3
        double bf = rec[3];
#pragma unroll 4
        for (int i = 0; i < N - 1; ++i) {
          const double un = off[i + 1];                  // zero past the end
          const double bn = rec[4 * i + 7];
          const bool sw = fabs(di) < fabs(li);
          const double p = sw ? li : di, o = sw ? di : li;
          const double r1 = sw ? -ls : ui, o1 = sw ? ui : -ls;
          const double rp = svt_rcp(fabs(p) < tiny ? (p < 0.0 ? -tiny : tiny) : p);
          const double f0 = o * rp;
          const double fct = __hiloint2double(__double2hiint(f0), (__double2loint(f0) & ~1) | int(sw));
          const double rb = sw ? bn : bf, ob = sw ? bf : bn;
          bf = ob - fct * rb;
          reinterpret_cast<d2v*>(rec + 4 * i)[0] = d2v{rp, r1};
          reinterpret_cast<d2v*>(rec + 4 * i + 2)[0] = d2v{fct, rb};
          di = o1 - fct * r1;
          ui = sw ? -fct * un : un;
          li = un;
        }
        rec[4 * (N - 1)] = svt_rcp(fabs(di) < tiny ? (di < 0.0 ? -tiny : tiny) : di);
        bfw = bf;
      }
    }
    for (int it = 0; it < SVT_ITERS; ++it) {
      // a solve from a unit right side whose solution reaches max |x_i| >=
      // 1 / (sqrt(N) eps ||T||) has a residual at the rounding level already
      // (the inverse-iteration stopping test of LAPACK's dstein, with its
      // extra step): when every value of the batch passes it on the second
      // solve, the third is skipped
      bool conv = true;
      if (tid < kb && !zv) {
        double* rec = iib + (int64_t)tid * pstr;
        // Both solves run in blocks of 8 steps: the block's records are read
        // first, the dependent chain runs in registers, the results are
        // stored last (LDS reads and writes complete in order, so a store
        // between two reads would make the wait for the later read cover it).
        // forward: the right side (slot 3) through the swaps and multipliers
        double bi = rec[3];
        auto fstep = [&](double fct, double bn) {
          const bool sw = __double2loint(fct) & 1;
          const double rb = sw ? bn : bi, ob = sw ? bi : bn;
          bi = ob - fct * rb;
          return rb;
        };
        int i = 0;
        if (it == 0) {
          bi = bfw;                                      // ran with the factorisation
        } else {
          for (const int r = (N - 1) & 7; i < r; ++i) rec[4 * i + 3] = fstep(rec[4 * i + 2], rec[4 * i + 7]);
          for (; i < N - 1; i += 8) {
            d2v fb[9];                                   // (multiplier, b) of steps i .. i+8
#pragma unroll
            for (int t = 0; t < 9; ++t) fb[t] = reinterpret_cast<const d2v*>(rec + 4 * (i + t) + 2)[0];
            double rb[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) rb[t] = fstep(fb[t][0], fb[t + 1][1]);
#pragma unroll
            for (int t = 0; t < 8; ++t) rec[4 * (i + t) + 3] = rb[t];
          }
        }
        // back substitution in place, the last two values in registers.  A
        // tiny pivot can multiply the solution by up to 1/eps: after every
        // block (at most 8 steps, far too few to overflow from 2^500) the
        // solution so far and the rest of the right side (sc) are scaled by
        // 2^-500 while the carried values exceed 2^500
        double x1 = bi * rec[4 * (N - 1)], x2 = 0.0, sc = 1.0;
        rec[4 * (N - 1) + 3] = x1;
        double mx = fabs(x1);
        auto bstep = [&](d2v a, d2v b, double o) {
          const int msk = -(__double2loint(b[0]) & 1);   // all ones after a swap
          const double r2 = __hiloint2double(__double2hiint(o) & msk, __double2loint(o) & msk);
          const double xi = (b[1] * sc - a[1] * x1 - r2 * x2) * a[0];
          x2 = x1;
          x1 = xi;
          mx = fmax(mx, fabs(xi));
          return xi;
        };
        auto rescale = [&](int i0) {     // entries i0 .. N-1 are stored
          for (int t = 0; t < 3 && (fabs(x1) > 0x1p500 || fabs(x2) > 0x1p500); ++t) {
            for (int q = i0; q < N; ++q) rec[4 * q + 3] *= 0x1p-500;
            x1 *= 0x1p-500;
            x2 *= 0x1p-500;
            sc *= 0x1p-500;
            mx *= 0x1p-500;
          }
        };
        i = N - 2;
        for (const int r = (N - 1) & 7; i > N - 2 - r; --i) {
          const d2v* ri = reinterpret_cast<const d2v*>(rec + 4 * i);
          rec[4 * i + 3] = bstep(ri[0], ri[1], off[i + 1]);
        }
        rescale(i + 1);
        for (; i >= 0; i -= 8) {
          d2v a[8], b[8];
          double o[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const d2v* ri = reinterpret_cast<const d2v*>(rec + 4 * (i - t));
            a[t] = ri[0];
            b[t] = ri[1];
            o[t] = off[i - t + 1];
          }
          double xs[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) xs[t] = bstep(a[t], b[t], o[t]);
#pragma unroll
          for (int t = 0; t < 8; ++t) rec[4 * (i - t) + 3] = xs[t];
          rescale(i - 7);
        }
        conv = sc < 1.0 || mx >= ctol;
      }
      const bool all_conv = __syncthreads_and(conv) != 0;
      if (wave < kb) {
        const int v = v0b + wave;
        bool cl = false;
        for (int u = lane; u < v; u += 64) cl |= fabs(sig[u] - sig[v]) < ortol;
        if (__ballot(cl) == 0) {
          double* x = iib + (int64_t)wave * pstr + 3;     // x_i = x[4 i]
          double s = 0.0;
          for (int i = lane; i < N; i += 64) s += x[4 * i] * x[4 * i];
          s = wave_sum_all(s);
          const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
          for (int i = lane; i < N; i += 64) x[4 * i] *= inv;
        }
      }
      __syncthreads();
      if (wave == 0) {
        for (int vb = 0; vb < kb; ++vb) {
          const int v = v0b + vb;
          bool cl = false;
          for (int u = lane; u < v; u += 64) cl |= fabs(sig[u] - sig[v]) < ortol;
          if (__ballot(cl) == 0) continue;
          double* x = iib + (int64_t)vb * pstr + 3;
          // against earlier close values (finished ones are in the work buffer)
          for (int u = 0; u < v; ++u) {
            if (fabs(sig[u] - sig[v]) >= ortol) continue;
            double s = 0.0;
            if (u >= v0b) {
              const double* y = iib + (int64_t)(u - v0b) * pstr + 3;
              for (int i = lane; i < N; i += 64) s += y[4 * i] * x[4 * i];
              s = wave_sum_all(s);
              for (int i = lane; i < N; i += 64) x[4 * i] -= s * y[4 * i];
            } else {
              const gptr<const double> y = pv + (int64_t)u * svt_stride(m, n);
              for (int i = lane; i < N; i += 64) s += y[i] * x[4 * i];
              s = wave_sum_all(s);
              for (int i = lane; i < N; i += 64) x[4 * i] -= s * y[i];
            }
          }
          double s = 0.0;
          for (int i = lane; i < N; i += 64) s += x[4 * i] * x[4 * i];
          s = wave_sum_all(s);
          const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
          for (int i = lane; i < N; i += 64) x[4 * i] *= inv;
        }
      }
      __syncthreads();
      if (it >= 1 && all_conv) break;
    }
    // keep the batch's eigenvectors in the work buffer
    for (int e = tid; e < kb * N; e += SVT_THREADS) {
      const int vb = e / N, i = e % N;
      pv[(int64_t)(v0b + vb) * svt_stride(m, n) + i] = iib[(int64_t)vb * pstr + 4 * i + 3];
    }
    __syncthreads();
  }
  // the values (zero at or below the noise floor) and the unit phases D_L
  // for k_svd_back
  const gptr<cplx> php = to_global(dsc.work + svt_ph_off(m, n, k));
  for (int v = tid; v < k; v += SVT_THREADS) sgout[v] = sig[v] * sig[v] <= floor2 ? 0.0 : sig[v];
  for (int j = tid; j < n; j += SVT_THREADS) php[j] = pL[j];
}

// Stage 4 of the top-k SVD, U = Q_L D_L u, one wave per kept value (lane r
// holds rows r + 64 t), SVK_VALS values per workgroup, so that the values of
// one block spread over several CUs.  The left reflectors pass through LDS
// in chunks of SVK_CH, double-buffered: the next chunk's global loads are in
// flight while the current chunk is applied.
__global__ __launch_bounds__(256) void k_svd_back(const JacobiDesc* __restrict__ descs) {
  const JacobiDesc dsc = descs[blockIdx.y];
  const int m = dsc.rows, n = dsc.cols, k = dsc.keep;
  if (n > SVT_MAXN || m > SVT_MAXN || n > m || k > n || n < 1) return;   // excluded by the plan
  const int v0 = blockIdx.x * SVK_VALS;
  if (v0 >= k) return;                                  // uniform: the grid covers the largest keep
  const int nt = (m + 15) / 16, mp = nt * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int v = v0 + wave;
  const bool mine = v < k;                              // wave-uniform
  const gptr<const cplx> W = to_global(dsc.work);      // reflectors, mp x n column-major
  const gptr<const cplx> bd = W + svt_bd_off(m, n);
  const gptr<const double> pv = to_global(reinterpret_cast<const double*>(dsc.work + svt_pv_off(m, n)));
  const gptr<const cplx> php = W + svt_ph_off(m, n, k);
  const gptr<cplx> Uout = to_global(dsc.U);
  const gptr<const double> sgv = to_global(dsc.sigma);
  __shared__ cplx chb[2][SVK_CH * SVT_MAXN];             // [c][row], rows 0..mp-1
  __shared__ double tau_s[SVT_MAXN];
  for (int j = tid; j < n; j += 256) tau_s[j] = bd[2 * n + j].re;
  constexpr int T = 3;                                  // rows per lane: 64 * 3 >= SVT_MAXN
  constexpr int E = SVK_CH * SVT_MAXN / 256;            // chunk elements per thread
  static_assert(E * 256 == SVK_CH * SVT_MAXN, "chunk split");
  // u = D_L z_u / ||z_u|| (the u half of the Golub-Kahan eigenvector)
  cplx uc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) uc[t] = cplx{0.0, 0.0};
  if (mine) {
    const gptr<const double> z = pv + (int64_t)v * svt_stride(m, n);
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = lane + 64 * t;
      if (i < n) s += z[2 * i + 1] * z[2 * i + 1];
    }
    s = wave_sum_all(s);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    if (sgv[v] != 0.0) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int i = lane + 64 * t;
        if (i < n) {
          const cplx ph = php[i];
          const double x = z[2 * i + 1] * inv;
          uc[t] = cplx{ph.re * x, ph.im * x};
        }
      }
    }
  }
  // reflectors j0 .. j0 + SVK_CH - 1 (those below 0 or at n and above are
  // zero), element e = c mp + i of the chunk
  cplx nx[E];
  auto fetch = [&](int j0) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int e = tid + 256 * q;
      const int c = e / mp, i = e - c * mp, j = j0 + c;
      const bool ok = c < SVK_CH && j >= 0 && j < n && i >= j && i < m;
      nx[q] = ok ? cplx(W[(int64_t)j * mp + i]) : cplx{0.0, 0.0};
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int e = tid + 256 * q;
      if (e < SVK_CH * mp) chb[b][e] = nx[q];
    }
  };
  const int nch = (n + SVK_CH - 1) / SVK_CH;
  int j0 = n - SVK_CH;                                  // the last chunk first
  fetch(j0);
  put(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c, j0 -= SVK_CH) {
    const int b = c & 1;
    if (c + 1 < nch) fetch(j0 - SVK_CH);                // in flight while this chunk is applied
    if (mine) {
      const int jlo = j0 > 0 ? j0 : 0;
      for (int j = j0 + SVK_CH - 1; j >= jlo; --j) {
        const double tau = tau_s[j];                    // tau = 0 leaves uc exactly as it is
        const cplx* const a0 = &chb[b][(j - j0) * mp];
        cplx a[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int i = lane + 64 * t;                  // rows past mp read zero
          a[t] = a0[i < mp ? i : 0];
          if (i >= mp) a[t] = cplx{0.0, 0.0};
        }
        double wr = 0.0, wi = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          wr = fma(a[t].re, uc[t].re, fma(a[t].im, uc[t].im, wr));
          wi = fma(a[t].re, uc[t].im, fma(-a[t].im, uc[t].re, wi));
        }
        wr = tau * wave_sum_all(wr);
        wi = tau * wave_sum_all(wi);
#pragma unroll
        for (int t = 0; t < T; ++t) {
          uc[t].re = fma(-a[t].re, wr, fma(a[t].im, wi, uc[t].re));
          uc[t].im = fma(-a[t].re, wi, fma(-a[t].im, wr, uc[t].im));
        }
      }
    }
    if (c + 1 < nch) put(b ^ 1);                        // read by every wave after the barrier
    __syncthreads();
  }
  if (!mine) return;
  // column gauge (when asked): the entry of largest modulus, the first row
  // on ties, made real and positive.  |u_i|^2 is the rounded sum of the
  // rounded squares, so that ties fall as in a plain evaluation
  if (dsc.gauge) {
    double best = -1.0;
    int bi = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = lane + 64 * t;
      double q;
      {
#pragma clang fp contract(off)
        q = uc[t].re * uc[t].re + uc[t].im * uc[t].im;
      }
      if (i < m && q > best) {
        best = q;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    cplx x = uc[0];
#pragma unroll
    for (int t = 1; t < T; ++t)
      if (t == (bi >> 6)) x = uc[t];
    x = cplx{__shfl(x.re, bi & 63), __shfl(x.im, bi & 63)};
    const double a = sqrt(x.re * x.re + x.im * x.im);
    if (a > 0.0) {
      const cplx ph = {x.re / a, x.im / a};
#pragma unroll
      for (int t = 0; t < T; ++t)
        uc[t] = cplx{uc[t].re * ph.re + uc[t].im * ph.im, uc[t].im * ph.re - uc[t].re * ph.im};
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int i = lane + 64 * t;
    if (i < m) Uout[(int64_t)i * k + v] = uc[t];
  }
}


__global__ __launch_bounds__(256) void k_colphase(const ColPhaseDesc* __restrict__ descs) {
  const ColPhaseDesc d = descs[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // four columns per workgroup (one per wave), column groups over blockIdx.y
  for (int j = blockIdx.y * 4 + wave; j < d.keep; j += 4 * gridDim.y) {
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

// C = alpha * sum_s P_s (see SumDesc); grid (element blocks, items).  The
// partials are loaded SUM_BATCH at a time, all in flight together, and added
// in order s = 0, 1, ... (a loop of single loads would wait out one memory
// round trip per partial).
constexpr int SUM_BATCH = 8;
__global__ __launch_bounds__(256) void k_sum_parts(const SumDesc* __restrict__ descs) {
  const SumDesc d = descs[blockIdx.y];
  const int64_t mn = (int64_t)d.M * d.N;
  const gptr<const cplx> P = to_global(d.P);
  const gptr<cplx> C = to_global(d.C);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mn; e += (int64_t)gridDim.x * 256) {
    double r = 0.0, i = 0.0;
    for (int s0 = 0; s0 < d.S; s0 += SUM_BATCH) {
      cplx v[SUM_BATCH];
#pragma unroll
      for (int t = 0; t < SUM_BATCH; ++t)   // past S: partial 0 again, not added
        v[t] = P[(s0 + t < d.S ? s0 + t : 0) * mn + e];
      __builtin_amdgcn_sched_barrier(0);   // keep the batch's loads ahead of its adds
#pragma unroll
      for (int t = 0; t < SUM_BATCH; ++t)
        if (s0 + t < d.S) {
          r += v[t].re;
          i += v[t].im;
        }
    }
    const int64_t row = e / d.N, col = e - row * d.N;
    C[row * d.ldc + col] = cplx{d.alpha.re * r - d.alpha.im * i, d.alpha.re * i + d.alpha.im * r};
  }
}

// chunk c of an item covers elements [c * step, min(len, (c + 1) * step)),
// step a multiple of 256 (blockIdx.x: chunk, blockIdx.y: item)
__device__ __forceinline__ int64_t norm_step(int64_t len) {
  return ((len + NORM_CHUNKS - 1) / NORM_CHUNKS + 255) / 256 * 256;
}

__global__ __launch_bounds__(256) void k_norm_partial(const NormDesc* __restrict__ descs) {
  const NormDesc d = descs[blockIdx.y];
  __shared__ double sh[8];
  const int64_t step = norm_step(d.len), lo = blockIdx.x * step;
  const int64_t hi = lo + step < d.len ? lo + step : d.len;
  const gptr<const cplx> x = to_global((const cplx*)d.x);
  double part = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
    const cplx v = x[e];
    part += v.re * v.re + v.im * v.im;
  }
  part = block_sum<256>(part, sh);
  if (threadIdx.x == 0) d.part[blockIdx.x] = part;
}

__global__ __launch_bounds__(256) void k_norm_apply(const NormDesc* __restrict__ descs) {
  const NormDesc d = descs[blockIdx.y];
  double t = 0.0;
  for (int c = 0; c < NORM_CHUNKS; ++c) t += d.part[c];   // same order in every chunk
  const double nrm = sqrt(t), inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  const int64_t step = norm_step(d.len), lo = blockIdx.x * step;
  const int64_t hi = lo + step < d.len ? lo + step : d.len;
  const gptr<cplx> x = to_global(d.x);
  for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
    const cplx v = x[e];
    x[e] = cplx{v.re * inv, v.im * inv};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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

// <O_k> = Tr(rho O_k) / Tr(rho) for bond sel[b] (rho_mat holds 16 complex
// per bond, [(p_i p_j), (p_i' p_j')]; O_k row-major in the (p_i p_j) basis),
// one thread per (bond, operator), out[b * nops + k]
__global__ void k_rho_ops(const cplx* __restrict__ rho_mat, const int32_t* __restrict__ sel,
                          int nsel, const cplx* __restrict__ ops, int nops, cplx* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsel * nops) return;
  const int b = t / nops, k = t - b * nops;
  const cplx* r = rho_mat + 16 * sel[b];
  const cplx* o = ops + 16 * k;
  double tr = 0.0, ti = 0.0, sr = 0.0, si = 0.0;
  for (int a = 0; a < 4; ++a) {
    tr += r[a * 4 + a].re;
    ti += r[a * 4 + a].im;
    for (int c = 0; c < 4; ++c) {
      const cplx x = r[a * 4 + c], y = o[c * 4 + a];
      sr += x.re * y.re - x.im * y.im;
      si += x.re * y.im + x.im * y.re;
    }
  }
  const double den = tr * tr + ti * ti;
  out[t] = cplx{(sr * tr + si * ti) / den, (si * tr - sr * ti) / den};
}

// ------------------------------------------------- two-site rho measures
// Eigenvalues (and with V, eigenvectors as columns) of a 4 x 4 Hermitian
// matrix by cyclic complex Jacobi rotations: for the pair (p, q) with
// A_pq = |a| e^{i phi}, the rotation G = diag(1, e^{-i phi}) [[c, s], [-s, c]]
// (on rows/columns p, q) makes G^H A G real symmetric in that pair and zeroes
// it; sweeps stop when the off-diagonal part is below 1e-30 of the
// Frobenius norm squared.
__device__ void herm_eig4(cplx A[4][4], double w[4], cplx V[4][4], bool vecs) {
  if (vecs)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) V[i][j] = cplx{i == j ? 1.0 : 0.0, 0.0};
  double fro = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) fro += A[i][j].re * A[i][j].re + A[i][j].im * A[i][j].im;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (i != j) off += A[i][j].re * A[i][j].re + A[i][j].im * A[i][j].im;
    if (!(off > 1e-30 * fro)) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        const double ab = sqrt(A[p][q].re * A[p][q].re + A[p][q].im * A[p][q].im);
        if (!(ab > 0.0)) continue;
        const cplx e = cplx{A[p][q].re / ab, A[p][q].im / ab};   // e^{i phi}
        const double tau = (A[q][q].re - A[p][p].re) / (2.0 * ab);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        // G = [[c, s], [-s conj(e), c conj(e)]] on (p, q): columns A <- A G
        for (int k = 0; k < 4; ++k) {
          const cplx ap = A[k][p], aq = A[k][q];
          // aq * conj(e)
          const cplx qe = cplx{aq.re * e.re + aq.im * e.im, aq.im * e.re - aq.re * e.im};
          A[k][p] = cplx{c * ap.re - sn * qe.re, c * ap.im - sn * qe.im};
          A[k][q] = cplx{sn * ap.re + c * qe.re, sn * ap.im + c * qe.im};
          if (vecs) {
            const cplx vp = V[k][p], vq = V[k][q];
            const cplx ve = cplx{vq.re * e.re + vq.im * e.im, vq.im * e.re - vq.re * e.im};
            V[k][p] = cplx{c * vp.re - sn * ve.re, c * vp.im - sn * ve.im};
            V[k][q] = cplx{sn * vp.re + c * ve.re, sn * vp.im + c * ve.im};
          }
        }
        // rows A <- G^H A: row p = c A_p - s e A_q, row q = s A_p + c e A_q
        for (int k = 0; k < 4; ++k) {
          const cplx ap = A[p][k], aq = A[q][k];
          const cplx qe = cplx{aq.re * e.re - aq.im * e.im, aq.im * e.re + aq.re * e.im};
          A[p][k] = cplx{c * ap.re - sn * qe.re, c * ap.im - sn * qe.im};
          A[q][k] = cplx{sn * ap.re + c * qe.re, sn * ap.im + c * qe.im};
        }
        A[p][q] = cplx{0.0, 0.0};
        A[q][p] = cplx{0.0, 0.0};
        A[p][p].im = 0.0;
        A[q][q].im = 0.0;
      }
  }
  for (int i = 0; i < 4; ++i) w[i] = A[i][i].re;
}

// rho / Tr rho, Hermitian part, from 16 complex values [(p_i p_j), (p_i' p_j')]
__device__ void unit_hermitian4(const cplx* r, cplx X[4][4]) {
  double tr = 0.0, ti = 0.0;
  for (int a = 0; a < 4; ++a) {
    tr += r[a * 4 + a].re;
    ti += r[a * 4 + a].im;
  }
  const double den = tr * tr + ti * ti;
  cplx Y[4][4];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) {
      const cplx x = r[a * 4 + c];
      Y[a][c] = cplx{(x.re * tr + x.im * ti) / den, (x.im * tr - x.re * ti) / den};
    }
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c)
      X[a][c] = cplx{0.5 * (Y[a][c].re + Y[c][a].re), 0.5 * (Y[a][c].im - Y[c][a].im)};
}

// Per selected bond b (one thread each): out[2 b] = negativity of
// rho_mat[sel[b]] (Eq. res:negativity, partial transpose on the second
// site), out[2 b + 1] = fidelity with sigma[b] (Eq. metrics:fidelity; NaN
// without sigma).  Both matrices are normalised to unit trace and taken
// Hermitian; negative eigenvalues (rounding) count as zero under the square
// roots.
__global__ void k_rho_measures(const cplx* __restrict__ rho_mat, const int32_t* __restrict__ sel,
                               int nsel, const cplx* __restrict__ sigma, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nsel) return;
  cplx X[4][4], P[4][4], V[4][4];
  double w[4];
  unit_hermitian4(rho_mat + 16 * sel[b], X);
  // partial transpose on the second site: (a b),(c d) <- (a d),(c b)
  for (int a = 0; a < 2; ++a)
    for (int bb = 0; bb < 2; ++bb)
      for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) P[a * 2 + bb][c * 2 + d] = X[a * 2 + d][c * 2 + bb];
  herm_eig4(P, w, V, false);
  out[2 * b] = 0.5 * (fabs(w[0]) + fabs(w[1]) + fabs(w[2]) + fabs(w[3]) - 1.0);
  if (!sigma) {
    out[2 * b + 1] = NAN;
    return;
  }
  // sqrt(rho) = V diag(sqrt(max(w, 0))) V^H
  herm_eig4(X, w, V, true);
  cplx S[4][4], Sg[4][4], M[4][4], T[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 4; ++k) {
        const double sq = sqrt(fmax(w[k], 0.0));
        // V[i][k] sq conj(V[j][k])
        re += sq * (V[i][k].re * V[j][k].re + V[i][k].im * V[j][k].im);
        im += sq * (V[i][k].im * V[j][k].re - V[i][k].re * V[j][k].im);
      }
      S[i][j] = cplx{re, im};
    }
  unit_hermitian4(sigma + 16 * b, Sg);
  for (int i = 0; i < 4; ++i)   // T = S Sg
    for (int j = 0; j < 4; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 4; ++k) {
        re += S[i][k].re * Sg[k][j].re - S[i][k].im * Sg[k][j].im;
        im += S[i][k].re * Sg[k][j].im + S[i][k].im * Sg[k][j].re;
      }
      T[i][j] = cplx{re, im};
    }
  for (int i = 0; i < 4; ++i)   // M = T S
    for (int j = 0; j < 4; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 4; ++k) {
        re += T[i][k].re * S[k][j].re - T[i][k].im * S[k][j].im;
        im += T[i][k].re * S[k][j].im + T[i][k].im * S[k][j].re;
      }
      M[i][j] = cplx{re, im};
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j <= i; ++j) {
      const cplx h = cplx{0.5 * (M[i][j].re + M[j][i].re), 0.5 * (M[i][j].im - M[j][i].im)};
      M[i][j] = h;
      M[j][i] = cplx{h.re, -h.im};
    }
  herm_eig4(M, w, V, false);
  const double f = sqrt(fmax(w[0], 0.0)) + sqrt(fmax(w[1], 0.0)) + sqrt(fmax(w[2], 0.0)) +
                   sqrt(fmax(w[3], 0.0));
  out[2 * b + 1] = f * f;
}
}  // namespace pn
