// Blocked Householder QR for gfx950.
//
// Panel factorization: shifted Cholesky QR with three passes (Fukaya,
// Nakatsukasa, Yanagisawa, Yamamoto 2020) carried out in FP64 arithmetic,
// followed by Householder reconstruction (Ballard, Demmel, Grigori, Jacquelin,
// Knight, Nguyen 2015): the orthonormal panel basis Q1 is turned into unit
// lower trapezoidal Householder vectors Y and the compact-WY triangle T with
// Q1 S = (I - Y T Y^T)[I; 0], S = diag(+-1).  Every step of the panel is a
// row-parallel pass or a 64 x 64 problem in one work-group; nothing waits on
// a reduction over the full column per Householder vector.
//
// Trailing updates C <- (I - Y T Y^T)^T C = C - (Y T^T)(Y^T C) are two MFMA
// GEMMs: W = Y^T C (split over rows, reduced deterministically) and
// C -= Yhat W with Yhat = Y T^T.  MFMA inputs are rounded to the factorization
// precision (fp32, bf16, fp16 or fp64); accumulation is fp32 (fp64 for fp64).
//
// The reflectors are the same as those of a Householder QR (Section 4.1,
// assumption on xGEQRF); the application of the orthogonal factor to vectors
// (xORMQR on a vector) applies the panels' block reflectors in sequence.
#include <hip/hip_fp8.h>

#include "engine.hpp"
#include "wg64.hpp"

namespace lsq {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

// ---------------------------------------------------------------------------
// Gram accumulation: G (upper triangle, column-major ld 64) += tile^T tile for
// the 64 x 64 FP64 LDS tile (columns >= jb are zero).  FP64 MFMA, then FP64
// atomics from the upper quadrants into copy (row tile mod copies) of G; the
// readers sum the copies in order.  One copy measured fastest on the
// 4096-row panels (more divide the atomic contention but multiply the
// readers' traffic).  The deterministic mode gives every row tile a copy of
// its own: each copy then receives one sum, and the readers' fixed order makes
// the Gram independent of the order in which the work-groups finish.
// ---------------------------------------------------------------------------
template <int NW>
__device__ __forceinline__ void gram_atomic(const double* tile, int jb, double* __restrict__ Gbase, int copies) {
  constexpr int BR = 8 / NW;
  double* __restrict__ G = Gbase + (size_t)(blockIdx.x % copies) * 4096;
  f64x4 acc[BR][2];
  mm64_acc<NW>(tile, true, tile, acc);
  const int w = threadIdx.x >> 6;
  if (16 * BR * (w >> 1) >= 32 * (w & 1) + 32) return;   // the wave's block lies below the diagonal
#pragma unroll
  for (int bi = 0; bi < BR; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mm64_row<NW>(bi, r), j = mm64_col<NW>(bj);
        if (i <= j && j < jb) atomicAdd(&G[i + j * 64], acc[bi][bj][r]);
      }
}

// The 64 x 64 panel problems run on work-groups of kPW waves.
constexpr int kPW = 8;
constexpr int kPT = 64 * kPW;
constexpr int kPR = 64 / kPW;   // register rows per thread

// Gram of the first panel: G += X^T X over 64-row tiles.  Later panels get
// theirs from the trailing update that produces them (k_wy_u).
template <typename Tin>
__global__ __launch_bounds__(kPT) void k_panel_gram(const Tin* __restrict__ X, int ldx, int mr,
                                                    int jb, double* __restrict__ G, int copies) {
  __shared__ double tile[64 * kLdt];
  LSQ_LDS_POISON(tile);
  const int rb = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += kPT) {
    const int i = e & 63, j = e >> 6;
    tile[i * kLdt + j] = (rb + i < mr && j < jb) ? (double)X[(size_t)(rb + i) + (size_t)j * ldx] : 0.0;
  }
  __syncthreads();
  gram_atomic<kPW>(tile, jb, G, copies);
}

// Loads the Gram accumulated in Gin as a symmetric LDS matrix, adds the
// shift of shifted Cholesky QR when asked and pads it with the identity
// beyond jb.  sigma = 11 (mr jb + jb (jb + 1)) u tr(G).
__device__ __forceinline__ void load_gram(const double* Gin, int copies, int jb, int mr, int shift, double* S,
                                          double* red) {
  for (int e = threadIdx.x; e < 4096; e += kPT) {
    const int i = e & 63, j = e >> 6;
    const int src = (i <= j) ? i + j * 64 : j + i * 64;
    double v = 0.0;
    for (int c = 0; c < copies; ++c) v += Gin[(size_t)c * 4096 + src];
    S[i * kLdt + j] = v;
  }
  __syncthreads();
  if (shift) {
    double tr = 0.0;
    for (int i = threadIdx.x; i < jb; i += kPT) tr += S[i * kLdt + i];
    tr = block_sum(tr, red);
    const double sigma = 11.0 * ((double)mr * jb + (double)jb * (jb + 1)) * kU64 * tr;
    if (threadIdx.x < jb) S[threadIdx.x * kLdt + threadIdx.x] += sigma;
    __syncthreads();
  }
  pad_identity<kPW>(S, jb);
}

// One Cholesky QR pass on a 64-row tile per work-group: R = chol(G (+ shift)),
// Xout = X R^{-1}, Gout += Xout^T Xout.  Every work-group factors G itself (a
// 64 x 64 problem, identical in all of them); work-group 0 also accumulates
// Racc <- R Racc (Racc <- R when first).
template <typename Tin>
__global__ __launch_bounds__(kPT) void k_panel_cholpass(
    const double* __restrict__ Gin, int shift, int first, double* __restrict__ Racc,
    int* __restrict__ status, const Tin* __restrict__ X, int ldx, int mr, int jb,
    double* __restrict__ Xout, int ldo, double* __restrict__ Gout, int copies) {
  __shared__ double S0[64 * kLdt];
  __shared__ double S1[64 * kLdt];
  __shared__ double S2[64 * kLdt];
  __shared__ double buf[512];
  __shared__ double red[kPW];
  LSQ_LDS_POISON(S0);
  LSQ_LDS_POISON(S1);
  LSQ_LDS_POISON(S2);
  LSQ_LDS_POISON(buf);
  LSQ_LDS_POISON(red);
  const int t = threadIdx.x;
  load_gram(Gin, copies, jb, mr, shift, S0, red);
  double x[kPR], z[kPR];
  regs_load<kPW>(S0, x);
  const bool ok = reg_cholesky_inv<kPW>(x, z, buf);
  if (!ok && blockIdx.x == 0 && t == 0) atomicOr(status, 1);
  regs_store_t<kPW>(S1, z, jb);                      // S1 = R^{-1} (zero outside jb x jb)
  __syncthreads();
  if (blockIdx.x == 0) {
    regs_store<kPW>(S0, x);                          // S0 = R
    if (first) {
      wg_store64<kPW>(S0, Racc);
    } else {
      __syncthreads();
      wg_load64<kPW>(Racc, S2);
      wg_matmul<kPW>(S0, S2, S2);
      wg_store64<kPW>(S2, Racc);
    }
  }
  const int rb = blockIdx.x * 64;
  for (int e = t; e < 64 * 64; e += kPT) {
    const int i = e & 63, j = e >> 6;
    S0[i * kLdt + j] = (rb + i < mr && j < jb) ? (double)X[(size_t)(rb + i) + (size_t)j * ldx] : 0.0;
  }
  __syncthreads();
  wg_matmul<kPW>(S0, S1, S0);
  for (int e = t; e < 64 * 64; e += kPT) {
    const int i = e & 63, j = e >> 6;
    if (rb + i < mr && j < jb) Xout[(size_t)(rb + i) + (size_t)j * ldo] = S0[i * kLdt + j];
  }
  gram_atomic<kPW>(S0, jb, Gout, copies);
}

// Last Cholesky QR pass fused with the Householder reconstruction and the
// Householder vectors of the work-group's 64-row tile.
//
// With R2 = chol(Q1^T Q1), the orthonormal basis is Q2 = Q1 R2^{-1}.  The
// modified LU without pivoting Q2top - S = L1 U (S = diag(-sign of the pivot))
// gives the vectors Y = [L1; Q2bot U^{-1}], T = -U S L1^{-T} and R = S R_total
// with R_total = R2 Racc.  One right-looking 64-step loop produces L1, U,
// V = U^{-T} and W = L1^{-1} together (row k of U and column k of L1 are final
// at step k, which is all the two forward substitutions need), so that
// Mmat = R2^{-1} V^T and T = -U S W^T are plain products.  Every work-group
// computes the 64 x 64 part (identically); work-group 0 writes R, L1, T and
// Racc, and each work-group writes Y = Q1 Mmat and Yhat = Y T^T of its rows.
template <typename Tw, typename Acc>
__global__ __launch_bounds__(kPT) void k_panel_final_y(
    const double* __restrict__ Gin, int jb, int mr,
    const double* __restrict__ Q1, int ldq,           // FP64 panel basis before the last pass
    double* __restrict__ Racc, Tw* __restrict__ Mst, int ldm, int j0,
    Tw* __restrict__ Tout, Tw* __restrict__ Yhat, int ldy, int* __restrict__ status,
    const Tw* __restrict__ Cn, int ncn, Acc* __restrict__ Wpart, int copies) {
  __shared__ double A0[64 * kLdt];     // U rows (published step by step), then -U S, then T
  __shared__ double A1[64 * kLdt];     // R2^{-1}, then W^T, then the Y tile
  __shared__ double A2[64 * kLdt];     // scratch, V^T -> Mmat, then T^T
  __shared__ double A3[64 * kLdt];     // L1 (strictly lower, zero elsewhere)
  __shared__ double buf[512];
  __shared__ double cbuf[128];
  __shared__ double sgn[64];
  __shared__ double red[kPW];
  LSQ_LDS_POISON(A0);
  LSQ_LDS_POISON(A1);
  LSQ_LDS_POISON(A2);
  LSQ_LDS_POISON(A3);
  LSQ_LDS_POISON(buf);
  LSQ_LDS_POISON(cbuf);
  LSQ_LDS_POISON(sgn);
  LSQ_LDS_POISON(red);
  const int t = threadIdx.x;
  const Own<kPW> o;
  double x[kPR], v[kPR], w[kPR];
  // R2 and R2^{-1}
  load_gram(Gin, copies, jb, mr, 0, A0, red);
  regs_load<kPW>(A0, x);
  {
    double z[kPR];
    if (!reg_cholesky_inv<kPW>(x, z, buf) && blockIdx.x == 0 && t == 0) atomicOr(status, 1);
    __syncthreads();
    regs_store<kPW>(A0, x);                                 // A0 = R2
    regs_store_t<kPW>(A1, z);                               // A1 = R2^{-1}
  }
  if (blockIdx.x == 0) {                               // Racc <- R2 Racc (A2 as scratch)
    __syncthreads();
    wg_load64<kPW>(Racc, A2);
    wg_matmul<kPW>(A0, A2, A2);
    wg_store64<kPW>(A2, Racc);
  }
  // A2 = Q2top = Q1top R2^{-1} (zero outside jb x jb), identity-padded
  for (int e = t; e < 4096; e += kPT) {
    const int i = e & 63, j = e >> 6;
    A2[i * kLdt + j] = (i < jb && j < jb) ? Q1[i + (size_t)j * ldq] : 0.0;
  }
  __syncthreads();
  wg_matmul<kPW>(A2, A1, A2);
  pad_identity<kPW>(A2, jb);
  regs_load<kPW>(A2, x);
#pragma unroll
  for (int qq = 0; qq < kPR; ++qq) {
    v[qq] = (o.r0 + qq == o.c) ? 1.0 : 0.0;
    w[qq] = v[qq];
  }
  // Modified LU of Q2top - S with V = U^{-T} and W = L1^{-1}.  Row k of U is
  // published (zero left of the diagonal) into row k of A0 and then cleared in
  // the registers, so the column published next holds zeros above the diagonal
  // and the updates need no masks; rows k of V and W are restored by their
  // owner after the update.
  for (int wk = 0; wk < kPW; ++wk)
#pragma unroll
  for (int q = 0; q < kPR; ++q) {
    const int k = kPR * wk + q;
    double* rk = A0 + k * kLdt;                        // row k of U
    double* cb = cbuf + (q & 1) * 64;                  // column k of the active matrix
    double* rv = buf + (q & 1) * 128;                  // row k of V (unscaled)
    double* rw = rv + 64;                              // row k of W
    if (o.w == wk) {
      rk[o.c] = (o.c >= k) ? x[q] : 0.0;
      rv[o.c] = v[q];
      rw[o.c] = w[q];
    }
    if (o.c == k) {
#pragma unroll
      for (int qq = 0; qq < kPR; ++qq) cb[o.r0 + qq] = x[qq];
    }
    __syncthreads();
    const double dkk = rk[k];
    const double sg = dkk >= 0.0 ? -1.0 : 1.0;
    const double piv = dkk - sg, ip = rcp64(piv);
    const double uk2 = rk[o.c] * ip;
    const double vkc = rv[o.c] * ip;
    const double wkc = rw[o.c];
    const double wk2 = wkc * ip;
#pragma unroll
    for (int qq = 0; qq < kPR; ++qq) {
      const double cik = cb[o.r0 + qq];                // L1[i][k] * piv below the diagonal
      x[qq] = fma(-cik, uk2, x[qq]);
      v[qq] = fma(-rk[o.r0 + qq], vkc, v[qq]);
      w[qq] = fma(-cik, wk2, w[qq]);
    }
    if (o.w == wk) {
      x[q] = 0.0;
      v[q] = vkc;
      w[q] = wkc;
    }
    if (o.w == 0) A3[o.c * kLdt + k] = (o.c > k) ? cb[o.c] * ip : 0.0;
    if (t == 0) sgn[k] = sg;
  }
  __syncthreads();
  // Mmat = R2^{-1} V^T -> A2
  regs_store_t<kPW>(A2, v);
  __syncthreads();
  wg_matmul<kPW>(A1, A2, A2);
  // T = -U S W^T -> A0 (U has the modified pivots dkk - sg on its diagonal)
  regs_store_t<kPW>(A1, w);
#pragma unroll
  for (int qq = 0; qq < kPR; ++qq) {
    const int i = o.r0 + qq;
    const double u = A0[i * kLdt + o.c];
    const double uv = (i == o.c) ? u - sgn[i] : u;
    A0[i * kLdt + o.c] = -uv * sgn[o.c];
  }
  __syncthreads();
  wg_matmul<kPW>(A0, A1, A0);
  // T rounded to the storage precision (the same values Yhat and the stored T use)
  for (int e = t; e < 4096; e += kPT) {
    const int i = e & 63, j = e >> 6;
    const double tv = (i <= j && i < jb && j < jb) ? (double)(Tw)A0[i * kLdt + j] : 0.0;
    A0[i * kLdt + j] = tv;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = t; e < 4096; e += kPT) Tout[e] = (Tw)A0[(e & 63) * kLdt + (e >> 6)];
    // R = S R_total and the strictly lower L1 into the factor storage
    __threadfence();
    __syncthreads();
    for (int e = t; e < 4096; e += kPT) {
      const int i = e & 63, j = e >> 6;
      if (i < jb && j < jb) {
        const double rv = (i <= j) ? sgn[i] * Racc[i + j * 64] : A3[i * kLdt + j];
        Mst[(size_t)(j0 + i) + (size_t)(j0 + j) * ldm] = (Tw)rv;
      }
    }
  }
  // this tile's Householder vectors: rows >= jb from Q1 Mmat, rows < jb from L1
  const int rb = blockIdx.x * 64;
  for (int e = t; e < 4096; e += kPT) {
    const int i = e & 63, j = e >> 6;
    A1[i * kLdt + j] = (rb + i < mr && rb + i >= jb && j < jb) ? Q1[(size_t)(rb + i) + (size_t)j * ldq] : 0.0;
  }
  __syncthreads();
  wg_matmul<kPW>(A1, A2, A1);
  for (int e = t; e < 4096; e += kPT) {
    const int i = e & 63, j = e >> 6, row = rb + i;
    double y = (double)(Tw)A1[i * kLdt + j];
    if (row < jb) y = (row > j) ? (double)(Tw)A3[row * kLdt + j] : (row == j ? 1.0 : 0.0);
    if (row >= mr || j >= jb) y = 0.0;
    A1[i * kLdt + j] = y;
    if (row >= jb && row < mr && j < jb) Mst[(size_t)(j0 + row) + (size_t)(j0 + j) * ldm] = (Tw)y;
    A2[j * kLdt + i] = A0[i * kLdt + j];               // A2 = T^T (Mmat no longer needed)
  }
  __syncthreads();
  if (Wpart) {
    // look-ahead: this tile's share of W = Y^T C for the next ncn columns
    // (C = Cn, rows of the panel), reduced over the tiles by k_wy_reduce
    for (int e = t; e < 4096; e += kPT) {
      const int i = e & 63, c = e >> 6;
      A3[i * kLdt + c] = (rb + i < mr && c < ncn) ? (double)Cn[(size_t)(rb + i) + (size_t)c * ldm] : 0.0;
    }
    __syncthreads();
    wg_matmul<kPW>(A1, A3, A0, true);
    for (int e = t; e < 64 * ncn; e += kPT)
      Wpart[(size_t)blockIdx.x * 64 * ncn + e] = (Acc)A0[(e & 63) * kLdt + (e >> 6)];
  }
  wg_matmul<kPW>(A1, A2, A1);
  for (int e = t; e < 4096; e += kPT) {
    const int i = e & 63, j = e >> 6, row = rb + i;
    if (row < mr) Yhat[(size_t)row + (size_t)j * ldy] = (Tw)A1[i * kLdt + j];
  }
}

// ---------------------------------------------------------------------------
// MFMA tiles: 64 x 64 output per 256-thread work-group, 2 x 2 waves of 32 x 32,
// each wave 2 x 2 blocks of 16 x 16.  Operands live in LDS with K contiguous.
// Fragment layout (16x16xK): lane l supplies A[l%16][kl*(l/16) .. +kl) and
// B[kl*(l/16) .. +kl)[l%16]; accumulator register r holds column l%16 and the
// row given by MmaT::row (4*(l/16)+r for the fp32-accumulating forms).
// ---------------------------------------------------------------------------
template <Mma MT> struct MmaT;
template <> struct MmaT<Mma::F32> {
  using In = float; using Acc = float; using V = f32x4;
  static constexpr int KI = 4, KL = 1, PAD = 4;
  static constexpr bool kScaled = false;
  __device__ static V mma(const In* a, const In* b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return (float)v; }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MmaT<Mma::F64> {
  using In = double; using Acc = double; using V = f64x4;
  static constexpr int KI = 4, KL = 1, PAD = 2;
  static constexpr bool kScaled = false;
  __device__ static V mma(const In* a, const In* b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return v; }
  // fp64 16x16x4: accumulator register r of lane l holds row 4 r + l/16
  __device__ static int row(int l, int r) { return 4 * r + (l >> 4); }
};
template <> struct MmaT<Mma::BF16> {
  using In = __bf16; using Acc = float; using V = f32x4;
  static constexpr int KI = 32, KL = 8, PAD = 8;
  static constexpr bool kScaled = false;
  __device__ static V mma(const In* a, const In* b, V c) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(a);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return (__bf16)(float)v; }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MmaT<Mma::F16> {
  using In = _Float16; using Acc = float; using V = f32x4;
  static constexpr int KI = 32, KL = 8, PAD = 8;
  static constexpr bool kScaled = false;
  __device__ static V mma(const In* a, const In* b, V c) {
    const f16x8 av = *reinterpret_cast<const f16x8*>(a);
    const f16x8 bv = *reinterpret_cast<const f16x8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return (_Float16)(float)v; }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// FP8 e4m3 (OCP): one byte per input; 16x16x32 fragments with the same lane
// layout as the bf16 form (eight consecutive K values per lane, packed into
// 64 bits).  Inputs are scaled by powers of two per tile (kScaled) so that
// the tile's largest magnitude lands in [128, 256), below the e4m3 maximum 448.
template <> struct MmaT<Mma::F8> {
  using In = unsigned char; using Acc = float; using V = f32x4;
  static constexpr int KI = 32, KL = 8, PAD = 16;
  static constexpr bool kScaled = true;
  __device__ static V mma(const In* a, const In* b, V c) {
    const long av = *reinterpret_cast<const long*>(a);
    const long bv = *reinterpret_cast<const long*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return __hip_fp8_e4m3((float)v).__x; }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Power-of-two scale that maps a tile maximum m into [128, 256) (1 for m = 0).
__device__ __forceinline__ double fp8_scale(double m) {
  if (!(m > 0.0) || !isfinite(m)) return 1.0;
  int e;
  frexp(m, &e);
  return ldexp(1.0, 8 - e);
}

template <Mma MT, int BK>
__device__ __forceinline__ void mma_block(const typename MmaT<MT>::In* As,
                                          const typename MmaT<MT>::In* Bs,
                                          typename MmaT<MT>::V acc[2][2]) {
  using T = MmaT<MT>;
  constexpr int LD = BK + T::PAD;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int k0 = 0; k0 < BK; k0 += T::KI) {
    const typename T::In* ap[2];
    const typename T::In* bp[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      ap[b] = As + (32 * wr + 16 * b + (l & 15)) * LD + k0 + T::KL * (l >> 4);
      bp[b] = Bs + (32 * wc + 16 * b + (l & 15)) * LD + k0 + T::KL * (l >> 4);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = T::mma(ap[bi], bp[bj], acc[bi][bj]);
  }
}

// W partial: Wpart[s] (64 x nc, ld 64) = Y^T C over rows [s*kch, (s+1)*kch) of the panel.
// Y is read from the factor storage with the unit-lower mask.  The next
// 32-row chunk is fetched into registers while the MFMAs of the current one run.
template <typename Tw, Mma MT>
__global__ __launch_bounds__(256) void k_wy_t(
    const Tw* __restrict__ Y, int ldy, int mr, int jb,      // Y = &M[j0 + j0*ld]
    const Tw* __restrict__ C, int ldc, int nc, int kch,     // C = &target[j0 + cstart*ldc]
    typename MmaT<MT>::Acc* __restrict__ Wpart) {  // [gridDim.y][64 x nc], ld 64
  using T = MmaT<MT>;
  constexpr int BK = 32;
  constexpr int LD = BK + T::PAD;
  __shared__ __attribute__((aligned(16))) typename T::In As[64 * LD];
  __shared__ __attribute__((aligned(16))) typename T::In Bs[64 * LD];
  LSQ_LDS_POISON(As);
  LSQ_LDS_POISON(Bs);
  const int t = threadIdx.x;
  const int c0 = blockIdx.x * 64;
  const int kbeg = blockIdx.y * kch;
  const int kend = min(mr, kbeg + kch);
  typename T::V acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
  double ya[8], cb[8];
  auto fetch = [&](int k) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q, kk = e & (BK - 1), a = e / BK, i = k + kk;
      double y = 0.0, c = 0.0;
      if (i < kend && a < jb) y = i > a ? (double)Y[(size_t)i + (size_t)a * ldy] : (i == a ? 1.0 : 0.0);
      if (i < kend && c0 + a < nc) c = (double)C[(size_t)i + (size_t)(c0 + a) * ldc];
      ya[q] = y;
      cb[q] = c;
    }
  };
  __shared__ double red[8];
  if (kbeg < kend) fetch(kbeg);
  for (int k = kbeg; k < kend; k += BK) {
    double sa = 1.0, sb = 1.0;
    if constexpr (T::kScaled) {
      double ma = 0.0, mb = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ma = fmax(ma, fabs(ya[q]));
        mb = fmax(mb, fabs(cb[q]));
      }
      sa = fp8_scale(block_max(ma, red));
      sb = fp8_scale(block_max(mb, red));
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q, kk = e & (BK - 1), a = e / BK;
      As[a * LD + kk] = T::cvt(ya[q] * sa);
      Bs[a * LD + kk] = T::cvt(cb[q] * sb);
    }
    __syncthreads();
    if (k + BK < kend) fetch(k + BK);
    if constexpr (T::kScaled) {
      typename T::V tmp[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) tmp[i][j][r] = 0;
      mma_block<MT, BK>(As, Bs, tmp);
      const float inv = (float)(1.0 / (sa * sb));
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] += tmp[i][j][r] * inv;
    } else {
      mma_block<MT, BK>(As, Bs, acc);
    }
  }
  const int l = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 32 * wr + 16 * bi + T::row(l, r);
        const int c = c0 + 32 * wc + 16 * bj + (l & 15);
        if (c < nc) Wpart[(size_t)blockIdx.y * 64 * nc + a + (size_t)c * 64] = acc[bi][bj][r];
      }
}

template <typename Acc>
__global__ void k_wy_reduce(const Acc* __restrict__ Wpart, int nsplit, int total, Acc* __restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  Acc s = 0;
  for (int q = 0; q < nsplit; ++q) s += Wpart[(size_t)q * total + e];
  W[e] = s;
}

// C (mr x nc) -= Yhat (mr x jb) * W (jb x nc).  The C tile is read and
// written with row-contiguous accesses through LDS (fetched into registers
// before the MFMAs).  With Gnext, the work-groups of the first column tile
// below the first 64 rows also accumulate the Gram of the updated tile (its
// first jbn columns): the next panel's first Gram.
template <typename Tw, Mma MT>
__global__ __launch_bounds__(256) void k_wy_u(
    const Tw* __restrict__ Yhat, int ldy, int mr, int jb,
    const typename MmaT<MT>::Acc* __restrict__ W, Tw* __restrict__ C, int ldc, int nc,
    double* __restrict__ Gnext, int jbn, int copies) {
  using T = MmaT<MT>;
  using In = typename T::In;
  constexpr int BK = 64;
  constexpr int LD = BK + T::PAD;
  constexpr size_t kOps = 2 * 64 * LD * sizeof(In), kTile = 64 * kLdt * sizeof(double);
  __shared__ __attribute__((aligned(16))) char smem[kOps > kTile ? kOps : kTile];
  LSQ_LDS_POISON(smem);
  In* As = reinterpret_cast<In*>(smem);
  In* Bs = As + 64 * LD;
  double* tile = reinterpret_cast<double*>(smem);
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  double cv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + 256 * q, i = e & 63, c = e >> 6;
    cv[q] = (r0 + i < mr && c0 + c < nc) ? (double)C[(size_t)(r0 + i) + (size_t)(c0 + c) * ldc] : 0.0;
  }
  double av[16], bv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + 256 * q, i = e & 63, a = e >> 6;
    av[q] = (r0 + i < mr && a < jb) ? (double)Yhat[(size_t)(r0 + i) + (size_t)a * ldy] : 0.0;
    bv[q] = (i < jb && c0 + a < nc) ? (double)W[i + (size_t)(c0 + a) * 64] : 0.0;
  }
  double sa = 1.0, sb = 1.0;
  if constexpr (T::kScaled) {
    __shared__ double red[8];
    double ma = 0.0, mb = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      ma = fmax(ma, fabs(av[q]));
      mb = fmax(mb, fabs(bv[q]));
    }
    sa = fp8_scale(block_max(ma, red));
    sb = fp8_scale(block_max(mb, red));
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + 256 * q, i = e & 63, a = e >> 6;
    As[i * LD + a] = T::cvt(av[q] * sa);     // As[row][k]
    Bs[a * LD + i] = T::cvt(bv[q] * sb);     // Bs[col][k]
  }
  __syncthreads();
  typename T::V acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
  mma_block<MT, BK>(As, Bs, acc);
  if constexpr (T::kScaled) {
    const float inv = (float)(1.0 / (sa * sb));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] *= inv;
  }
  __syncthreads();                                 // the tile reuses the operand buffers
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + 256 * q, i = e & 63, c = e >> 6;
    tile[i * kLdt + c] = cv[q];
  }
  __syncthreads();
  const int l = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int il = 32 * wr + 16 * bi + T::row(l, r), cl = 32 * wc + 16 * bj + (l & 15);
        double* p = &tile[il * kLdt + cl];
        *p = (double)(Tw)(*p - (double)acc[bi][bj][r]);
      }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + 256 * q, i = e & 63, c = e >> 6;
    if (r0 + i < mr && c0 + c < nc) C[(size_t)(r0 + i) + (size_t)(c0 + c) * ldc] = (Tw)tile[i * kLdt + c];
  }
  if (Gnext != nullptr && blockIdx.y == 0 && blockIdx.x > 0) gram_atomic<4>(tile, jbn, Gnext, copies);
}

// ---------------------------------------------------------------- host side

static size_t elem(int tw) { return (size_t)tw; }

void qr_alloc(Ctx& ctx, QRFactor& f, int r, int c, int tw, Mma mt, int nb) {
  f.r = r; f.c = c; f.k = r < c ? r : c; f.ld = r > 1 ? r : 1;
  f.nb = nb; f.np = ceil_div(f.k, nb); f.tw = tw; f.mt = mt;
  f.passes = tw == 8 ? 3 : 2;
  f.M = ctx.ws->alloc(elem(tw) * (size_t)f.ld * (c > 0 ? c : 1));
  f.T = ctx.ws->alloc(elem(tw) * 4096 * (size_t)(f.np > 0 ? f.np : 1));
  f.yoff.resize(f.np);
  size_t tot = 0;
  for (int j = 0; j < f.np; ++j) {
    f.yoff[j] = tot;
    tot += (size_t)(r - j * nb) * 64;
  }
  f.Yhat = ctx.ws->alloc(elem(tw) * (tot > 0 ? tot : 1));
  f.status = ctx.ws->get<int>(1);
  LSQ_HIP(hipMemsetAsync(f.status, 0, sizeof(int), ctx.stream));
}

template <typename Tw, Mma MT>
static void wy_apply(Ctx& ctx, const Tw* Y, int ldy, int mr, int jb, const Tw* Yhat, int ldyh,
                     Tw* C, int ldc, int nc, double* Gnext = nullptr, int jbn = 0, int gcopies = 1) {
  using Acc = typename MmaT<MT>::Acc;
  if (nc <= 0 || mr <= 0) return;
  const int nct = ceil_div(nc, 64);
  int nsplit = ceil_div(768, nct);
  int maxsplit = ceil_div(mr, 128);
  if (maxsplit > 32) maxsplit = 32;
  if (nsplit > maxsplit) nsplit = maxsplit;
  if (nsplit < 1) nsplit = 1;
  int kch = ceil_div(ceil_div(mr, nsplit), 32) * 32;
  nsplit = ceil_div(mr, kch);
  Acc* Wpart = ctx.ws->get<Acc>((size_t)nsplit * 64 * nc);
  Acc* W = ctx.ws->get<Acc>((size_t)64 * nc);
  ktimer_begin(ctx, kKWyT, 2.0 * mr * jb * nc, (double)mr * (jb + nc) * sizeof(Tw));
  hipLaunchKernelGGL((k_wy_t<Tw, MT>), dim3(nct, nsplit), dim3(256), 0, ctx.stream,
                     Y, ldy, mr, jb, C, ldc, nc, kch, Wpart);
  ktimer_end(ctx, kKWyT);
  const int total = 64 * nc;
  hipLaunchKernelGGL((k_wy_reduce<Acc>), dim3(ceil_div(total, 256)), dim3(256), 0, ctx.stream,
                     Wpart, nsplit, total, W);
  LSQ_LAUNCH_CHECK();
  ktimer_begin(ctx, kKWyU, 2.0 * mr * jb * nc, (double)mr * (jb + 2.0 * nc) * sizeof(Tw));
  hipLaunchKernelGGL((k_wy_u<Tw, MT>), dim3(ceil_div(mr, 64), nct), dim3(256), 0, ctx.stream,
                     Yhat, ldyh, mr, jb, W, C, ldc, nc, Gnext, jbn, gcopies);
  ktimer_end(ctx, kKWyU);
  LSQ_LAUNCH_CHECK();
}

template <typename Tw, Mma MT>
static void qr_factor_t(Ctx& ctx, QRFactor& f) {
  using Acc = typename MmaT<MT>::Acc;
  Tw* M = static_cast<Tw*>(f.M);
  Tw* Tb = static_cast<Tw*>(f.T);
  Tw* Yh = static_cast<Tw*>(f.Yhat);
  const int r = f.r, ld = f.ld;
  double* Q0 = ctx.ws->get<double>((size_t)r * 64);
  double* Q1 = ctx.ws->get<double>((size_t)r * 64);
  // three Gram accumulators per panel (gcopies copies each: one, or one per
  // row tile in the deterministic mode), zeroed once
  const int gcopies = ctx.deterministic ? ceil_div(r, 64) : 1;
  const size_t gstride = (size_t)gcopies * 4096;
  double* Gall = ctx.ws->get<double>((size_t)f.np * 3 * gstride);
  LSQ_HIP(hipMemsetAsync(Gall, 0, sizeof(double) * (size_t)f.np * 3 * gstride, ctx.stream));
  double* Racc = ctx.ws->get<double>(4096);
  const bool lookahead = ctx.lookahead && ctx.side != nullptr && ctx.events != nullptr && f.np > 1;
  Ctx sctx = ctx;
  sctx.stream = ctx.side;
  int side_pending = -1;            // last step whose side-stream update is not yet awaited
  {
    const int jb = f.k < f.nb ? f.k : f.nb;
    hipLaunchKernelGGL((k_panel_gram<Tw>), dim3(ceil_div(r, 64)), dim3(kPT), 0, ctx.stream,
                       M, ld, r, jb, Gall, gcopies);
  }
  for (int j = 0; j < f.np; ++j) {
    const int j0 = j * f.nb;
    const int jb = (f.k - j0) < f.nb ? (f.k - j0) : f.nb;
    const int mr = r - j0;
    const int tiles = ceil_div(mr, 64);
    double* G0 = Gall + (size_t)j * 3 * gstride;
    double* G1 = G0 + gstride;
    double* G2 = G1 + gstride;
    Tw* P = M + (size_t)j0 + (size_t)j0 * ld;
    // shifted pass: Q0 = P R0^{-1}, R0 = chol(P^T P + sigma I)
    // algorithmic work of a pass: X R^{-1} and the Gram (2 mr jb^2 each), the
    // Cholesky with its inverse (2 jb^3 / 3); bytes: X in, Xout out
    const double pass_flops = 4.0 * mr * jb * jb + 2.0 * jb * jb * jb / 3.0;
    ktimer_begin(ctx, kKPanelCholPass, pass_flops, (double)mr * jb * (sizeof(Tw) + 8));
    hipLaunchKernelGGL((k_panel_cholpass<Tw>), dim3(tiles), dim3(kPT), 0, ctx.stream,
                       G0, 1, 1, Racc, f.status, P, ld, mr, jb, Q0, mr, G1, gcopies);
    ktimer_end(ctx, kKPanelCholPass);
    const double* Qlast = Q0;
    const double* Glast = G1;
    if (f.passes >= 3) {
      ktimer_begin(ctx, kKPanelCholPass, pass_flops, (double)mr * jb * 16);
      hipLaunchKernelGGL((k_panel_cholpass<double>), dim3(tiles), dim3(kPT), 0, ctx.stream,
                         G1, 0, 0, Racc, f.status, Q0, mr, mr, jb, Q1, mr, G2, gcopies);
      ktimer_end(ctx, kKPanelCholPass);
      Qlast = Q1;
      Glast = G2;
    }
    // Trailing update of columns j0 + jb .. c-1.  With look-ahead, the next
    // panel's columns are updated on the main stream: W = Y^T C for them is
    // formed inside the reconstruction kernel (which holds Y), then reduced and
    // applied together with the next panel's Gram.  The remaining columns are
    // updated on the side stream, overlapping the next panel's factorization;
    // that update must finish before the next reconstruction reads the
    // columns after it.
    const int nc = f.c - j0 - jb;
    double* Gnext = nullptr;
    int jbn = 0;
    if (j + 1 < f.np) {
      Gnext = Gall + (size_t)(j + 1) * 3 * gstride;
      jbn = (f.k - j0 - f.nb) < f.nb ? (f.k - j0 - f.nb) : f.nb;
    }
    Tw* Ctr = M + (size_t)j0 + (size_t)(j0 + jb) * ld;
    const bool la = lookahead && j + 1 < f.np && nc > jbn;
    Acc* Wpart = la ? ctx.ws->get<Acc>((size_t)tiles * 64 * jbn) : nullptr;
    if (side_pending >= 0) {
      LSQ_HIP(hipStreamWaitEvent(ctx.stream, ctx_event(ctx, 2 * side_pending + 1), 0));
      side_pending = -1;
    }
    // algorithmic work: the Householder factorization of the mr x jb panel
    // (2 mr jb^2 - 2 jb^3 / 3 flops, Section 4.1's xGEQRF), which this kernel
    // completes; the Cholesky-QR passes and the reconstruction are how it is
    // computed, not extra work of the method.  Bytes: Q1 in, Y and Yhat out.
    ktimer_begin(ctx, kKPanelFinal, 2.0 * mr * jb * jb - 2.0 * jb * jb * jb / 3.0,
                 (double)mr * jb * (8 + 2 * sizeof(Tw)));
    hipLaunchKernelGGL((k_panel_final_y<Tw, Acc>), dim3(tiles), dim3(kPT), 0, ctx.stream,
                       Glast, jb, mr, Qlast, mr, Racc, M, ld, j0, Tb + (size_t)j * 4096,
                       Yh + f.yoff[j], mr, f.status, (const Tw*)Ctr, la ? jbn : 0, Wpart, gcopies);
    ktimer_end(ctx, kKPanelFinal);
    LSQ_LAUNCH_CHECK();
    if (la) {
      hipEvent_t panel_done = ctx_event(ctx, 2 * j);
      LSQ_HIP(hipEventRecord(panel_done, ctx.stream));
      Acc* W = ctx.ws->get<Acc>((size_t)64 * jbn);
      hipLaunchKernelGGL((k_wy_reduce<Acc>), dim3(ceil_div(64 * jbn, 256)), dim3(256), 0, ctx.stream,
                         Wpart, tiles, 64 * jbn, W);
      hipLaunchKernelGGL((k_wy_u<Tw, MT>), dim3(tiles, 1), dim3(256), 0, ctx.stream,
                         Yh + f.yoff[j], mr, mr, jb, W, Ctr, ld, jbn, Gnext, jbn, gcopies);
      LSQ_LAUNCH_CHECK();
      LSQ_HIP(hipStreamWaitEvent(sctx.stream, panel_done, 0));
      wy_apply<Tw, MT>(sctx, P, ld, mr, jb, Yh + f.yoff[j], mr, Ctr + (size_t)jbn * ld, ld,
                       nc - jbn);
      LSQ_HIP(hipEventRecord(ctx_event(ctx, 2 * j + 1), sctx.stream));
      side_pending = j;
    } else {
      wy_apply<Tw, MT>(ctx, P, ld, mr, jb, Yh + f.yoff[j], mr, Ctr, ld, nc, Gnext, jbn, gcopies);
    }
  }
  if (side_pending >= 0) LSQ_HIP(hipStreamWaitEvent(ctx.stream, ctx_event(ctx, 2 * side_pending + 1), 0));
}

void qr_factor(Ctx& ctx, QRFactor& f) {
  if (f.k <= 0) return;
  if (f.tw == 8) {
    qr_factor_t<double, Mma::F64>(ctx, f);
  } else {
    switch (f.mt) {
      case Mma::F8: qr_factor_t<float, Mma::F8>(ctx, f); break;
      case Mma::BF16: qr_factor_t<float, Mma::BF16>(ctx, f); break;
      case Mma::F16: qr_factor_t<float, Mma::F16>(ctx, f); break;
      default: qr_factor_t<float, Mma::F32>(ctx, f); break;
    }
  }
}

template <typename Tw, Mma MT>
static void apply_left_t(Ctx& ctx, const QRFactor& f, Tw* C, int ldc, int ncols) {
  const Tw* M = static_cast<const Tw*>(f.M);
  const Tw* Yh = static_cast<const Tw*>(f.Yhat);
  for (int j = 0; j < f.np; ++j) {
    const int j0 = j * f.nb;
    const int jb = (f.k - j0) < f.nb ? (f.k - j0) : f.nb;
    const int mr = f.r - j0;
    wy_apply<Tw, MT>(ctx, M + (size_t)j0 + (size_t)j0 * f.ld, f.ld, mr, jb, Yh + f.yoff[j], mr,
                     C + j0, ldc, ncols);
  }
}

void qr_apply_left_T(Ctx& ctx, const QRFactor& f, void* C, int ldc, int ncols) {
  if (f.k <= 0 || ncols <= 0) return;
  if (f.tw == 8) {
    apply_left_t<double, Mma::F64>(ctx, f, static_cast<double*>(C), ldc, ncols);
  } else {
    switch (f.mt) {
      case Mma::F8: apply_left_t<float, Mma::F8>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
      case Mma::BF16: apply_left_t<float, Mma::BF16>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
      case Mma::F16: apply_left_t<float, Mma::F16>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
      default: apply_left_t<float, Mma::F32>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
    }
  }
}

}  // namespace lsq
