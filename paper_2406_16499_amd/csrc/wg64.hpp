// 64 x 64 FP64 building blocks for one work-group of NW waves (gfx950).
#pragma once
#include "common.hpp"

namespace lsq {

constexpr int kLdt = kMaxNb + 1;   // padded LDS row stride for 64-wide FP64 tiles

// ---------------------------------------------------------------------------
// 64 x 64 dense kernels for one work-group of NW waves (64 NW threads).
//
// Thread t owns column c = t & 63 of rows r0 .. r0 + R - 1 (R = 64 / NW,
// r0 = R (t >> 6)) and keeps those R entries in registers.  The sequential
// algorithms (Cholesky with its inverse factor, the modified LU of the panel
// kernels) are right-looking; in each step only the pivot rows or column travel through a
// double-buffered LDS line, so there is one barrier per step and no LDS
// read-modify-write traffic.  With NW = 8 two waves share each SIMD and hide
// each other's LDS and dependency latency.  Dense 64 x 64 products run on
// FP64 MFMA from row-major LDS tiles [64][kLdt].
// ---------------------------------------------------------------------------
template <int NW>
struct Own {
  static constexpr int R = 64 / NW;
  int c, w, r0;      // w and r0 are wave-uniform (scalar registers)
  __device__ Own()
      : c(threadIdx.x & 63), w(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)), r0(R * w) {}
};

template <int NW>
__device__ __forceinline__ void regs_load(const double* S, double* x) {
  const Own<NW> o;
#pragma unroll
  for (int q = 0; q < Own<NW>::R; ++q) x[q] = S[(o.r0 + q) * kLdt + o.c];
}
template <int NW>
__device__ __forceinline__ void regs_store(double* S, const double* x) {
  const Own<NW> o;
#pragma unroll
  for (int q = 0; q < Own<NW>::R; ++q) S[(o.r0 + q) * kLdt + o.c] = x[q];
}
// S = x^T restricted to the leading jb x jb block (zero elsewhere): the
// thread's register column becomes row c of S.
template <int NW>
__device__ __forceinline__ void regs_store_t(double* S, const double* x, int jb = 64) {
  const Own<NW> o;
#pragma unroll
  for (int q = 0; q < Own<NW>::R; ++q)
    S[o.c * kLdt + o.r0 + q] = (o.c < jb && o.r0 + q < jb) ? x[q] : 0.0;
}

// acc = op(A) * B for 64 x 64 LDS matrices.  The 4 x 4 grid of 16 x 16 blocks
// is split over the waves: wave w takes BR = 8 / NW block rows starting at
// 16 BR (w >> 1) and the two block columns starting at 32 (w & 1).
// fp64 16x16x4 fragments: lane l supplies A[l%16][k + l/16], B[k + l/16][l%16];
// accumulator register r holds row 4r + l/16, column l%16.
template <int NW>
__device__ __forceinline__ void mm64_acc(const double* A, bool transA, const double* B,
                                         f64x4 acc[8 / NW][2]) {
  constexpr int BR = 8 / NW;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rb = 16 * BR * (w >> 1), cb = 32 * (w & 1);
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
#pragma unroll 4
  for (int k0 = 0; k0 < 64; k0 += 4) {
    double a[BR], b[2];
    const int kk = k0 + (l >> 4);
#pragma unroll
    for (int q = 0; q < BR; ++q) {
      const int row = rb + 16 * q + (l & 15);
      a[q] = transA ? A[kk * kLdt + row] : A[row * kLdt + kk];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) b[q] = B[kk * kLdt + cb + 16 * q + (l & 15)];
#pragma unroll
    for (int bi = 0; bi < BR; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
}
// (row, column) of accumulator element (bi, bj, r) of this lane
template <int NW>
__device__ __forceinline__ int mm64_row(int bi, int r) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  return 16 * (8 / NW) * (w >> 1) + 16 * bi + 4 * r + (l >> 4);
}
template <int NW>
__device__ __forceinline__ int mm64_col(int bj) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  return 32 * (w & 1) + 16 * bj + (l & 15);
}
template <int NW>
__device__ __forceinline__ void mm64_store(const f64x4 acc[8 / NW][2], double* C) {
#pragma unroll
  for (int bi = 0; bi < 8 / NW; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) C[mm64_row<NW>(bi, r) * kLdt + mm64_col<NW>(bj)] = acc[bi][bj][r];
}
// C = op(A) * B; C may alias A or B.
template <int NW>
__device__ __forceinline__ void wg_matmul(const double* A, const double* B, double* C, bool transA = false) {
  f64x4 acc[8 / NW][2];
  mm64_acc<NW>(A, transA, B, acc);
  __syncthreads();
  mm64_store<NW>(acc, C);
  __syncthreads();
}

// Reciprocal and reciprocal square root in FP64 from the hardware
// approximations refined by Newton steps (no IEEE division / sqrt sequences on
// the sequential path).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// In-register Cholesky with the inverse factor.  On entry x holds this
// thread's entries of a symmetric positive definite G (identity-padded beyond
// jb).  On exit x holds R (upper, G = R^T R, zeros below the diagonal) and z
// holds Z = R^{-T} (lower): rows of Z follow from forward substitution with
// R^T, which needs exactly the rows of R produced in the same step, so both
// run in one loop.  Each step eliminates a 2 x 2 pivot block (rows k, k+1 of
// one wave): one barrier and one pivot chain per two columns.  The pivot rows
// are published with zeros left of their diagonal, so the updates need no
// masks: finished rows see zero multipliers, and the pivot rows themselves are
// overwritten by their owner after the update.  buf: 8 x 64 LDS doubles.
template <int NW>
__device__ __forceinline__ bool reg_cholesky_inv(double* x, double* z, double* buf) {
  constexpr int R = Own<NW>::R;
  const Own<NW> o;
  bool ok = true;
#pragma unroll
  for (int qq = 0; qq < R; ++qq) z[qq] = (o.r0 + qq == o.c) ? 1.0 : 0.0;
  for (int wk = 0; wk < NW; ++wk) {
#pragma unroll
    for (int q = 0; q < R; q += 2) {
      const int k = R * wk + q;
      double* g0 = buf + ((k >> 1) & 1) * 256;        // row k of G, row k + 1, rows k, k + 1 of z
      double* g1 = g0 + 64;
      double* z0 = g0 + 128;
      double* z1 = g0 + 192;
      if (o.w == wk) {
        g0[o.c] = (o.c >= k) ? x[q] : 0.0;
        g1[o.c] = (o.c >= k + 1) ? x[q + 1] : 0.0;
        z0[o.c] = z[q];
        z1[o.c] = z[q + 1];
      }
      __syncthreads();
      // 2 x 2 pivot block [g00 g01; g01 g11] = R_kk^T R_kk
      double g00 = g0[k];
      ok = ok && (g00 > 0.0);
      g00 = g00 > 0.0 ? g00 : 1e-300;
      const double i0 = rsqrt64(g00);
      const double r01 = g0[k + 1] * i0;
      double d1 = g1[k + 1] - r01 * r01;
      ok = ok && (d1 > 0.0);
      d1 = d1 > 0.0 ? d1 : 1e-300;
      const double i1 = rsqrt64(d1);
      // rows k, k + 1 of R and Z in this thread's column
      const double R0 = g0[o.c] * i0;
      const double R1 = (g1[o.c] - r01 * R0) * i1;
      const double Z0 = z0[o.c] * i0;
      const double Z1 = (z1[o.c] - r01 * Z0) * i1;
      // x_i -= R0_i R0 + R1_i R1 with R0_i = g0_i i0, R1_i = (g1_i - r01 R0_i) i1,
      // regrouped as g0_i a + g1_i b (likewise for z)
      const double t = r01 * i0 * i1;
      const double ax = R0 * i0 - t * R1, bx = R1 * i1;
      const double az = Z0 * i0 - t * Z1, bz = Z1 * i1;
#pragma unroll
      for (int qq = 0; qq < R; ++qq) {
        const double a0 = g0[o.r0 + qq], a1 = g1[o.r0 + qq];
        x[qq] = fma(-a1, bx, fma(-a0, ax, x[qq]));
        z[qq] = fma(-a1, bz, fma(-a0, az, z[qq]));
      }
      if (o.w == wk) {
        x[q] = R0;
        x[q + 1] = (o.c >= k + 1) ? R1 : 0.0;
        z[q] = Z0;
        z[q + 1] = Z1;
      }
    }
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Blocked inverse of a 64 x 64 upper triangle as a 4 x 4 grid of 16 x 16
// blocks: each diagonal block is inverted by one wave in registers (16 steps
// that need no work-group barrier, rows travelling by lane shuffles), four
// waves at once; the off-diagonal blocks follow by distance from the diagonal
// (one barrier per distance) as 16 x 16 x 16 FP64 MFMA products, one block
// per wave.
// ---------------------------------------------------------------------------

// fp64 16x16x4 operand fragments of block (bi, bj) of S, for K steps s = 0..3:
// as the A operand lane l supplies M[l%16][4s + l/16], as the B operand
// M[4s + l/16][l%16], M the block.
__device__ __forceinline__ void frag_a(const double* S, int bi, int bj, double a[4]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) a[s] = S[(16 * bi + (l & 15)) * kLdt + 16 * bj + 4 * s + (l >> 4)];
}
__device__ __forceinline__ void frag_b(const double* S, int bi, int bj, double b[4]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) b[s] = S[(16 * bi + 4 * s + (l >> 4)) * kLdt + 16 * bj + (l & 15)];
}
// Accumulator register r of lane l holds row 4 r + l/16, column l%16 of the
// block: the B-operand layout, so a product can feed the next one directly.
__device__ __forceinline__ void blk_store(double* S, int bi, int bj, const f64x4& acc) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) S[(16 * bi + 4 * r + (l >> 4)) * kLdt + 16 * bj + (l & 15)] = acc[r];
}
__device__ __forceinline__ f64x4 blk_zero() {
  f64x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = 0.0;
  return acc;
}
// acc += sign * A B for fragments a (A operand) and b (B operand)
__device__ __forceinline__ f64x4 blk_mma(const double a[4], const double b[4], f64x4 acc, double sign = 1.0) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * a[s], b[s], acc, 0, 0, 0);
  return acc;
}
__device__ __forceinline__ f64x4 blk_mma_acc(const double a[4], const f64x4& b, f64x4 acc, double sign = 1.0) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * a[s], b[s], acc, 0, 0, 0);
  return acc;
}
// Zero the blocks strictly below (lower = true) or above the diagonal.
template <int NW>
__device__ __forceinline__ void zero_off_blocks(double* S, bool lower) {
  for (int e = threadIdx.x; e < 4096; e += 64 * NW) {
    const int i = e >> 6, j = e & 63;
    if (lower ? (i >> 4) > (j >> 4) : (i >> 4) < (j >> 4)) S[i * kLdt + j] = 0.0;
  }
}

// One wave: X(b, b) = R(b, b)^{-1} for an upper triangular diagonal block, by
// back substitution on [R(b, b) | I] (the triangle itself needs no update:
// column k of the rows above k is read as it was); rows travel by lane
// shuffles.
__device__ __forceinline__ void wave_uinv16(const double* R, double* X, int b) {
  const int l = threadIdx.x & 63, i = l & 15, q = l >> 4, o = 16 * b;
  double r[4], x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    r[j] = R[(o + i) * kLdt + o + 4 * q + j];
    x[j] = (4 * q + j == i) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int k = 15; k >= 0; --k) {
    const double rkk = __shfl(r[k & 3], ((k >> 2) << 4) + k, 64);
    const double rik = __shfl(r[k & 3], ((k >> 2) << 4) + i, 64);    // R[i][k]
    const double ip = rcp64(rkk);
    double xk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) xk[j] = __shfl(x[j], (q << 4) + k, 64) * ip;   // row k of the inverse
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = (i < k) ? fma(-rik, xk[j], x[j]) : (i == k ? xk[j] : x[j]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) X[(o + i) * kLdt + o + 4 * q + j] = x[j];
}

// X = R^{-1} for an upper triangular R (64 x 64 LDS, zeros below the
// diagonal, identity-padded where unused): the four diagonal blocks on four
// waves at once, then the off-diagonal blocks by distance from the diagonal.
template <int NW>
__device__ __forceinline__ void blk_upper_inverse(const double* R, double* X) {
  static_assert(NW >= 4, "one wave per diagonal block");
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  zero_off_blocks<NW>(X, true);
  if (w < 4) wave_uinv16(R, X, w);
  __syncthreads();
  for (int dd = 1; dd < 4; ++dd) {
    if (w < 4 - dd) {
      const int i = w, j = w + dd;
      f64x4 acc = blk_zero();
      for (int k = i + 1; k <= j; ++k) {
        double a[4], bb[4];
        frag_a(R, i, k, a);
        frag_b(X, k, j, bb);
        acc = blk_mma(a, bb, acc);
      }
      double a[4];
      frag_a(X, i, i, a);
      blk_store(X, i, j, blk_mma_acc(a, acc, blk_zero(), -1.0));
    }
    __syncthreads();
  }
}

// Identity padding of a 64 x 64 LDS matrix beyond jb (upper triangular or symmetric use).
template <int NW>
__device__ void pad_identity(double* S, int jb) {
  const Own<NW> o;
#pragma unroll
  for (int qq = 0; qq < Own<NW>::R; ++qq) {
    const int i = o.r0 + qq;
    if (i >= jb || o.c >= jb) S[i * kLdt + o.c] = (i == o.c) ? 1.0 : 0.0;
  }
  __syncthreads();
}

template <int NW>
__device__ void wg_load64(const double* g, double* s) {   // global col-major ld 64 -> LDS
  for (int e = threadIdx.x; e < 4096; e += 64 * NW) s[(e & 63) * kLdt + (e >> 6)] = g[e];
  __syncthreads();
}
template <int NW>
__device__ void wg_store64(const double* s, double* g) {
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 64 * NW) g[e] = s[(e & 63) * kLdt + (e >> 6)];
  __syncthreads();
}

}  // namespace lsq
