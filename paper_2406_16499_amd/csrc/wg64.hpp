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
// algorithms (Cholesky, triangular inverse, LU, triangular solve for T) are
// right-looking; in each step only the pivot rows or column travel through a
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

// x <- R^{-1} (upper) with R read from LDS (row-major, zero below the diagonal,
// identity-padded).  Right-looking back substitution with the diagonal
// reciprocals computed up front; the owner of the finished row restores it
// after the (unmasked) update.  buf: 2 x 64 + 64 doubles.
template <int NW>
__device__ __forceinline__ void reg_upper_inverse(const double* R, double* x, double* buf) {
  constexpr int RR = Own<NW>::R;
  const Own<NW> o;
  double* dinv = buf + 128;
  if (threadIdx.x < 64) dinv[threadIdx.x] = rcp64(R[threadIdx.x * kLdt + threadIdx.x]);
#pragma unroll
  for (int qq = 0; qq < RR; ++qq) x[qq] = (o.r0 + qq == o.c) ? 1.0 : 0.0;
  __syncthreads();
  for (int wi = NW - 1; wi >= 0; --wi) {
#pragma unroll
    for (int q = RR - 1; q >= 0; --q) {
      const int i = RR * wi + q;
      double* rb = buf + (i & 1) * 64;
      if (o.w == wi) rb[o.c] = x[q] * dinv[i];
      __syncthreads();
      const double xi = rb[o.c];
#pragma unroll
      for (int qq = 0; qq < RR; ++qq) x[qq] = fma(-R[(o.r0 + qq) * kLdt + i], xi, x[qq]);
      if (o.w == wi) x[q] = xi;
    }
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
