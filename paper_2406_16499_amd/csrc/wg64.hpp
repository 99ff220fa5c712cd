// 64 x 64 FP64 building blocks for one 256-thread work-group (gfx950).
#pragma once
#include "common.hpp"

namespace lsq {

constexpr int kLdt = kMaxNb + 1;   // padded LDS row stride for 64-wide FP64 tiles

// ---------------------------------------------------------------------------
// 64 x 64 dense kernels for one 256-thread work-group.
//
// Thread t owns column c = t & 63 of rows r0 .. r0+15, r0 = 16 (t >> 6), and
// keeps those 16 entries in registers.  The sequential algorithms (Cholesky,
// triangular inverse, LU, triangular solve for T) are right-looking; in each
// step only the pivot row or column travels through a double-buffered LDS line,
// so there is one barrier per step and no LDS read-modify-write traffic.
// Dense 64 x 64 products run on FP64 MFMA from row-major LDS tiles [64][kLdt].
// ---------------------------------------------------------------------------
struct Own {
  int c, w, r0;      // w and r0 are wave-uniform (scalar registers)
  __device__ Own()
      : c(threadIdx.x & 63), w(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)), r0(16 * w) {}
};

__device__ __forceinline__ void regs_load(const double* S, double x[16]) {
  const Own o;
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = S[(o.r0 + q) * kLdt + o.c];
}
__device__ __forceinline__ void regs_store(double* S, const double x[16]) {
  const Own o;
#pragma unroll
  for (int q = 0; q < 16; ++q) S[(o.r0 + q) * kLdt + o.c] = x[q];
}
// S = x^T restricted to the leading jb x jb block (zero elsewhere): the
// thread's register column becomes row c of S.
__device__ __forceinline__ void regs_store_t(double* S, const double x[16], int jb = 64) {
  const Own o;
#pragma unroll
  for (int q = 0; q < 16; ++q) S[o.c * kLdt + o.r0 + q] = (o.c < jb && o.r0 + q < jb) ? x[q] : 0.0;
}

// acc = op(A) * B for 64 x 64 LDS matrices; wave w computes the 32 x 32 quadrant
// (w >> 1, w & 1).  fp64 16x16x4 fragments: lane l supplies A[l%16][k + l/16],
// B[k + l/16][l%16]; accumulator register r holds row 4r + l/16, column l%16.
__device__ __forceinline__ void mm64_acc(const double* A, bool transA, const double* B, f64x4 acc[2][2]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
#pragma unroll 4
  for (int k0 = 0; k0 < 64; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int row = 32 * wr + 16 * q + (l & 15), kk = k0 + (l >> 4);
      a[q] = transA ? A[kk * kLdt + row] : A[row * kLdt + kk];
      b[q] = B[kk * kLdt + 32 * wc + 16 * q + (l & 15)];
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
}
__device__ __forceinline__ void mm64_store(const f64x4 acc[2][2], double* C) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        C[(32 * wr + 16 * bi + 4 * r + (l >> 4)) * kLdt + 32 * wc + 16 * bj + (l & 15)] = acc[bi][bj][r];
}
// C = op(A) * B; C may alias A or B.
__device__ __forceinline__ void wg_matmul(const double* A, const double* B, double* C, bool transA = false) {
  f64x4 acc[2][2];
  mm64_acc(A, transA, B, acc);
  __syncthreads();
  mm64_store(acc, C);
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
// holds Z = R^{-T} (lower): row k of Z follows from forward substitution with
// R^T, which needs exactly the row of R produced in step k, so both run in
// one loop.  The pivot row is published with zeros left of the diagonal, so
// the updates need no masks: finished rows see a zero multiplier, and the
// pivot row itself is overwritten by its owner after the update.
// buf: 4 x 64 LDS doubles.
__device__ __forceinline__ bool reg_cholesky_inv(double x[16], double z[16], double* buf) {
  const Own o;
  bool ok = true;
#pragma unroll
  for (int qq = 0; qq < 16; ++qq) z[qq] = (o.r0 + qq == o.c) ? 1.0 : 0.0;
  for (int wk = 0; wk < 4; ++wk) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 16 * wk + q;
      double* rg = buf + (q & 1) * 128;
      double* rz = rg + 64;
      if (o.w == wk) {
        rg[o.c] = (o.c >= k) ? x[q] : 0.0;
        rz[o.c] = z[q];
      }
      __syncthreads();
      double dkk = rg[k];
      ok = ok && (dkk > 0.0);
      dkk = dkk > 0.0 ? dkk : 1e-300;
      const double ip = rsqrt64(dkk), ip2 = ip * ip;
      const double gkc = rg[o.c], zkc = rz[o.c];
      const double rk2 = gkc * ip2, zk2 = zkc * ip2;
#pragma unroll
      for (int qq = 0; qq < 16; ++qq) {
        const double gki = rg[o.r0 + qq];
        x[qq] = fma(-gki, rk2, x[qq]);
        z[qq] = fma(-gki, zk2, z[qq]);
      }
      if (o.w == wk) {
        x[q] = gkc * ip;
        z[q] = zkc * ip;
      }
    }
  }
  return ok;
}

// x <- R^{-1} (upper) with R read from LDS (row-major, zero below the diagonal,
// identity-padded).  Right-looking back substitution with the diagonal
// reciprocals computed up front; the owner of the finished row restores it
// after the (unmasked) update.  buf: 2 x 64 + 64 doubles.
__device__ __forceinline__ void reg_upper_inverse(const double* R, double x[16], double* buf) {
  const Own o;
  double* dinv = buf + 128;
  if (threadIdx.x < 64) dinv[threadIdx.x] = rcp64(R[threadIdx.x * kLdt + threadIdx.x]);
#pragma unroll
  for (int qq = 0; qq < 16; ++qq) x[qq] = (o.r0 + qq == o.c) ? 1.0 : 0.0;
  __syncthreads();
  for (int wi = 3; wi >= 0; --wi) {
#pragma unroll
    for (int q = 15; q >= 0; --q) {
      const int i = 16 * wi + q;
      double* rb = buf + (q & 1) * 64;
      if (o.w == wi) rb[o.c] = x[q] * dinv[i];
      __syncthreads();
      const double xi = rb[o.c];
#pragma unroll
      for (int qq = 0; qq < 16; ++qq) x[qq] = fma(-R[(o.r0 + qq) * kLdt + i], xi, x[qq]);
      if (o.w == wi) x[q] = xi;
    }
  }
}

// Identity padding of a 64 x 64 LDS matrix beyond jb (upper triangular or symmetric use).
__device__ void pad_identity(double* S, int jb) {
  const Own o;
#pragma unroll
  for (int qq = 0; qq < 16; ++qq) {
    const int i = o.r0 + qq;
    if (i >= jb || o.c >= jb) S[i * kLdt + o.c] = (i == o.c) ? 1.0 : 0.0;
  }
  __syncthreads();
}

__device__ void wg_load64(const double* g, double* s) {   // global col-major ld 64 -> LDS
  for (int e = threadIdx.x; e < 4096; e += 256) s[(e & 63) * kLdt + (e >> 6)] = g[e];
  __syncthreads();
}
__device__ void wg_store64(const double* s, double* g) {
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) g[e] = s[(e & 63) * kLdt + (e >> 6)];
  __syncthreads();
}
// symmetric G from its accumulated upper storage (col-major, ld 64)
__device__ void wg_load_sym(const double* g, double* s) {
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int i = e & 63, j = e >> 6;
    s[i * kLdt + j] = (i <= j) ? g[i + j * 64] : g[j + i * 64];
  }
  __syncthreads();
}


}  // namespace lsq
