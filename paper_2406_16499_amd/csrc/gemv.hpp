// Masked skinny GEMV kernels (bandwidth-oriented) for the vector side of the
// refinement: triangular-inverse products, aggregated reflector application
// and products with blocks of the triangular factors.
//
// A is column-major (lda) in storage type S; vectors and arithmetic in TC.
// Masks relative to a diagonal offset d (entry (i, j) of the block):
//   kDense      every entry;
//   kUpper      entries with i - j <= d (an upper triangle shifted by d);
//   kUnitLower  entries with i - j > d, and 1 where i - j == d (unit lower).
// N: y[i] += alpha sum_j op(A)[i][j] x[j]   (one row per thread, 64 columns
//    per work-group, eight independent accumulators, atomic accumulation);
// T: s[j] += alpha sum_i op(A)[i][j] y[i]   (rows across the lanes, 16
//    columns per work-group, one accumulator per column, block reduction).
// Work-groups whose whole tile is masked out return at once.
#pragma once
#include <algorithm>
#include <cstdint>
#include "common.hpp"

namespace lsq {

enum GemvMask : int { kDense = 0, kUpper = 1, kUnitLower = 2 };

template <int MASK, typename TC>
__device__ __forceinline__ TC gemv_masked(TC a, int i, int j, int d) {
  if (MASK == kUpper) return (i - j <= d) ? a : (TC)0;
  if (MASK == kUnitLower) return (i - j > d) ? a : ((i - j == d) ? (TC)1 : (TC)0);
  return a;
}

template <typename S, typename TC, int MASK>
__global__ __launch_bounds__(256) void k_gemv_n(const S* __restrict__ A, int lda, int rows, int cols,
                                                int d, TC alpha, const TC* __restrict__ x,
                                                TC* __restrict__ y) {
  constexpr int CB = 64;
  __shared__ TC xs[CB];
  LSQ_LDS_POISON(xs);
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * 256, c0 = blockIdx.y * CB;
  const int ce = min(cols, c0 + CB);
  if (MASK == kUpper && r0 - (ce - 1) > d) return;          // every row below the band
  if (MASK == kUnitLower && (r0 + 255) - c0 < d) return;     // every row above the band
  if (t < CB) xs[t] = (c0 + t < cols) ? x[c0 + t] : (TC)0;
  __syncthreads();
  const int i = r0 + t;
  if (i >= rows) return;
  TC acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = (TC)0;
  int j = c0;
  for (; j + 8 <= ce; j += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const TC a = gemv_masked<MASK>((TC)A[(size_t)i + (size_t)(j + u) * lda], i, j + u, d);
      acc[u] = fma(a, xs[j + u - c0], acc[u]);
    }
  }
  for (; j < ce; ++j) {
    const TC a = gemv_masked<MASK>((TC)A[(size_t)i + (size_t)j * lda], i, j, d);
    acc[0] = fma(a, xs[j - c0], acc[0]);
  }
  const TC s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  if (s != (TC)0) atomicAdd(&y[i], alpha * s);
}

template <typename S, typename TC, int MASK>
__global__ __launch_bounds__(256) void k_gemv_t(const S* __restrict__ A, int lda, int rows, int cols,
                                                int d, TC alpha, const TC* __restrict__ yv,
                                                TC* __restrict__ s, int rows_per_block) {
  constexpr int NC = 16;
  __shared__ TC red[4][NC];
  LSQ_LDS_POISON(red);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c0 = blockIdx.x * NC;
  const int rb = blockIdx.y * rows_per_block, re = min(rows, rb + rows_per_block);
  const int cl = min(cols, c0 + NC) - 1;
  if (MASK == kUpper && rb - cl > d) return;
  if (MASK == kUnitLower && (re - 1) - c0 < d) return;
  TC acc[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) acc[u] = (TC)0;
  for (int i = rb + t; i < re; i += 256) {
    const TC yi = yv[i];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int j = c0 + u;
      if (j < cols) {
        const TC a = gemv_masked<MASK>((TC)A[(size_t)i + (size_t)j * lda], i, j, d);
        acc[u] = fma(a, yi, acc[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const TC v = wave_sum(acc[u]);
    if (lane == 0) red[w][u] = v;
  }
  __syncthreads();
  if (t < NC && c0 + t < cols) {
    const TC v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    if (v != (TC)0) atomicAdd(&s[c0 + t], alpha * v);
  }
}

// T with 16-byte loads: each lane takes VN = 16 / sizeof(S) consecutive rows
// of a column per load (a pass of the work-group covers 256 VN rows), eight
// columns per work-group, the column loads of a pass all issued before the
// first product.  Needs A 16-byte aligned, lda a multiple of VN and
// rows_per_block a multiple of 256 VN; a ragged last group of rows falls back
// to scalar loads.
template <typename S> struct Vec16 {};
template <> struct Vec16<float> { using T = float4; static constexpr int N = 4; };
template <> struct Vec16<double> { using T = double2; static constexpr int N = 2; };

template <typename S, typename TC, int MASK>
__global__ __launch_bounds__(256) void k_gemv_tv(const S* __restrict__ A, int lda, int rows, int cols,
                                                 int d, TC alpha, const TC* __restrict__ yv,
                                                 TC* __restrict__ s, int rows_per_block) {
  using V = typename Vec16<S>::T;
  constexpr int VN = Vec16<S>::N;
  constexpr int NC = 8;
  __shared__ TC red[4][NC];
  LSQ_LDS_POISON(red);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c0 = blockIdx.x * NC;
  const int rb = blockIdx.y * rows_per_block, re = min(rows, rb + rows_per_block);
  const int cl = min(cols, c0 + NC) - 1;
  if (MASK == kUpper && rb - cl > d) return;
  if (MASK == kUnitLower && (re - 1) - c0 < d) return;
  TC acc[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) acc[u] = (TC)0;
  for (int i0 = rb + VN * t; i0 < re; i0 += VN * 256) {
    if (i0 + VN <= re) {
      V a[NC];
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int j = c0 + u < cols ? c0 + u : cols - 1;     // a column past the end: re-read, unused
        a[u] = *reinterpret_cast<const V*>(A + (size_t)i0 + (size_t)j * lda);
      }
      TC yi[VN];
#pragma unroll
      for (int q = 0; q < VN; ++q) yi[q] = yv[i0 + q];
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        if (c0 + u >= cols) continue;
        const S* av = reinterpret_cast<const S*>(&a[u]);
#pragma unroll
        for (int q = 0; q < VN; ++q)
          acc[u] = fma(gemv_masked<MASK>((TC)av[q], i0 + q, c0 + u, d), yi[q], acc[u]);
      }
    } else {
      for (int i = i0; i < re; ++i) {
        const TC yi = yv[i];
#pragma unroll
        for (int u = 0; u < NC; ++u)
          if (c0 + u < cols)
            acc[u] = fma(gemv_masked<MASK>((TC)A[(size_t)i + (size_t)(c0 + u) * lda], i, c0 + u, d), yi, acc[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const TC v = wave_sum(acc[u]);
    if (lane == 0) red[w][u] = v;
  }
  __syncthreads();
  if (t < NC && c0 + t < cols) {
    const TC v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    if (v != (TC)0) atomicAdd(&s[c0 + t], alpha * v);
  }
}

// Launchers (stream-ordered; y / s must hold the values to accumulate onto).
// det: no two work-groups of one launch add into the same element, so the
// sums do not depend on the order the work-groups finish in (gemv_n then
// launches its 64-column blocks one after another; gemv_t gives each
// 16-column group one work-group for all the rows).
template <typename S, typename TC, int MASK>
void gemv_n(hipStream_t st, const S* A, int lda, int rows, int cols, int d, TC alpha, const TC* x, TC* y,
            bool det = false) {
  if (rows <= 0 || cols <= 0) return;
  if (det) {
    // block c holds columns 64 c .. : column j' of the block is j = j' + 64 c,
    // so the mask's offset becomes d + 64 c
    for (int c0 = 0; c0 < cols; c0 += 64)
      hipLaunchKernelGGL((k_gemv_n<S, TC, MASK>), dim3(ceil_div(rows, 256), 1), dim3(256), 0, st,
                         A + (size_t)c0 * lda, lda, rows, cols - c0 < 64 ? cols - c0 : 64, d + c0, alpha,
                         x + c0, y);
    return;
  }
  hipLaunchKernelGGL((k_gemv_n<S, TC, MASK>), dim3(ceil_div(rows, 256), ceil_div(cols, 64)), dim3(256), 0,
                     st, A, lda, rows, cols, d, alpha, x, y);
}

template <typename S, typename TC, int MASK>
void gemv_t(hipStream_t st, const S* A, int lda, int rows, int cols, int d, TC alpha, const TC* yv, TC* s,
            bool det = false) {
  if (rows <= 0 || cols <= 0) return;
  constexpr int VN = 16 / (int)sizeof(S);
  if constexpr (sizeof(S) == 4 || sizeof(S) == 8) {
    if (reinterpret_cast<uintptr_t>(A) % 16 == 0 && lda % VN == 0) {
      // one pass of 256 VN rows per work-group, up to about 4096 work-groups
      const int nbx = ceil_div(cols, 8), pass = 256 * VN;
      int nby = std::min(ceil_div(rows, pass), ceil_div(4096, nbx));
      if (nby < 1 || det) nby = 1;
      const int rpb = ceil_div(ceil_div(rows, nby), pass) * pass;
      nby = ceil_div(rows, rpb);
      hipLaunchKernelGGL((k_gemv_tv<S, TC, MASK>), dim3(nbx, nby), dim3(256), 0, st, A, lda, rows, cols, d,
                         alpha, yv, s, rpb);
      return;
    }
  }
  const int nbx = ceil_div(cols, 16);
  int nby = ceil_div(rows, 256);
  const int want = ceil_div(2048, nbx);
  if (nby > want) nby = want;
  if (nby < 1 || det) nby = 1;
  const int rpb = ceil_div(ceil_div(rows, nby), 256) * 256;
  nby = ceil_div(rows, rpb);
  hipLaunchKernelGGL((k_gemv_t<S, TC, MASK>), dim3(nbx, nby), dim3(256), 0, st, A, lda, rows, cols, d,
                     alpha, yv, s, rpb);
}

}  // namespace lsq
