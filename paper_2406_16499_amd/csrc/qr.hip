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
#include "engine.hpp"

namespace lsq {

constexpr int kLdt = kMaxNb + 1;   // padded LDS row stride for 64-wide FP64 tiles
constexpr int kPanRows = 256;      // rows per work-group in the panel passes
constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

// ---------------------------------------------------------------------------
// Panel pass: optional right-multiplication by an upper triangular Rinv,
// optional store of the product, and a partial Gram matrix per work-group.
// ---------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(256) void k_panel_pass(
    const Tin* __restrict__ X, int ldx, int mr, int jb,
    const double* __restrict__ Rinv,   // 64 x 64 column-major, zero outside the upper jb x jb
    double* __restrict__ Xout, int ldo,
    double* __restrict__ Gpart) {      // [gridDim.x][64 * 64]
  __shared__ double tile[64 * kLdt];
  __shared__ double rinv[64 * kLdt];
  const int t = threadIdx.x;
  const bool use_r = Rinv != nullptr;
  if (use_r) {
    for (int e = t; e < 64 * 64; e += 256) {
      const int i = e & 63, j = e >> 6;
      rinv[i * kLdt + j] = Rinv[i + j * 64];
    }
  }
  double g[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) g[q] = 0.0;
  const int a = t & 63, bq = (t >> 6) * 16;
  const int row0 = blockIdx.x * kPanRows;
  for (int sub = 0; sub < kPanRows; sub += 64) {
    const int rb = row0 + sub;
    if (rb >= mr) break;
    __syncthreads();
    for (int e = t; e < 64 * 64; e += 256) {
      const int i = e & 63, j = e >> 6;
      double v = 0.0;
      if (rb + i < mr && j < jb) v = (double)X[(size_t)(rb + i) + (size_t)j * ldx];
      tile[i * kLdt + j] = v;
    }
    __syncthreads();
    if (use_r) {
      const int i = t & 63, c0 = (t >> 6) * 16;
      double o[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) o[q] = 0.0;
      for (int kk = 0; kk < 64; ++kk) {
        const double v = tile[i * kLdt + kk];
#pragma unroll
        for (int q = 0; q < 16; ++q) o[q] += v * rinv[kk * kLdt + c0 + q];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 16; ++q) tile[i * kLdt + c0 + q] = o[q];
      __syncthreads();
      if (Xout) {
        for (int e = t; e < 64 * 64; e += 256) {
          const int ii = e & 63, j = e >> 6;
          if (rb + ii < mr && j < jb) Xout[(size_t)(rb + ii) + (size_t)j * ldo] = tile[ii * kLdt + j];
        }
      }
    }
    for (int i = 0; i < 64; ++i) {
      const double va = tile[i * kLdt + a];
#pragma unroll
      for (int q = 0; q < 16; ++q) g[q] += va * tile[i * kLdt + bq + q];
    }
  }
  double* out = Gpart + (size_t)blockIdx.x * 4096;
#pragma unroll
  for (int q = 0; q < 16; ++q) out[a + (bq + q) * 64] = g[q];
}

// --- small dense helpers for one 256-thread work-group, LDS row-major [64][kLdt]

// Cholesky G = R^T R in place (upper triangle of G becomes R).  Returns false
// (uniformly) if a pivot is not positive; the pivot is then replaced by a
// tiny positive value so that the computation stays finite.
__device__ bool wg_cholesky(double* G, int jb) {
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < jb; ++k) {
    if (t == 0) {
      double dkk = G[k * kLdt + k];
      if (!(dkk > 0.0)) {
        bad = 1;
        dkk = 1e-300;
      }
      G[k * kLdt + k] = sqrt(dkk);
    }
    __syncthreads();
    const double piv = G[k * kLdt + k];
    if (t > k && t < jb) G[k * kLdt + t] /= piv;
    __syncthreads();
    const int w = jb - k - 1;
    for (int e = t; e < w * w; e += 256) {
      const int i = k + 1 + e % w, j = k + 1 + e / w;
      if (i <= j) G[i * kLdt + j] -= G[k * kLdt + i] * G[k * kLdt + j];
    }
    __syncthreads();
  }
  // clear the strictly lower part so G holds exactly R
  for (int e = t; e < 64 * 64; e += 256) {
    const int i = e & 63, j = e >> 6;
    if (i > j || i >= jb || j >= jb) G[i * kLdt + j] = 0.0;
  }
  __syncthreads();
  return bad == 0;
}

// Inverse of an upper triangular R (jb x jb) into Ri (zero elsewhere).
__device__ void wg_upper_inverse(const double* R, double* Ri, int jb) {
  const int t = threadIdx.x;
  for (int e = t; e < 64 * 64; e += 256) Ri[(e & 63) * kLdt + (e >> 6)] = 0.0;
  __syncthreads();
  if (t < jb) {
    const int j = t;                   // column j of R^{-1}: back substitution
    Ri[j * kLdt + j] = 1.0 / R[j * kLdt + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int kk = i + 1; kk <= j; ++kk) s += R[i * kLdt + kk] * Ri[kk * kLdt + j];
      Ri[i * kLdt + j] = -s / R[i * kLdt + i];
    }
  }
  __syncthreads();
}

// C = A * B for 64 x 64 row-major LDS matrices (C must not alias A or B).
__device__ void wg_matmul(const double* A, const double* B, double* C) {
  const int t = threadIdx.x;
  for (int e = t; e < 64 * 64; e += 256) {
    const int i = e >> 6, j = e & 63;
    double s = 0.0;
    for (int kk = 0; kk < 64; ++kk) s += A[i * kLdt + kk] * B[kk * kLdt + j];
    C[i * kLdt + j] = s;
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
}

__device__ void wg_sum_parts(const double* Gpart, int nparts, double* G) {
  for (int e = threadIdx.x; e < 4096; e += 256) {
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += Gpart[(size_t)q * 4096 + e];
    G[(e & 63) * kLdt + (e >> 6)] = s;
  }
  __syncthreads();
}

// Cholesky step of a pass: G = sum of partials (+ shift), R = chol(G),
// Rinv = R^{-1}, Racc <- R * Racc (or R when first).
__global__ __launch_bounds__(256) void k_panel_chol(
    const double* __restrict__ Gpart, int nparts, int jb, int mr, int shift, int first,
    double* __restrict__ Rinv_out, double* __restrict__ Racc, int* __restrict__ status) {
  __shared__ double G[64 * kLdt];
  __shared__ double B1[64 * kLdt];
  __shared__ double B2[64 * kLdt];
  __shared__ double red[4];
  const int t = threadIdx.x;
  wg_sum_parts(Gpart, nparts, G);
  if (shift) {
    double tr = 0.0;
    for (int i = t; i < jb; i += 256) tr += G[i * kLdt + i];
    tr = block_sum(tr, red);
    const double sigma = 11.0 * ((double)mr * jb + (double)jb * (jb + 1)) * kU64 * tr;
    if (t < jb) G[t * kLdt + t] += sigma;
    __syncthreads();
  }
  const bool ok = wg_cholesky(G, jb);
  if (!ok && t == 0) atomicOr(status, 1);
  wg_upper_inverse(G, B1, jb);
  wg_store64(B1, Rinv_out);
  __syncthreads();
  if (first) {
    wg_store64(G, Racc);
  } else {
    wg_load64(Racc, B1);
    wg_matmul(G, B1, B2);
    wg_store64(B2, Racc);
  }
}

// Final panel step: last Cholesky, Householder reconstruction, compact-WY T.
// Q2 = Q1 R2^{-1} is the orthonormal basis; its top block gives the modified
// LU  Q2top - S = L1 U,  T = -U S L1^{-T},  R = S * R2 * Racc.  Mmat = (U R2)^{-1}
// maps Q1's lower rows to the lower Householder vectors.
template <typename Tw>
__global__ __launch_bounds__(256) void k_panel_final(
    const double* __restrict__ Gpart, int nparts, int jb,
    const double* __restrict__ Q1, int ldq,           // FP64 panel basis before the last pass
    double* __restrict__ Racc, Tw* __restrict__ Mst, int ldm, int j0,
    Tw* __restrict__ Tout, double* __restrict__ Mmat, int* __restrict__ status) {
  __shared__ double R2[64 * kLdt];
  __shared__ double A[64 * kLdt];
  __shared__ double B[64 * kLdt];
  __shared__ double sgn[64];
  const int t = threadIdx.x;
  wg_sum_parts(Gpart, nparts, R2);
  if (!wg_cholesky(R2, jb) && t == 0) atomicOr(status, 1);
  // Racc_final = R2 * Racc  -> B
  wg_load64(Racc, A);
  wg_matmul(R2, A, B);
  wg_store64(B, Racc);                       // keep R_total for the writer below
  // A = R2^{-1}
  __syncthreads();
  wg_upper_inverse(R2, A, jb);
  // B = Q2top = Q1top * R2^{-1}
  for (int e = t; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    double s = 0.0;
    if (i < jb && j < jb)
      for (int kk = 0; kk <= j; ++kk) s += Q1[i + (size_t)kk * ldq] * A[kk * kLdt + j];
    B[i * kLdt + j] = s;
  }
  __syncthreads();
  // modified LU without pivoting of B - S (in place: L strictly lower, U upper)
  for (int kk = 0; kk < jb; ++kk) {
    if (t == 0) {
      const double dkk = B[kk * kLdt + kk];
      const double s = dkk >= 0.0 ? -1.0 : 1.0;
      sgn[kk] = s;
      B[kk * kLdt + kk] = dkk - s;
    }
    __syncthreads();
    const double piv = B[kk * kLdt + kk];
    if (t > kk && t < jb) B[t * kLdt + kk] /= piv;
    __syncthreads();
    const int w = jb - kk - 1;
    for (int e = t; e < w * w; e += 256) {
      const int i = kk + 1 + e % w, j = kk + 1 + e / w;
      B[i * kLdt + j] -= B[i * kLdt + kk] * B[kk * kLdt + j];
    }
    __syncthreads();
  }
  // T = -U S L1^{-T}: row i of T solves L1 * T[i,:]^T = -(U S)[i,:]^T (forward subst.)
  // Store T in A (A's R2^{-1} is consumed below first: compute Mmat before T).
  // Mmat = (U R2)^{-1} = R2^{-1} U^{-1}:  first U^{-1} into R2's slot? R2 is needed;
  // compute P = U * R2 into the T-slot, invert it.
  __shared__ double P[64 * kLdt];
  for (int e = t; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    double s = 0.0;
    if (i < jb && j < jb && i <= j)
      for (int kk = i; kk <= j; ++kk) s += B[i * kLdt + kk] * R2[kk * kLdt + j];
    P[i * kLdt + j] = s;
  }
  __syncthreads();
  wg_upper_inverse(P, A, jb);                // A = (U R2)^{-1}
  wg_store64(A, Mmat);
  __syncthreads();
  // T into P
  if (t < jb) {
    const int i = t;
    for (int j = 0; j < 64; ++j) P[i * kLdt + j] = 0.0;
    // unknowns tr[j], j = 0..jb-1: sum_{k<=j} L1[j][k] tr[k] = -(U[i][j] * s_j), L1 unit lower
    for (int j = 0; j < jb; ++j) {
      double rhs = (j >= i) ? -B[i * kLdt + j] * sgn[j] : 0.0;
      for (int kk = 0; kk < j; ++kk) rhs -= B[j * kLdt + kk] * P[i * kLdt + kk];
      P[i * kLdt + j] = rhs;
    }
  }
  __syncthreads();
  for (int e = t; e < 4096; e += 256) {
    const int i = e & 63, j = e >> 6;
    Tout[e] = (i < jb && j < jb && i <= j) ? (Tw)P[i * kLdt + j] : (Tw)0;
  }
  // R_final = S * R_total (Racc): rows scaled by the signs; write R and L1 into M.
  for (int e = t; e < jb * jb; e += 256) {
    const int i = e % jb, j = e / jb;
    double v;
    if (i <= j) v = sgn[i] * Racc[i + j * 64];
    else v = B[i * kLdt + j];
    Mst[(size_t)(j0 + i) + (size_t)(j0 + j) * ldm] = (Tw)v;
  }
}

// Householder vectors of the rows below the panel's top block (Y = Q1 Mmat)
// and Yhat = Y T^T for all panel rows.
template <typename Tw>
__global__ __launch_bounds__(256) void k_panel_y(
    const double* __restrict__ Q1, int ldq, const double* __restrict__ Mmat,
    const Tw* __restrict__ Tin, Tw* __restrict__ Mst, int ldm, int j0, int mr, int jb,
    Tw* __restrict__ Yhat, int ldy) {
  __shared__ double tile[64 * kLdt];
  __shared__ double mm[64 * kLdt];
  __shared__ double tt[64 * kLdt];
  const int t = threadIdx.x;
  for (int e = t; e < 4096; e += 256) {
    mm[(e & 63) * kLdt + (e >> 6)] = Mmat[e];
    tt[(e & 63) * kLdt + (e >> 6)] = (double)Tin[e];
  }
  const int row0 = blockIdx.x * kPanRows;
  for (int sub = 0; sub < kPanRows; sub += 64) {
    const int rb = row0 + sub;
    if (rb >= mr) break;
    __syncthreads();
    for (int e = t; e < 4096; e += 256) {
      const int i = e & 63, j = e >> 6;
      tile[i * kLdt + j] = (rb + i < mr && j < jb) ? Q1[(size_t)(rb + i) + (size_t)j * ldq] : 0.0;
    }
    __syncthreads();
    const int i = t & 63, c0 = (t >> 6) * 16;
    const int row = rb + i;
    double y[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) y[q] = 0.0;
    if (row >= jb) {
      for (int kk = 0; kk < 64; ++kk) {
        const double v = tile[i * kLdt + kk];
#pragma unroll
        for (int q = 0; q < 16; ++q) y[q] += v * mm[kk * kLdt + c0 + q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = c0 + q;
        y[q] = (c < jb) ? (row > c ? (double)Mst[(size_t)(j0 + row) + (size_t)(j0 + c) * ldm]
                                   : (row == c ? 1.0 : 0.0))
                        : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + q;
      const Tw yr = (Tw)y[q];
      if (row >= jb && row < mr && c < jb) Mst[(size_t)(j0 + row) + (size_t)(j0 + c) * ldm] = yr;
      tile[i * kLdt + c] = (c < jb) ? (double)yr : 0.0;
    }
    __syncthreads();
    // Yhat[row][c] = sum_k Y[row][k] * T[c][k]   (T upper: k >= c)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + q;
      double s = 0.0;
      for (int kk = c; kk < 64; ++kk) s += tile[i * kLdt + kk] * tt[c * kLdt + kk];
      if (row < mr && c < 64) Yhat[(size_t)row + (size_t)c * ldy] = (Tw)s;
    }
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
  __device__ static V mma(const In* a, const In* b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return (float)v; }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MmaT<Mma::F64> {
  using In = double; using Acc = double; using V = f64x4;
  static constexpr int KI = 4, KL = 1, PAD = 2;
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
  __device__ static V mma(const In* a, const In* b, V c) {
    const f16x8 av = *reinterpret_cast<const f16x8*>(a);
    const f16x8 bv = *reinterpret_cast<const f16x8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
  __device__ static In cvt(double v) { return (_Float16)(float)v; }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

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
// Y is read from the factor storage with the unit-lower mask.
template <typename Tw, Mma MT>
__global__ __launch_bounds__(256) void k_wy_t(
    const Tw* __restrict__ Y, int ldy, int mr, int jb,      // Y = &M[j0 + j0*ld]
    const Tw* __restrict__ C, int ldc, int nc, int kch,     // C = &target[j0 + cstart*ldc]
    typename MmaT<MT>::Acc* __restrict__ Wpart) {
  using T = MmaT<MT>;
  constexpr int BK = (T::KI > 16) ? 32 : 32;
  constexpr int LD = BK + T::PAD;
  __shared__ __attribute__((aligned(16))) typename T::In As[64 * LD];
  __shared__ __attribute__((aligned(16))) typename T::In Bs[64 * LD];
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
  for (int k = kbeg; k < kend; k += BK) {
    __syncthreads();
    for (int e = t; e < 64 * BK; e += 256) {
      const int kk = e % BK, a = e / BK;
      const int i = k + kk;
      double v = 0.0;
      if (i < kend && a < jb) {
        if (i > a) v = (double)Y[(size_t)i + (size_t)a * ldy];
        else if (i == a) v = 1.0;
      }
      As[a * LD + kk] = T::cvt(v);
    }
    for (int e = t; e < 64 * BK; e += 256) {
      const int kk = e % BK, c = e / BK;
      const int i = k + kk;
      double v = 0.0;
      if (i < kend && c0 + c < nc) v = (double)C[(size_t)i + (size_t)(c0 + c) * ldc];
      Bs[c * LD + kk] = T::cvt(v);
    }
    __syncthreads();
    mma_block<MT, BK>(As, Bs, acc);
  }
  const int l = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  typename T::Acc* out = Wpart + (size_t)blockIdx.y * 64 * nc;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 32 * wr + 16 * bi + T::row(l, r);
        const int c = c0 + 32 * wc + 16 * bj + (l & 15);
        if (c < nc) out[a + (size_t)c * 64] = acc[bi][bj][r];
      }
}

template <typename Acc>
__global__ void k_wy_reduce(const Acc* __restrict__ Wpart, int nsplit, int total,
                            Acc* __restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  Acc s = 0;
  for (int q = 0; q < nsplit; ++q) s += Wpart[(size_t)q * total + e];
  W[e] = s;
}

// C (mr x nc) -= Yhat (mr x jb) * W (jb x nc).
template <typename Tw, Mma MT>
__global__ __launch_bounds__(256) void k_wy_u(
    const Tw* __restrict__ Yhat, int ldy, int mr, int jb,
    const typename MmaT<MT>::Acc* __restrict__ W, Tw* __restrict__ C, int ldc, int nc) {
  using T = MmaT<MT>;
  constexpr int BK = 64;
  constexpr int LD = BK + T::PAD;
  __shared__ __attribute__((aligned(16))) typename T::In As[64 * LD];
  __shared__ __attribute__((aligned(16))) typename T::In Bs[64 * LD];
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  for (int e = t; e < 64 * 64; e += 256) {
    const int i = e & 63, a = e >> 6;
    double v = (r0 + i < mr && a < jb) ? (double)Yhat[(size_t)(r0 + i) + (size_t)a * ldy] : 0.0;
    As[i * LD + a] = T::cvt(v);
  }
  for (int e = t; e < 64 * 64; e += 256) {
    const int a = e & 63, c = e >> 6;
    double v = (a < jb && c0 + c < nc) ? (double)W[a + (size_t)(c0 + c) * 64] : 0.0;
    Bs[c * LD + a] = T::cvt(v);
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
  const int l = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + 32 * wr + 16 * bi + T::row(l, r);
        const int c = c0 + 32 * wc + 16 * bj + (l & 15);
        if (i < mr && c < nc) {
          Tw* p = C + (size_t)i + (size_t)c * ldc;
          *p = (Tw)((double)*p - (double)acc[bi][bj][r]);
        }
      }
}

// ---------------------------------------------------------------------------
// Application of the block reflectors to a vector (cooperative launch).
// Each work-group owns a contiguous range of rows; per panel: partial
// s = Y^T y over own rows, grid barrier, s = sum of partials, t = T^T s
// (for Q^T) or T s (for Q), y -= Y t over own rows.
// ---------------------------------------------------------------------------
template <typename Tc>
__device__ __forceinline__ void butterfly64(Tc v[64]) {
  // reduce-scatter across the wave: afterwards v[0] of lane l holds the sum over
  // all lanes of the original v[l].
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int m = 32, c = 64; m >= 1; m >>= 1, c >>= 1) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < c / 2; ++i) {
      const Tc send = up ? v[i] : v[i + c / 2];
      const Tc keep = up ? v[i + c / 2] : v[i];
      v[i] = keep + __shfl_xor(send, m, 64);
    }
  }
}

template <typename Tw, typename Tc>
__global__ __launch_bounds__(256) void k_apply_q_vec(
    const Tw* __restrict__ M, int ld, int r, int k, int nb, const Tw* __restrict__ Tb,
    int trans, Tc* __restrict__ y, Tc* __restrict__ part, int rows_per_wg,
    unsigned* bar, int* err) {
  __shared__ Tc red[4][64];
  __shared__ Tc svec[64];
  __shared__ Tc tvec[64];
  __shared__ Tc tmat[64 * 65];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int np = ceil_div(k, nb);
  const int rbeg = g * rows_per_wg, rend = min(r, rbeg + rows_per_wg);
  for (int step = 0; step < np; ++step) {
    const int pj = trans ? step : (np - 1 - step);
    const int j0 = pj * nb, jb = min(nb, k - j0);
    const Tw* Y = M + (size_t)j0 * ld;     // column j0; rows indexed globally
    // partial s = sum_rows Y[row][a] y[row], rows in [max(rbeg, j0), rend)
    Tc acc[64];
#pragma unroll
    for (int a = 0; a < 64; ++a) acc[a] = 0;
    const int lo = max(rbeg, j0);
    for (int row = lo + t; row < rend; row += 256) {
      const Tc yr = y[row];
      const int rr = row - j0;
#pragma unroll
      for (int a = 0; a < 64; ++a) {
        Tc yv = 0;
        if (a < jb) yv = rr > a ? (Tc)Y[(size_t)row + (size_t)a * ld] : (rr == a ? (Tc)1 : (Tc)0);
        acc[a] += yv * yr;
      }
    }
    butterfly64<Tc>(acc);
    red[w][lane] = acc[0];
    __syncthreads();
    Tc* mypart = part + ((size_t)(step & 1) * G + g) * 64;
    if (t < 64) mypart[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    // load T_j while waiting
    const Tw* Tj = Tb + (size_t)pj * 4096;
    for (int e = t; e < 4096; e += 256) tmat[(e & 63) * 65 + (e >> 6)] = (Tc)Tj[e];
    grid_barrier(bar, G, err);
    if (t < 64) {
      Tc s = 0;
      const Tc* pp = part + (size_t)(step & 1) * G * 64;
      for (int q = 0; q < G; ++q) s += __hip_atomic_load(&pp[q * 64 + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      svec[t] = s;
    }
    __syncthreads();
    if (t < 64) {
      Tc s = 0;
      if (trans) {   // t = T^T s : t_i = sum_{k<=i} T[k][i] s_k
        for (int kk = 0; kk <= t; ++kk) s += tmat[kk * 65 + t] * svec[kk];
      } else {       // t = T s : t_i = sum_{k>=i} T[i][k] s_k
        for (int kk = t; kk < 64; ++kk) s += tmat[t * 65 + kk] * svec[kk];
      }
      tvec[t] = s;
    }
    __syncthreads();
    for (int row = lo + t; row < rend; row += 256) {
      const int rr = row - j0;
      Tc s = 0;
#pragma unroll
      for (int a = 0; a < 64; ++a) {
        Tc yv = 0;
        if (a < jb) yv = rr > a ? (Tc)Y[(size_t)row + (size_t)a * ld] : (rr == a ? (Tc)1 : (Tc)0);
        s += yv * tvec[a];
      }
      y[row] -= s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host side

static size_t elem(int tw) { return (size_t)tw; }

void qr_alloc(Ctx& ctx, QRFactor& f, int r, int c, int tw, Mma mt, int nb) {
  f.r = r; f.c = c; f.k = r < c ? r : c; f.ld = r > 1 ? r : 1;
  f.nb = nb; f.np = ceil_div(f.k, nb); f.tw = tw; f.mt = mt;
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
                     Tw* C, int ldc, int nc) {
  using Acc = typename MmaT<MT>::Acc;
  if (nc <= 0 || mr <= 0) return;
  const int nct = ceil_div(nc, 64);
  int nsplit = ceil_div(1024, nct);
  const int maxsplit = ceil_div(mr, 64);
  if (nsplit > maxsplit) nsplit = maxsplit;
  if (nsplit < 1) nsplit = 1;
  int kch = ceil_div(ceil_div(mr, nsplit), 32) * 32;
  nsplit = ceil_div(mr, kch);
  Acc* Wpart = ctx.ws->get<Acc>((size_t)nsplit * 64 * nc);
  Acc* W = ctx.ws->get<Acc>((size_t)64 * nc);
  hipLaunchKernelGGL((k_wy_t<Tw, MT>), dim3(nct, nsplit), dim3(256), 0, ctx.stream,
                     Y, ldy, mr, jb, C, ldc, nc, kch, Wpart);
  LSQ_LAUNCH_CHECK();
  const int total = 64 * nc;
  hipLaunchKernelGGL((k_wy_reduce<Acc>), dim3(ceil_div(total, 256)), dim3(256), 0, ctx.stream,
                     Wpart, nsplit, total, W);
  LSQ_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_wy_u<Tw, MT>), dim3(ceil_div(mr, 64), nct), dim3(256), 0, ctx.stream,
                     Yhat, ldyh, mr, jb, W, C, ldc, nc);
  LSQ_LAUNCH_CHECK();
}

template <typename Tw, Mma MT>
static void qr_factor_t(Ctx& ctx, QRFactor& f) {
  Tw* M = static_cast<Tw*>(f.M);
  Tw* Tb = static_cast<Tw*>(f.T);
  Tw* Yh = static_cast<Tw*>(f.Yhat);
  const int r = f.r, ld = f.ld;
  double* Q0 = ctx.ws->get<double>((size_t)r * 64);
  double* Q1 = ctx.ws->get<double>((size_t)r * 64);
  const int maxparts = ceil_div(r, kPanRows);
  double* Gpart = ctx.ws->get<double>((size_t)maxparts * 4096);
  double* Rinv = ctx.ws->get<double>(4096);
  double* Racc = ctx.ws->get<double>(4096);
  double* Mmat = ctx.ws->get<double>(4096);
  for (int j = 0; j < f.np; ++j) {
    const int j0 = j * f.nb;
    const int jb = (f.k - j0) < f.nb ? (f.k - j0) : f.nb;
    const int mr = r - j0;
    const int parts = ceil_div(mr, kPanRows);
    Tw* P = M + (size_t)j0 + (size_t)j0 * ld;
    // pass 0: Gram of P, shifted Cholesky
    hipLaunchKernelGGL((k_panel_pass<Tw>), dim3(parts), dim3(256), 0, ctx.stream,
                       P, ld, mr, jb, (const double*)nullptr, (double*)nullptr, 0, Gpart);
    hipLaunchKernelGGL(k_panel_chol, dim3(1), dim3(256), 0, ctx.stream,
                       Gpart, parts, jb, mr, 1, 1, Rinv, Racc, f.status);
    // pass 1: Q0 = P R0^{-1}, Gram of Q0
    hipLaunchKernelGGL((k_panel_pass<Tw>), dim3(parts), dim3(256), 0, ctx.stream,
                       P, ld, mr, jb, Rinv, Q0, mr, Gpart);
    hipLaunchKernelGGL(k_panel_chol, dim3(1), dim3(256), 0, ctx.stream,
                       Gpart, parts, jb, mr, 0, 0, Rinv, Racc, f.status);
    // pass 2: Q1 = Q0 R1^{-1}, Gram of Q1
    hipLaunchKernelGGL((k_panel_pass<double>), dim3(parts), dim3(256), 0, ctx.stream,
                       Q0, mr, mr, jb, Rinv, Q1, mr, Gpart);
    // last Cholesky + reconstruction
    hipLaunchKernelGGL((k_panel_final<Tw>), dim3(1), dim3(256), 0, ctx.stream,
                       Gpart, parts, jb, Q1, mr, Racc, M, ld, j0, Tb + (size_t)j * 4096, Mmat,
                       f.status);
    hipLaunchKernelGGL((k_panel_y<Tw>), dim3(parts), dim3(256), 0, ctx.stream,
                       Q1, mr, Mmat, Tb + (size_t)j * 4096, M, ld, j0, mr, jb,
                       Yh + f.yoff[j], mr);
    LSQ_LAUNCH_CHECK();
    // trailing update of columns j0 + jb .. c-1
    const int nc = f.c - j0 - jb;
    wy_apply<Tw, MT>(ctx, P, ld, mr, jb, Yh + f.yoff[j], mr,
                     M + (size_t)j0 + (size_t)(j0 + jb) * ld, ld, nc);
  }
}

void qr_factor(Ctx& ctx, QRFactor& f) {
  if (f.k <= 0) return;
  if (f.tw == 8) {
    qr_factor_t<double, Mma::F64>(ctx, f);
  } else {
    switch (f.mt) {
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
      case Mma::BF16: apply_left_t<float, Mma::BF16>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
      case Mma::F16: apply_left_t<float, Mma::F16>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
      default: apply_left_t<float, Mma::F32>(ctx, f, static_cast<float*>(C), ldc, ncols); break;
    }
  }
}

template <typename Tw, typename Tc>
static void apply_vec_t(Ctx& ctx, const QRFactor& f, bool trans, Tc* y) {
  int G = ceil_div(f.r, 512);
  if (G > ctx.max_coop_blocks) G = ctx.max_coop_blocks;
  if (G > 64) G = 64;
  if (G < 1) G = 1;
  int rows = ceil_div(f.r, G);
  G = ceil_div(f.r, rows);
  Tc* part = ctx.ws->get<Tc>((size_t)2 * G * 64);
  const Tw* M = static_cast<const Tw*>(f.M);
  const Tw* Tb = static_cast<const Tw*>(f.T);
  int ld = f.ld, r = f.r, k = f.k, nb = f.nb, tr = trans ? 1 : 0;
  unsigned* bar = ctx.sync;
  int* err = ctx.err;
  void* args[] = {(void*)&M, (void*)&ld, (void*)&r, (void*)&k, (void*)&nb, (void*)&Tb,
                  (void*)&tr, (void*)&y, (void*)&part, (void*)&rows, (void*)&bar, (void*)&err};
  LSQ_HIP(hipLaunchCooperativeKernel((const void*)k_apply_q_vec<Tw, Tc>, dim3(G), dim3(256), args,
                                     0, ctx.stream));
}

void qr_apply_vec(Ctx& ctx, const QRFactor& f, bool trans, void* y, int tc) {
  if (f.k <= 0) return;
  if (f.tw == 8) {
    if (tc == 8) apply_vec_t<double, double>(ctx, f, trans, static_cast<double*>(y));
    else apply_vec_t<double, float>(ctx, f, trans, static_cast<float*>(y));
  } else {
    if (tc == 8) apply_vec_t<float, double>(ctx, f, trans, static_cast<double*>(y));
    else apply_vec_t<float, float>(ctx, f, trans, static_cast<float*>(y));
  }
}

}  // namespace lsq
