// Dense building blocks on MFMA: a masked, batched GEMM, the inverse of an
// upper triangular matrix by recursive doubling, and the GEMV kernels that
// apply aggregated block reflectors to a vector.  None of these kernels waits
// on another work-group.
#include "engine.hpp"
#include "wg64.hpp"
#include "gemv.hpp"

namespace lsq {

template <typename T> struct MmaOf;
template <> struct MmaOf<float> {
  using V = f32x4;
  static constexpr int PAD = 4;
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MmaOf<double> {
  using V = f64x4;
  static constexpr int PAD = 2;
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int r) { return 4 * r + (l >> 4); }
};

// Buffer loads: an offset past the resource's extent (kOobB) reads zero, so
// every load can be issued without a branch.
constexpr uint32_t kOobB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename S> __device__ __forceinline__ S bld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float bld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double bld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Element (i, j) of a masked operand, v as loaded from storage.  mask: 0
// dense, 1 upper (zero when i + off > j), 2 unit lower (value when i + off >
// j, 1 on the diagonal, zero above).
template <typename S>
__device__ __forceinline__ double mval(S v, int i, int j, int mask, int off) {
  double x = (double)v;
  if (mask == 1) x = (i + off > j) ? 0.0 : x;
  else if (mask == 2) x = (i + off < j) ? 0.0 : ((i + off == j) ? 1.0 : x);
  return x;
}

// C = alpha * op(A) op(B) + beta * C, op(X) = X or X^T; batched over
// blockIdx.z with element strides.  64 x 64 tile per 256-thread work-group.
struct GemmArgs {
  const void* A; int lda; long long sa; int ta; int ma; int oa;
  const void* B; int ldb; long long sb; int tb; int mb; int ob;
  void* C; int ldc; long long sc;
  int m, n, k;
  double alpha, beta;
  int ksplit;            // > 1: partial products over k-chunks go to Cpart[z % ksplit] (m x n, ld m)
  int kchunk;
  void* Cpart;
  // two-level batch: with bper > 0, batch entry z is item z % bper of group
  // z / bper, at offset (z % bper) s + (z / bper) s2 for each operand
  int bper;
  long long sa2, sb2, sc2;
};

template <typename SA, typename SB, typename TC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  using Mt = MmaOf<TC>;
  constexpr int BK = 32;
  constexpr int LD = BK + Mt::PAD;
  __shared__ TC As[64 * LD];
  __shared__ TC Bs[64 * LD];
  LSQ_LDS_POISON(As);
  LSQ_LDS_POISON(Bs);
  const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const int ks = g.ksplit > 1 ? g.ksplit : 1;
  const int bz = blockIdx.z / ks, kz = blockIdx.z % ks;
  const int bi = g.bper > 0 ? bz % g.bper : bz, bg = g.bper > 0 ? bz / g.bper : 0;
  const SA* A = static_cast<const SA*>(g.A) + (long long)bi * g.sa + (long long)bg * g.sa2;
  const SB* B = static_cast<const SB*>(g.B) + (long long)bi * g.sb + (long long)bg * g.sb2;
  TC* C = static_cast<TC*>(g.C) + (long long)bi * g.sc + (long long)bg * g.sc2;
  const int kbeg = ks > 1 ? kz * g.kchunk : 0;
  const int kend = ks > 1 ? min(g.k, kbeg + g.kchunk) : g.k;
  typename Mt::V acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
  // The next 32-deep chunk of op(A) and op(B) is fetched into registers while
  // the MFMAs of the current one run.  op(A)(row, kk): storage (row, kk) or
  // (kk, row); the fast index of each thread's elements follows storage rows.
  // Buffer loads over each operand's extent: out-of-range elements read as
  // zero, and the masks are applied to the loaded values.
  const int ta = g.ta, tb = g.tb, ma = g.ma, mb = g.mb, oa = g.oa, ob = g.ob;
  const size_t extA = g.k > 0 ? (ta ? (size_t)(g.m - 1) * g.lda + g.k : (size_t)(g.k - 1) * g.lda + g.m) : 1;
  const size_t extB = g.k > 0 ? (tb ? (size_t)(g.k - 1) * g.ldb + g.n : (size_t)(g.n - 1) * g.ldb + g.k) : 1;
  const auto rsA = brsrc(A, extA * sizeof(SA));
  const auto rsB = brsrc(B, extB * sizeof(SB));
  TC av[8], bv[8];
  auto fetch = [&](int k0) {
    SA ra[8];
    SB rb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      int row, kk;
      if (!ta) { row = e & 63; kk = e >> 6; } else { kk = e % BK; row = e / BK; }
      const int gi = r0 + row, gka = k0 + kk;
      const size_t oa_ = ta ? (size_t)gka + (size_t)gi * g.lda : (size_t)gi + (size_t)gka * g.lda;
      ra[q] = bld<SA>(rsA, ((gi < g.m) & (gka < kend)) ? (uint32_t)(oa_ * sizeof(SA)) : kOobB);
      int col, kb;
      if (!tb) { kb = e % BK; col = e / BK; } else { col = e & 63; kb = e >> 6; }
      const int gj = c0 + col, gkb = k0 + kb;
      const size_t ob_ = tb ? (size_t)gj + (size_t)gkb * g.ldb : (size_t)gkb + (size_t)gj * g.ldb;
      rb[q] = bld<SB>(rsB, ((gj < g.n) & (gkb < kend)) ? (uint32_t)(ob_ * sizeof(SB)) : kOobB);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      int row, kk;
      if (!ta) { row = e & 63; kk = e >> 6; } else { kk = e % BK; row = e / BK; }
      const int gi = r0 + row, gka = k0 + kk;
      av[q] = (TC)(ta ? mval(ra[q], gka, gi, ma, oa) : mval(ra[q], gi, gka, ma, oa));
      int col, kb;
      if (!tb) { kb = e % BK; col = e / BK; } else { col = e & 63; kb = e >> 6; }
      const int gj = c0 + col, gkb = k0 + kb;
      bv[q] = (TC)(tb ? mval(rb[q], gj, gkb, mb, ob) : mval(rb[q], gkb, gj, mb, ob));
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      int row, kk, col, kb;
      if (!g.ta) { row = e & 63; kk = e >> 6; } else { kk = e % BK; row = e / BK; }
      if (!g.tb) { kb = e % BK; col = e / BK; } else { col = e & 63; kb = e >> 6; }
      As[row * LD + kk] = av[q];
      Bs[col * LD + kb] = bv[q];
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TC a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a[q] = As[(32 * wr + 16 * q + (l & 15)) * LD + kk + (l >> 4)];
        b[q] = Bs[(32 * wc + 16 * q + (l & 15)) * LD + kk + (l >> 4)];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mt::mma(a[bi], b[bj], acc[bi][bj]);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + 32 * wr + 16 * bi + Mt::row(l, r);
        const int j = c0 + 32 * wc + 16 * bj + (l & 15);
        if (i < g.m && j < g.n && ks > 1) {
          static_cast<TC*>(g.Cpart)[(size_t)kz * g.m * g.n + i + (size_t)j * g.m] = acc[bi][bj][r];
        } else if (i < g.m && j < g.n) {
          TC* p = C + (size_t)i + (size_t)j * g.ldc;
          const double old = g.beta != 0.0 ? (double)*p : 0.0;
          *p = (TC)(g.alpha * (double)acc[bi][bj][r] + g.beta * old);
        }
      }
}

template <typename TC>
__global__ void k_ksum(const TC* __restrict__ part, int ks, int m, int n, double alpha, double beta,
                       TC* __restrict__ C, int ldc) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  double s = 0.0;
  for (int q = 0; q < ks; ++q) s += (double)part[(size_t)q * m * n + e];
  TC* p = C + (size_t)i + (size_t)j * ldc;
  *p = (TC)(alpha * s + (beta != 0.0 ? beta * (double)*p : 0.0));
}

// Launch; with few output tiles and a long k, the product is split over k
// (deterministic partials + one reduction kernel; batch must be 1 then).
template <typename SA, typename SB, typename TC>
static void gemm(Ctx& ctx, GemmArgs g, int batch) {
  if (g.m <= 0 || g.n <= 0 || batch <= 0) return;
  const int tiles = ceil_div(g.m, 64) * ceil_div(g.n, 64) * batch;
  g.ksplit = 1;
  if (batch == 1 && tiles < 256 && g.k >= 512) {
    int ks = ceil_div(512, tiles);
    const int kmax = g.k / 128;
    if (ks > kmax) ks = kmax;
    if (ks > 32) ks = 32;
    if (ks > 1) {
      g.kchunk = ceil_div(ceil_div(g.k, ks), 32) * 32;
      ks = ceil_div(g.k, g.kchunk);
      g.ksplit = ks;
      g.Cpart = ctx.ws->alloc(sizeof(TC) * (size_t)ks * g.m * g.n);
    }
  }
  dim3 grid(ceil_div(g.m, 64), ceil_div(g.n, 64), batch * g.ksplit);
  hipLaunchKernelGGL((k_gemm<SA, SB, TC>), grid, dim3(256), 0, ctx.stream, g);
  if (g.ksplit > 1) {
    const long long tot = (long long)g.m * g.n;
    hipLaunchKernelGGL((k_ksum<TC>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx.stream,
                       static_cast<const TC*>(g.Cpart), g.ksplit, g.m, g.n, g.alpha, g.beta,
                       static_cast<TC*>(g.C), g.ldc);
  }
  LSQ_LAUNCH_CHECK();
}

// ----------------------------------------------------- triangular inverse --
// Inverse of each 64 x 64 diagonal block; one work-group per block, FP64,
// blocked (16 x 16 diagonal blocks on four waves at once, MFMA products for
// the rest).  blockIdx.y selects the matrix of a batch (strides su, sx).
template <typename S, typename TC>
__global__ __launch_bounds__(512) void k_diag_inv(const S* __restrict__ U, int ldu, long long su, int mask,
                                                  int nn, TC* __restrict__ X, int ldx, long long sx) {
  __shared__ double R[64 * kLdt];
  __shared__ double Xs[64 * kLdt];
  LSQ_LDS_POISON(R);
  LSQ_LDS_POISON(Xs);
  U += (long long)blockIdx.y * su;
  X += (long long)blockIdx.y * sx;
  const int I = blockIdx.x, i0 = I * 64, ib = min(64, nn - i0);
  const int t = threadIdx.x;
  for (int e = t; e < 4096; e += 512) {
    const int i = e & 63, j = e >> 6;
    double v = 0.0;
    if (i < ib && j < ib && i <= j) v = mval(U[(size_t)(i0 + i) + (size_t)(i0 + j) * ldu], i0 + i, i0 + j, mask, 0);
    if (i == j && i >= ib) v = 1.0;
    R[i * kLdt + j] = v;
  }
  __syncthreads();
  blk_upper_inverse<8>(R, Xs);
  for (int e = t; e < 4096; e += 512) {
    const int i = e & 63, j = e >> 6;
    if (i < ib && j < ib) X[(size_t)(i0 + i) + (size_t)(i0 + j) * ldx] = (TC)Xs[i * kLdt + j];
  }
}

template <typename TC>
__global__ void k_zero_lower(TC* X, int ldx, long long sx, int nn, int nmat) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)nn * nn;
  if (e >= per * nmat) return;
  const long long q = e / per, r = e % per;
  const int i = (int)(r % nn), j = (int)(r / nn);
  if (i > j) X[q * sx + (size_t)i + (size_t)j * ldx] = (TC)0;
}

// X_q (nn x nn, ld ldx, type TC) = U_q^{-1} for the upper triangles of nmat
// matrices U_q = U + q su, X_q = X + q sx (type S, masked upper).  Off-diagonal
// blocks by recursive doubling: for a diagonal pair [A B; 0 C] of size 2b,
// X12 = -A^{-1} B C^{-1}; the pairs of every matrix at one level share two
// batched GEMMs.
template <typename S, typename TC>
void tri_inverse_batched(Ctx& ctx, const S* U, int ldu, long long su, int nn, TC* X, int ldx,
                         long long sx, int nmat) {
  if (nn <= 0 || nmat <= 0) return;
  const int nblk = ceil_div(nn, 64);
  const long long tot = (long long)nn * nn * nmat;
  hipLaunchKernelGGL((k_zero_lower<TC>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx.stream,
                     X, ldx, sx, nn, nmat);
  hipLaunchKernelGGL((k_diag_inv<S, TC>), dim3(nblk, nmat), dim3(512), 0, ctx.stream, U, ldu, su, 1, nn,
                     X, ldx, sx);
  LSQ_LAUNCH_CHECK();
  const long long tper = (long long)nn * 64 + (long long)nn * nn / 2 + 64;   // tmp per matrix
  TC* tmp = ctx.ws->get<TC>((size_t)tper * nmat);
  for (int b = 64; b < nn; b *= 2) {
    const int npairs = ceil_div(nn, 2 * b);
    // full pairs share one batched launch; a ragged last pair is launched alone
    const int full = nn / (2 * b);
    for (int pass = 0; pass < 2; ++pass) {
      const int cnt = pass == 0 ? full : npairs - full;
      if (cnt <= 0) continue;
      const int p0 = pass == 0 ? 0 : full;
      const int a0 = p0 * 2 * b, c0 = a0 + b;
      const int bw = min(b, nn - c0);          // width of the C block
      if (bw <= 0) continue;
      // tmp = B * C^{-1}   (b x bw);  B = U[a0:a0+b, c0:c0+bw],  C^{-1} = X[c0.., c0..]
      GemmArgs g1{};
      g1.A = U + (size_t)a0 + (size_t)c0 * ldu; g1.lda = ldu; g1.sa = (long long)2 * b * (ldu + 1); g1.ta = 0; g1.ma = 0; g1.oa = 0;
      g1.B = X + (size_t)c0 + (size_t)c0 * ldx; g1.ldb = ldx; g1.sb = (long long)2 * b * (ldx + 1); g1.tb = 0; g1.mb = 0; g1.ob = 0;
      g1.C = tmp; g1.ldc = b; g1.sc = (long long)b * b;
      g1.m = b; g1.n = bw; g1.k = bw; g1.alpha = 1.0; g1.beta = 0.0;
      g1.bper = cnt; g1.sa2 = su; g1.sb2 = sx; g1.sc2 = tper;
      gemm<S, TC, TC>(ctx, g1, cnt * nmat);
      // X12 = -A^{-1} tmp   (b x bw)
      GemmArgs g2{};
      g2.A = X + (size_t)a0 + (size_t)a0 * ldx; g2.lda = ldx; g2.sa = (long long)2 * b * (ldx + 1); g2.ta = 0; g2.ma = 0; g2.oa = 0;
      g2.B = tmp; g2.ldb = b; g2.sb = (long long)b * b; g2.tb = 0; g2.mb = 0; g2.ob = 0;
      g2.C = X + (size_t)a0 + (size_t)c0 * ldx; g2.ldc = ldx; g2.sc = (long long)2 * b * (ldx + 1);
      g2.m = b; g2.n = bw; g2.k = b; g2.alpha = -1.0; g2.beta = 0.0;
      g2.bper = cnt; g2.sa2 = sx; g2.sb2 = tper; g2.sc2 = sx;
      gemm<TC, TC, TC>(ctx, g2, cnt * nmat);
    }
  }
}

template <typename S, typename TC>
void tri_inverse(Ctx& ctx, const S* U, int ldu, int nn, TC* X, int ldx) {
  tri_inverse_batched<S, TC>(ctx, U, ldu, 0, nn, X, ldx, 0, 1);
}

// ------------------------------------------------- inverse-based solves --
// y += op(X) x for a dense upper triangular X (nn x nn): X x or X^T x.
// Partial row sums are added atomically into y, which holds the values to
// accumulate onto.
template <typename TC>
void trmv_dense(Ctx& ctx, const TC* X, int ldx, int nn, bool trans, const TC* x, TC* y) {
  if (nn <= 0) return;
  if (!trans)
    gemv_n<TC, TC, kUpper>(ctx.stream, X, ldx, nn, nn, 0, (TC)1, x, y, ctx.deterministic);
  else
    gemv_t<TC, TC, kUpper>(ctx.stream, X, ldx, nn, nn, 0, (TC)1, x, y, ctx.deterministic);
  LSQ_LAUNCH_CHECK();
}
// ---------------------------------------- aggregated reflector application --
// G = striu(Y^T Y) + diag(Y^T Y) / 2 for a unit-lower Y (rows x cols), dense
// output; nmat matrices n x n stored one after another (ld n).
template <typename TC>
__global__ void k_ut_fix(TC* G, int n, int nmat) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)n * n;
  if (e >= per * nmat) return;
  const long long r = e % per;
  const int i = (int)(r % n), j = (int)(r / n);
  TC* p = G + e;
  if (i > j) *p = (TC)0;
  else if (i == j) *p = (TC)((double)*p * 0.5);
}

// ------------------------------------------------------------- host side --
template <typename TC>
__global__ void k_cast(const double* __restrict__ s, TC* __restrict__ d, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = (TC)s[e];
}

void agg_prepare(Ctx& ctx, QRFactor& f, int tc, int panels_per_block) {
  f.agg.clear();
  f.agg_tc = tc;
  const int width = 64 * (panels_per_block > 0 ? panels_per_block : 1);
  std::vector<AggBlock> blocks;
  for (int J0 = 0; J0 < f.k; J0 += width) {
    AggBlock b;
    b.J0 = J0;
    b.w = min(width, f.k - J0);
    blocks.push_back(b);
  }
  // Consecutive blocks of one width form a group: their Grams are formed one
  // by one (the row counts differ) into consecutive w x w slots, and the
  // triangular inverses of the group run as one batch.
  const bool f64 = tc == 8 || f.tw == 8;   // FP64 Gram and inverse (GMRES, FP64 path)
  size_t i = 0;
  while (i < blocks.size()) {
    size_t j = i;
    while (j < blocks.size() && blocks[j].w == blocks[i].w) ++j;
    const int w = blocks[i].w, nm = (int)(j - i);
    const long long tot = (long long)w * w;
    void* G = ctx.ws->alloc((f64 ? 8 : 4) * (size_t)(tot * nm));
    for (size_t q = i; q < j; ++q) {
      const int J0 = blocks[q].J0, rows = f.r - J0;
      GemmArgs g{};
      g.A = f.tw == 8 ? (const void*)(static_cast<const double*>(f.M) + (size_t)J0 + (size_t)J0 * f.ld)
                      : (const void*)(static_cast<const float*>(f.M) + (size_t)J0 + (size_t)J0 * f.ld);
      g.lda = f.ld; g.ta = 1; g.ma = 2; g.oa = 0;
      g.B = g.A; g.ldb = f.ld; g.tb = 0; g.mb = 2; g.ob = 0;
      g.ldc = w; g.m = w; g.n = w; g.k = rows; g.alpha = 1.0; g.beta = 0.0;
      if (f64) {
        g.C = static_cast<double*>(G) + (size_t)(q - i) * tot;
        if (f.tw == 8) gemm<double, double, double>(ctx, g, 1); else gemm<float, float, double>(ctx, g, 1);
      } else {
        g.C = static_cast<float*>(G) + (size_t)(q - i) * tot;
        gemm<float, float, float>(ctx, g, 1);
      }
    }
    const unsigned nbk = (unsigned)((tot * nm + 255) / 256);
    void* T = ctx.ws->alloc((size_t)tc * (size_t)(tot * nm));
    if (f64) {
      double* G64 = static_cast<double*>(G);
      hipLaunchKernelGGL((k_ut_fix<double>), dim3(nbk), dim3(256), 0, ctx.stream, G64, w, nm);
      double* T64 = tc == 8 ? static_cast<double*>(T) : ctx.ws->get<double>((size_t)(tot * nm));
      tri_inverse_batched<double, double>(ctx, G64, w, tot, w, T64, w, tot, nm);
      if (tc != 8)
        hipLaunchKernelGGL((k_cast<float>), dim3(nbk), dim3(256), 0, ctx.stream, T64, static_cast<float*>(T),
                           tot * nm);
    } else {
      float* G32 = static_cast<float*>(G);
      hipLaunchKernelGGL((k_ut_fix<float>), dim3(nbk), dim3(256), 0, ctx.stream, G32, w, nm);
      tri_inverse_batched<float, float>(ctx, G32, w, tot, w, static_cast<float*>(T), w, tot, nm);
    }
    LSQ_LAUNCH_CHECK();
    for (size_t q = i; q < j; ++q) blocks[q].T = static_cast<char*>(T) + (size_t)tc * (size_t)(q - i) * tot;
    i = j;
  }
  size_t acc = 0;
  for (auto& b : blocks) {
    b.acc = acc;
    acc += 2 * (size_t)b.w;
  }
  f.agg_acc_len = acc;
  f.agg_acc = ctx.ws->alloc((size_t)tc * (acc > 0 ? acc : 1));
  vec_zero(ctx, f.agg_acc, tc, (int)acc);
  f.agg = blocks;
}

template <typename S, typename TC>
static void agg_apply_t(Ctx& ctx, const QRFactor& f, bool trans, TC* y) {
  const int nb = (int)f.agg.size();
  TC* acc = static_cast<TC*>(f.agg_acc);
  for (int q = 0; q < nb; ++q) {
    const AggBlock& b = f.agg[trans ? q : nb - 1 - q];
    const int rows = f.r - b.J0;
    const S* Y = static_cast<const S*>(f.M) + (size_t)b.J0 + (size_t)b.J0 * f.ld;
    TC* yy = y + b.J0;
    TC* s = acc + b.acc;                 // zero on entry
    TC* tv = s + b.w;                    // zero on entry
    // one read of the block's reflectors (rows x w in S) per product
    const double fl = 2.0 * rows * b.w, by = (double)rows * b.w * sizeof(S);
    // s = Y^T y (unit-lower Y)
    ktimer_begin(ctx, kKAggGemv, fl, by);
    gemv_t<S, TC, kUnitLower>(ctx.stream, Y, f.ld, rows, b.w, 0, (TC)1, yy, s, ctx.deterministic);
    ktimer_end(ctx, kKAggGemv);
    // Q^T = I - Y T^T Y^T  -> t = T^T s ;  Q = I - Y T Y^T -> t = T s
    trmv_dense<TC>(ctx, static_cast<const TC*>(b.T), b.w, b.w, trans, s, tv);
    // y -= Y t
    ktimer_begin(ctx, kKAggGemv, fl, by);
    gemv_n<S, TC, kUnitLower>(ctx.stream, Y, f.ld, rows, b.w, 0, (TC)-1, tv, yy, ctx.deterministic);
    ktimer_end(ctx, kKAggGemv);
    LSQ_LAUNCH_CHECK();
  }
  // every block's accumulators back to zero for the next application (a fill
  // kernel: this path may be graph-captured)
  vec_zero(ctx, acc, (int)sizeof(TC), (int)f.agg_acc_len);
}

void agg_apply(Ctx& ctx, const QRFactor& f, bool trans, void* y, int tc) {
  if (f.k <= 0) return;
  if (tc != f.agg_tc) throw HipError{hipErrorInvalidValue, "aggregated reflectors prepared for another precision"};
  if (f.tw == 8) {
    if (tc == 8) agg_apply_t<double, double>(ctx, f, trans, static_cast<double*>(y));
    else agg_apply_t<double, float>(ctx, f, trans, static_cast<float*>(y));
  } else {
    if (tc == 8) agg_apply_t<float, double>(ctx, f, trans, static_cast<double*>(y));
    else agg_apply_t<float, float>(ctx, f, trans, static_cast<float*>(y));
  }
}

// Dense inverse of the upper triangular block U = f.M[o:o+nn, o:o+nn] in TC.
void tri_inverse_factor(Ctx& ctx, const QRFactor& f, int o, int nn, void* X, int tc) {
  if (nn <= 0) return;
  if (f.tw == 8) {
    const double* U = static_cast<const double*>(f.M) + (size_t)o + (size_t)o * f.ld;
    if (tc == 8) tri_inverse<double, double>(ctx, U, f.ld, nn, static_cast<double*>(X), nn);
    else tri_inverse<double, float>(ctx, U, f.ld, nn, static_cast<float*>(X), nn);
  } else {
    const float* U = static_cast<const float*>(f.M) + (size_t)o + (size_t)o * f.ld;
    if (tc == 8) tri_inverse<float, double>(ctx, U, f.ld, nn, static_cast<double*>(X), nn);
    else tri_inverse<float, float>(ctx, U, f.ld, nn, static_cast<float*>(X), nn);
  }
}

void trmv_acc(Ctx& ctx, const void* X, int nn, bool trans, const void* x, void* y, int tc) {
  if (tc == 8) trmv_dense<double>(ctx, static_cast<const double*>(X), nn, nn, trans, static_cast<const double*>(x), static_cast<double*>(y));
  else trmv_dense<float>(ctx, static_cast<const float*>(X), nn, nn, trans, static_cast<const float*>(x), static_cast<float*>(y));
}

}  // namespace lsq
