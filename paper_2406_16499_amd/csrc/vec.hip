// Vector-side kernels: triangular solves on factor blocks, masked GEMV,
// conversions / reversals, and the FP64 augmented-residual sweeps with the
// stop test (eq. lse-stop / eq. gls-stop).
#include "engine.hpp"
#include "gemv.hpp"

namespace lsq {

// ------------------------------------------------------------ triangular --
void trsv_prepare(Ctx& ctx, TriBlock& tb, const QRFactor& f, int o, int nn, int tc) {
  tb.f = &f; tb.o = o; tb.nn = nn; tb.tc = tc;
  tb.inv = ctx.ws->alloc((size_t)tc * (nn > 0 ? (size_t)nn * nn : 1));
  tb.tmp = ctx.ws->alloc((size_t)tc * (nn > 0 ? nn : 1));
  vec_zero(ctx, tb.tmp, tc, nn);
  tri_inverse_factor(ctx, f, o, nn, tb.inv, tc);
}

// tmp (zero between solves) accumulates op(U^{-1}) x, then moves into x and
// is cleared in the same pass.
void trsv(Ctx& ctx, const TriBlock& tb, bool trans, void* x) {
  if (tb.nn <= 0) return;
  trmv_acc(ctx, tb.inv, tb.nn, trans, x, tb.tmp, tb.tc);
  vec_move(ctx, x, tb.tmp, tb.tc, tb.nn);
}

// ------------------------------------------------------------ masked GEMV --
void gemv_upper(Ctx& ctx, const QRFactor& f, int ro, int co, int nr, int nc, bool trans,
                double alpha, const void* x, void* y, int tc) {
  if (nr <= 0 || nc <= 0) return;
  // the block's entries with global row <= global column: i - j <= co - ro
#define LSQ_GEMV(TW, TC)                                                                        \
  {                                                                                             \
    const TW* A = static_cast<const TW*>(f.M) + (size_t)ro + (size_t)co * f.ld;                 \
    if (!trans)                                                                                 \
      gemv_n<TW, TC, kUpper>(ctx.stream, A, f.ld, nr, nc, co - ro, (TC)alpha,                   \
                             static_cast<const TC*>(x), static_cast<TC*>(y), ctx.deterministic); \
    else                                                                                        \
      gemv_t<TW, TC, kUpper>(ctx.stream, A, f.ld, nr, nc, co - ro, (TC)alpha,                   \
                             static_cast<const TC*>(x), static_cast<TC*>(y), ctx.deterministic); \
  }
  if (f.tw == 8) {
    if (tc == 8) { LSQ_GEMV(double, double) } else { LSQ_GEMV(double, float) }
  } else {
    if (tc == 8) { LSQ_GEMV(float, double) } else { LSQ_GEMV(float, float) }
  }
#undef LSQ_GEMV
  LSQ_LAUNCH_CHECK();
}

// ------------------------------------------------------- elementwise ops --
template <typename Td, typename Ts>
__global__ void k_vec_convert(Td* __restrict__ dst, const Ts* __restrict__ src, int n, int rev,
                              double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (double)src[rev ? (n - 1 - i) : i];
  dst[i] = (Td)(v * scale);
}

template <typename Ty, typename Tx>
__global__ void k_vec_axpy(Ty* __restrict__ y, double a, const Tx* __restrict__ x, int n, int rev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = (Ty)((double)y[i] + a * (double)x[rev ? (n - 1 - i) : i]);
}

template <typename T>
__global__ void k_vec_zero(T* __restrict__ y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)0;
}

#define LSQ_DISPATCH2(td, ts, F)                         \
  if ((td) == 8 && (ts) == 8) { F(double, double) }      \
  else if ((td) == 8) { F(double, float) }               \
  else if ((ts) == 8) { F(float, double) }               \
  else { F(float, float) }

void vec_convert(Ctx& ctx, void* dst, int td, const void* src, int ts, int n, bool reverse,
                 double scale) {
  if (n <= 0) return;
#define F(TD, TS)                                                                               \
  hipLaunchKernelGGL((k_vec_convert<TD, TS>), dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream, \
                     static_cast<TD*>(dst), static_cast<const TS*>(src), n, reverse ? 1 : 0, scale);
  LSQ_DISPATCH2(td, ts, F)
#undef F
  LSQ_LAUNCH_CHECK();
}

void vec_axpy(Ctx& ctx, void* y, int ty, double a, const void* x, int tx, int n, bool reverse_x) {
  if (n <= 0) return;
#define F(TY, TX)                                                                            \
  hipLaunchKernelGGL((k_vec_axpy<TY, TX>), dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream, \
                     static_cast<TY*>(y), a, static_cast<const TX*>(x), n, reverse_x ? 1 : 0);
  LSQ_DISPATCH2(ty, tx, F)
#undef F
  LSQ_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_vec_move(T* __restrict__ dst, T* __restrict__ src, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = src[i];
  src[i] = (T)0;
}

void vec_move(Ctx& ctx, void* dst, void* src, int t, int n) {
  if (n <= 0) return;
  if (t == 8)
    hipLaunchKernelGGL((k_vec_move<double>), dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream,
                       static_cast<double*>(dst), static_cast<double*>(src), n);
  else
    hipLaunchKernelGGL((k_vec_move<float>), dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream,
                       static_cast<float*>(dst), static_cast<float*>(src), n);
  LSQ_LAUNCH_CHECK();
}

void vec_zero(Ctx& ctx, void* y, int ty, int n) {
  if (n <= 0) return;
  if (ty == 8)
    hipLaunchKernelGGL((k_vec_zero<double>), dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream,
                       static_cast<double*>(y), n);
  else
    hipLaunchKernelGGL((k_vec_zero<float>), dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream,
                       static_cast<float*>(y), n);
  LSQ_LAUNCH_CHECK();
}

// dst (dr x dc) [i][j] = src[a][b], (a, b) = trans ? (j, i) : (i, j), reversed per flags
// against the source extents (sr x sc).  64 x 64 tiles through LDS.
template <typename Td, typename Ts>
__global__ __launch_bounds__(256) void k_mat_convert(Td* __restrict__ dst, int ldd,
                                                     const Ts* __restrict__ src, int lds, int dr,
                                                     int dc, int trans, int rev_r, int rev_c,
                                                     int sr, int sc, double scale) {
  __shared__ double tile[64 * 65];
  LSQ_LDS_POISON(tile);
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int t = threadIdx.x;
  for (int e = t; e < 4096; e += 256) {
    const int fast = e & 63, slow = e >> 6;
    const int i = trans ? i0 + slow : i0 + fast;
    const int j = trans ? j0 + fast : j0 + slow;
    double v = 0.0;
    if (i < dr && j < dc) {
      int a = trans ? j : i, b = trans ? i : j;
      if (rev_r) a = sr - 1 - a;
      if (rev_c) b = sc - 1 - b;
      v = (double)src[(size_t)a + (size_t)b * lds] * scale;
    }
    tile[(i - i0) * 65 + (j - j0)] = v;
  }
  __syncthreads();
  for (int e = t; e < 4096; e += 256) {
    const int i = i0 + (e & 63), j = j0 + (e >> 6);
    if (i < dr && j < dc) dst[(size_t)i + (size_t)j * ldd] = (Td)tile[(i - i0) * 65 + (j - j0)];
  }
}

void mat_convert(Ctx& ctx, void* dst, int td, int ldd, const void* src, int ts, int lds,
                 int dr, int dc, bool trans, bool rev_r, bool rev_c, double scale) {
  if (dr <= 0 || dc <= 0) return;
  const int sr = trans ? dc : dr, sc = trans ? dr : dc;
  dim3 grid(ceil_div(dr, 64), ceil_div(dc, 64));
#define F(TD, TS)                                                                       \
  hipLaunchKernelGGL((k_mat_convert<TD, TS>), grid, dim3(256), 0, ctx.stream,           \
                     static_cast<TD*>(dst), ldd, static_cast<const TS*>(src), lds, dr, dc, \
                     trans ? 1 : 0, rev_r ? 1 : 0, rev_c ? 1 : 0, sr, sc, scale);
  LSQ_DISPATCH2(td, ts, F)
#undef F
  LSQ_LAUNCH_CHECK();
}

// Entries on and above the diagonal of the first k rows, times s.
template <typename T>
__global__ __launch_bounds__(256) void k_scale_upper(T* __restrict__ M, int ld, int k, int c, double s) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (j < c && i < k && i <= j) M[(size_t)i + (size_t)j * ld] = (T)((double)M[(size_t)i + (size_t)j * ld] * s);
}

void scale_upper(Ctx& ctx, QRFactor& f, double s) {
  if (f.k <= 0 || f.c <= 0 || s == 1.0) return;
  const dim3 grid(ceil_div(f.k, 256), f.c);
  if (f.tw == 8)
    hipLaunchKernelGGL((k_scale_upper<double>), grid, dim3(256), 0, ctx.stream, static_cast<double*>(f.M),
                       f.ld, f.k, f.c, s);
  else
    hipLaunchKernelGGL((k_scale_upper<float>), grid, dim3(256), 0, ctx.stream, static_cast<float*>(f.M),
                       f.ld, f.k, f.c, s);
  LSQ_LAUNCH_CHECK();
}

// ----------------------------------------------------- FP64 dual GEMV ----
// Work-group tile: 256 rows x 64 columns.  Each lane owns one row; the column
// sums M^T w are reduced across the wave with a reduce-scatter butterfly.
__global__ __launch_bounds__(256) void k_dual_gemv(const double* __restrict__ M, int ld, int rows,
                                                   int cols, const double* __restrict__ u,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ rowp,
                                                   double* __restrict__ colp) {
  __shared__ double us[64];
  __shared__ double red[4][64];
  LSQ_LDS_POISON(us);
  LSQ_LDS_POISON(red);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int r0 = blockIdx.x * 256, c0 = blockIdx.y * 64;
  if (t < 64) us[t] = (c0 + t < cols) ? u[c0 + t] : 0.0;
  __syncthreads();
  const int row = r0 + t;
  const bool rin = row < rows;
  const double wr = rin ? w[row] : 0.0;
  double racc = 0.0;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    double cp[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int col = c0 + half * 32 + c;
      const double v = (rin && col < cols) ? M[(size_t)row + (size_t)col * ld] : 0.0;
      racc += v * us[half * 32 + c];
      cp[c] = v * wr;
    }
    // 32 values over 64 lanes: exchange across lane bits 5..1, then add lane pairs
    {
#pragma unroll
      for (int m = 32, c = 32; c > 1; m >>= 1, c >>= 1) {
        const bool up = (lane & m) != 0;
#pragma unroll
        for (int i = 0; i < c / 2; ++i) {
          const double send = up ? cp[i] : cp[i + c / 2];
          const double keep = up ? cp[i + c / 2] : cp[i];
          cp[i] = keep + __shfl_xor(send, m, 64);
        }
      }
      cp[0] += __shfl_xor(cp[0], 1, 64);
    }
    // lane l now holds the wave sum of column index (l >> 1): bits 5..1 select it
    if ((lane & 1) == 0) red[wv][half * 32 + (lane >> 1)] = cp[0];
  }
  if (rin) rowp[(size_t)blockIdx.y * rows + row] = racc;
  __syncthreads();
  if (t < 64 && c0 + t < cols)
    colp[(size_t)blockIdx.x * cols + c0 + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

void dual_parts_alloc(Ctx& ctx, int rows, int cols, DualParts& out) {
  out.nrb = ceil_div(rows, 256);
  out.ncb = ceil_div(cols, 64);
  out.rowp = ctx.ws->get<double>((size_t)out.ncb * (rows > 0 ? rows : 1));
  out.colp = ctx.ws->get<double>((size_t)out.nrb * (cols > 0 ? cols : 1));
}

void dual_gemv(Ctx& ctx, const double* M, int ld, int rows, int cols, const double* u,
               const double* w, DualParts& out) {
  if (!out.rowp) dual_parts_alloc(ctx, rows, cols, out);
  out.nrb = ceil_div(rows, 256);
  out.ncb = ceil_div(cols, 64);
  if (rows <= 0 || cols <= 0) {
    out.nrb = out.ncb = 0;
    return;
  }
  // 4 flops per matrix element (two products), one FP64 read of the matrix
  ktimer_begin(ctx, kKDualGemv, 4.0 * rows * cols, 8.0 * rows * cols);
  hipLaunchKernelGGL(k_dual_gemv, dim3(out.nrb, out.ncb), dim3(256), 0, ctx.stream, M, ld, rows,
                     cols, u, w, out.rowp, out.colp);
  ktimer_end(ctx, kKDualGemv);
  LSQ_LAUNCH_CHECK();
}

// ------------------------------------------ double-double residual sweep --
// Extra-precise residual (u_r = u^2, Table 2's "quad" rows): every product
// and sum of the residual is carried as an unevaluated pair hi + lo with
// error-free transformations (Knuth's TwoSum, an FMA-based TwoProduct), and
// the residual blocks are rounded to FP64 only at the end.  Two passes over
// the matrix (M u, then M^T w); an optional mode, so plainness beats fusion.
// The transformations are exact only if every product and sum is rounded on
// its own: FP contraction (an FMA formed from a product and a later sum) is
// off inside them.
struct DD { double hi, lo; };
__device__ __forceinline__ DD dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ DD dd_quick(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ DD dd_add(DD a, DD b) {
#pragma clang fp contract(off)
  const DD s = dd_two_sum(a.hi, b.hi);
  return dd_quick(s.hi, s.lo + (a.lo + b.lo));
}
__device__ __forceinline__ DD dd_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ DD dd_shfl_xor(DD a, int m) {
  return {__shfl_xor(a.hi, m, 64), __shfl_xor(a.lo, m, 64)};
}

// rowp[cb][i] = sum over the 64 columns of block cb of M[i][j] u[j] (hi / lo arrays)
__global__ __launch_bounds__(256) void k_gemv_n_dd(const double* __restrict__ M, int ld, int rows,
                                                   int cols, const double* __restrict__ u,
                                                   double* __restrict__ hi, double* __restrict__ lo) {
  __shared__ double us[64];
  const int t = threadIdx.x, r = blockIdx.x * 256 + t, c0 = blockIdx.y * 64;
  if (t < 64) us[t] = (c0 + t < cols) ? u[c0 + t] : 0.0;
  __syncthreads();
  if (r >= rows) return;
  DD acc = {0.0, 0.0};
  const int ce = min(cols, c0 + 64);
  for (int j = c0; j < ce; ++j) acc = dd_add(acc, dd_prod(M[(size_t)r + (size_t)j * ld], us[j - c0]));
  hi[(size_t)blockIdx.y * rows + r] = acc.hi;
  lo[(size_t)blockIdx.y * rows + r] = acc.lo;
}

// colp[rb][j] = sum over the 256 rows of block rb of M[i][j] w[i]: each wave
// takes 16 columns, each lane four rows of a column, then a pairwise reduction.
__global__ __launch_bounds__(256) void k_gemv_t_dd(const double* __restrict__ M, int ld, int rows,
                                                   int cols, const double* __restrict__ w,
                                                   double* __restrict__ hi, double* __restrict__ lo) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 256, c0 = blockIdx.x * 64 + 16 * wv;
  double wr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = r0 + lane + 64 * k;
    wr[k] = i < rows ? w[i] : 0.0;
  }
  for (int c = 0; c < 16; ++c) {
    const int j = c0 + c;
    if (j >= cols) break;
    DD acc = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = r0 + lane + 64 * k;
      if (i < rows) acc = dd_add(acc, dd_prod(M[(size_t)i + (size_t)j * ld], wr[k]));
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc = dd_add(acc, dd_shfl_xor(acc, m));
    if (lane == 0) {
      hi[(size_t)blockIdx.y * cols + j] = acc.hi;
      lo[(size_t)blockIdx.y * cols + j] = acc.lo;
    }
  }
}

// Partial sums of one product in double-double: part q of element i is
// hi[q len + i] + lo[q len + i].
struct PartsDD {
  const double* hi; const double* lo; int nparts; int len;
  __device__ DD sum(int i) const {
    DD s = {0.0, 0.0};
    for (int q = 0; q < nparts; ++q)
      s = dd_add(s, DD{hi[(size_t)q * len + i], lo[(size_t)q * len + i]});
    return s;
  }
};
__device__ __forceinline__ DD dd_neg(DD a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ DD dd_from(double a) { return {a, 0.0}; }
__device__ __forceinline__ double dd_round(DD a) { return a.hi + a.lo; }

// ------------------------------------------------------- residual finish --
struct PartsView {
  const double* p; int nparts; int len;
  __device__ double sum(int i) const {
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += p[(size_t)q * len + i];
    return s;
  }
};

// Scaled sums of squares of six per-thread values over a work-group of 256:
// for each slot k, the work-group's largest magnitude 2^e (frexp exponent e)
// and the sum of (value 2^-e)^2 go to out[k] and out[6 + k].  The squares of
// the scaled values lie in [0, 1), so no sum overflows or underflows for any
// finite input; the stop test combines the blocks' (sum, e) pairs.
__device__ __forceinline__ void scaled_sumsq6(const double val[6], double* __restrict__ out) {
  __shared__ double red[4][6];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    a[k] = fabs(val[k]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a[k] = fmax(a[k], __shfl_xor(a[k], o, 64));
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[w][k] = a[k];
  __syncthreads();
  int e[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double mx = fmax(fmax(red[0][k], red[1][k]), fmax(red[2][k], red[3][k]));
    e[k] = 0;
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e[k]);   // inf / NaN stay inf / NaN below
    const double t = ldexp(val[k], -e[k]);
    a[k] = t * t;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a[k] += __shfl_xor(a[k], o, 64);
  }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[w][k] = a[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      out[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
      out[6 + k] = (double)e[k];
    }
}

// LSE: f1 = b - r - A x, f2 = d - B x, f3 = -A^T r + B^T v, plus the scaled
// sums of squares of f1, f2, f3, x, r, v into normp[block][12].
__global__ __launch_bounds__(256) void k_lse_finish(int m, int n, int p, const double* __restrict__ b,
                                                    const double* __restrict__ d,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ v, PartsView Ax,
                                                    PartsView Atr, PartsView Bx, PartsView Btv,
                                                    double* __restrict__ f1, double* __restrict__ f2,
                                                    double* __restrict__ f3,
                                                    double* __restrict__ normp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (i < m) {
    const double val = b[i] - r[i] - Ax.sum(i);
    f1[i] = val;
    s[0] = val;
    s[4] = r[i];
  }
  if (i < p) {
    const double val = d[i] - Bx.sum(i);
    f2[i] = val;
    s[1] = val;
    s[5] = v[i];
  }
  if (i < n) {
    const double val = -Atr.sum(i) + Btv.sum(i);
    f3[i] = val;
    s[2] = val;
    s[3] = x[i];
  }
  scaled_sumsq6(s, normp + (size_t)blockIdx.x * kNormSlots);
}

// GLS: f1 = -y + V^T z, f2 = d - W x - V y, f3 = W^T z; scaled sums of squares
// of f1, f2, f3, x, y, z.
__global__ __launch_bounds__(256) void k_gls_finish(int n, int m, int p, const double* __restrict__ d,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ z, PartsView Wx,
                                                    PartsView Wtz, PartsView Vy, PartsView Vtz,
                                                    double* __restrict__ f1, double* __restrict__ f2,
                                                    double* __restrict__ f3,
                                                    double* __restrict__ normp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (i < p) {
    const double val = -y[i] + Vtz.sum(i);
    f1[i] = val;
    s[0] = val;
    s[4] = y[i];
  }
  if (i < n) {
    const double val = d[i] - Wx.sum(i) - Vy.sum(i);
    f2[i] = val;
    s[1] = val;
    s[5] = z[i];
  }
  if (i < m) {
    const double val = Wtz.sum(i);
    f3[i] = val;
    s[2] = val;
    s[3] = x[i];
  }
  scaled_sumsq6(s, normp + (size_t)blockIdx.x * kNormSlots);
}

// Double-double versions of the two finish kernels: the residual blocks
// are formed from the FP64 inputs and iterate and the double-double partial
// products, and rounded once.
__global__ __launch_bounds__(256) void k_lse_finish_dd(int m, int n, int p, const double* __restrict__ b,
                                                       const double* __restrict__ d,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ r,
                                                       const double* __restrict__ v, PartsDD Ax,
                                                       PartsDD Atr, PartsDD Bx, PartsDD Btv,
                                                       double* __restrict__ f1, double* __restrict__ f2,
                                                       double* __restrict__ f3,
                                                       double* __restrict__ normp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (i < m) {
    const double val = dd_round(dd_add(dd_two_sum(b[i], -r[i]), dd_neg(Ax.sum(i))));
    f1[i] = val;
    s[0] = val;
    s[4] = r[i];
  }
  if (i < p) {
    const double val = dd_round(dd_add(dd_from(d[i]), dd_neg(Bx.sum(i))));
    f2[i] = val;
    s[1] = val;
    s[5] = v[i];
  }
  if (i < n) {
    const double val = dd_round(dd_add(dd_neg(Atr.sum(i)), Btv.sum(i)));
    f3[i] = val;
    s[2] = val;
    s[3] = x[i];
  }
  scaled_sumsq6(s, normp + (size_t)blockIdx.x * kNormSlots);
}

__global__ __launch_bounds__(256) void k_gls_finish_dd(int n, int m, int p, const double* __restrict__ d,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z, PartsDD Wx,
                                                       PartsDD Wtz, PartsDD Vy, PartsDD Vtz,
                                                       double* __restrict__ f1, double* __restrict__ f2,
                                                       double* __restrict__ f3,
                                                       double* __restrict__ normp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (i < p) {
    const double val = dd_round(dd_add(dd_from(-y[i]), Vtz.sum(i)));
    f1[i] = val;
    s[0] = val;
    s[4] = y[i];
  }
  if (i < n) {
    const double val = dd_round(dd_add(dd_add(dd_from(d[i]), dd_neg(Wx.sum(i))), dd_neg(Vy.sum(i))));
    f2[i] = val;
    s[1] = val;
    s[5] = z[i];
  }
  if (i < m) {
    const double val = dd_round(Wtz.sum(i));
    f3[i] = val;
    s[2] = val;
    s[3] = x[i];
  }
  scaled_sumsq6(s, normp + (size_t)blockIdx.x * kNormSlots);
}

// Stop test.  normp: per block the scaled sums of squares and exponents of
// [f1, f2, f3, x, a1, a2] (k_lse_finish / k_gls_finish).
// matnorms: [||A||_F, ||B||_F, ||rhs1||, ||rhs2||].
// LSE (gls = 0): scale1 = ||b|| + ||r|| + ||A|| ||x||, scale2 = ||d|| + ||B|| ||x||,
//                scale3 = ||A|| ||r|| + ||B|| ||v||              (a1 = r, a2 = v)
// GLS (gls = 1): scale1 = ||y|| + ||V|| ||z||, scale2 = ||d|| + ||W|| ||x|| + ||V|| ||y||,
//                scale3 = ||W|| ||z||    (A = W, B = V, a1 = y, a2 = z, rhs1 = ||d||)
__global__ void k_stop(const double* __restrict__ normp, int nblk, const double* __restrict__ matnorms,
                       int gls, double tol, StopStatus* __restrict__ st) {
  __shared__ double red[4];
  __shared__ double nrm[6];
  for (int k = 0; k < 6; ++k) {
    // common exponent E = the largest block exponent among nonzero blocks,
    // then the sum of the blocks' scaled sums brought to 2^E
    // (exponents offset by 4096 so that they are positive; 0 = no nonzero block)
    double ev = 0.0;
    for (int q = threadIdx.x; q < nblk; q += blockDim.x)
      if (normp[(size_t)q * kNormSlots + k] > 0.0)
        ev = fmax(ev, normp[(size_t)q * kNormSlots + 6 + k] + 4096.0);
    ev = block_max(ev, red);
    const int E = ev > 0.0 ? (int)ev - 4096 : 0;
    double s = 0.0;
    for (int q = threadIdx.x; q < nblk; q += blockDim.x) {
      const double part = normp[(size_t)q * kNormSlots + k];
      if (part > 0.0) s += ldexp(part, 2 * ((int)normp[(size_t)q * kNormSlots + 6 + k] - E));
      else if (part != 0.0) s += part;   // NaN: the norm becomes NaN
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) nrm[k] = ldexp(sqrt(s), E);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double nf1 = nrm[0], nf2 = nrm[1], nf3 = nrm[2];
  const double nx = nrm[3], na1 = nrm[4], na2 = nrm[5];
  const double nA = matnorms[0], nB = matnorms[1], nr1 = matnorms[2], nr2 = matnorms[3];
  double sc[3];
  if (!gls) {
    sc[0] = nr1 + na1 + nA * nx;
    sc[1] = nr2 + nB * nx;
    sc[2] = nA * na1 + nB * na2;
  } else {
    sc[0] = na1 + nB * na2;
    sc[1] = nr1 + nA * nx + nB * na1;
    sc[2] = nA * na2;
  }
  const double nf[3] = {nf1, nf2, nf3};
  int conv = 1, bad = 0;
  double bm = 0.0;
  for (int k = 0; k < 3; ++k) {
    st->nf[k] = nf[k];
    st->scale[k] = sc[k];
    double e = 0.0;
    if (nf[k] > 0.0) e = sc[k] > 0.0 ? nf[k] / sc[k] : INFINITY;
    st->berr[k] = e;
    if (!(nf[k] <= tol * sc[k])) conv = 0;
    if (!isfinite(nf[k]) || !isfinite(sc[k])) bad = 1;
    bm = e > bm ? e : bm;
  }
  if (!isfinite(nx) || !isfinite(na1) || !isfinite(na2)) bad = 1;
  st->berr_max = bm;
  st->converged = conv && !bad;
  st->nonfinite = bad;
}

// Double-double partial products of M (rows x cols): Mu parts (one per
// 64-column block, length rows) and M^T w parts (one per 256-row block,
// length cols), from the workspace.
struct DualDD { PartsDD mu, mtw; };
static DualDD dual_dd(Ctx& ctx, const double* M, int ld, int rows, int cols, const double* u,
                      const double* w) {
  DualDD o;
  const int ncb = ceil_div(cols, 64), nrb = ceil_div(rows, 256);
  if (rows <= 0 || cols <= 0) {
    o.mu = {nullptr, nullptr, 0, rows};
    o.mtw = {nullptr, nullptr, 0, cols};
    return o;
  }
  double* rh = ctx.ws->get<double>((size_t)ncb * rows);
  double* rl = ctx.ws->get<double>((size_t)ncb * rows);
  double* ch = ctx.ws->get<double>((size_t)nrb * cols);
  double* cl = ctx.ws->get<double>((size_t)nrb * cols);
  hipLaunchKernelGGL(k_gemv_n_dd, dim3(nrb, ncb), dim3(256), 0, ctx.stream, M, ld, rows, cols, u, rh, rl);
  hipLaunchKernelGGL(k_gemv_t_dd, dim3(ncb, nrb), dim3(256), 0, ctx.stream, M, ld, rows, cols, w, ch, cl);
  LSQ_LAUNCH_CHECK();
  o.mu = {rh, rl, ncb, rows};
  o.mtw = {ch, cl, nrb, cols};
  return o;
}

void residual_scratch_alloc(Ctx& ctx, int r1, int c1, int r2, int c2, int len, ResidualScratch& rs) {
  dual_parts_alloc(ctx, r1, c1, rs.p1);
  dual_parts_alloc(ctx, r2, c2, rs.p2);
  rs.normp = ctx.ws->get<double>((size_t)ceil_div(len > 0 ? len : 1, 256) * kNormSlots);
}

void lse_residual(Ctx& ctx, int m, int n, int p, const double* A, int lda, const double* B,
                  int ldb, const double* b, const double* d, const double* x, const double* r,
                  const double* v, double* f1, double* f2, double* f3, const double* matnorms,
                  double tol, StopStatus* st, bool dd, ResidualScratch* rs) {
  // the partial sums live only until the finish kernel below has read them:
  // the memory goes back to the workspace (stream order keeps it safe)
  const Arena::Mark mk = ctx.ws->mark();
  const int len = m > n ? (m > p ? m : p) : (n > p ? n : p);
  const int nblk = ceil_div(len, 256);
  if (dd) rs = nullptr;
  double* normp = rs ? rs->normp : ctx.ws->get<double>((size_t)nblk * kNormSlots);
  if (dd) {
    const DualDD pa = dual_dd(ctx, A, lda, m, n, x, r), pb = dual_dd(ctx, B, ldb, p, n, x, v);
    hipLaunchKernelGGL(k_lse_finish_dd, dim3(nblk), dim3(256), 0, ctx.stream, m, n, p, b, d, x, r, v,
                       pa.mu, pa.mtw, pb.mu, pb.mtw, f1, f2, f3, normp);
  } else {
    DualParts pa, pb;
    if (rs) { pa = rs->p1; pb = rs->p2; }
    dual_gemv(ctx, A, lda, m, n, x, r, pa);
    dual_gemv(ctx, B, ldb, p, n, x, v, pb);
    PartsView Ax{pa.rowp, pa.ncb, m}, Atr{pa.colp, pa.nrb, n}, Bx{pb.rowp, pb.ncb, p},
        Btv{pb.colp, pb.nrb, n};
    hipLaunchKernelGGL(k_lse_finish, dim3(nblk), dim3(256), 0, ctx.stream, m, n, p, b, d, x, r, v, Ax,
                       Atr, Bx, Btv, f1, f2, f3, normp);
  }
  hipLaunchKernelGGL(k_stop, dim3(1), dim3(256), 0, ctx.stream, normp, nblk, matnorms, 0, tol, st);
  LSQ_LAUNCH_CHECK();
  ctx.ws->rewind(mk);
}

void gls_residual(Ctx& ctx, int n, int m, int p, const double* W, int ldw, const double* V,
                  int ldv, const double* d, const double* x, const double* y, const double* z,
                  double* f1, double* f2, double* f3, const double* matnorms, double tol,
                  StopStatus* st, bool dd, ResidualScratch* rs) {
  // the partial sums live only until the finish kernel below has read them:
  // the memory goes back to the workspace (stream order keeps it safe)
  const Arena::Mark mk = ctx.ws->mark();
  const int len = m > n ? (m > p ? m : p) : (n > p ? n : p);
  const int nblk = ceil_div(len, 256);
  if (dd) rs = nullptr;
  double* normp = rs ? rs->normp : ctx.ws->get<double>((size_t)nblk * kNormSlots);
  if (dd) {
    const DualDD pw = dual_dd(ctx, W, ldw, n, m, x, z), pv = dual_dd(ctx, V, ldv, n, p, y, z);
    hipLaunchKernelGGL(k_gls_finish_dd, dim3(nblk), dim3(256), 0, ctx.stream, n, m, p, d, x, y, z,
                       pw.mu, pw.mtw, pv.mu, pv.mtw, f1, f2, f3, normp);
  } else {
    DualParts pw, pv;
    if (rs) { pw = rs->p1; pv = rs->p2; }
    dual_gemv(ctx, W, ldw, n, m, x, z, pw);
    dual_gemv(ctx, V, ldv, n, p, y, z, pv);
    PartsView Wx{pw.rowp, pw.ncb, n}, Wtz{pw.colp, pw.nrb, m}, Vy{pv.rowp, pv.ncb, n},
        Vtz{pv.colp, pv.nrb, p};
    hipLaunchKernelGGL(k_gls_finish, dim3(nblk), dim3(256), 0, ctx.stream, n, m, p, d, x, y, z, Wx,
                       Wtz, Vy, Vtz, f1, f2, f3, normp);
  }
  hipLaunchKernelGGL(k_stop, dim3(1), dim3(256), 0, ctx.stream, normp, nblk, matnorms, 1, tol, st);
  LSQ_LAUNCH_CHECK();
  ctx.ws->rewind(mk);
}

// --------------------------------------------------------------- norms ----
// One read of each input yields its Frobenius norm, its largest magnitude and
// whether it holds a non-finite value.  The sum of squares is kept three times
// (entries scaled by 2^-600, unscaled, scaled by 2^600) so that the norm is
// right over the whole FP64 range: the unscaled sum when it neither overflows
// nor underflows, else the scaled one that does not.
// Work items are 1024-row segments of one column (contiguous reads); each
// work-group writes per slot k: lo, mid, hi sums and the max (NaN when a
// non-finite entry was seen) at part[(4 k + s) * per + block].
constexpr double kTwo600 = 4.149515568880993e180;    // 2^600
constexpr double kTwoM600 = 2.409919865102884e-181;  // 2^-600

__global__ __launch_bounds__(256) void k_sumsq_mat(const double* __restrict__ M, int ld, int rows,
                                                   int cols, double* __restrict__ part, int per) {
  __shared__ double red[4];
  double lo = 0.0, mid = 0.0, hi = 0.0, mx = 0.0, bad = 0.0;
  const int nseg = (rows + 1023) / 1024;
  const long long items = (long long)nseg * cols;
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const int j = (int)(it / nseg), i0 = (int)(it % nseg) * 1024;
    const double* col = M + (size_t)j * ld;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + q * 256 + threadIdx.x;
      if (i < rows) {
        const double v = col[i];
        if (!isfinite(v)) {
          bad = 1.0;
        } else {
          const double a = fabs(v);
          mx = fmax(mx, a);
          const double vl = v * kTwoM600, vh = v * kTwo600;
          lo = fma(vl, vl, lo);
          mid = fma(v, v, mid);
          hi = fma(vh, vh, hi);
        }
      }
    }
  }
  lo = block_sum(lo, red);
  mid = block_sum(mid, red);
  hi = block_sum(hi, red);
  bad = block_sum(bad, red);
  mx = block_max(mx, red);
  if (threadIdx.x == 0) {
    part[(size_t)0 * per + blockIdx.x] = lo;
    part[(size_t)1 * per + blockIdx.x] = mid;
    part[(size_t)2 * per + blockIdx.x] = hi;
    part[(size_t)3 * per + blockIdx.x] = bad > 0.0 ? NAN : mx;
  }
}

// out[k] = ||input k|| (k < 4), out[4 + k] = its largest magnitude, NaN when
// it holds a non-finite value.
__global__ void k_norms_final(const double* __restrict__ part, int per, double* __restrict__ out) {
  __shared__ double red[4];
  for (int k = 0; k < 4; ++k) {
    const double* pk = part + (size_t)4 * k * per;
    double lo = 0.0, mid = 0.0, hi = 0.0, mx = 0.0, bad = 0.0;
    for (int q = threadIdx.x; q < per; q += blockDim.x) {
      lo += pk[q];
      mid += pk[per + q];
      hi += pk[2 * per + q];
      const double m = pk[3 * per + q];
      if (isnan(m)) bad = 1.0; else mx = fmax(mx, m);
    }
    lo = block_sum(lo, red);
    mid = block_sum(mid, red);
    hi = block_sum(hi, red);
    bad = block_sum(bad, red);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) {
      double nrm;
      if (!isfinite(mid)) nrm = sqrt(lo) * kTwo600;              // squares overflow
      else if (mid < 0x1p-960 && hi > 0.0) nrm = sqrt(hi) * kTwoM600;   // squares underflow
      else nrm = sqrt(mid);
      out[k] = nrm;
      out[4 + k] = bad > 0.0 ? NAN : mx;
    }
  }
}

void frob_norms(Ctx& ctx, const double* A, int lda, int ar, int ac, const double* B, int ldb,
                int br, int bc, const double* v1, int n1, const double* v2, int n2,
                double* matnorms) {
  const int per = 512;
  double* part = ctx.ws->get<double>(16 * per);
  vec_zero(ctx, part, 8, 16 * per);
  const double* mats[4] = {A, B, v1, v2};
  const int rr[4] = {ar, br, n1, n2}, cc[4] = {ac, bc, 1, 1}, ll[4] = {lda, ldb, n1 > 0 ? n1 : 1, n2 > 0 ? n2 : 1};
  for (int k = 0; k < 4; ++k) {
    if (!mats[k] || rr[k] <= 0 || cc[k] <= 0) continue;
    const long long items = (long long)ceil_div(rr[k], 1024) * cc[k];
    const int g = (int)(items < per ? items : per);
    hipLaunchKernelGGL(k_sumsq_mat, dim3(g), dim3(256), 0, ctx.stream, mats[k], ll[k], rr[k], cc[k],
                       part + (size_t)4 * k * per, per);
  }
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(256), 0, ctx.stream, part, per, matnorms);
  LSQ_LAUNCH_CHECK();
}

// --------------------------------------------------------- complex data --
// Real embedding of a complex column-major matrix M (rows x cols, interleaved
// (re, im) pairs, ld in complex elements): E = [Re M, -Im M; Im M, Re M]
// (2 rows x 2 cols, ld 2 rows).  M u = w over C is E [Re u; Im u] = [Re w; Im w],
// and E^T is the embedding of M^H.  One thread per complex element, rows fastest.
__global__ __launch_bounds__(256) void k_embed_mat(const double2* __restrict__ M, int ld, int rows,
                                                   int cols, double* __restrict__ E) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const int i = (int)(e % rows), j = (int)(e / rows);
  const double2 z = M[(size_t)i + (size_t)j * ld];
  const size_t le = 2 * (size_t)rows;
  E[(size_t)i + (size_t)j * le] = z.x;
  E[(size_t)i + (size_t)(cols + j) * le] = -z.y;
  E[(size_t)(rows + i) + (size_t)j * le] = z.y;
  E[(size_t)(rows + i) + (size_t)(cols + j) * le] = z.x;
}
// [Re u; Im u] (2n) from an interleaved complex vector u (n), and back.
__global__ void k_embed_vec(const double2* __restrict__ u, int n, double* __restrict__ e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 z = u[i];
  e[i] = z.x;
  e[n + i] = z.y;
}
__global__ void k_unembed_vec(const double* __restrict__ e, int n, double2* __restrict__ u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[i] = make_double2(e[i], e[n + i]);
}
__global__ void k_scale_first(double* __restrict__ v, int n, double s) {
  const int i = threadIdx.x;
  if (i < n) v[i] *= s;
}

void embed_mat(Ctx& ctx, const double* M, int ld, int rows, int cols, double* E) {
  const long long tot = (long long)rows * cols;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_embed_mat, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx.stream,
                     reinterpret_cast<const double2*>(M), ld, rows, cols, E);
  LSQ_LAUNCH_CHECK();
}
void embed_vec(Ctx& ctx, const double* u, int n, double* e) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_embed_vec, dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream,
                     reinterpret_cast<const double2*>(u), n, e);
  LSQ_LAUNCH_CHECK();
}
void unembed_vec(Ctx& ctx, const double* e, int n, double* u) {
  if (n <= 0 || !u) return;
  hipLaunchKernelGGL(k_unembed_vec, dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream, e, n,
                     reinterpret_cast<double2*>(u));
  LSQ_LAUNCH_CHECK();
}
void scale_first(Ctx& ctx, double* v, int n, double s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale_first, dim3(1), dim3(64), 0, ctx.stream, v, n, s);
  LSQ_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ copy --
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                size_t n16) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}
__global__ void k_copy1(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                        size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

void dev_copy(Ctx& ctx, void* dst, const void* src, size_t bytes) {
  const size_t n16 = bytes / 16;
  if (n16 > 0) {
    size_t g = (n16 + 255) / 256;
    const size_t cap = (size_t)ctx.num_cu * 16;
    if (g > cap) g = cap;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)g), dim3(256), 0, ctx.stream,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  }
  const size_t tail = bytes - n16 * 16;
  if (tail > 0)
    hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, ctx.stream,
                       static_cast<const unsigned char*>(src) + n16 * 16,
                       static_cast<unsigned char*>(dst) + n16 * 16, tail);
  LSQ_LAUNCH_CHECK();
}

}  // namespace lsq
