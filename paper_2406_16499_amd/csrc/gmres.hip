// Restarted GMRES in FP64 on the device (the inner solver of GMRES-IR,
// Section 5: GMRES on the preconditioned augmented system, FP64 arithmetic
// with the factors stored at u_f).
//
// Arnoldi with classical Gram-Schmidt applied twice (CGS2): per pass one
// kernel forms the partial dot products V_k^T w per 256-row block, the next
// sums them and subtracts V_k h from w (the second pass also accumulates
// ||w||^2 per block).  A one-wave kernel then applies the Givens rotations
// to the new Hessenberg column on the device and records the residual
// estimate and a done flag; the host enqueues the next iteration before it
// reads the previous one's flag (one iteration in flight beyond the test),
// so no iteration waits for a host round trip.  After convergence the
// kernels of an iteration already queued return at once.  The basis is
// column-major N x (restart + 1) in FP64.
#include "engine.hpp"
#include "segs.hpp"

namespace lsq {

constexpr int kCgsRows = 256;        // rows per work-group in the CGS kernels
constexpr int kCgsMax = 32;          // at most restart + 1 <= 32 basis vectors

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// part[b * kCgsMax + j] = sum over the rows of block b of V[i, j] w[i], j < kc.
// Row i of the basis, columns j < kc, into registers (zero elsewhere).  The
// loads are unconditional, at indexes clamped into the basis (rows past N
// read row N - 1, columns past kc read column kc - 1, both then discarded),
// so the compiler issues all of them before the first use: a pass waits for
// memory once, not once per column.  Needs N >= 1 and kc >= 1.
__device__ __forceinline__ void cgs_load_row(const double* __restrict__ V, int ldv, int N, int kc, int i,
                                             double (&v)[kCgsMax]) {
  const size_t ic = (size_t)(i < N ? i : N - 1);
#pragma unroll
  for (int j = 0; j < kCgsMax; ++j) {
    const double x = V[ic + (size_t)(j < kc ? j : kc - 1) * ldv];
    v[j] = (i < N && j < kc) ? x : 0.0;
  }
}

// Block sums of v[j] * wi into part[b * kCgsMax + j] for j < kc (b = this
// block).  Each wave reduces its 32 products with a reduce-scatter over lane
// bits 5..1 (every step halves the values a lane holds; 32 exchanges in all
// instead of 6 per column), after which lane l holds the wave sum of column
// l >> 1; the four waves' sums are added in a fixed order.
static_assert(kCgsMax == 32, "the reduce-scatter maps 32 columns onto lane pairs");
__device__ __forceinline__ void cgs_block_dots(const double (&v)[kCgsMax], double wi, int kc,
                                               double (*red)[kCgsMax], double* __restrict__ part) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double cp[kCgsMax];
#pragma unroll
  for (int j = 0; j < kCgsMax; ++j) cp[j] = v[j] * wi;
#pragma unroll
  for (int m = 32, c = kCgsMax; c > 1; m >>= 1, c >>= 1) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int q = 0; q < c / 2; ++q) {
      const double send = up ? cp[q] : cp[q + c / 2];
      const double keep = up ? cp[q + c / 2] : cp[q];
      cp[q] = keep + __shfl_xor(send, m, 64);
    }
  }
  cp[0] += __shfl_xor(cp[0], 1, 64);
  if ((lane & 1) == 0) red[wv][lane >> 1] = cp[0];
  __syncthreads();
  if (t < kc) part[(size_t)blockIdx.x * kCgsMax + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

__global__ __launch_bounds__(256) void k_cgs_dot(const double* __restrict__ V, int ldv, int N, int kc,
                                                 const double* __restrict__ w, double* __restrict__ part,
                                                 const double* __restrict__ stat) {
  __shared__ double red[4][kCgsMax];
  LSQ_LDS_POISON(red);
  if (stat && stat[2] != 0.0) return;        // converged at an earlier iteration
  const int i = blockIdx.x * kCgsRows + threadIdx.x;
  double v[kCgsMax];
  cgs_load_row(V, ldv, N, kc, i, v);
  const double wi = i < N ? w[i] : 0.0;
  cgs_block_dots(v, wi, kc, red, part);
}

// h = sum of the block partials; w -= V h; hacc (+)= h (written by block 0);
// with nrm, nrm[b] = sum over block b of the updated w[i]^2; with part_next,
// the next pass's partials of V^T w from the updated rows (the sums of
// k_cgs_dot, in its order; a buffer of their own, since other blocks may
// still read part).
__global__ __launch_bounds__(256) void k_cgs_update(const double* __restrict__ V, int ldv, int N, int kc,
                                                    const double* __restrict__ part, int nblk,
                                                    double* __restrict__ w, double* __restrict__ hacc,
                                                    int accumulate, double* __restrict__ nrm,
                                                    const double* __restrict__ stat,
                                                    double* __restrict__ part_next) {
  __shared__ double h[kCgsMax];
  __shared__ double hp[8][kCgsMax];
  __shared__ double red[4];
  __shared__ double red2[4][kCgsMax];
  LSQ_LDS_POISON(h);
  LSQ_LDS_POISON(hp);
  LSQ_LDS_POISON(red);
  LSQ_LDS_POISON(red2);
  if (stat && stat[2] != 0.0) return;        // converged at an earlier iteration
  const int t = threadIdx.x;
  const int i = blockIdx.x * kCgsRows + t;
  double v[kCgsMax];
  cgs_load_row(V, ldv, N, kc, i, v);          // in flight while h is summed
  {
    // the block partials of column j = t & 31, every eighth one per group of
    // 32 threads, then the eight group sums in a fixed order
    const int j = t & (kCgsMax - 1), g = t / kCgsMax;
    double s = 0.0;
    if (j < kc)
      for (int b = g; b < nblk; b += 8) s += part[(size_t)b * kCgsMax + j];
    hp[g][j] = s;
  }
  __syncthreads();
  if (t < kCgsMax) {
    double s = 0.0;
    if (t < kc) {
      s = ((hp[0][t] + hp[1][t]) + (hp[2][t] + hp[3][t])) + ((hp[4][t] + hp[5][t]) + (hp[6][t] + hp[7][t]));
      if (blockIdx.x == 0) hacc[t] = accumulate ? hacc[t] + s : s;
    }
    h[t] = s;                                   // zero past kc: those fma terms leave wi unchanged
  }
  __syncthreads();
  double wi = i < N ? w[i] : 0.0;
#pragma unroll
  for (int j = 0; j < kCgsMax; ++j) wi = fma(-v[j], h[j], wi);
  double sq = wi * wi;
  if (i < N) w[i] = wi;
  if (nrm) {
    sq = block_sum(sq, red);
    if (t == 0) nrm[blockIdx.x] = sq;
  }
  if (part_next) cgs_block_dots(v, wi, kc, red2, part_next);
}

// Device state of one restart cycle: the rotated Hessenberg matrix H
// ((restart + 1) x restart, column-major), the rotations cs, sn and the
// right-hand side g of the small least-squares problem, and
// stat = [|g_{k+1}|, h_{k+1,k}, done, iterations].
struct GivensState {
  double* H; int ldh;
  double* cs; double* sn; double* g;
  double* stat;
};

// Iteration k: the new column h (k + 1 entries from CGS2) and h_{k+1,k} =
// ||w|| (block partial sums of squares) are rotated by the k earlier
// rotations, the new rotation zeroes h_{k+1,k}, and g is updated.  done is
// set once |g_{k+1}| <= tol_abs or h_{k+1,k} = 0 (breakdown: the Krylov space
// holds the solution).  One wave; the work is O(k).
__global__ void k_givens(int k, const double* __restrict__ hcol, const double* __restrict__ nrm,
                         int nblk, GivensState st, double tol_abs) {
  if (st.stat[2] != 0.0) return;
  double sq = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) sq += nrm[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(sq);
  double* col = st.H + (size_t)k * st.ldh;
  for (int i = 0; i <= k; ++i) col[i] = hcol[i];
  col[k + 1] = hn;
  for (int i = 0; i < k; ++i) {
    const double t0 = st.cs[i] * col[i] + st.sn[i] * col[i + 1];
    col[i + 1] = -st.sn[i] * col[i] + st.cs[i] * col[i + 1];
    col[i] = t0;
  }
  const double rho = hypot(col[k], col[k + 1]);
  const double c = rho > 0.0 ? col[k] / rho : 1.0, sn = rho > 0.0 ? col[k + 1] / rho : 0.0;
  st.cs[k] = c;
  st.sn[k] = sn;
  col[k] = rho;
  col[k + 1] = 0.0;
  const double gk = st.g[k];
  st.g[k + 1] = -sn * gk;
  st.g[k] = c * gk;
  st.stat[0] = fabs(st.g[k + 1]);
  st.stat[1] = hn;
  st.stat[3] = (double)(k + 1);
  if (fabs(st.g[k + 1]) <= tol_abs || hn == 0.0) st.stat[2] = 1.0;
}

// v = w / h_{k+1,k} (the next basis vector) into v and, if set, v2 (the
// operator graph's input), unless h is 0 or an earlier iteration converged.
// v may be w itself.
__global__ __launch_bounds__(256) void k_scale_basis(const double* w, double* v, double* __restrict__ v2,
                                                     int N, const double* __restrict__ stat, int k) {
  if (stat[2] != 0.0 && stat[3] < (double)(k + 1)) return;
  const double hn = stat[1];
  if (!(hn > 0.0)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const double x = w[i] * (1.0 / hn);
  v[i] = x;
  if (v2) v2[i] = x;
}

// x += V[:, 0:kc] y
__global__ __launch_bounds__(256) void k_basis_combine(const double* __restrict__ V, int ldv, int N,
                                                       int kc, const double* __restrict__ y,
                                                       double* __restrict__ x) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int j = 0; j < kc; ++j) s = fma(V[(size_t)i + (size_t)j * ldv], y[j], s);
  x[i] += s;
}

// out[i] = c0 x0[i] + c1 sum_q p1[q][i] + c2 sum_q p2[q][i]  (null terms skipped)
__global__ __launch_bounds__(256) void k_combine(double* __restrict__ out, int n, double c0,
                                                 const double* __restrict__ x0, double c1,
                                                 const double* __restrict__ p1, int np1, double c2,
                                                 const double* __restrict__ p2, int np2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = x0 ? c0 * x0[i] : 0.0;
  if (p1) {
    double a = 0.0;
    for (int q = 0; q < np1; ++q) a += p1[(size_t)q * n + i];
    s = fma(c1, a, s);
  }
  if (p2) {
    double a = 0.0;
    for (int q = 0; q < np2; ++q) a += p2[(size_t)q * n + i];
    s = fma(c2, a, s);
  }
  out[i] = s;
}

__global__ __launch_bounds__(256) void k_sumsq_vec(const double* __restrict__ x, int n,
                                                   double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) s = fma(x[i], x[i], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename Tw>
__global__ __launch_bounds__(256) void k_min_abs_diag(const Tw* __restrict__ M, int ld, int nn,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double m = INFINITY;
  for (int i = threadIdx.x; i < nn; i += 256) m = fmin(m, fabs((double)M[(size_t)i + (size_t)i * ld]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <typename Tw>
__global__ __launch_bounds__(256) void k_diag_minmax(const Tw* __restrict__ M, int ld, int nn,
                                                     double* __restrict__ out) {
  __shared__ double rmin[256];
  __shared__ double rmax[256];
  double lo = INFINITY, hi = 0.0;
  for (int i = threadIdx.x; i < nn; i += 256) {
    const double a = fabs((double)M[(size_t)i + (size_t)i * ld]);
    lo = isnan(a) ? a : fmin(lo, a);
    hi = isnan(a) ? a : fmax(hi, a);
  }
  rmin[threadIdx.x] = lo;
  rmax[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double a = rmin[threadIdx.x], b = rmin[threadIdx.x + s];
      const double c = rmax[threadIdx.x], d = rmax[threadIdx.x + s];
      rmin[threadIdx.x] = (isnan(a) || isnan(b)) ? NAN : fmin(a, b);
      rmax[threadIdx.x] = (isnan(c) || isnan(d)) ? NAN : fmax(c, d);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = rmin[0];
    out[1] = rmax[0];
  }
}

// out[2 b] = max |cur - old|, out[2 b + 1] = max |cur| over block b's stride.
__global__ __launch_bounds__(256) void k_change_max(const double* __restrict__ old,
                                                    const double* __restrict__ cur, int n,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  double dm = 0.0, xm = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double c = cur[i];
    dm = fmax(dm, fabs(c - old[i]));
    xm = fmax(xm, fabs(c));
    if (c != c) dm = c;                      // NaN propagates
  }
  dm = block_max(dm, red);
  xm = block_max(xm, red);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = dm;
    out[2 * blockIdx.x + 1] = xm;
  }
}

// Independent FP64 vector segments in one launch (blockIdx.y = segment): the
// copies, reversals, scalings and partial additions between the solves of
// the preconditioners, which would otherwise be one small launch each.
__global__ __launch_bounds__(256) void k_vec_segs(VecSegs v) {
  const VecSeg g = v.s[blockIdx.y];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < g.n; i += gridDim.x * 256) {
    const int j = g.rev ? g.n - 1 - i : i;
    double val = g.src ? g.a * g.src[j] : 0.0;
    if (g.src2 && j >= g.lo) val = val + g.b * g.src2[j];
    g.dst[i] = val * g.c;
  }
}

// Mixed-precision segments (segs.hpp), blockIdx.y = segment.
__device__ __forceinline__ double seg_ld(const void* p, int t, int i) {
  return t == 8 ? static_cast<const double*>(p)[i] : (double)static_cast<const float*>(p)[i];
}
__global__ __launch_bounds__(256) void k_vec_segs_t(VecSegsT v) {
  const VecSegT g = v.s[blockIdx.y];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < g.n; i += gridDim.x * 256) {
    const int j1 = g.rev ? g.n - 1 - i : i, j2 = g.rev2 ? g.n - 1 - i : i;
    double val = g.src ? g.a * seg_ld(g.src, g.ts, j1) : 0.0;
    if (g.src2 && j2 >= g.lo) val = val + g.b * seg_ld(g.src2, g.ts2, j2);
    val = val * g.c;
    if (g.td == 8) static_cast<double*>(g.dst)[i] = val;
    else static_cast<float*>(g.dst)[i] = (float)val;
  }
}

// The operator's three combines in one launch (blockIdx.y = block of F u).
// A work-group covers 64 outputs; its four waves each add every fourth
// partial product of both sums (the partials of one index are 64 contiguous
// words per wave), and the first wave adds the four subtotals in a fixed
// order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_combine3(CombineArgs a0, CombineArgs a1, CombineArgs a2) {
  __shared__ double red[2][4][64];
  LSQ_LDS_POISON(red);
  const CombineArgs a = blockIdx.y == 0 ? a0 : (blockIdx.y == 1 ? a1 : a2);
  if ((int)blockIdx.x * 64 >= a.n) return;      // the whole work-group: no barrier is skipped by part of it
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double t1 = 0.0, t2 = 0.0;
  if (i < a.n) {
    if (a.p1)
      for (int q = wv; q < a.np1; q += 4) t1 += a.p1[(size_t)q * a.n + i];
    if (a.p2)
      for (int q = wv; q < a.np2; q += 4) t2 += a.p2[(size_t)q * a.n + i];
  }
  red[0][wv][lane] = t1;
  red[1][wv][lane] = t2;
  __syncthreads();
  if (wv != 0 || i >= a.n) return;
  double s = a.x0 ? a.c0 * a.x0[i] : 0.0;
  if (a.p1) s = fma(a.c1, (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]), s);
  if (a.p2) s = fma(a.c2, (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]), s);
  a.out[i] = s;
}

// ------------------------------------------------------------------ host --
void vec_segs(Ctx& ctx, std::initializer_list<VecSeg> segs) {
  VecSegs v{};
  int nmax = 0;
  for (const VecSeg& g : segs) {
    if (g.n <= 0) continue;
    if (v.count == kVecSegs) throw std::runtime_error("vec_segs: too many segments");
    if (g.rev && (g.dst == g.src || g.dst == g.src2))
      throw std::runtime_error("vec_segs: a reversed segment cannot work in place");
    v.s[v.count++] = g;
    nmax = std::max(nmax, g.n);
  }
  if (v.count == 0) return;
  const int gx = std::min(ceil_div(nmax, 256), 64);
  hipLaunchKernelGGL(k_vec_segs, dim3(gx, v.count), dim3(256), 0, ctx.stream, v);
  LSQ_LAUNCH_CHECK();
}

void vec_segs_t(Ctx& ctx, std::initializer_list<VecSegT> segs) {
  VecSegsT v{};
  int nmax = 0;
  for (const VecSegT& g : segs) {
    if (g.n <= 0) continue;
    if (v.count == kVecSegsT) throw std::runtime_error("vec_segs_t: too many segments");
    if ((g.rev && g.src == g.dst) || (g.rev2 && g.src2 == g.dst))
      throw std::runtime_error("vec_segs_t: a reversed source cannot be the destination");
    v.s[v.count++] = g;
    nmax = std::max(nmax, g.n);
  }
  if (v.count == 0) return;
  const int gx = std::min(ceil_div(nmax, 256), 64);
  hipLaunchKernelGGL(k_vec_segs_t, dim3(gx, v.count), dim3(256), 0, ctx.stream, v);
  LSQ_LAUNCH_CHECK();
}

void combine3(Ctx& ctx, const CombineArgs& a0, const CombineArgs& a1, const CombineArgs& a2) {
  const int nmax = std::max(a0.n, std::max(a1.n, a2.n));
  if (nmax <= 0) return;
  hipLaunchKernelGGL(k_combine3, dim3(ceil_div(nmax, 64), 3), dim3(256), 0, ctx.stream, a0, a1, a2);
  LSQ_LAUNCH_CHECK();
}

void combine(Ctx& ctx, double* out, int n, double c0, const double* x0, double c1, const double* p1,
             int np1, double c2, const double* p2, int np2) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_combine, dim3(ceil_div(n, 256)), dim3(256), 0, ctx.stream, out, n, c0, x0, c1,
                     p1, np1, c2, p2, np2);
  LSQ_LAUNCH_CHECK();
}

double dev_norm2(Ctx& ctx, const double* x, int n) {
  if (n <= 0) return 0.0;
  int g = ceil_div(n, 256);
  if (g > 64) g = 64;
  double* part = ctx.ws->get<double>(64);
  hipLaunchKernelGGL(k_sumsq_vec, dim3(g), dim3(256), 0, ctx.stream, x, n, part);
  LSQ_LAUNCH_CHECK();
  LSQ_HIP(hipMemcpyAsync(ctx.pin, part, sizeof(double) * g, hipMemcpyDeviceToHost, ctx.stream));
  LSQ_HIP(hipStreamSynchronize(ctx.stream));
  double s = 0.0;
  for (int q = 0; q < g; ++q) s += ctx.pin[q];
  return std::sqrt(s);
}

double rel_change(Ctx& ctx, const double* old, const double* cur, int n) {
  if (n <= 0) return 0.0;
  int g = ceil_div(n, 256);
  if (g > 64) g = 64;
  double* part = ctx.ws->get<double>(128);
  hipLaunchKernelGGL(k_change_max, dim3(g), dim3(256), 0, ctx.stream, old, cur, n, part);
  LSQ_LAUNCH_CHECK();
  LSQ_HIP(hipMemcpyAsync(ctx.pin, part, sizeof(double) * 2 * g, hipMemcpyDeviceToHost, ctx.stream));
  LSQ_HIP(hipStreamSynchronize(ctx.stream));
  double dm = 0.0, xm = 0.0;
  for (int q = 0; q < g; ++q) {
    if (!(ctx.pin[2 * q] <= dm)) dm = ctx.pin[2 * q];
    xm = std::max(xm, ctx.pin[2 * q + 1]);
  }
  if (!(dm == dm)) return INFINITY;
  return xm > 0.0 ? dm / xm : (dm > 0.0 ? INFINITY : 0.0);
}

double min_abs_diag(Ctx& ctx, const QRFactor& f, int o, int nn) {
  if (nn <= 0) return 0.0;
  double* out = ctx.ws->get<double>(1);
  if (f.tw == 8)
    hipLaunchKernelGGL((k_min_abs_diag<double>), dim3(1), dim3(256), 0, ctx.stream,
                       static_cast<const double*>(f.M) + (size_t)o * (f.ld + 1), f.ld, nn, out);
  else
    hipLaunchKernelGGL((k_min_abs_diag<float>), dim3(1), dim3(256), 0, ctx.stream,
                       static_cast<const float*>(f.M) + (size_t)o * (f.ld + 1), f.ld, nn, out);
  LSQ_LAUNCH_CHECK();
  LSQ_HIP(hipMemcpyAsync(ctx.pin, out, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  LSQ_HIP(hipStreamSynchronize(ctx.stream));
  return ctx.pin[0];
}

void diag_minmax(Ctx& ctx, const QRFactor& f, int o, int nn, double* out) {
  out[0] = out[1] = 0.0;
  if (nn <= 0) return;
  double* d = ctx.ws->get<double>(2);
  if (f.tw == 8)
    hipLaunchKernelGGL((k_diag_minmax<double>), dim3(1), dim3(256), 0, ctx.stream,
                       static_cast<const double*>(f.M) + (size_t)o * (f.ld + 1), f.ld, nn, d);
  else
    hipLaunchKernelGGL((k_diag_minmax<float>), dim3(1), dim3(256), 0, ctx.stream,
                       static_cast<const float*>(f.M) + (size_t)o * (f.ld + 1), f.ld, nn, d);
  LSQ_LAUNCH_CHECK();
  LSQ_HIP(hipMemcpyAsync(ctx.pin, d, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  LSQ_HIP(hipStreamSynchronize(ctx.stream));
  out[0] = ctx.pin[0];
  out[1] = ctx.pin[1];
}

// The operator as a replayable HIP graph: apply() is captured once from a
// fixed input buffer to a fixed output buffer; run(u, y) copies u in, replays
// the graph and copies the result out.  If capture is not possible the
// operator runs eagerly (same kernels, launched one by one).
struct GraphOp {
  Ctx& ctx;
  const std::function<void(const double*, double*)>& apply;
  int N;
  double* in = nullptr;
  double* out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  GraphOp(Ctx& c, const std::function<void(const double*, double*)>& f, int n, bool use_graph)
      : ctx(c), apply(f), N(n) {
    // capture on the context's side stream (the caller's stream may be the
    // null stream, which cannot be captured); replays go to ctx.stream
    if (!use_graph || N <= 0 || !ctx.side) return;
    in = ctx.ws->get<double>(N);
    out = ctx.ws->get<double>(N);
    vec_zero(ctx, in, 8, N);
    KernelTimer* saved_timer = ctx.timer;     // no event records inside the graph
    hipStream_t saved_stream = ctx.stream;
    ctx.timer = nullptr;
    ctx.stream = ctx.side;
    bool ok = hipStreamBeginCapture(ctx.side, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      try {
        apply(in, out);
      } catch (const HipError&) {
        ok = false;
      }
      hipGraph_t g = nullptr;
      const bool ended = hipStreamEndCapture(ctx.side, &g) == hipSuccess;
      graph = g;
      ok = ok && ended && graph != nullptr;
    }
    ctx.timer = saved_timer;
    ctx.stream = saved_stream;
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
  }
  ~GraphOp() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  void run(const double* u, double* y) {
    if (!exec) { apply(u, y); return; }
    vec_convert(ctx, in, 8, u, 8, N, false);
    LSQ_HIP(hipGraphLaunch(exec, ctx.stream));
    vec_convert(ctx, y, 8, out, 8, N, false);
  }
};

// Restarted GMRES(restart) from x = 0 on apply(u) = M u, stopping when the
// Arnoldi residual estimate reaches tol ||rhs|| or after maxit iterations in
// total; after every cycle the residual is recomputed from x.
GmresOut gmres(Ctx& ctx, int N, const std::function<void(const double*, double*)>& apply_eager,
               const double* rhs, double* x, int restart, double tol, int maxit, bool use_graph,
               bool give_up) {
  GmresOut out;
  GraphOp op(ctx, apply_eager, N, use_graph);
  auto apply = [&](const double* u, double* y) { op.run(u, y); };
  out.graph = op.exec != nullptr;
  vec_zero(ctx, x, 8, N);
  if (N <= 0) { out.converged = true; return out; }
  if (restart > kCgsMax - 1) restart = kCgsMax - 1;
  if (restart < 1) restart = 1;
  const int nblk = ceil_div(N, kCgsRows);
  const int ldh = restart + 1;
  double* Vb = ctx.ws->get<double>((size_t)N * (restart + 1));
  double* r = ctx.ws->get<double>(N);
  double* part = ctx.ws->get<double>((size_t)nblk * kCgsMax);
  double* part2 = ctx.ws->get<double>((size_t)nblk * kCgsMax);
  // with the operator captured, the Arnoldi loop feeds its fixed input and
  // orthogonalizes its fixed output in place: no copies around the replays
  const bool direct = op.exec != nullptr;
  double* hdev = ctx.ws->get<double>(kCgsMax);
  double* nrm = ctx.ws->get<double>(nblk);
  double* ydev = ctx.ws->get<double>(kCgsMax);
  // device Givens state: H, cs, sn, g, stat (one allocation)
  double* gs = ctx.ws->get<double>((size_t)ldh * restart + 3 * kCgsMax + 4);
  GivensState st{gs, ldh, gs + (size_t)ldh * restart, gs + (size_t)ldh * restart + kCgsMax,
                 gs + (size_t)ldh * restart + 2 * kCgsMax, gs + (size_t)ldh * restart + 3 * kCgsMax};
  // pinned host staging: g and stat for the cycle start, two stat slots for
  // the per-iteration reads, H, g and stat at the cycle end
  double* pin = ctx.pin;
  const size_t hstage = (size_t)ldh * restart + 3 * kCgsMax + 4;
  if (hstage + kCgsMax + 4 + 8 > (size_t)kPinDoubles - 16)
    throw HipError{hipErrorInvalidValue, "GMRES: restart too long for the pinned staging"};
  double* pin_start = pin;                              // g (kCgsMax) then stat (4)
  double* pin_stat = pin + kCgsMax + 4;                 // 2 slots of 4
  double* pin_end = pin_stat + 8;                       // H, cs, sn, g, stat
  hipEvent_t evs[2] = {ctx_event(ctx, 200), ctx_event(ctx, 201)};
  std::vector<double> y(restart);

  vec_convert(ctx, r, 8, rhs, 8, N, false);
  const double beta0 = dev_norm2(ctx, r, N);
  if (beta0 == 0.0) { out.converged = true; return out; }
  double beta = beta0;
  while (out.iters < maxit) {
    if (beta <= tol * beta0) { out.converged = true; break; }
    const double beta_start = beta;
    const int kmax = std::min(restart, maxit - out.iters);
    for (int q = 0; q < kCgsMax + 4; ++q) pin_start[q] = 0.0;
    pin_start[0] = beta;                                // g = beta e1; stat = 0
    LSQ_HIP(hipMemcpyAsync(st.g, pin_start, sizeof(double) * kCgsMax, hipMemcpyHostToDevice, ctx.stream));
    LSQ_HIP(hipMemcpyAsync(st.stat, pin_start + kCgsMax, sizeof(double) * 4, hipMemcpyHostToDevice,
                           ctx.stream));
    vec_segs(ctx, {seg_copy(Vb, r, N, false, 1.0 / beta), seg_copy(direct ? op.in : nullptr, r, direct ? N : 0,
                                                                    false, 1.0 / beta)});
    // iteration k is enqueued before the flag of iteration k - 1 is read
    int launched = 0;
    for (int k = 0; k < kmax; ++k) {
      double* vnext = Vb + (size_t)(k + 1) * N;
      double* w = direct ? op.out : vnext;
      if (direct) LSQ_HIP(hipGraphLaunch(op.exec, ctx.stream));
      else apply(Vb + (size_t)k * N, w);
      const int kc = k + 1;
      // CGS2: the first pass's update also forms the second pass's dots
      hipLaunchKernelGGL(k_cgs_dot, dim3(nblk), dim3(256), 0, ctx.stream, Vb, N, N, kc, w, part, st.stat);
      hipLaunchKernelGGL(k_cgs_update, dim3(nblk), dim3(256), 0, ctx.stream, Vb, N, N, kc, part, nblk, w, hdev,
                         0, nullptr, st.stat, part2);
      hipLaunchKernelGGL(k_cgs_update, dim3(nblk), dim3(256), 0, ctx.stream, Vb, N, N, kc, part2, nblk, w,
                         hdev, 1, nrm, st.stat, nullptr);
      hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, ctx.stream, k, hdev, nrm, nblk, st,
                         tol * beta0);
      hipLaunchKernelGGL(k_scale_basis, dim3(ceil_div(N, 256)), dim3(256), 0, ctx.stream, w, vnext,
                         direct ? op.in : nullptr, N, st.stat, k);
      LSQ_LAUNCH_CHECK();
      LSQ_HIP(hipMemcpyAsync(pin_stat + 4 * (k & 1), st.stat, sizeof(double) * 4, hipMemcpyDeviceToHost,
                             ctx.stream));
      LSQ_HIP(hipEventRecord(evs[k & 1], ctx.stream));
      launched = k + 1;
      if (k >= 1) {
        LSQ_HIP(hipEventSynchronize(evs[(k - 1) & 1]));
        if (pin_stat[4 * ((k - 1) & 1) + 2] != 0.0) break;    // converged at iteration k - 1
      }
    }
    // the cycle's state: H, g and stat after the last queued iteration
    LSQ_HIP(hipMemcpyAsync(pin_end, gs, sizeof(double) * hstage, hipMemcpyDeviceToHost, ctx.stream));
    LSQ_HIP(hipStreamSynchronize(ctx.stream));
    const double* Hh = pin_end;
    const double* g = pin_end + (size_t)ldh * restart + 2 * kCgsMax;
    const double* sth = pin_end + (size_t)ldh * restart + 3 * kCgsMax;
    const int kdone = std::min((int)sth[3], launched);
    const bool done = sth[2] != 0.0;
    out.iters += kdone;
    // y = H(0:kdone, 0:kdone)^{-1} g, x += V y, r = rhs - M x
    for (int i = kdone - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int jj = i + 1; jj < kdone; ++jj) sacc -= Hh[(size_t)i + (size_t)jj * ldh] * y[jj];
      const double hii = Hh[(size_t)i + (size_t)i * ldh];
      y[i] = hii != 0.0 ? sacc / hii : 0.0;
    }
    for (int i = 0; i < kdone; ++i) pin[i] = y[i];
    LSQ_HIP(hipMemcpyAsync(ydev, pin, sizeof(double) * kdone, hipMemcpyHostToDevice, ctx.stream));
    hipLaunchKernelGGL(k_basis_combine, dim3(ceil_div(N, 256)), dim3(256), 0, ctx.stream, Vb, N, N,
                       kdone, ydev, x);
    LSQ_LAUNCH_CHECK();
    apply(x, r);
    vec_axpy(ctx, r, 8, -1.0, rhs, 8, N, false);          // r = M x - rhs
    beta = dev_norm2(ctx, r, N);
    vec_convert(ctx, r, 8, r, 8, N, false, -1.0);           // r = rhs - M x
    if (done && kdone > 0 && std::fabs(g[kdone]) <= tol * beta0) { out.converged = true; break; }
    if (give_up && !(beta <= tol * beta0) && out.iters < maxit) {
      // the cycle reduced the residual by beta / beta_start over kdone
      // iterations; at that rate the rest of the way to tol takes
      // log(tol beta0 / beta) / log(rate) more
      const double ratio = beta / beta_start;
      const double need = ratio > 0.0 && ratio < 1.0 && kdone > 0
                              ? std::log(tol * beta0 / beta) / (std::log(ratio) / kdone)
                              : INFINITY;
      if (!(need <= (double)(maxit - out.iters))) { out.hopeless = true; break; }
    }
    if (kdone == 0) break;
  }
  if (!out.converged) out.converged = beta <= tol * beta0;
  return out;
}

// Y[:, j] = M U[:, j] for k columns (N x k, column-major) through the
// captured graph, one replay per column (the copies in and out run eagerly
// between replays).  *graph_used reports whether capture succeeded.
void graph_apply_columns(Ctx& ctx, int N, const std::function<void(const double*, double*)>& apply,
                         const double* U, double* Y, int k, bool* graph_used) {
  GraphOp op(ctx, apply, N, true);
  if (graph_used) *graph_used = op.exec != nullptr;
  for (int j = 0; j < k; ++j) op.run(U + (size_t)j * N, Y + (size_t)j * N);
}

}  // namespace lsq
