// Persistent batched solver: one work-group per instance.
//
// A batch of small LSE / GLS instances is solved by one launch of one or two
// work-groups per compute unit (batch_blocks_per_cu).  Each work-group takes the
// next instance from a device counter (the host orders the instances longest
// first) and carries out the whole method for it: the generalized RQ (LSE) or
// generalized QR (GLS) factorization of Section 3 in precision T, then
// classical refinement (Algorithms 2 and 4) with the correction solves of
// Algorithms 1 and 3 in T and the augmented residual and stop test
// (eq. lse-stop / gls-stop) in FP64.  Nothing waits on another work-group and
// every work-group leaves the loop once the counter passes the batch, so the
// grid always drains.
//
// The factorizations are blocked Householder QR (LAPACK's convention: H = I -
// tau v v^T, v(j) = 1): each 16-column panel is factored in registers (one
// work-group reduction per column), its compact-WY T comes from an MFMA Gram,
// and the trailing columns are updated on MFMA by all four waves, 16 columns
// per wave at a time.  The correction solves also run on all waves: Q and Q^T
// are applied one panel at a time through the stored T blocks, and the
// triangular solves go in 16-row blocks (one wave solves the diagonal block,
// every thread updates its rows).
#include <chrono>
#include <stdexcept>
#include <thread>
#include <type_traits>

#include "engine.hpp"

namespace lsq {

namespace {

constexpr int kBT = 256;                 // threads per work-group
constexpr int kBW = kBT / 64;            // waves per work-group
constexpr int kVecs = 9;                 // LDS vectors of length kBatchMaxDim
constexpr double kMaxPredictedSteps = 6.0;
constexpr int kRQ = kBatchMaxDim / kBT;  // row slots per thread (rows t + kBT q)

// The out-of-line device functions below take their pointers in explicit
// address spaces, so that their memory operations compile to global and LDS
// instructions rather than generic (flat) ones.
#define LSQ_GLB __attribute__((address_space(1)))
#define LSQ_LDS __attribute__((address_space(3)))

// Buffer loads with the hardware range check: an offset at or beyond the
// resource's byte size reads as 0, so masked loads need neither a branch nor a
// select on the loaded value (either would serialize the loads in flight).
constexpr uint32_t kOob = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

template <typename T> __device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ void bstore<float>(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0)), v), r, off, 0, 0);
}
template <> __device__ __forceinline__ void bstore<double>(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, off, 0, 0);
}

typedef float f32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4v bload4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(f32x4v, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ void bstore4(f32x4v v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b128(
      __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0)), v), r, off, 0, 0);
}

// Wave-uniform copies of values the compiler cannot prove uniform (the
// arguments of out-of-line functions arrive in vector registers).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}
template <typename P>
__device__ __forceinline__ LSQ_LDS P* uni(LSQ_LDS P* p) {
  return (LSQ_LDS P*)(size_t)(unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(size_t)p);
}

// Wave sum with DPP: quad and row-mirror exchanges give every lane its
// 16-lane row sum, and the four row sums are read out as scalars (the result
// is uniform).  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_val(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ T wsum(T v) {
  v += dpp<0xB1>(v);     // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);     // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);    // row_half_mirror
  v += dpp<0x140>(v);    // row_mirror
  return (lane_val(v, 0) + lane_val(v, 16)) + (lane_val(v, 32) + lane_val(v, 48));
}

// Panel width of the blocked QR (a multiple of the 16-row MFMA tile) and
// resident work-groups per compute unit: the LDS panel (kBatchMaxDim x
// (NB + 1)) takes about 70 KB in FP32 (two work-groups per compute unit) and
// 140 KB in FP64 (one).  A work-group is bound by the memory requests its
// compute unit keeps in flight and by the latency of the sequential panel
// steps; wider panels cut the passes over the trailing matrix but lengthen
// every panel step.
template <typename T> struct QrCfg;
template <> struct QrCfg<float> { static constexpr int NB = 16, BLOCKS = 2; };
template <> struct QrCfg<double> { static constexpr int NB = 16, BLOCKS = 1; };

// 16 x 16 x 4 MFMA per precision.  Lane l supplies A[l%16][k] and B[k][l%16]
// for the K index k it holds; accumulator register r of lane l holds row
// drow(l, r) of column l%16.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using V = f32x4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
  using V = f64x4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int l, int r) { return 4 * r + (l >> 4); }
};

template <typename T>
struct BLds {
  static constexpr int NB = QrCfg<T>::NB, PS = NB + 1;
  union {
    struct {
      T Ys[kBatchMaxDim * PS];       // panel, row-major with row stride PS
      T Ts[NB * NB];                 // compact-WY triangle (row-major, upper)
      T Gs[NB * NB];                 // Gram of the panel's reflectors
      T beta[NB], tau[NB];
    } f;
    T vec[kVecs][kBatchMaxDim];      // vectors of the correction solves
  } u;
  static_assert(kVecs * sizeof(float) >= 4 * sizeof(double), "four FP64 vectors fit over the correction vectors");
  static_assert(sizeof(u) >= (kVecs + kBW) * kBatchMaxDim * sizeof(T), "the block products' scratch fits");
  // FP64 vector k (k < 4) of the residual, over the correction vectors
  __device__ double* dvec(int k) { return reinterpret_cast<double*>(&u.vec[0][0]) + kBatchMaxDim * k; }
  // kBW x kBatchMaxDim words after the correction vectors (the panel's
  // space, unused while refining): per-wave partial sums of the block products
  __device__ T* wscratch() { return &u.vec[0][0] + kVecs * kBatchMaxDim; }
  T red[kBW];
  T vred[2 * (kBW + 1) * NB];        // reductions of the register panel and vector kernels
  double dred[kBW * 6];
  int next;
};

__device__ __forceinline__ size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Sum over the work-group; every thread receives it.
template <typename T>
__device__ __forceinline__ T wg_sum1(T v, T* red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < kBW; ++i) s += red[i];
  return s;
}

// max |d_i| / min |d_i| over the diagonal d_i = F[i + i ld], i < nn, of the
// triangle of one factorization (1 for nn = 0; a zero pivot gives infinity).
// Every thread receives it.  red: kBW * 6 doubles.
template <typename T>
__device__ __forceinline__ double wg_diag_ratio(const T* F, int ld, int nn, double* red) {
  double mx = 0.0, mn = INFINITY;
  for (int i = threadIdx.x; i < nn; i += kBT) {
    const double a = fabs((double)F[i + (size_t)i * ld]);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    mn = fmin(mn, __shfl_xor(mn, o, 64));
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[(threadIdx.x >> 6) * 2] = mx;
    red[(threadIdx.x >> 6) * 2 + 1] = mn;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBW; ++i) {
    mx = fmax(mx, red[2 * i]);
    mn = fmin(mn, red[2 * i + 1]);
  }
  __syncthreads();
  if (nn <= 0) return 1.0;
  return mn > 0.0 ? mx / mn : INFINITY;
}

__device__ __forceinline__ void wg_sum6(double v[6], double* red) {
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wsum(v[k]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[(threadIdx.x >> 6) * 6 + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double s = 0.0;
    for (int i = 0; i < kBW; ++i) s += red[i * 6 + k];
    v[k] = s;
  }
}

// f(integral_constant<int, I>) for I = B .. E - 1, so that register arrays
// are only ever indexed by constants.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// -------------------------------------------------- lane exchanges --
// Pairwise exchanges for the reduce-scatter: the gfx950 permlane swaps pair
// lane l with l ^ 32 (l ^ 16); for X, Y in every lane, afterwards X + Y is the
// lane's own value plus its partner's, taken from X in the lower and from Y
// in the upper lane of each pair.
__device__ __forceinline__ void lane_swap32(unsigned& x, unsigned& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
__device__ __forceinline__ void lane_swap16(unsigned& x, unsigned& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
template <int MASK>
__device__ __forceinline__ float pair_sum(float lo, float hi) {
  unsigned x = __float_as_uint(lo), y = __float_as_uint(hi);
  if constexpr (MASK == 32) lane_swap32(x, y); else lane_swap16(x, y);
  return __uint_as_float(x) + __uint_as_float(y);
}
template <int MASK>
__device__ __forceinline__ double pair_sum(double lo, double hi) {
  const unsigned long long a = (unsigned long long)__double_as_longlong(lo);
  const unsigned long long b = (unsigned long long)__double_as_longlong(hi);
  unsigned xl = (unsigned)a, xh = (unsigned)(a >> 32), yl = (unsigned)b, yh = (unsigned)(b >> 32);
  if constexpr (MASK == 32) { lane_swap32(xl, yl); lane_swap32(xh, yh); }
  else { lane_swap16(xl, yl); lane_swap16(xh, yh); }
  const double x = __longlong_as_double((long long)(((unsigned long long)xh << 32) | xl));
  const double y = __longlong_as_double((long long)(((unsigned long long)yh << 32) | yl));
  return x + y;
}
// DPP exchanges pairing each lane with one whose bit MASK differs and whose
// higher bits agree (within a row of 16): xor 8, mirror within 8, mirror
// within 4, xor 1.
template <int MASK> struct PairDpp;
template <> struct PairDpp<8> { static constexpr int ctrl = 0x128; };   // row_ror:8
template <> struct PairDpp<4> { static constexpr int ctrl = 0x141; };   // row_half_mirror
template <> struct PairDpp<2> { static constexpr int ctrl = 0x1B; };    // quad_perm [3,2,1,0]
template <> struct PairDpp<1> { static constexpr int ctrl = 0xB1; };    // quad_perm [1,0,3,2]

// Reduce-scatter of NV (a power of two <= 64) per-lane values over the wave:
// every lane returns the wave total of value index lane >> (6 - log2 NV).
// Each halving step keeps the half of the values selected by one lane bit and
// adds the partner lane's copy of it.
template <typename T, int NV, int HALF, int MASK>
__device__ __forceinline__ void rs_step(T (&v)[NV], int lane) {
  if constexpr (HALF >= 1) {
    if constexpr (MASK >= 16) {
#pragma unroll
      for (int k = 0; k < HALF; ++k) v[k] = pair_sum<MASK>(v[k], v[k + HALF]);
    } else {
      const bool up = (lane & MASK) != 0;
#pragma unroll
      for (int k = 0; k < HALF; ++k) {
        const T keep = up ? v[k + HALF] : v[k];
        const T send = up ? v[k] : v[k + HALF];
        v[k] = keep + dpp<PairDpp<MASK>::ctrl>(send);
      }
    }
    rs_step<T, NV, HALF / 2, MASK / 2>(v, lane);
  }
}
template <typename T, int MASK>
__device__ __forceinline__ T rs_tail(T r) {
  if constexpr (MASK >= 1) {
    r += dpp<PairDpp<MASK>::ctrl>(r);
    return rs_tail<T, MASK / 2>(r);
  }
  return r;
}
template <typename T, int NV>
__device__ __forceinline__ T wave_reduce_scatter(T (&v)[NV]) {
  static_assert(NV >= 4 && NV <= 64, "the tail exchanges stay inside a row of 16");
  const int lane = threadIdx.x & 63;
  rs_step<T, NV, NV / 2, 32>(v, lane);
  return rs_tail<T, 32 / NV>(v[0]);
}

typedef double f64x2v __attribute__((ext_vector_type(2)));

// Rows g .. g + 3 of a padded column at byte offset off (zeros when !ok).
template <typename T>
__device__ __forceinline__ void load_rows4(__amdgpu_buffer_rsrc_t rs, bool ok, uint32_t off, T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    const f32x4v x = bload4(rs, ok ? off : kOob);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = x[e];
  } else {
    const f64x2v a = __builtin_bit_cast(f64x2v, __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? off : kOob, 0, 0));
    const f64x2v b = __builtin_bit_cast(f64x2v, __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? off + 16 : kOob, 0, 0));
    v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
  }
}
template <typename T>
__device__ __forceinline__ void store_rows4(__amdgpu_buffer_rsrc_t rs, bool ok, uint32_t off, const T (&v)[4]) {
  using R = decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0));
  if constexpr (sizeof(T) == 4) {
    bstore4(f32x4v{v[0], v[1], v[2], v[3]}, rs, ok ? off : kOob);
  } else {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(R, f64x2v{v[0], v[1]}), rs, ok ? off : kOob, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(R, f64x2v{v[2], v[3]}), rs, ok ? off + 16 : kOob, 0, 0);
  }
}

// ------------------------------------------------------------ Householder --
// Blocked Householder QR (LAPACK's convention: H = I - tau v v^T, v(j) = 1;
// Q = H_0 ... H_{k-1}; per panel H_j0 ... H_{j0+nb-1} = I - Y T Y^T with T
// upper triangular).  A panel of NB columns is factored in LDS; its T comes
// from the Gram Y^T Y; the trailing columns are updated with
// C <- C - Y (T^T (Y^T C)), each wave streaming CG columns at a time through
// registers (one read and one write of C per panel).

// Panel rows j0 .. j0 + Lr of columns j0 .. j0 + nbj of M into Ys (columns
// beyond nbj zero).  unit: load the reflector view (1 on the diagonal, 0
// above) of a factored panel instead of the raw columns.
template <typename T>
__device__ __forceinline__ void stage_panel(const T* M, int ld, int j0, int nbj, int Lr, T* Ys,
                                            bool unit) {
  constexpr int NB = QrCfg<T>::NB, PS = NB + 1, RS = kBatchMaxDim / kBT;
  const T* base = M + j0 + (size_t)j0 * ld;
  const auto rs = rsrc(base, ((size_t)(NB - 1) * ld + Lr) * sizeof(T));
  T v[RS][NB];
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int i = threadIdx.x + kBT * s;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const bool in = i < Lr && a < nbj && (!unit || i > a);
      v[s][a] = bload<T>(rs, in ? (uint32_t)((i + (size_t)a * ld) * sizeof(T)) : kOob);
      if (unit && i == a && a < nbj) v[s][a] += (T)1;
    }
  }
  const int Lr16 = (Lr + 15) & ~15;          // rows Lr .. Lr16 zero (see panel_factor)
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int i = threadIdx.x + kBT * s;
    if (i < Lr16)
#pragma unroll
      for (int a = 0; a < NB; ++a) Ys[i * PS + a] = v[s][a];
  }
  __syncthreads();
}

// Householder QR of the panel M[j0 : j0 + Lr, j0 : j0 + nbj) (nbj <= Lr) in
// registers: thread t holds panel rows 4t .. 4t + 3 of the NB columns.  For
// column a one work-group reduction gives both ||x(a+1:)||^2 and the products
// x(a+1:)^T c_b with the later columns b (wave reduce-scatter, then the four
// waves' partials and row a through LDS, one barrier); every thread then
// derives H_a = I - tau v v^T (v = [1; x(a+1:) / (alpha - beta)]) and applies
// it to its rows.  On return M holds R on and above the diagonal and the
// reflectors below it, Ys the reflectors (unit diagonal, zeros above, zero
// columns beyond nbj), f.beta the diagonal of R and f.tau the scalars.
template <typename T>
__device__ __forceinline__ void panel_factor(BLds<T>& L, T* M, int ld, int j0, int nbj, int Lr) {
  constexpr int NB = QrCfg<T>::NB, PS = NB + 1;
  static_assert(kBT * 4 == kBatchMaxDim, "thread t holds rows 4t .. 4t + 3");
  T* Ys = L.u.f.Ys;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g0 = 4 * t;
  const bool rok = g0 < Lr;
  const auto rs = rsrc(M + j0 + (size_t)j0 * ld, ((size_t)(nbj - 1) * ld + ((Lr + 3) & ~3)) * sizeof(T));
  T P[NB][4];
#pragma unroll
  for (int c = 0; c < NB; ++c) load_rows4(rs, rok && c < nbj, (uint32_t)((g0 + (size_t)c * ld) * sizeof(T)), P[c]);
  static_for<0, NB>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    if (a < nbj) {
      T* buf = L.vred + (a & 1) * (kBW + 1) * NB;
      T s[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        s[b] = 0;
        if (b < a) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) s[b] += (g0 + e > a ? P[a][e] : (T)0) * P[b][e];
      }
      const T sv = wave_reduce_scatter<T, NB>(s);
      if ((lane & 3) == 0) buf[w * NB + (lane >> 2)] = sv;
      if (t == (a >> 2)) {
#pragma unroll
        for (int b = a; b < NB; ++b) buf[kBW * NB + b] = P[b][a & 3];
      }
      __syncthreads();
      T S[NB], Ra[NB];
#pragma unroll
      for (int b = a; b < NB; ++b) {
        S[b] = (buf[b] + buf[NB + b]) + (buf[2 * NB + b] + buf[3 * NB + b]);
        Ra[b] = buf[kBW * NB + b];
      }
      const T alpha = Ra[a], ss = S[a];
      T tau = 0, scal = 1, beta = alpha;
      if (ss > (T)0) {
        const T nrm = sqrt(alpha * alpha + ss);
        beta = alpha >= (T)0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = (T)1 / (alpha - beta);
      }
      T v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = g0 + e;
        v[e] = row > a ? P[a][e] * scal : (row == a ? (T)1 : (T)0);
      }
#pragma unroll
      for (int b = a + 1; b < NB; ++b) {
        const T d = tau * (Ra[b] + scal * S[b]);
#pragma unroll
        for (int e = 0; e < 4; ++e) P[b][e] -= d * v[e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = g0 + e;
        P[a][e] = row > a ? v[e] : (row == a ? beta : P[a][e]);
      }
      if (t == 0) {
        L.u.f.beta[a] = beta;
        L.u.f.tau[a] = tau;
      }
    }
  });
#pragma unroll
  for (int c = 0; c < NB; ++c) store_rows4(rs, rok && c < nbj, (uint32_t)((g0 + (size_t)c * ld) * sizeof(T)), P[c]);
  // rows Lr .. 16 ceil(Lr / 16) are zero, so that the MFMA loops over
  // 16-row chunks need no row masks
  const int Lr16 = (Lr + 15) & ~15;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = g0 + e;
    if (row >= Lr16) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      Ys[row * PS + c] = (c < nbj && row < Lr) ? (row > c ? P[c][e] : (row == c ? (T)1 : (T)0)) : (T)0;
  }
  __syncthreads();
}

// Ts (upper, row-major NB x NB) of the panel in Ys with scalars tau[0:nbj):
// T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) (Y(:, 0:j)^T y_j), the
// Gram Y^T Y from MFMA over 16-row chunks (16 x 16 blocks).  One wave.
template <typename T>
__device__ __forceinline__ void panel_t(BLds<T>& L, int nbj, int Lr, const T* tau) {
  constexpr int NB = QrCfg<T>::NB, PS = NB + 1, NBB = NB / 16;
  using MF = Mfma<T>;
  const T* Ys = L.u.f.Ys;
  T* Ts = L.u.f.Ts;
  T* Gs = L.u.f.Gs;
  const int lane = threadIdx.x & 63, w = uni(threadIdx.x >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  if (w == 0) {
    typename MF::V g[NBB][NBB];
#pragma unroll
    for (int bi = 0; bi < NBB; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBB; ++bj) g[bi][bj] = typename MF::V{0, 0, 0, 0};
    const int nk = (Lr + 15) >> 4;
    for (int kc = 0; kc < nk; ++kc) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = 16 * kc + 4 * lg + t;
        const bool ok = row < Lr;
        T yv[NBB];
#pragma unroll
        for (int b = 0; b < NBB; ++b) {
          const T y = Ys[(ok ? row : 0) * PS + 16 * b + lc];
          yv[b] = ok ? y : (T)0;
        }
#pragma unroll
        for (int bi = 0; bi < NBB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NBB; ++bj) g[bi][bj] = MF::mma(yv[bi], yv[bj], g[bi][bj]);
      }
    }
    // upper blocks from the products; the lower ones are written as zeros (the
    // recurrence multiplies them by zeros, and LDS may hold any bit pattern)
#pragma unroll
    for (int bi = 0; bi < NBB; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBB; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Gs[(16 * bi + MF::drow(lane, r)) * NB + 16 * bj + lc] = bj >= bi ? g[bi][bj][r] : (T)0;
    // lane i keeps row i of T in registers; column j of G is read in one
    // batch of (broadcast) LDS loads per step
    T trow[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) trow[l] = 0;
    for (int j = 0; j < nbj; ++j) {
      const T tj = tau[j];
      T sacc = 0;
#pragma unroll
      for (int l = 0; l < NB; ++l) sacc += trow[l] * Gs[l * NB + j];
      const T val = lane < j ? -tj * sacc : (lane == j ? tj : (T)0);
#pragma unroll
      for (int l = 0; l < NB; ++l) trow[l] = (l == j) ? val : trow[l];
    }
    if (lane < NB)
#pragma unroll
      for (int l = 0; l < NB; ++l) Ts[lane * NB + l] = trow[l];
  }
  __syncthreads();
}

// C (Lr x nc, ldc) <- C - Y (T^T (Y^T C)) with Y = Ys (Lr x NB), T = Ts, on
// MFMA: each wave takes 16 columns at a time.  W = Y^T C accumulates over
// 16-row chunks (lane l supplies four consecutive rows of its column), W' =
// T^T W and C - Y W' take their B operand from the accumulator registers
// themselves: every product is a sum over an index whose order the lanes
// agree on, so the K order may follow the accumulator layout.  The panel's
// NB columns form NB / 16 blocks of the 16 x 16 tiles.
// Lp >= Lr rows of each column are addressable (zero padding beyond Lr), and
// groups of 4 rows starting at a multiple of 4 never cross Lp: the W pass
// moves such a group with one (FP32) or two (FP64) 16-byte accesses per lane,
// and so does the update in FP32.
// LP (FP32 storage only): the BF16 factorization.  The two products with the
// panel take BF16 inputs (rounded to nearest even) with FP32 accumulation: a
// lane's four rows of two consecutive chunks are the eight K values of one
// 16 x 16 x 32 BF16 MFMA in the W pass, and its four values of W' the four of
// one 16 x 16 x 16 BF16 MFMA in the update (A and B take the same lane slots,
// so the K order is again the lanes' own).  W' = T^T W stays in FP32.
template <typename T, bool LP = false>
__device__ __forceinline__ void apply_block_qt(BLds<T>& L, int Lr, int Lp, T* C, int ldc, int nc) {
  static_assert(!LP || sizeof(T) == 4, "BF16 updates of FP32 storage");
  constexpr int NB = QrCfg<T>::NB, PS = NB + 1, NBB = NB / 16;
  constexpr int KB = sizeof(T) == 4 ? 8 : 4;    // 16-row chunks per batch of loads
  using MF = Mfma<T>;
  using V = typename MF::V;
  const T* Ys = L.u.f.Ys;
  const T* Ts = L.u.f.Ts;
  const int lane = threadIdx.x & 63, w = uni(threadIdx.x >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  if (nc <= 0) return;
  const auto rs = rsrc(C, ((size_t)(nc - 1) * ldc + Lp) * sizeof(T));
  const int nk = (Lr + 15) >> 4;
  for (int c0 = 16 * w; c0 < nc; c0 += 16 * kBW) {
    const int col = c0 + lc;
    const bool cok = col < nc;
    // Both passes run over batches of KB 16-row chunks with two register
    // sets: the next batch's loads are issued before the current batch's
    // MFMAs, and loads beyond the last chunk read zeros (out of range).
    // W = Y^T C (block b holds rows 16 b .. 16 b + 15 of W); lane l supplies
    // rows g .. g + 3 of its column, g = 16 chunk + 4 (l / 16).
    // FP32: lane l supplies rows g .. g + 3 of its column, g = 16 chunk +
    // 4 (l / 16), one 16-byte load.  FP64: rows 2 (l / 16) + {0, 1} and
    // 8 + 2 (l / 16) + {0, 1} (krow), two 16-byte loads that each cover 64
    // contiguous bytes of the column across the four lane groups.
    auto krow = [&](int t) { return sizeof(T) == 4 ? 4 * lg + t : (t < 2 ? 2 * lg + t : 6 + 2 * lg + t); };
    auto load1 = [&](int kb, T (&cv)[KB][4]) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        if constexpr (sizeof(T) == 4) {
          const int g = 16 * (kb + u) + 4 * lg;
          load_rows4(rs, g < Lr && cok, (uint32_t)((g + (size_t)col * ldc) * sizeof(T)), cv[u]);
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int g = 16 * (kb + u) + 8 * h + 2 * lg;
            const f64x2v v = __builtin_bit_cast(f64x2v, __builtin_amdgcn_raw_buffer_load_b128(
                rs, (g < Lr && cok) ? (uint32_t)((g + (size_t)col * ldc) * sizeof(T)) : kOob, 0, 0));
            cv[u][2 * h] = v[0];
            cv[u][2 * h + 1] = v[1];
          }
        }
      }
    };
    // two accumulators (even and odd chunks) halve the dependent MFMA chain
    V acc[NBB], acc2[NBB];
#pragma unroll
    for (int b = 0; b < NBB; ++b) acc[b] = acc2[b] = V{0, 0, 0, 0};
    auto comp1 = [&](int kb, const T (&cv)[KB][4]) {
      // the batch's Y values first; chunks past the last one (whose C rows
      // read as zeros) take the last chunk's finite Y rows, as Ys rows from
      // 16 nk on are not zeroed
      T yv[KB][4][NBB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int ch = kb + u < nk ? kb + u : nk - 1;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int b = 0; b < NBB; ++b) yv[u][t][b] = Ys[(16 * ch + krow(t)) * PS + 16 * b + lc];
      }
      if constexpr (LP) {
        static_assert(KB % 2 == 0, "chunk pairs");
#pragma unroll
        for (int u = 0; u < KB; u += 2)
#pragma unroll
          for (int b = 0; b < NBB; ++b) {
            bf16x8 av, bv;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              av[t] = (__bf16)(float)yv[u][t][b];
              av[4 + t] = (__bf16)(float)yv[u + 1][t][b];
              bv[t] = (__bf16)(float)cv[u][t];
              bv[4 + t] = (__bf16)(float)cv[u + 1][t];
            }
            if ((u >> 1) & 1) acc2[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc2[b], 0, 0, 0);
            else acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[b], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int u = 0; u < KB; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int b = 0; b < NBB; ++b) {
              if (u & 1) acc2[b] = MF::mma(yv[u][t][b], cv[u][t], acc2[b]);
              else acc[b] = MF::mma(yv[u][t][b], cv[u][t], acc[b]);
            }
      }
    };
    {
      // (the scheduling barriers keep each batch's loads ahead of the
      // previous batch's MFMAs)
      T ca[KB][4], cb[KB][4];
      load1(0, ca);
      for (int kb = 0; kb < nk; kb += 2 * KB) {
        load1(kb + KB, cb);
        __builtin_amdgcn_sched_barrier(0);
        comp1(kb, ca);
        load1(kb + 2 * KB, ca);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + KB < nk) comp1(kb + KB, cb);
      }
    }
#pragma unroll
    for (int b = 0; b < NBB; ++b) acc[b] += acc2[b];
    // W' = T^T W; T is upper triangular, so block o takes blocks i <= o
    V wp[NBB];
#pragma unroll
    for (int o = 0; o < NBB; ++o) {
      wp[o] = V{0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i <= o; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int b = 16 * i + MF::drow(lane, t);
          wp[o] = MF::mma(Ts[b * NB + 16 * o + lc], acc[i][t], wp[o]);
        }
    }
    // C <- C - Y W' in the accumulator layout
    auto load2 = [&](int kb, V (&d)[KB]) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        if constexpr (sizeof(T) == 4) {
          const int g = 16 * (kb + u) + 4 * lg;         // accumulator rows g .. g + 3
          d[u] = bload4(rs, (g < Lr && cok) ? (uint32_t)((g + (size_t)col * ldc) * 4) : kOob);
        } else {
          // FP64 computes the transposed tile: register r of lane l holds row
          // 16 chunk + l % 16 of column c0 + drow(l, r)
          const int row = 16 * (kb + u) + lc;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cc = c0 + MF::drow(lane, r);
            d[u][r] = bload<T>(rs, (row < Lr && cc < nc) ? (uint32_t)((row + (size_t)cc * ldc) * sizeof(T)) : kOob);
          }
        }
      }
    };
    auto comp2 = [&](int kb, V (&d)[KB]) {
      T yv[KB][NBB][4];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int ch = kb + u < nk ? kb + u : nk - 1;
#pragma unroll
        for (int b = 0; b < NBB; ++b)
#pragma unroll
          for (int t = 0; t < 4; ++t) yv[u][b][t] = Ys[(16 * ch + lc) * PS + 16 * b + MF::drow(lane, t)];
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {                  // (chunks past the last one are not stored)
#pragma unroll
        for (int b = 0; b < NBB; ++b) {
          if constexpr (LP) {
            bf16x4 av, bv;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              av[t] = (__bf16)(float)-yv[u][b][t];
              bv[t] = (__bf16)(float)wp[b][t];
            }
            d[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, av),
                                                             __builtin_bit_cast(s16x4, bv), d[u], 0, 0, 0);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              // FP32: (-Y) W'; FP64: W'^T (-Y)^T, the same K order (wp[b][t]
              // of lane l is W' row 16 b + drow(l, t) = 16 b + 4 t + l / 16)
              if constexpr (sizeof(T) == 4) d[u] = MF::mma(-yv[u][b][t], wp[b][t], d[u]);
              else d[u] = MF::mma(wp[b][t], -yv[u][b][t], d[u]);
            }
          }
        }
        if constexpr (sizeof(T) == 4) {
          const int g = 16 * (kb + u) + 4 * lg;
          bstore4(d[u], rs, (g < Lr && cok) ? (uint32_t)((g + (size_t)col * ldc) * 4) : kOob);
        } else {
          const int row = 16 * (kb + u) + lc;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cc = c0 + MF::drow(lane, r);
            bstore<T>(d[u][r], rs, (row < Lr && cc < nc) ? (uint32_t)((row + (size_t)cc * ldc) * sizeof(T)) : kOob);
          }
        }
      }
    };
    {
      V da[KB], db[KB];
      load2(0, da);
      for (int kb = 0; kb < nk; kb += 2 * KB) {
        load2(kb + KB, db);
        __builtin_amdgcn_sched_barrier(0);
        comp2(kb, da);
        load2(kb + 2 * KB, da);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + KB < nk) comp2(kb + KB, db);
      }
    }
  }
}

// Householder QR of the r x c matrix M (ld) in place: R on and above the
// diagonal, the reflectors below, tau[min(r, c)], and each panel's T
// (NB x NB, row-major) at Tst + panel * NB * NB.
template <typename T, bool LP>
__device__ __noinline__ void wg_geqrf_impl(LSQ_GLB T* Mg, int ld, int r, int c, LSQ_GLB T* taug,
                                           LSQ_GLB T* Tstg, LSQ_LDS BLds<T>* Lp) {
  T* M = (T*)uni(Mg);
  T* tau = (T*)uni(taug);
  T* Tst = (T*)uni(Tstg);
  BLds<T>& L = *(BLds<T>*)uni(Lp);
  ld = uni(ld); r = uni(r); c = uni(c);
  constexpr int NB = QrCfg<T>::NB;
  const int kq = r < c ? r : c;
  for (int j0 = 0, pan = 0; j0 < kq; j0 += NB, ++pan) {
    const int nbj = kq - j0 < NB ? kq - j0 : NB, Lr = r - j0;
    panel_factor(L, M, ld, j0, nbj, Lr);
    panel_t(L, nbj, Lr, L.u.f.tau);
    // scalars and T to storage
    for (int e = threadIdx.x; e < NB * NB; e += kBT) Tst[(size_t)pan * NB * NB + e] = L.u.f.Ts[e];
    if (threadIdx.x < nbj) tau[j0 + threadIdx.x] = L.u.f.tau[threadIdx.x];
    apply_block_qt<T, LP>(L, Lr, ld - j0, M + j0 + (size_t)(j0 + nbj) * ld, ld, c - j0 - nbj);
    __syncthreads();
  }
}

template <typename T, bool LP = false>
__device__ __forceinline__ void wg_geqrf(T* M, int ld, int r, int c, T* tau, T* Tst, BLds<T>& L) {
  wg_geqrf_impl<T, LP>((LSQ_GLB T*)M, ld, r, c, (LSQ_GLB T*)tau, (LSQ_GLB T*)Tst, (LSQ_LDS BLds<T>*)&L);
}

// X (r x ncols, ldx) <- Q^T X for the k reflectors stored in M (ld) by
// wg_geqrf, panel by panel.
template <typename T, bool LP>
__device__ __noinline__ void wg_apply_qt_impl(const LSQ_GLB T* Mg, int ld, int r, int k,
                                              const LSQ_GLB T* Tstg, LSQ_GLB T* Xg, int ldx,
                                              int ncols, LSQ_LDS BLds<T>* Lp) {
  const T* M = (const T*)uni(Mg);
  const T* Tst = (const T*)uni(Tstg);
  T* X = (T*)uni(Xg);
  BLds<T>& L = *(BLds<T>*)uni(Lp);
  ld = uni(ld); r = uni(r); k = uni(k); ldx = uni(ldx); ncols = uni(ncols);
  constexpr int NB = QrCfg<T>::NB;
  for (int j0 = 0, pan = 0; j0 < k; j0 += NB, ++pan) {
    const int nbj = k - j0 < NB ? k - j0 : NB, Lr = r - j0;
    for (int e = threadIdx.x; e < NB * NB; e += kBT) L.u.f.Ts[e] = Tst[(size_t)pan * NB * NB + e];
    stage_panel(M, ld, j0, nbj, Lr, L.u.f.Ys, true);
    apply_block_qt<T, LP>(L, Lr, ldx - j0, X + j0, ldx, ncols);
    __syncthreads();
  }
}

template <typename T, bool LP = false>
__device__ __forceinline__ void wg_apply_qt(const T* M, int ld, int r, int k, const T* Tst, T* X,
                                            int ldx, int ncols, BLds<T>& L) {
  wg_apply_qt_impl<T, LP>((const LSQ_GLB T*)M, ld, r, k, (const LSQ_GLB T*)Tst, (LSQ_GLB T*)X, ldx,
                      ncols, (LSQ_LDS BLds<T>*)&L);
}

// ------------------------------------------- work-group vector kernels --
// The correction solves on all waves.  A vector of length <= kBatchMaxDim
// lives in LDS; for the matrix work thread t owns rows 4t .. 4t + 3, which a
// padded column delivers in one (FP32) or two (FP64) 16-byte loads.

// y (LDS, length r) <- Q^T y (trans) or Q y, Q = H_0 ... H_{k-1} from the
// reflectors of M (ld) and the panels' T (NB x NB, row-major, at Tst; the
// panel's product is I - Y T Y^T), one panel at a time: z = Y^T y by a wave
// reduce-scatter and LDS, w = T^T z (T z) on NB lanes of each wave, y -= Y w.
// In FP32 the next panel's columns load while the current one is reduced.
template <typename T, bool TRANS>
__device__ __forceinline__ void wg_apply_q_vec_impl(const LSQ_GLB T* Mg, int ld, int r, int k,
                                                 const LSQ_GLB T* Tstg, LSQ_LDS T* yl,
                                                 LSQ_LDS T* redl) {
  constexpr bool trans = TRANS;
  constexpr int NB = QrCfg<T>::NB;
  static_assert(NB == 16 && kBT * 4 == kBatchMaxDim, "thread t owns rows 4t .. 4t + 3");
  constexpr bool PF = sizeof(T) == 4;
  const T* M = (const T*)uni(Mg);
  const LSQ_GLB T* Tst = uni(Tstg);
  LSQ_LDS T* y = uni(yl);
  LSQ_LDS T* red = uni(redl);
  ld = uni(ld); r = uni(r); k = uni(k);
  const int t = threadIdx.x, lane = t & 63, w = uni(t >> 6), g0 = 4 * t;
  const int np = (k + NB - 1) / NB;
  T yv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) yv[e] = g0 + e < r ? y[g0 + e] : (T)0;
  auto panel = [&](int b) { return trans ? b : np - 1 - b; };
  // (b >= np loads nothing: every offset is out of range; it keeps the
  // prefetch unconditional, so the compiler waits only for the panel in use)
  auto load = [&](int b, T (&Yv)[NB][4], T (&Tv)[NB]) {
    const bool valid = b < np;
    const int j0 = valid ? panel(b) * NB : 0, nbj = valid ? (k - j0 < NB ? k - j0 : NB) : 1;
    const auto rs = rsrc(M + (size_t)j0 * ld, (size_t)nbj * ld * sizeof(T));
    const bool act = valid & (g0 + 3 >= j0) & (g0 < r);   // (no short-circuit branches)
#pragma unroll
    for (int c = 0; c < NB; ++c) load_rows4(rs, act, (uint32_t)((g0 + (size_t)c * ld) * sizeof(T)), Yv[c]);
    // lane c < NB of every wave: column c of T (w = T^T z) or row c (w = T z)
    const auto rt = rsrc((const T*)Tst + (size_t)(j0 / NB) * NB * NB, NB * NB * sizeof(T));
#pragma unroll
    for (int i = 0; i < NB; ++i)
      Tv[i] = bload<T>(rt, (valid & (lane < NB) & (i < nbj)) ? (uint32_t)((trans ? i * NB + lane : lane * NB + i) * sizeof(T)) : kOob);
  };
  auto step = [&](int b, T (&Yv)[NB][4], T (&Tv)[NB], T (&Yn)[NB][4], T (&Tn)[NB]) {
    const int j0 = panel(b) * NB, nbj = k - j0 < NB ? k - j0 : NB;
    // the diagonal block (1 on it, 0 above) lies in the rows of one wave,
    // which alone takes the (uniform) branch
    if (w == j0 / (4 * 64)) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = g0 + e;
          Yv[c][e] = row < j0 + c ? (T)0 : (row == j0 + c ? (c < nbj ? (T)1 : (T)0) : Yv[c][e]);
        }
    }
    T pz[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) pz[c] = (Yv[c][0] * yv[0] + Yv[c][1] * yv[1]) + (Yv[c][2] * yv[2] + Yv[c][3] * yv[3]);
    if constexpr (PF) {
      load(b + 1, Yn, Tn);
      __builtin_amdgcn_sched_barrier(0);
    }
    const T zc = wave_reduce_scatter<T, NB>(pz);    // lanes 4c .. 4c + 3: the wave's z_c
    // the four waves' partials meet in LDS (two buffers by panel parity, so
    // one barrier per panel suffices); every wave then forms w on its lanes
    // 0 .. NB - 1 and broadcasts it with readlanes
    LSQ_LDS T* buf = red + (b & 1) * kBW * NB;
    if ((lane & 3) == 0) buf[w * NB + (lane >> 2)] = zc;
    __syncthreads();
    T acc = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const T zi = (buf[i] + buf[NB + i]) + (buf[2 * NB + i] + buf[3 * NB + i]);
      acc += Tv[i] * zi;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const T wc = lane_val(acc, c);
#pragma unroll
      for (int e = 0; e < 4; ++e) yv[e] -= Yv[c][e] * wc;
    }
  };
  if constexpr (PF) {
    T Ya[NB][4], Yb[NB][4], Ta[NB], Tb[NB];
    if (np > 0) load(0, Ya, Ta);
    for (int b = 0; b < np; b += 2) {
      step(b, Ya, Ta, Yb, Tb);
      if (b + 1 < np) step(b + 1, Yb, Tb, Ya, Ta);
    }
  } else {
    T Ya[NB][4], Ta[NB];
    for (int b = 0; b < np; ++b) {
      load(b, Ya, Ta);
      step(b, Ya, Ta, Ya, Ta);
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (g0 + e < r) y[g0 + e] = yv[e];
  __syncthreads();
}

// Out-of-line copy: the FP32 kernel keeps these steps as calls (its 256
// registers per lane cannot hold them inline); the FP64 kernel, with twice
// the register file per wave, inlines them and saves the callee-saved
// register spills of every call.
template <typename T, bool TRANS>
__device__ __noinline__ void wg_apply_q_vec_call(const LSQ_GLB T* Mg, int ld, int r, int k,
                                                 const LSQ_GLB T* Tstg, LSQ_LDS T* yl,
                                                 LSQ_LDS T* redl) {
  wg_apply_q_vec_impl<T, TRANS>(Mg, ld, r, k, Tstg, yl, redl);
}
template <typename T>
__device__ __forceinline__ void wg_apply_q_vec(const T* M, int ld, int r, int k, const T* Tst, T* y,
                                               T* red, bool trans) {
  const auto Mg = (const LSQ_GLB T*)M;
  const auto Tg = (const LSQ_GLB T*)Tst;
  const auto yl = (LSQ_LDS T*)y;
  const auto rl = (LSQ_LDS T*)red;
  if constexpr (sizeof(T) == 4) {
    if (trans) wg_apply_q_vec_call<T, true>(Mg, ld, r, k, Tg, yl, rl);
    else wg_apply_q_vec_call<T, false>(Mg, ld, r, k, Tg, yl, rl);
  } else {
    if (trans) wg_apply_q_vec_impl<T, true>(Mg, ld, r, k, Tg, yl, rl);
    else wg_apply_q_vec_impl<T, false>(Mg, ld, r, k, Tg, yl, rl);
  }
}

// y (LDS, length nn) <- U^{-1} y (TRANS = false) or U^{-T} y, U the upper
// triangle of M[0:nn, 0:nn] (ld), in blocks of 16 rows.  The wave that owns
// a block's rows (thread t holds rows 4t .. 4t + 3) solves its diagonal block
// on lanes 0 .. 15 (lane i holds row i of it, or column i for U^T; a partial
// last block is padded with the identity) right after its own update, then
// every thread subtracts the block's contribution from its unsolved rows: one
// barrier per block.  The update's columns load before the diagonal solve.  A
// zero pivot gives a non-finite result, which the stop test reports.
template <typename T, bool TRANS>
__device__ __forceinline__ void wg_trsv_vec_impl(const LSQ_GLB T* Mg, int ld, int nn, LSQ_LDS T* yl) {
  constexpr int NB = 16;
  const T* M = (const T*)uni(Mg);
  LSQ_LDS T* y = uni(yl);
  ld = uni(ld); nn = uni(nn);
  const int t = threadIdx.x, lane = t & 63, w = uni(t >> 6), g0 = 4 * t;
  const int nbk = (nn + NB - 1) / NB;
  for (int b = 0; b < nbk; ++b) {
    const int j0 = (TRANS ? b : nbk - 1 - b) * NB, nbj = nn - j0 < NB ? nn - j0 : NB;
    // the update's part of U: columns j0 .. j0 + nbj of rows g0 .. g0 + 3
    // (U), or rows j0 .. j0 + nbj of columns g0 .. g0 + 3 (U^T)
    T Uv[NB][4];
    const bool act = TRANS ? (g0 >= j0 + NB && g0 < nn) : g0 < j0;
    if constexpr (!TRANS) {
      const auto rs = rsrc(M + (size_t)j0 * ld, (size_t)nbj * ld * sizeof(T));
#pragma unroll
      for (int c = 0; c < NB; ++c) load_rows4(rs, act, (uint32_t)((g0 + (size_t)c * ld) * sizeof(T)), Uv[c]);
    } else {
      const auto rs = rsrc(M + j0, ((size_t)(nn - 1) * ld + nbj) * sizeof(T));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool ok = act && g0 + e < nn;
#pragma unroll
        for (int c4 = 0; c4 < NB; c4 += 4) {
          T v[4];
          load_rows4(rs, ok, (uint32_t)((c4 + (size_t)(g0 + e) * ld) * sizeof(T)), v);
#pragma unroll
          for (int q = 0; q < 4; ++q) Uv[c4 + q][e] = v[q];
        }
      }
    }
    if (w == j0 / (4 * 64)) {                     // the block's rows are this wave's
      const auto rd = rsrc(M + j0 + (size_t)j0 * ld, ((size_t)(nbj - 1) * ld + nbj) * sizeof(T));
      T ud[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const size_t e = TRANS ? (size_t)c + (size_t)lane * ld : (size_t)lane + (size_t)c * ld;
        const T v = bload<T>(rd, (lane < nbj && c < nbj) ? (uint32_t)(e * sizeof(T)) : kOob);
        ud[c] = (c == lane && c >= nbj) ? (T)1 : v;
      }
      T yi = lane < nbj ? y[j0 + (lane < nbj ? lane : 0)] : (T)0;
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        const int j = TRANS ? s : NB - 1 - s;
        const T xj = lane_val(yi, j) / lane_val(ud[j], j);
        const T upd = yi - ud[j] * xj;
        yi = lane == j ? xj : ((TRANS ? lane > j : lane < j) ? upd : yi);
      }
      if (lane < nbj) y[j0 + lane] = yi;
    }
    __syncthreads();
    if (act) {
      T xb[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) xb[c] = c < nbj ? y[j0 + c] : (T)0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (g0 + e >= nn) continue;
        T acc = 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) acc += Uv[c][e] * xb[c];
        y[g0 + e] -= acc;
      }
    }
  }
  __syncthreads();
}

template <typename T, bool TRANS>
__device__ __noinline__ void wg_trsv_vec_call(const LSQ_GLB T* Mg, int ld, int nn, LSQ_LDS T* yl) {
  wg_trsv_vec_impl<T, TRANS>(Mg, ld, nn, yl);
}
template <typename T>
__device__ __forceinline__ void wg_trsv_vec(const T* M, int ld, int nn, T* y, bool trans) {
  const auto Mg = (const LSQ_GLB T*)M;
  const auto yl = (LSQ_LDS T*)y;
  if constexpr (sizeof(T) == 4) {
    if (trans) wg_trsv_vec_call<T, true>(Mg, ld, nn, yl);
    else wg_trsv_vec_call<T, false>(Mg, ld, nn, yl);
  } else {
    if (trans) wg_trsv_vec_impl<T, true>(Mg, ld, nn, yl);
    else wg_trsv_vec_impl<T, false>(Mg, ld, nn, yl);
  }
}

// Products with the upper part of the column block F[:, k : k + nc) (ld; rows
// i <= k + c of column k + c, i < r, r <= kBatchMaxDim): the off-diagonal
// blocks of the second factorization's triangle in the correction solves.
// Thread t owns rows 4t .. 4t + 3, which a padded column delivers in one
// (FP32) or two (FP64) 16-byte loads; the columns go in chunks of 16 (FP32) or
// 8 (FP64), the next chunk's loads in flight while the current one is used.
template <typename T>
struct Rows4 {
  T v[4];
};
template <typename T>
struct UpperBlock {
  static constexpr int CB = sizeof(T) == 4 ? 16 : 8;   // two chunks in registers: 128 VGPRs
  const T* F;
  int ld, r, k, nc, g0;
  __amdgpu_buffer_rsrc_t rs;
  __device__ UpperBlock(const T* F_, int ld_, int r_, int k_, int nc_)
      : F(F_), ld(ld_), r(r_), k(k_), nc(nc_), g0(4 * (int)threadIdx.x),
        rs(rsrc(F_ + (size_t)k_ * ld_, (size_t)(nc_ > 0 ? nc_ : 1) * ld_ * sizeof(T))) {}
  // (chunks past nc load nothing: every offset is out of range)
  __device__ __forceinline__ void load(int c0, T (&Yv)[CB][4]) const {
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const bool ok = (g0 < r) & (c0 + c < nc) & (g0 <= k + c0 + c);
      load_rows4(rs, ok, (uint32_t)((g0 + (size_t)(c0 + c) * ld) * sizeof(T)), Yv[c]);
    }
  }
  // element (g0 + e, k + c0 + c) of the upper part, else 0
  __device__ __forceinline__ T at(const T (&Yv)[CB][4], int c0, int c, int e) const {
    return (g0 + e <= k + c0 + c) & (g0 + e < r) ? Yv[c][e] : (T)0;
  }
};

// Rows 4t .. 4t + 3 of F[:, k : k + nc) h over the upper part (h: LDS,
// length nc).  No barrier.
template <typename T>
__device__ __forceinline__ Rows4<T> wg_upper_gemv_n_impl(const LSQ_GLB T* Fg, int ld, int r, int k, int nc,
                                                      const LSQ_LDS T* hg) {
  constexpr int CB = UpperBlock<T>::CB;
  const LSQ_LDS T* h = uni(hg);
  const UpperBlock<T> U((const T*)uni(Fg), uni(ld), uni(r), uni(k), uni(nc));
  Rows4<T> o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o.v[e] = 0;
  auto step = [&](int c0, const T (&Yv)[CB][4]) {
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const T hc0 = h[c0 + c < U.nc ? c0 + c : 0];
      const T hc = c0 + c < U.nc ? hc0 : (T)0;
#pragma unroll
      for (int e = 0; e < 4; ++e) o.v[e] += U.at(Yv, c0, c, e) * hc;
    }
  };
  T Ya[CB][4], Yb[CB][4];
  U.load(0, Ya);
  for (int c0 = 0; c0 < U.nc; c0 += 2 * CB) {
    U.load(c0 + CB, Yb);
    __builtin_amdgcn_sched_barrier(0);
    step(c0, Ya);
    U.load(c0 + 2 * CB, Ya);
    __builtin_amdgcn_sched_barrier(0);
    if (c0 + CB < U.nc) step(c0 + CB, Yb);
  }
  return o;
}

// out(c) = sum_i F(i, k + c) g(i) over the upper part, c < nc (g, out: LDS;
// wbuf: LDS scratch of kBW x kBatchMaxDim words).  Each chunk's column sums
// are reduced over the wave and the four waves' partials meet in wbuf: one
// barrier at the end, and one after out is written.
template <typename T>
__device__ __forceinline__ void wg_upper_gemv_t_impl(const LSQ_GLB T* Fg, int ld, int r, int k, int nc,
                                                   const LSQ_LDS T* gg, LSQ_LDS T* outg, LSQ_LDS T* wbufg) {
  constexpr int CB = UpperBlock<T>::CB;
  const LSQ_LDS T* g = uni(gg);
  LSQ_LDS T* out = uni(outg);
  LSQ_LDS T* wbuf = uni(wbufg);
  const UpperBlock<T> U((const T*)uni(Fg), uni(ld), uni(r), uni(k), uni(nc));
  const int lane = threadIdx.x & 63, w = uni((int)threadIdx.x >> 6);
  T gv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const T v = g[U.g0 + e < U.r ? U.g0 + e : 0];
    gv[e] = U.g0 + e < U.r ? v : (T)0;
  }
  auto step = [&](int c0, const T (&Yv)[CB][4]) {
    T pz[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c)
      pz[c] = (U.at(Yv, c0, c, 0) * gv[0] + U.at(Yv, c0, c, 1) * gv[1]) +
              (U.at(Yv, c0, c, 2) * gv[2] + U.at(Yv, c0, c, 3) * gv[3]);
    // lanes (64 / CB) c .. (64 / CB) (c + 1) - 1: the wave's sum of column c
    const T zc = wave_reduce_scatter<T, CB>(pz);
    constexpr int LPC = 64 / CB;
    const int c = c0 + lane / LPC;
    if (lane % LPC == 0 && c < U.nc) wbuf[w * kBatchMaxDim + c] = zc;
  };
  T Ya[CB][4], Yb[CB][4];
  U.load(0, Ya);
  for (int c0 = 0; c0 < U.nc; c0 += 2 * CB) {
    U.load(c0 + CB, Yb);
    __builtin_amdgcn_sched_barrier(0);
    step(c0, Ya);
    U.load(c0 + 2 * CB, Ya);
    __builtin_amdgcn_sched_barrier(0);
    if (c0 + CB < U.nc) step(c0 + CB, Yb);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < U.nc; c += kBT)
    out[c] = (wbuf[c] + wbuf[kBatchMaxDim + c]) + (wbuf[2 * kBatchMaxDim + c] + wbuf[3 * kBatchMaxDim + c]);
  __syncthreads();
}

// Out-of-line copies for the FP32 kernel (see wg_apply_q_vec_call).
template <typename T>
__device__ __noinline__ Rows4<T> wg_upper_gemv_n_call(const LSQ_GLB T* Fg, int ld, int r, int k, int nc,
                                                     const LSQ_LDS T* hg) {
  return wg_upper_gemv_n_impl<T>(Fg, ld, r, k, nc, hg);
}
template <typename T>
__device__ __noinline__ void wg_upper_gemv_t_call(const LSQ_GLB T* Fg, int ld, int r, int k, int nc,
                                                  const LSQ_LDS T* gg, LSQ_LDS T* outg, LSQ_LDS T* wbufg) {
  wg_upper_gemv_t_impl<T>(Fg, ld, r, k, nc, gg, outg, wbufg);
}
template <typename T>
__device__ __forceinline__ Rows4<T> wg_upper_gemv_n(const T* F, int ld, int r, int k, int nc, const T* h) {
  const auto Fg = (const LSQ_GLB T*)F;
  const auto hl = (const LSQ_LDS T*)h;
  if constexpr (sizeof(T) == 4) return wg_upper_gemv_n_call<T>(Fg, ld, r, k, nc, hl);
  else return wg_upper_gemv_n_impl<T>(Fg, ld, r, k, nc, hl);
}
template <typename T>
__device__ __forceinline__ void wg_upper_gemv_t(const T* F, int ld, int r, int k, int nc, const T* g, T* out,
                                                T* wbuf) {
  const auto Fg = (const LSQ_GLB T*)F;
  const auto gl = (const LSQ_LDS T*)g;
  const auto ol = (LSQ_LDS T*)out;
  const auto wl = (LSQ_LDS T*)wbuf;
  if constexpr (sizeof(T) == 4) wg_upper_gemv_t_call<T>(Fg, ld, r, k, nc, gl, ol, wl);
  else wg_upper_gemv_t_impl<T>(Fg, ld, r, k, nc, gl, ol, wl);
}

// ------------------------------------------------------------- staging --
// dst = src^T with optional reversals, through an LDS tile: src is sr x sc
// (column-major, lds), dst is sc x sr (ldd) with dst(x', y') = src(y, x),
// x' = sc - 1 - x if rx, y' = sr - 1 - y if ry; dst rows sc .. ldd - 1 are
// zero filled.  A tile is 64 columns of src by kBT rows: the loads run down
// the columns of src and the stores down the columns of dst.  Returns this
// thread's part of the squared Frobenius norm of src.
template <typename T, typename S>
__device__ __noinline__ double wg_transpose_impl(const LSQ_GLB S* srcg, int lds, int sr, int sc,
                                                 LSQ_GLB T* dstg, int ldd, int rx, int ry,
                                                 LSQ_LDS T* tileg) {
  constexpr int TX = 64, TY = kBT, TS = TY + 1, UB = 16;
  const S* src = (const S*)uni(srcg);
  LSQ_GLB T* dst = uni(dstg);
  LSQ_LDS T* tile = uni(tileg);
  lds = uni(lds); sr = uni(sr); sc = uni(sc); ldd = uni(ldd); rx = uni(rx); ry = uni(ry);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const auto rs = rsrc(src, ((size_t)(sc > 0 ? sc - 1 : 0) * lds + sr) * sizeof(S));
  double ss = 0.0;
  for (int x0 = 0; x0 < ldd; x0 += TX) {
    for (int y0 = 0; y0 < sr; y0 += TY) {
      const int y = y0 + t;
#pragma unroll
      for (int xb = 0; xb < TX; xb += UB) {
        S v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int x = x0 + xb + u;
          v[u] = bload<S>(rs, (x < sc && y < sr) ? (uint32_t)((y + (size_t)x * lds) * sizeof(S)) : kOob);
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          ss += (double)v[u] * (double)v[u];
          tile[(xb + u) * TS + t] = (T)v[u];
        }
      }
      __syncthreads();
      const int x = x0 + lane;
      const int xd = x < sc ? (rx ? sc - 1 - x : x) : x;
      const int ny = sr - y0 < TY ? sr - y0 : TY;
      if (x < ldd)
        for (int yy = w; yy < ny; yy += kBW) {
          const int yd = ry ? sr - 1 - (y0 + yy) : y0 + yy;
          dst[(size_t)xd + (size_t)yd * ldd] = tile[lane * TS + yy];
        }
      __syncthreads();
    }
  }
  return ss;
}
template <typename T, typename S>
__device__ __forceinline__ double wg_transpose(const S* src, int lds, int sr, int sc, T* dst, int ldd,
                                               bool rx, bool ry, T* tile) {
  return wg_transpose_impl<T, S>((const LSQ_GLB S*)src, lds, sr, sc, (LSQ_GLB T*)dst, ldd, rx, ry,
                                 (LSQ_LDS T*)tile);
}

// dst (rows x cols, ldd; rows .. ldd - 1 zero filled) = src (lds), UB columns
// of loads in flight per thread.  Returns this thread's part of the squared
// Frobenius norm of src.
template <typename T>
__device__ __noinline__ double wg_copy_impl(const LSQ_GLB double* srcg, int lds, int rows, int cols,
                                            LSQ_GLB T* dstg, int ldd) {
  constexpr int UB = 8;
  const double* src = (const double*)uni(srcg);
  LSQ_GLB T* dst = uni(dstg);
  lds = uni(lds); rows = uni(rows); cols = uni(cols); ldd = uni(ldd);
  const auto rs = rsrc(src, ((size_t)(cols > 0 ? cols - 1 : 0) * lds + rows) * sizeof(double));
  double ss = 0.0;
  for (int j0 = 0; j0 < cols; j0 += UB)
    for (int i = threadIdx.x; i < ldd; i += kBT) {
      double v[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u)
        v[u] = bload<double>(rs, (i < rows && j0 + u < cols) ? (uint32_t)((i + (size_t)(j0 + u) * lds) * sizeof(double)) : kOob);
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        ss += v[u] * v[u];
        if (j0 + u < cols) dst[(size_t)i + (size_t)(j0 + u) * ldd] = (T)v[u];
      }
    }
  return ss;
}
template <typename T>
__device__ __forceinline__ double wg_copy(const double* src, int lds, int rows, int cols, T* dst, int ldd) {
  return wg_copy_impl<T>((const LSQ_GLB double*)src, lds, rows, cols, (LSQ_GLB T*)dst, ldd);
}

// ---------------------------------------------------------- residuals --
// One pass of the FP64 augmented residual over M (rows x cols, ld, column-
// major): thread t owns rows t + kBT q (q < kRQ), so that each load covers 64
// consecutive rows, and returns its row sums sum_j M(i, j) xs(j); the column
// sums sum_i M(i, j) ws(i) are added to cs[j] (LDS, zeroed by the caller)
// through a wave reduce-scatter of CB columns at a time and LDS atomics.
// xs and ws are LDS vectors; CB columns of loads are in flight per thread.
struct RowSums {
  double v[kRQ];
};
__device__ __noinline__ RowSums wg_resid_pass_impl(const LSQ_GLB double* Mg, int ld, int rows, int cols,
                                                   const LSQ_LDS double* xsg, const LSQ_LDS double* wsg,
                                                   LSQ_LDS double* csg) {
  constexpr int CB = 8;
  const double* M = (const double*)uni(Mg);
  const LSQ_LDS double* xs = uni(xsg);
  const LSQ_LDS double* ws = uni(wsg);
  LSQ_LDS double* cs = uni(csg);
  ld = uni(ld); rows = uni(rows); cols = uni(cols);
  const int t = threadIdx.x, lane = t & 63;
  const auto rs = rsrc(M, ((size_t)(cols > 0 ? cols - 1 : 0) * ld + rows) * sizeof(double));
  RowSums o;
  double w[kRQ];
#pragma unroll
  for (int q = 0; q < kRQ; ++q) {
    const int i = t + kBT * q;
    o.v[q] = 0.0;
    w[q] = ws[i < rows ? i : 0];
    w[q] = i < rows ? w[q] : 0.0;
  }
  for (int j0 = 0; j0 < cols; j0 += CB) {
    double a[CB][kRQ];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int q = 0; q < kRQ; ++q) {
        const int i = t + kBT * q;
        a[c][q] = bload<double>(rs, (i < rows && j0 + c < cols) ? (uint32_t)((i + (size_t)(j0 + c) * ld) * 8) : kOob);
      }
    double csum[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const bool cin = j0 + c < cols;
      const double xc0 = xs[cin ? j0 + c : 0];
      const double xc = cin ? xc0 : 0.0;
      double ps = 0.0;
#pragma unroll
      for (int q = 0; q < kRQ; ++q) {
        o.v[q] += a[c][q] * xc;
        ps += a[c][q] * w[q];
      }
      csum[c] = ps;
    }
    const double tot = wave_reduce_scatter<double, CB>(csum);   // lanes 8c .. 8c + 7: column c
    const int c = lane >> 3;
    if ((lane & 7) == 0 && j0 + c < cols)
      __hip_atomic_fetch_add(&cs[j0 + c], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return o;
}
__device__ __forceinline__ RowSums wg_resid_pass(const double* M, int ld, int rows, int cols,
                                                 const double* xs, const double* ws, double* cs) {
  return wg_resid_pass_impl((const LSQ_GLB double*)M, ld, rows, cols, (const LSQ_LDS double*)xs,
                            (const LSQ_LDS double*)ws, (LSQ_LDS double*)cs);
}

// ----------------------------------------------------------- workspaces --
template <typename T>
struct LseWs {
  T *Fb, *taub, *Tb, *X, *Fa, *taua, *Ta;
  double *r, *v, *f1, *f2, *f3;
};
template <typename T>
struct GlsWs {
  T *Fw, *taw, *Tw, *X, *Fv, *tav, *Tv;
  double *z, *f1, *f2, *f3;
};

// Leading dimension of the workspace matrices: rows padded to a multiple of 4
// (zero-filled), so that every aligned group of 4 rows lies in its column.
__host__ __device__ constexpr int ldpad(int r) { return (r + 3) & ~3; }

// Byte offsets of an instance's workspace regions for element size esz and
// panel width nb, computed by one function on the host (sizing) and on the
// device (use).  LSE: Fb, taub, Tb, X, Fa, taua, Ta, r, v, f1, f2, f3;
// GLS: Fw, taw, Tw, X, Fv, tav, Tv, z, f1, f2, f3.  Returns the total.
__host__ __device__ inline size_t ws_layout(int type, int m, int n, int p, int esz, int nb,
                                            size_t* off) {
  size_t o = 0;
  int k = 0;
  auto take = [&](size_t bytes) {
    off[k++] = o;
    o += (bytes + 255) & ~(size_t)255;
  };
  auto tblk = [&](int refl) { return (size_t)((refl + nb - 1) / nb) * nb * nb * esz; };
  const size_t e = (size_t)esz, M = m, N = n, Pp = p;
  const size_t LM = ldpad(m), LN = ldpad(n), LP = ldpad(p);
  if (type == 0) {
    const int ka = m < n ? m : n;
    take(e * LN * Pp); take(e * Pp); take(tblk(p)); take(e * LN * M); take(e * LM * N);
    take(e * ka); take(tblk(ka));
    take(8 * M); take(8 * Pp); take(8 * M); take(8 * Pp); take(8 * N);
  } else {
    const int kv = p < n ? p : n;
    take(e * LN * M); take(e * M); take(tblk(m)); take(e * LN * Pp); take(e * LP * N);
    take(e * kv); take(tblk(kv));
    take(8 * N); take(8 * Pp); take(8 * N); take(8 * M);
  }
  return o;
}

template <typename T>
__device__ __forceinline__ LseWs<T> lse_ws(char* base, int m, int n, int p) {
  size_t off[12];
  ws_layout(0, m, n, p, (int)sizeof(T), QrCfg<T>::NB, off);
  LseWs<T> w;
  w.Fb = (T*)(base + off[0]);
  w.taub = (T*)(base + off[1]);
  w.Tb = (T*)(base + off[2]);
  w.X = (T*)(base + off[3]);
  w.Fa = (T*)(base + off[4]);
  w.taua = (T*)(base + off[5]);
  w.Ta = (T*)(base + off[6]);
  w.r = (double*)(base + off[7]);
  w.v = (double*)(base + off[8]);
  w.f1 = (double*)(base + off[9]);
  w.f2 = (double*)(base + off[10]);
  w.f3 = (double*)(base + off[11]);
  return w;
}
template <typename T>
__device__ __forceinline__ GlsWs<T> gls_ws(char* base, int n, int m, int p) {
  size_t off[12];
  ws_layout(1, m, n, p, (int)sizeof(T), QrCfg<T>::NB, off);
  GlsWs<T> w;
  w.Fw = (T*)(base + off[0]);
  w.taw = (T*)(base + off[1]);
  w.Tw = (T*)(base + off[2]);
  w.X = (T*)(base + off[3]);
  w.Fv = (T*)(base + off[4]);
  w.tav = (T*)(base + off[5]);
  w.Tv = (T*)(base + off[6]);
  w.z = (double*)(base + off[7]);
  w.f1 = (double*)(base + off[8]);
  w.f2 = (double*)(base + off[9]);
  w.f3 = (double*)(base + off[10]);
  return w;
}

template <typename PD>
__device__ __forceinline__ double wg_fro(PD M, int ld, int rows, int cols, double* red) {
  double s = 0.0;
  for (int j = 0; j < cols; ++j)
    for (int i = threadIdx.x; i < rows; i += kBT) {
      const double a = M[(size_t)i + (size_t)j * ld];
      s += a * a;
    }
  return sqrt(wg_sum1(s, red));
}

// Stop test on the squared norms [f1, f2, f3, x, a1, a2] with the scales of
// eq. lse-stop (gls = 0; a1 = r, a2 = v) or eq. gls-stop (gls = 1; a1 = y,
// a2 = z).  mat: [||A||, ||B||, ||rhs1||, ||rhs2||].
struct StopOut {
  bool conv, bad;
  double berr[3], bmax;
};
__device__ __forceinline__ StopOut stop_test(const double s[6], const double mat[4], int gls, double tol) {
  const double nf[3] = {sqrt(s[0]), sqrt(s[1]), sqrt(s[2])};
  const double nx = sqrt(s[3]), na1 = sqrt(s[4]), na2 = sqrt(s[5]);
  double sc[3];
  if (!gls) {
    sc[0] = mat[2] + na1 + mat[0] * nx;
    sc[1] = mat[3] + mat[1] * nx;
    sc[2] = mat[0] * na1 + mat[1] * na2;
  } else {
    sc[0] = na1 + mat[1] * na2;
    sc[1] = mat[2] + mat[0] * nx + mat[1] * na1;
    sc[2] = mat[0] * na2;
  }
  StopOut o;
  o.conv = true;
  o.bad = !isfinite(nx) || !isfinite(na1) || !isfinite(na2);
  o.bmax = 0.0;
  for (int k = 0; k < 3; ++k) {
    double e = 0.0;
    if (nf[k] > 0.0) e = sc[k] > 0.0 ? nf[k] / sc[k] : INFINITY;
    o.berr[k] = e;
    if (!(nf[k] <= tol * sc[k])) o.conv = false;
    if (!isfinite(nf[k]) || !isfinite(sc[k])) o.bad = true;
    o.bmax = e > o.bmax ? e : o.bmax;
  }
  o.conv = o.conv && !o.bad;
  return o;
}

// Classical refinement driver shared by both problems: `correct(first)` adds
// one correction (the initial solve when first), `residual(s)` evaluates the
// FP64 residual and the six squared norms.  Divergence / stagnation: stop when
// an iterate is not finite or the backward error has not halved over the last
// three steps.
template <typename Correct, typename Residual>
__device__ __forceinline__ void refine(Correct correct, Residual residual, const double mat[4], int gls,
                                      double tol, int maxit, double polish, bool fast_exit, BatchOut* out,
                                      unsigned long long t0, bool skip) {
  const unsigned long long t1 = wall_clock64();
  if (skip) {
    // routed to the next rung on the strength of the factors alone
    if (threadIdx.x == 0) {
      out->info = 3;
      out->steps = -1;
      for (int k = 0; k < 3; ++k) out->berr[k] = INFINITY;
      out->berr_max = INFINITY;
      out->t0 = t0;
      out->t1 = t1;
      out->t2 = t1;
    }
    return;
  }
  correct(true);
  double hist[4] = {0, 0, 0, 0};
  int it = 0;
  StopOut so;
  bool polished = false;
  for (;; ++it) {
    double s[6];
    residual(s);
    so = stop_test(s, mat, gls, tol);
    hist[0] = hist[1]; hist[1] = hist[2]; hist[2] = hist[3]; hist[3] = so.bmax;
    if (so.conv) {
      // one more correction toward the limiting accuracy while the backward
      // error is still above `polish` (polish <= 0: stop at once)
      if (polished || !(polish > 0.0) || so.bmax <= polish || it >= maxit) break;
      polished = true;
      correct(false);
      continue;
    }
    bool stalled = it >= 3 && !(hist[3] <= 0.5 * hist[0]);
    if (fast_exit && it >= 1) {
      // a higher-precision rung follows: leave once the observed contraction
      // of the last step predicts more than kMaxPredictedSteps further steps
      const double rho = hist[3] / hist[2];
      stalled = stalled || !(rho < 1.0) ||
                log(hist[3] / tol) > kMaxPredictedSteps * log(1.0 / rho);
    }
    if (so.bad || it >= maxit || stalled) break;
    correct(false);
  }
  if (threadIdx.x == 0) {
    out->info = so.conv ? 0 : (so.bad ? 5 : 3);
    out->steps = it;
    for (int k = 0; k < 3; ++k) out->berr[k] = so.berr[k];
    out->berr_max = so.bmax;
    out->t0 = t0;
    out->t1 = t1;
    out->t2 = wall_clock64();
  }
}

// ------------------------------------------------------------------ LSE --
// Layout as the single-instance path: Bt = J_n B^T J_p = Qt [Rt; 0] (Fb),
// Abar = A J Qt J = Za [T; 0] (Fa), k = n - p, T11 = T[0:k, 0:k],
// T12 = T[0:k, k:n], T22 = T[k:m, k:n] (upper part).
template <typename T, bool LP = false>
__device__ __forceinline__ void lse_instance(const BatchProb& P, char* base, double tol, int maxit, double polish,
                                             bool fast_exit, double route, BatchOut* out,
                             BLds<T>& L) {
  const unsigned long long t_start = wall_clock64();
  const int m = P.m, n = P.n, p = P.p, k = n - p, kqa = m < n ? m : n;
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const LseWs<T> W = lse_ws<T>(base, m, n, p);
  // the instance's arrays, typed as global memory
  const LSQ_GLB double* A = (const LSQ_GLB double*)P.A;
  const LSQ_GLB double* B = (const LSQ_GLB double*)P.B;
  const LSQ_GLB double* bvec = (const LSQ_GLB double*)P.b;
  const LSQ_GLB double* dvec = (const LSQ_GLB double*)P.d;
  LSQ_GLB double* x = (LSQ_GLB double*)P.x;
  // factorization in T: Bt = J_n B^T J_p = Qt [Rt; 0]; X = Qt^T (J_n A^T);
  // Abar = A J Qt J = (J_n X)^T = Za [T; 0]
  const int ldn = ldpad(n), ldm = ldpad(m);
  double mat[4];
  mat[0] = sqrt(wg_sum1(wg_transpose((const double*)A, P.lda, m, n, W.X, ldn, true, false, L.u.f.Ys), L.dred));
  mat[1] = sqrt(wg_sum1(wg_transpose((const double*)B, P.ldb, p, n, W.Fb, ldn, true, true, L.u.f.Ys), L.dred));
  mat[2] = wg_fro(bvec, m, m, 1, L.dred);
  mat[3] = wg_fro(dvec, p, p, 1, L.dred);
  __syncthreads();
  wg_geqrf<T, LP>(W.Fb, ldn, n, p, W.taub, W.Tb, L);
  wg_apply_qt<T, LP>(W.Fb, ldn, n, p, W.Tb, W.X, ldn, m, L);
  wg_transpose(W.X, ldn, n, m, W.Fa, ldm, false, true, L.u.f.Ys);   // Fa[j][n-1-i] = X[i][j]
  __syncthreads();
  wg_geqrf<T, LP>(W.Fa, ldm, m, n, W.taua, W.Ta, L);
  __syncthreads();
  // with a higher rung to follow, an instance whose triangles Rt or T11 show
  // a diagonal ratio above `route` (a lower bound on their condition number)
  // goes on to it without refining
  const bool skip = fast_exit && route > 0.0 &&
                    !(fmax(wg_diag_ratio(W.Fb, ldn, p, L.dred), wg_diag_ratio(W.Fa, ldm, k, L.dred)) <= route);
  for (int i = t; i < n; i += kBT) x[i] = 0.0;
  for (int i = t; i < m; i += kBT) W.r[i] = 0.0;
  for (int i = t; i < p; i += kBT) W.v[i] = 0.0;
  __syncthreads();

  T* U = L.u.vec[0];
  T* Wv = L.u.vec[1];
  T* Y2 = L.u.vec[2];
  T* Y2n = L.u.vec[3];
  T* Qv = L.u.vec[4];
  T* Y1 = L.u.vec[5];
  T* S = L.u.vec[6];
  T* X2 = L.u.vec[7];
  T* Yt = L.u.vec[8];
  const T* Fa = W.Fa;
  // Algorithm 1 on (f1, f2, f3), f3 = 0 for the initial solve; adds the
  // corrections to (x, r, v).
  auto correct = [&](bool first) {
    const LSQ_GLB double* f1 = first ? bvec : (const LSQ_GLB double*)W.f1;
    const LSQ_GLB double* f2 = first ? dvec : (const LSQ_GLB double*)W.f2;
    for (int i = t; i < n; i += kBT) U[i] = first ? (T)0 : (T)W.f3[n - 1 - i];
    for (int i = t; i < m; i += kBT) Wv[i] = (T)f1[i];
    for (int i = t; i < p; i += kBT) Y2[i] = (T)f2[p - 1 - i];
    __syncthreads();
    // u~ = Qt^T (J f3); w = Z^T f1; Rt^T (J y2) = J f2
    wg_apply_q_vec(W.Fb, ldn, n, p, W.Tb, U, L.vred, true);
    wg_apply_q_vec(W.Fa, ldm, m, kqa, W.Ta, Wv, L.vred, true);
    wg_trsv_vec(W.Fb, ldn, p, Y2, true);
    for (int i = t; i < p; i += kBT) Y2n[i] = Y2[p - 1 - i];
    for (int i = t; i < k; i += kBT) Qv[i] = U[p + k - 1 - i];
    __syncthreads();
    wg_trsv_vec(Fa, ldm, k, Qv, true);                    // T11^T q1 = u1
    {
      // w1 - T12 y2 (rows < k) and q2 = w2 - T22 y2 (rows >= k)
      const Rows4<T> ty = wg_upper_gemv_n(Fa, ldm, m, k, p, Y2n);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 4 * t + e;
        if (i < k) Y1[i] = Wv[i] - ty.v[e] - Qv[i];
        else if (i < m) Qv[i] = Wv[i] - ty.v[e];
      }
    }
    __syncthreads();
    wg_trsv_vec(Fa, ldm, k, Y1, false);                   // T11 y1 = w1 - q1 - T12 y2
    // s = [T12; T22]^T q - u2
    wg_upper_gemv_t(Fa, ldm, m, k, p, Qv, S, L.wscratch());
    for (int i = t; i < p; i += kBT) X2[i] = S[p - 1 - i] - U[i];
    for (int i = t; i < p; i += kBT) Yt[i] = Y2[i];
    for (int i = t; i < k; i += kBT) Yt[p + i] = Y1[k - 1 - i];
    __syncthreads();
    wg_trsv_vec(W.Fb, ldn, p, X2, false);                 // R^T dv = s
    for (int i = t; i < p; i += kBT) W.v[i] += (double)X2[p - 1 - i];
    wg_apply_q_vec(W.Fa, ldm, m, kqa, W.Ta, Qv, L.vred, false);   // dr = Z q
    for (int i = t; i < m; i += kBT) W.r[i] += (double)Qv[i];
    wg_apply_q_vec(W.Fb, ldn, n, p, W.Tb, Yt, L.vred, false);     // dx = J Qt (J y)
    for (int i = t; i < n; i += kBT) x[i] += (double)Yt[n - 1 - i];
    __syncthreads();
  };
  // f1 = b - r - A x, f2 = d - B x, f3 = -A^T r + B^T v (FP64): one pass
  // over A and one over B (row sums per thread, column sums through LDS)
  auto residual = [&](double s[6]) {
    double* cs = L.dvec(0);
    double* xl = L.dvec(1);
    double* rl = L.dvec(2);                             // -r
    double* vl = L.dvec(3);
    for (int j = t; j < n; j += kBT) {
      cs[j] = 0.0;
      xl[j] = x[j];
    }
    for (int i = t; i < m; i += kBT) rl[i] = -W.r[i];
    for (int i = t; i < p; i += kBT) vl[i] = W.v[i];
    __syncthreads();
    const RowSums ax = wg_resid_pass((const double*)A, P.lda, m, n, xl, rl, cs);
    const RowSums bx = wg_resid_pass((const double*)B, P.ldb, p, n, xl, vl, cs);
    __syncthreads();
    for (int q = 0; q < 6; ++q) s[q] = 0.0;
#pragma unroll
    for (int q = 0; q < kRQ; ++q) {
      const int i = t + kBT * q;
      if (i < m) {
        const double ri = -rl[i];
        const double val = bvec[i] - ri - ax.v[q];
        W.f1[i] = val;
        s[0] += val * val;
        s[4] += ri * ri;
      }
      if (i < p) {
        const double val = dvec[i] - bx.v[q];
        W.f2[i] = val;
        s[1] += val * val;
        s[5] += vl[i] * vl[i];
      }
    }
    for (int j = t; j < n; j += kBT) {
      const double val = cs[j];
      W.f3[j] = val;
      s[2] += val * val;
      s[3] += xl[j] * xl[j];
    }
    wg_sum6(s, L.dred);
  };
  refine(correct, residual, mat, 0, tol, maxit, polish, fast_exit, out, t_start, skip);
}

// ------------------------------------------------------------------ GLS --
// Layout as the single-instance path: W = Qw [Rw; 0] (Fw),
// Vt = J_p (Qw^T V)^T J_n = Qv Tv (Fv, p x n), k = n - m,
// A11 = Tv[0:k, 0:k], A12 = Tv[0:k, k:n], A22 = Tv[k:p, k:n] (upper part).
template <typename T, bool LP = false>
__device__ __forceinline__ void gls_instance(const BatchProb& P, char* base, double tol, int maxit, double polish,
                                             bool fast_exit, double route, BatchOut* out,
                             BLds<T>& L) {
  const unsigned long long t_start = wall_clock64();
  const int n = P.n, m = P.m, p = P.p, k = n - m, kqv = p < n ? p : n;
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
  const GlsWs<T> W = gls_ws<T>(base, n, m, p);
  // the instance's arrays, typed as global memory
  const LSQ_GLB double* A = (const LSQ_GLB double*)P.A;
  const LSQ_GLB double* B = (const LSQ_GLB double*)P.B;
  const LSQ_GLB double* dvec = (const LSQ_GLB double*)P.d;
  LSQ_GLB double* x = (LSQ_GLB double*)P.x;
  LSQ_GLB double* y = (LSQ_GLB double*)P.y;
  // factorization in T: W = Qw [Rw; 0]; X = Qw^T V;
  // Vt = J_p X^T J_n = Qv Tv
  const int ldn = ldpad(n), ldp = ldpad(p);            // rows beyond n (p) are zero padding
  double mat[4];
  mat[0] = sqrt(wg_sum1(wg_copy((const double*)A, P.lda, n, m, W.Fw, ldn), L.dred));
  mat[1] = sqrt(wg_sum1(wg_copy((const double*)B, P.ldb, n, p, W.X, ldn), L.dred));
  mat[2] = wg_fro(dvec, n, n, 1, L.dred);
  mat[3] = 0.0;
  __syncthreads();
  wg_geqrf<T, LP>(W.Fw, ldn, n, m, W.taw, W.Tw, L);
  wg_apply_qt<T, LP>(W.Fw, ldn, n, m, W.Tw, W.X, ldn, p, L);
  wg_transpose(W.X, ldn, n, p, W.Fv, ldp, true, true, L.u.f.Ys);    // Fv[p-1-j][n-1-i] = X[i][j]
  __syncthreads();
  wg_geqrf<T, LP>(W.Fv, ldp, p, n, W.tav, W.Tv, L);
  __syncthreads();
  // route as for the LSE: triangles Rw and A11 = Tv[0:k, 0:k]
  const bool skip = fast_exit && route > 0.0 &&
                    !(fmax(wg_diag_ratio(W.Fw, ldn, m, L.dred), wg_diag_ratio(W.Fv, ldp, k, L.dred)) <= route);
  for (int i = t; i < m; i += kBT) x[i] = 0.0;
  for (int i = t; i < p; i += kBT) y[i] = 0.0;
  for (int i = t; i < n; i += kBT) W.z[i] = 0.0;
  __syncthreads();

  T* U = L.u.vec[0];
  T* Wt = L.u.vec[1];
  T* H1 = L.u.vec[2];
  T* H1t = L.u.vec[3];
  T* G = L.u.vec[4];
  T* H2t = L.u.vec[5];
  T* S = L.u.vec[6];
  T* X = L.u.vec[7];
  T* Hv = L.u.vec[8];
  const T* Fv = W.Fv;
  // Algorithm 3 on (f1, f2, f3), f1 = f3 = 0 for the initial solve; adds the
  // corrections to (x, y, z) with dz = -Q h.
  auto correct = [&](bool first) {
    const LSQ_GLB double* f2 = first ? dvec : (const LSQ_GLB double*)W.f2;
    for (int i = t; i < n; i += kBT) U[i] = (T)f2[i];
    for (int i = t; i < p; i += kBT) Wt[i] = first ? (T)0 : (T)W.f1[p - 1 - i];
    for (int i = t; i < m; i += kBT) H1[i] = first ? (T)0 : (T)W.f3[i];
    __syncthreads();
    // u = Q^T f2; J w = Zt^T (J f1); R^T h1 = f3
    wg_apply_q_vec(W.Fw, ldn, n, m, W.Tw, U, L.vred, true);
    wg_apply_q_vec(W.Fv, ldp, p, kqv, W.Tv, Wt, L.vred, true);
    wg_trsv_vec(W.Fw, ldn, m, H1, true);
    for (int i = t; i < m; i += kBT) H1t[i] = H1[m - 1 - i];
    for (int i = t; i < k; i += kBT) G[i] = U[m + k - 1 - i];
    __syncthreads();
    wg_trsv_vec(Fv, ldp, k, G, true);                     // A11^T (J g2) = J u2
    {
      // J w2 - A12 J h1 - J g2 (rows < k) and J g1 = J w1 - A22 J h1 (rows >= k)
      const Rows4<T> ah = wg_upper_gemv_n(Fv, ldp, p, k, m, H1t);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 4 * t + e;
        if (i < k) H2t[i] = Wt[i] - ah.v[e] - G[i];
        else if (i < p) G[i] = Wt[i] - ah.v[e];
      }
    }
    __syncthreads();
    wg_trsv_vec(Fv, ldp, k, H2t, false);                  // A11 (J h2) = J w2 - J g2 - A12 J h1
    // s = Tv[:, k:n]^T (J g)
    wg_upper_gemv_t(Fv, ldp, p, k, m, G, S, L.wscratch());
    for (int i = t; i < m; i += kBT) X[i] = U[i] - S[m - 1 - i];
    for (int i = t; i < m; i += kBT) Hv[i] = H1[i];
    for (int i = t; i < k; i += kBT) Hv[m + i] = H2t[k - 1 - i];
    __syncthreads();
    wg_trsv_vec(W.Fw, ldn, m, X, false);                  // R dx = u1 - J s
    for (int i = t; i < m; i += kBT) x[i] += (double)X[i];
    wg_apply_q_vec(W.Fw, ldn, n, m, W.Tw, Hv, L.vred, false);     // dz = -Q h
    for (int i = t; i < n; i += kBT) W.z[i] -= (double)Hv[i];
    wg_apply_q_vec(W.Fv, ldp, p, kqv, W.Tv, G, L.vred, false);    // dy = J Zt (J g)
    for (int i = t; i < p; i += kBT) y[i] += (double)G[p - 1 - i];
    __syncthreads();
  };
  // f1 = -y + V^T z, f2 = d - W x - V y, f3 = W^T z (FP64): one pass over W
  // and one over V (row sums per thread, column sums through LDS)
  auto residual = [&](double s[6]) {
    double* cw = L.dvec(0);                             // W^T z
    double* cv = L.dvec(1);                             // V^T z
    double* zl = L.dvec(2);
    double* xy = L.dvec(3);                             // x, then y
    for (int j = t; j < m; j += kBT) {
      cw[j] = 0.0;
      xy[j] = x[j];
    }
    for (int j = t; j < p; j += kBT) cv[j] = 0.0;
    for (int i = t; i < n; i += kBT) zl[i] = W.z[i];
    __syncthreads();
    const RowSums wx = wg_resid_pass((const double*)A, P.lda, n, m, xy, zl, cw);
    __syncthreads();
    for (int j = t; j < p; j += kBT) xy[j] = y[j];
    __syncthreads();
    const RowSums vy = wg_resid_pass((const double*)B, P.ldb, n, p, xy, zl, cv);
    __syncthreads();
    for (int q = 0; q < 6; ++q) s[q] = 0.0;
#pragma unroll
    for (int q = 0; q < kRQ; ++q) {
      const int i = t + kBT * q;
      if (i < n) {
        const double val = dvec[i] - wx.v[q] - vy.v[q];
        W.f2[i] = val;
        s[1] += val * val;
        s[5] += zl[i] * zl[i];
      }
    }
    for (int j = t; j < m; j += kBT) {
      const double val = cw[j];
      W.f3[j] = val;
      s[2] += val * val;
      s[3] += x[j] * x[j];
    }
    for (int j = t; j < p; j += kBT) {
      const double yj = xy[j];
      const double val = -yj + cv[j];
      W.f1[j] = val;
      s[0] += val * val;
      s[4] += yj * yj;
    }
    wg_sum6(s, L.dred);
  };
  refine(correct, residual, mat, 1, tol, maxit, polish, fast_exit, out, t_start, skip);
}

template <typename T, bool LP = false>
__global__ __launch_bounds__(kBT, QrCfg<T>::BLOCKS) void k_batch(const BatchProb* __restrict__ probs,
                                                  const int* __restrict__ order, int count,
                                                  int* __restrict__ counter, char* __restrict__ ws,
                                                  size_t ws_stride, double tol, int maxit, double polish,
                                                  int fast_exit, double route, BatchOut* __restrict__ out,
                                                  EscQueue* __restrict__ esc, int esc_big) {
  __shared__ BLds<T> L;
  char* mine = ws + (size_t)blockIdx.x * ws_stride;
  for (;;) {
    if (threadIdx.x == 0) L.next = atomicAdd(counter, 1);
    __syncthreads();
    const int q = uni(L.next);
    __syncthreads();
    if (q >= count) break;
    const int idx = order[q];
    const BatchProb P = probs[idx];
    LSQ_LDS_POISON(L.u);
    LSQ_LDS_POISON(L.red);
    LSQ_LDS_POISON(L.vred);
    LSQ_LDS_POISON(L.dred);
    if (P.type == 0) lse_instance<T, LP>(P, mine, tol, maxit, polish, fast_exit != 0, route, out + idx, L);
    else gls_instance<T, LP>(P, mine, tol, maxit, polish, fast_exit != 0, route, out + idx, L);
    __syncthreads();
    if (esc && threadIdx.x == 0) {
      // a failure goes to the FP64 launch beside this one: claim a slot,
      // write the instance, then publish it; the first esc_big instances of
      // the order (the longest) use their own queue, which the consumers
      // drain first.  Every instance counts as done.
      if (out[idx].info != 0) {
        const int qi = q < esc_big ? 1 : 0;
        int* slot = reinterpret_cast<int*>(esc + 1) + 2 * count * qi;
        int* ready = slot + count;
        const int pos = __hip_atomic_fetch_add(&esc->tail[qi], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        slot[pos] = idx;
        __hip_atomic_store(&ready[pos], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_fetch_add(&esc->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// FP64 consumer of the escalation queue.  Thread 0 claims the next published
// slot; with the queue empty it sleeps until the FP32 launch has finished
// every instance (then leaves once the queue is drained) or until spin_ticks
// of the wall clock pass without a slot, when it leaves as well: the host
// solves whatever was not taken.  No work-group ever waits on another
// without that bound.
__global__ __launch_bounds__(kBT, QrCfg<double>::BLOCKS) void k_batch_esc(
    const BatchProb* __restrict__ probs, int count, EscQueue* __restrict__ esc,
    char* __restrict__ ws, size_t ws_stride, double tol, int maxit, double polish, BatchOut* __restrict__ out,
    unsigned long long spin_ticks, int* started) {
  __shared__ BLds<double> L;
  char* mine = ws + (size_t)blockIdx.x * ws_stride;
  // residency count for the host (pinned memory), which holds the FP32
  // launch back until the consumers own their compute units
  if (started && threadIdx.x == 0) __hip_atomic_fetch_add(started, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  // claims the next published slot of queue qi: 1 claimed (item set, -1 if
  // its producer never published within the bound), 0 empty, -1 lost a race
  auto claim = [&](int qi, unsigned long long t0, int& item) {
    int* slot = reinterpret_cast<int*>(esc + 1) + 2 * count * qi;
    int* ready = slot + count;
    const int h = __hip_atomic_load(&esc->head[qi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int t = __hip_atomic_load(&esc->tail[qi], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (h >= t) return 0;
    int expect = h;
    if (!__hip_atomic_compare_exchange_strong(&esc->head[qi], &expect, h + 1, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return -1;
    // the producer publishes right after claiming the slot
    while (!__hip_atomic_load(&ready[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) &&
           wall_clock64() - t0 < spin_ticks)
      __builtin_amdgcn_s_sleep(8);
    item = __hip_atomic_load(&ready[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) ? slot[h] : -1;
    return 1;
  };
  for (;;) {
    if (threadIdx.x == 0) {
      int item = -1;
      const unsigned long long t0 = wall_clock64();
      for (;;) {
        const int cb = claim(1, t0, item);
        if (cb > 0) break;
        if (cb < 0) continue;
        const int cs = claim(0, t0, item);
        if (cs > 0) break;
        if (cs < 0) continue;
        if (__hip_atomic_load(&esc->done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= count) {
          // every FP32 instance is finished: leave once both queues are drained
          bool empty = true;
          for (int qi = 0; qi < 2; ++qi)
            empty = empty && __hip_atomic_load(&esc->tail[qi], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <=
                                 __hip_atomic_load(&esc->head[qi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (empty) break;
          continue;
        }
        if (wall_clock64() - t0 >= spin_ticks) break;
        __builtin_amdgcn_s_sleep(32);
      }
      L.next = item;
    }
    __syncthreads();
    const int idx = uni(L.next);
    __syncthreads();
    if (idx < 0) break;
    const BatchProb P = probs[idx];
    LSQ_LDS_POISON(L.u);
    LSQ_LDS_POISON(L.red);
    LSQ_LDS_POISON(L.vred);
    LSQ_LDS_POISON(L.dred);
    if (P.type == 0) lse_instance<double>(P, mine, tol, maxit, polish, false, 0.0, out + idx, L);
    else gls_instance<double>(P, mine, tol, maxit, polish, false, 0.0, out + idx, L);
    __syncthreads();
  }
}

// Queue 1 (drained first by the FP64 consumers) preloaded with the first
// `pre` entries of the order, which the FP32 launch then skips: its counter
// and the done count start at pre.
__global__ void k_esc_preload(const int* __restrict__ order, int count, int pre, int* __restrict__ counter,
                              EscQueue* __restrict__ esc) {
  int* slot = reinterpret_cast<int*>(esc + 1) + 2 * count;
  int* ready = slot + count;
  for (int i = threadIdx.x; i < pre; i += blockDim.x) {
    slot[i] = order[i];
    ready[i] = 1;
  }
  if (threadIdx.x == 0) {
    esc->tail[1] = pre;
    esc->done = pre;
    *counter = pre;
  }
}

// n words of p set to v (graph capture records kernels, not memsets).
__global__ void k_fill_words(unsigned* __restrict__ p, size_t n, unsigned v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Holds the stream until `target` FP64 consumers have counted themselves in
// *started, or `ticks` of the wall clock pass: the device-side form of the
// host's wait in batch_launch_escalating, for a captured graph.
__global__ void k_wait_resident(const int* __restrict__ started, int target, unsigned long long ticks) {
  if (threadIdx.x != 0) return;
  const unsigned long long t0 = wall_clock64();
  while (__hip_atomic_load(started, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target &&
         wall_clock64() - t0 < ticks)
    __builtin_amdgcn_s_sleep(8);
}

void fill_words(hipStream_t s, void* p, size_t bytes, unsigned v) {
  const size_t n = bytes / 4;
  if (n == 0) return;
  const int grid = (int)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_words, dim3(grid), dim3(256), 0, s, static_cast<unsigned*>(p), n, v);
  LSQ_LAUNCH_CHECK();
}

}  // namespace

size_t batch_ws_bytes(const BatchProb& P) {
  size_t off[12];
  const size_t a = ws_layout(P.type, P.m, P.n, P.p, 4, QrCfg<float>::NB, off);
  const size_t b = ws_layout(P.type, P.m, P.n, P.p, 8, QrCfg<double>::NB, off);
  return a > b ? a : b;
}

int batch_blocks_per_cu(int tw) { return tw == 8 ? QrCfg<double>::BLOCKS : QrCfg<float>::BLOCKS; }

bool batch_eligible(const BatchProb& P) {
  const int lim = kBatchMaxDim;
  return P.m >= 1 && P.n >= 1 && P.p >= 1 && P.m <= lim && P.n <= lim && P.p <= lim;
}

// Householder QR of an r x c matrix: 2 c^2 (r - c/3) for r >= c, 2 r^2 (c - r/3)
// otherwise; applying k reflectors of length c from the right to r rows:
// 4 r (c - j) for reflector j.
static double qr_flops(double r, double c) {
  return r >= c ? 2.0 * c * c * (r - c / 3.0) : 2.0 * r * r * (c - r / 3.0);
}
static double right_flops(double r, double c, int k) {
  double f = 0.0;
  for (int j = 0; j < k; ++j) f += 4.0 * r * (c - j);
  return f;
}

double batch_factor_flops(const BatchProb& P) {
  if (P.type == 0) return qr_flops(P.n, P.p) + right_flops(P.m, P.n, P.p) + qr_flops(P.m, P.n);
  return qr_flops(P.n, P.m) + right_flops(P.p, P.n, P.m) + qr_flops(P.p, P.n);
}

void batch_launch(Ctx& ctx, int tw, const BatchProb* probs, const int* order, int count,
                  int* counter, char* ws, size_t ws_stride, int grid, double tol, int maxit, double polish,
                  bool fast_exit, double route, BatchOut* out, double flops, bool lowp) {
  if (count <= 0 || grid <= 0) return;
  LSQ_HIP(hipMemsetAsync(counter, 0, sizeof(int), ctx.stream));
  const int kind = tw == 8 ? kKBatch64 : kKBatch32;
  ktimer_begin(ctx, kind, flops, 0.0);
  if (tw == 8)
    hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(kBT), 0, ctx.stream, probs, order, count,
                       counter, ws, ws_stride, tol, maxit, polish, fast_exit ? 1 : 0, route, out, nullptr, 0);
  else if (lowp)
    hipLaunchKernelGGL((k_batch<float, true>), dim3(grid), dim3(kBT), 0, ctx.stream, probs, order, count,
                       counter, ws, ws_stride, tol, maxit, polish, fast_exit ? 1 : 0, route, out, nullptr, 0);
  else
    hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(kBT), 0, ctx.stream, probs, order, count,
                       counter, ws, ws_stride, tol, maxit, polish, fast_exit ? 1 : 0, route, out, nullptr, 0);
  LSQ_LAUNCH_CHECK();
  ktimer_end(ctx, kind);
}

size_t esc_queue_bytes(int count) { return sizeof(EscQueue) + 4 * sizeof(int) * (size_t)(count > 0 ? count : 0); }

void batch_launch_escalating(Ctx& ctx, const BatchProb* probs, const int* order, int count,
                             int* counter, char* ws, size_t ws_stride, int grid, char* ws64,
                             int grid64a, int grid64b, EscQueue* q, double tol, int maxit, double polish,
                             double route, BatchOut* out, BatchOut* out64, double flops, double spin_ms,
                             int* started, int big_count, int pre, bool lowp) {
  if (count <= 0 || grid <= 0) return;
  if (!ctx.side || grid64a <= 0) throw std::runtime_error("batch_launch_escalating: no side stream");
  if (pre < 0 || pre > count) throw std::runtime_error("batch_launch_escalating: pre outside [0, count]");
  LSQ_HIP(hipMemsetAsync(q, 0, esc_queue_bytes(count), ctx.stream));
  LSQ_HIP(hipMemsetAsync(out64, 0xff, sizeof(BatchOut) * (size_t)count, ctx.stream));   // info = -1
  hipLaunchKernelGGL(k_esc_preload, dim3(1), dim3(kBT), 0, ctx.stream, order, count, pre, counter, q);
  LSQ_LAUNCH_CHECK();
  hipEvent_t ready = ctx_event(ctx, 0), joined = ctx_event(ctx, 1);
  LSQ_HIP(hipEventRecord(ready, ctx.stream));
  const unsigned long long ticks = (unsigned long long)(spin_ms * 1e5);   // 100 MHz wall clock
  // consumers on the compute units the FP32 grid leaves free, from the start
  LSQ_HIP(hipStreamWaitEvent(ctx.side, ready, 0));
  if (started) __atomic_store_n(started, 0, __ATOMIC_RELEASE);
  ktimer_begin_on(ctx, kKBatchEsc, ctx.side, 0.0, 0.0);
  hipLaunchKernelGGL(k_batch_esc, dim3(grid64a), dim3(kBT), 0, ctx.side, probs, count, q, ws64,
                     ws_stride, tol, maxit, polish, out64, ticks, started);
  LSQ_LAUNCH_CHECK();
  ktimer_end_on(ctx, kKBatchEsc, ctx.side);
  LSQ_HIP(hipEventRecord(joined, ctx.side));
  if (started) {
    // the work-groups of two launches are placed in no fixed order: the FP32
    // grid would spread over every compute unit and leave none whole for a
    // consumer, so it waits (at most 20 ms) until the consumers are resident
    const auto t0 = std::chrono::steady_clock::now();
    while (__atomic_load_n(started, __ATOMIC_ACQUIRE) < grid64a &&
           std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(20))
      std::this_thread::yield();
  }
  ktimer_begin(ctx, kKBatch32, flops, 0.0);
  if (lowp)
    hipLaunchKernelGGL((k_batch<float, true>), dim3(grid), dim3(kBT), 0, ctx.stream, probs, order, count,
                       counter, ws, ws_stride, tol, maxit, polish, 1, route, out, q, big_count);
  else
    hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(kBT), 0, ctx.stream, probs, order, count,
                       counter, ws, ws_stride, tol, maxit, polish, 1, route, out, q, big_count);
  LSQ_LAUNCH_CHECK();
  ktimer_end(ctx, kKBatch32);
  // more consumers once the FP32 launch is over, for what is still queued
  if (grid64b > 0) {
    ktimer_begin(ctx, kKBatchEsc, 0.0, 0.0);
    hipLaunchKernelGGL(k_batch_esc, dim3(grid64b), dim3(kBT), 0, ctx.stream, probs, count, q,
                       ws64 + (size_t)grid64a * ws_stride, ws_stride, tol, maxit, polish, out64, ticks,
                       nullptr);
    LSQ_LAUNCH_CHECK();
    ktimer_end(ctx, kKBatchEsc);
  }
  LSQ_HIP(hipStreamWaitEvent(ctx.stream, joined, 0));
}

void batch_capture_escalating(Ctx& ctx, const BatchProb* probs, const int* order, int count, int* counter,
                              char* ws, size_t ws_stride, int grid, char* ws64, int grid64a, int grid64b,
                              EscQueue* q, double tol, int maxit, double polish, double route, BatchOut* out,
                              BatchOut* out64, double spin_ms, int* started, int big_count, int pre) {
  if (count <= 0 || grid <= 0) return;
  if (!ctx.side || grid64a <= 0) throw std::runtime_error("batch_capture_escalating: no side stream");
  if (pre < 0 || pre > count) throw std::runtime_error("batch_capture_escalating: pre outside [0, count]");
  fill_words(ctx.stream, q, esc_queue_bytes(count), 0u);
  fill_words(ctx.stream, out64, sizeof(BatchOut) * (size_t)count, 0xffffffffu);   // info = -1
  fill_words(ctx.stream, started, sizeof(int), 0u);
  hipLaunchKernelGGL(k_esc_preload, dim3(1), dim3(kBT), 0, ctx.stream, order, count, pre, counter, q);
  LSQ_LAUNCH_CHECK();
  hipEvent_t ready = ctx_event(ctx, 0), joined = ctx_event(ctx, 1);
  LSQ_HIP(hipEventRecord(ready, ctx.stream));
  const unsigned long long ticks = (unsigned long long)(spin_ms * 1e5);   // 100 MHz wall clock
  LSQ_HIP(hipStreamWaitEvent(ctx.side, ready, 0));
  hipLaunchKernelGGL(k_batch_esc, dim3(grid64a), dim3(kBT), 0, ctx.side, probs, count, q, ws64,
                     ws_stride, tol, maxit, polish, out64, ticks, started);
  LSQ_LAUNCH_CHECK();
  LSQ_HIP(hipEventRecord(joined, ctx.side));
  // (at most 20 ms, as the host's wait)
  hipLaunchKernelGGL(k_wait_resident, dim3(1), dim3(64), 0, ctx.stream, started, grid64a,
                     (unsigned long long)(20.0 * 1e5));
  LSQ_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(kBT), 0, ctx.stream, probs, order, count,
                     counter, ws, ws_stride, tol, maxit, polish, 1, route, out, q, big_count);
  LSQ_LAUNCH_CHECK();
  if (grid64b > 0) {
    hipLaunchKernelGGL(k_batch_esc, dim3(grid64b), dim3(kBT), 0, ctx.stream, probs, count, q,
                       ws64 + (size_t)grid64a * ws_stride, ws_stride, tol, maxit, polish, out64, ticks,
                       nullptr);
    LSQ_LAUNCH_CHECK();
  }
  LSQ_HIP(hipStreamWaitEvent(ctx.stream, joined, 0));
}

}  // namespace lsq
