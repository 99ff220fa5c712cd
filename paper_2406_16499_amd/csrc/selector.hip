// Learned precision / solver selector.
//
// Features (16, FP32) of an instance come from FP64 norms of the inputs and
// from the diagonals of the triangular factors of its FP32 generalized
// factorization, the first rung of the plain ladder (whose factors are reused
// when the selector picks an FP32 rung).  An
// MLP 16 -> 64 -> 64 -> 7 (ReLU, FP32) maps the standardized features to two
// heads: 5 logits for the factorization precision {FP8-e4m3, BF16, FP16,
// FP32, FP64 direct} and 2 for the refinement solver {classical IR, GMRES-IR}.
#include "engine.hpp"

namespace lsq {

// |diag| statistics of the upper triangular block f.M[o:o+nn, o:o+nn]:
// out = {log10 max, log10 min, mean log10}.
template <typename Tw>
__global__ __launch_bounds__(256) void k_diag_stats(const Tw* __restrict__ M, int ld, int nn,
                                                    float* __restrict__ out) {
  __shared__ double smax[256], smin[256], ssum[256];
  double mx = 0.0, mn = INFINITY, sm = 0.0;
  for (int i = threadIdx.x; i < nn; i += 256) {
    const double a = fabs((double)M[(size_t)i + (size_t)i * ld]);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
    sm += log10(fmax(a, 1e-300));
  }
  smax[threadIdx.x] = mx; smin[threadIdx.x] = mn; ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      ssum[threadIdx.x] += ssum[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (nn > 0) {
      out[0] = (float)log10(fmax(smax[0], 1e-300));
      out[1] = (float)log10(fmax(smin[0], 1e-300));
      out[2] = (float)(ssum[0] / nn);
    } else {
      out[0] = out[1] = out[2] = 0.0f;
    }
  }
}

// Assembles the feature vector.  st1: first triangle (R of B / R of W);
// st2: the block that decides uniqueness (T11 / the n-m leading block of the
// second triangle); st3: the whole second triangle.
__global__ void k_features(int type, int m, int n, int p, const double* __restrict__ matnorms,
                           const float* __restrict__ st1, const float* __restrict__ st2,
                           const float* __restrict__ st3, float* __restrict__ f) {
  if (threadIdx.x != 0) return;
  auto lg = [](double v) { return (float)log10(fmax(v, 1e-300)); };
  f[0] = (float)type;
  f[1] = log2f((float)m + 1.0f);
  f[2] = log2f((float)n + 1.0f);
  f[3] = log2f((float)p + 1.0f);
  f[4] = lg(matnorms[0]);
  f[5] = lg(matnorms[1]);
  f[6] = lg(matnorms[2] + 1e-300);
  f[7] = lg(matnorms[3] + 1e-300);
  f[8] = st1[0] - st1[1];
  f[9] = st2[0] - st2[1];
  f[10] = st3[0] - st3[1];
  f[11] = st1[2] - st1[0];
  f[12] = st2[2] - st2[0];
  f[13] = st3[2] - st3[0];
  f[14] = f[4] - f[5];
  f[15] = f[2] - f[1];
}

// MLP inference, one 64-thread block: standardize, two ReLU layers, the two
// heads and their argmax.  W packs (mean[16], std[16], W1[64][16], b1[64],
// W2[64][64], b2[64], W3[7][64], b3[7]).
__global__ __launch_bounds__(64) void k_mlp(const float* __restrict__ W, const float* __restrict__ f,
                                            float* __restrict__ logits, int* __restrict__ cls) {
  __shared__ float x[kSelFeatures], h1[kSelHidden], h2[kSelHidden], lo[kSelOut];
  LSQ_LDS_POISON(x);
  LSQ_LDS_POISON(h1);
  LSQ_LDS_POISON(h2);
  LSQ_LDS_POISON(lo);
  const int t = threadIdx.x;
  const float* mean = W;
  const float* sd = W + kSelFeatures;
  const float* W1 = sd + kSelFeatures;
  const float* b1 = W1 + kSelHidden * kSelFeatures;
  const float* W2 = b1 + kSelHidden;
  const float* b2 = W2 + kSelHidden * kSelHidden;
  const float* W3 = b2 + kSelHidden;
  const float* b3 = W3 + kSelOut * kSelHidden;
  if (t < kSelFeatures) x[t] = (f[t] - mean[t]) / sd[t];
  __syncthreads();
  float s = b1[t];
  for (int i = 0; i < kSelFeatures; ++i) s = fmaf(W1[t * kSelFeatures + i], x[i], s);
  h1[t] = fmaxf(s, 0.0f);
  __syncthreads();
  s = b2[t];
  for (int i = 0; i < kSelHidden; ++i) s = fmaf(W2[t * kSelHidden + i], h1[i], s);
  h2[t] = fmaxf(s, 0.0f);
  __syncthreads();
  if (t < kSelOut) {
    float o = b3[t];
    for (int i = 0; i < kSelHidden; ++i) o = fmaf(W3[t * kSelHidden + i], h2[i], o);
    lo[t] = o;
    logits[t] = o;
  }
  __syncthreads();
  if (t == 0) {
    int bp = 0;
    for (int c = 1; c < kSelPrec; ++c)
      if (lo[c] > lo[bp]) bp = c;
    cls[0] = bp;
    cls[1] = lo[kSelPrec + 1] > lo[kSelPrec] ? 1 : 0;
  }
}

// ------------------------------------------------------------------ host --
void diag_stats(Ctx& ctx, const QRFactor& f, int o, int nn, float* out) {
  if (f.tw == 8)
    hipLaunchKernelGGL((k_diag_stats<double>), dim3(1), dim3(256), 0, ctx.stream,
                       static_cast<const double*>(f.M) + (size_t)o * (f.ld + 1), f.ld, nn, out);
  else
    hipLaunchKernelGGL((k_diag_stats<float>), dim3(1), dim3(256), 0, ctx.stream,
                       static_cast<const float*>(f.M) + (size_t)o * (f.ld + 1), f.ld, nn, out);
  LSQ_LAUNCH_CHECK();
}

void features(Ctx& ctx, int type, int m, int n, int p, const double* matnorms, const float* st1,
              const float* st2, const float* st3, float* feats) {
  hipLaunchKernelGGL(k_features, dim3(1), dim3(64), 0, ctx.stream, type, m, n, p, matnorms, st1,
                     st2, st3, feats);
  LSQ_LAUNCH_CHECK();
}

void mlp_select(Ctx& ctx, const float* weights, const float* feats, float* logits, int* cls) {
  hipLaunchKernelGGL(k_mlp, dim3(1), dim3(64), 0, ctx.stream, weights, feats, logits, cls);
  LSQ_LAUNCH_CHECK();
}

}  // namespace lsq
