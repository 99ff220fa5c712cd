// Host-side driver for sanitizer builds of liblsq (AddressSanitizer or
// ThreadSanitizer on the host code only; the device code is built as usual).
// It exercises the paths whose host code runs on several threads or keeps
// state across calls: the batched entry point with concurrent workers (one
// host thread, stream and workspace each), the persistent batch, the single
// solves with the escalation ladder, factor-once objects and handle teardown.
//
//   lsq_sanitize_driver [count] [workers]
//
// Prints one line per phase and exits non-zero if a solve fails to certify.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "lsq.h"

namespace {

#define CHECK_HIP(e)                                                            \
  do {                                                                          \
    hipError_t err_ = (e);                                                      \
    if (err_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s failed: %s\n", #e, hipGetErrorString(err_));     \
      std::exit(2);                                                             \
    }                                                                           \
  } while (0)

double* to_device(const std::vector<double>& h) {
  double* d = nullptr;
  CHECK_HIP(hipMalloc(&d, sizeof(double) * (h.empty() ? 1 : h.size())));
  if (!h.empty()) CHECK_HIP(hipMemcpy(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
  return d;
}

struct Instance {
  lsq_problem prob{};
  std::vector<double*> owned;
};

// A Gaussian instance (well conditioned with high probability): LSE with
// (m, n, p) or GLS with (n, m, p) = (rows, columns of W, columns of V).
Instance make_instance(std::mt19937_64& rng, int type, int a, int b, int c) {
  std::normal_distribution<double> g(0.0, 1.0);
  auto vec = [&](size_t k) {
    std::vector<double> v(k);
    for (auto& t : v) t = g(rng);
    return v;
  };
  Instance in;
  lsq_problem& P = in.prob;
  P.type = type;
  if (type == LSQ_LSE) {
    const int m = a, n = b, p = c;
    P.m = m; P.n = n; P.p = p;
    P.A = to_device(vec((size_t)m * n)); P.lda = m;
    P.B = to_device(vec((size_t)p * n)); P.ldb = p;
    P.b = to_device(vec(m));
    P.d = to_device(vec(p));
    P.x = to_device(std::vector<double>(n, 0.0));
    P.y = nullptr;
  } else {
    const int n = a, m = b, p = c;
    P.n = n; P.m = m; P.p = p;
    P.A = to_device(vec((size_t)n * m)); P.lda = n;
    P.B = to_device(vec((size_t)n * p)); P.ldb = n;
    P.b = nullptr;
    P.d = to_device(vec(n));
    P.x = to_device(std::vector<double>(m, 0.0));
    P.y = to_device(std::vector<double>(p, 0.0));
  }
  for (const void* q : {(const void*)P.A, (const void*)P.B, (const void*)P.b, (const void*)P.d,
                        (const void*)P.x, (const void*)P.y})
    if (q) in.owned.push_back(const_cast<double*>(static_cast<const double*>(q)));
  return in;
}

int report(const char* what, int rc, const std::vector<lsq_result>& res) {
  int bad = 0;
  for (const auto& r : res)
    if (r.info != 0 || !(r.berr_max <= 1e-14)) ++bad;
  std::printf("%s: rc=%d, %d of %zu instances not certified\n", what, rc, bad, res.size());
  std::fflush(stdout);
  return bad;
}

}  // namespace

int main(int argc, char** argv) {
  const int count = argc > 1 ? std::atoi(argv[1]) : 48;
  const int workers = argc > 2 ? std::atoi(argv[2]) : 8;
  std::mt19937_64 rng(20260);
  std::uniform_int_distribution<int> um(64, 400);
  std::vector<Instance> inst;
  for (int i = 0; i < count; ++i) {
    const int type = i % 2 == 0 ? LSQ_LSE : LSQ_GLS;
    const int big = um(rng), mid = std::max(8, big / 2 - (int)(rng() % 16)), small = std::max(2, mid / 5);
    if (type == LSQ_LSE) inst.push_back(make_instance(rng, type, big, mid, small));
    else inst.push_back(make_instance(rng, type, mid, small, big));
  }
  std::vector<lsq_problem> probs;
  for (auto& in : inst) probs.push_back(in.prob);
  int fails = 0;
  for (int round = 0; round < 2; ++round) {
    lsq_handle h = nullptr;
    if (lsq_create(&h, 0) != 0) {
      std::fprintf(stderr, "lsq_create failed\n");
      return 2;
    }
    lsq_opts o;
    lsq_opts_default(&o);
    std::vector<lsq_result> res(count);
    // concurrent workers, every rung of the ladder from BF16 up
    lsq_set_batch_workers(h, workers);
    lsq_set_batch_mode(h, LSQ_BATCH_WORKERS);
    o.prec = LSQ_PREC_BF16;
    int rc = lsq_solve_batched(h, count, probs.data(), &o, res.data());
    fails += report("workers, bf16 ladder", rc, res);
    o.prec = LSQ_PREC_FP32;
    o.solver = LSQ_SOLVER_GMRES_IR;
    rc = lsq_solve_batched(h, count, probs.data(), &o, res.data());
    fails += report("workers, fp32 gmres-ir", rc, res);
    // the persistent batch, FP32 with the FP64 rung beside it
    lsq_set_batch_mode(h, LSQ_BATCH_AUTO);
    o.solver = LSQ_SOLVER_IR;
    rc = lsq_solve_batched(h, count, probs.data(), &o, res.data());
    fails += report("persistent, fp32 then fp64", rc, res);
    // factor once, solve twice, then destroy the factors before the handle
    const lsq_problem& P = probs[0];
    lsq_factors f = nullptr;
    rc = lse_factor(h, P.m, P.n, P.p, P.A, P.lda, P.B, P.ldb, LSQ_PREC_FP32, &f);
    lsq_result r1{};
    for (int k = 0; k < 2 && rc == 0; ++k) {
      rc = lse_solve_factored(h, f, P.b, P.d, P.x, nullptr, nullptr, nullptr, &r1);
    }
    std::printf("factored: rc=%d berr=%.2e\n", rc, r1.berr_max);
    fails += rc != 0;
    lsq_factors_destroy(f);
    lsq_destroy(h);
  }
  for (auto& in : inst)
    for (double* q : in.owned) CHECK_HIP(hipFree(q));
  std::printf("done: %d failures\n", fails);
  return fails == 0 ? 0 : 1;
}
