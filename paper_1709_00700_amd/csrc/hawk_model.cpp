// Learned cost model behind the C ABI: parameters on the device, training by
// mini-batch Adam with the library's own forward/backward kernels, and
// per-query variant picks (argmin of the predicted time over the variant
// space). Exhaustive search and Algorithm 1 stay available as the fallback
// and as the reference the picks are scored against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hawk.h"
#include "hawk_internal.h"
#include "hawk_mlp.h"

struct hawk_model {
  hawk_ctx* ctx = nullptr;
  float* p = nullptr;     // parameters (device)
  float* m1 = nullptr;    // Adam moments
  float* m2 = nullptr;
  float* mu = nullptr;    // feature standardisation (device)
  float* sd = nullptr;
  int64_t step = 0;
};

namespace {

uint64_t sm64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double unit(uint64_t& s) { return (static_cast<double>(sm64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
double normal(uint64_t& s) {  // Box-Muller
  const double u = unit(s), v = unit(s);
  return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
}

hawk_status dev_err(hawk_ctx* ctx, hipError_t e, const char* where) {
  return set_error(ctx, HAWK_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define CK(call, where)                                              \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) return dev_err(M->ctx, e_, where);         \
  } while (0)

struct DevBuf {
  hawk_ctx* ctx;
  std::vector<void*> ps;
  explicit DevBuf(hawk_ctx* c) : ctx(c) {}
  void* get(size_t bytes) {
    void* p = ctx->pool.get(bytes);
    if (p) ps.push_back(p);
    return p;
  }
  ~DevBuf() {
    for (void* p : ps) ctx->pool.put(p);
  }
};

}  // namespace

extern "C" hawk_status hawk_model_create(hawk_ctx* ctx, uint64_t seed, hawk_model** out) {
  if (!ctx || !out) return HAWK_E_ARG;
  *out = nullptr;
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  hawk_model* M = new hawk_model();
  M->ctx = ctx;
  ctx->models.insert(M);
  const size_t bytes = MLP_NPARAMS * sizeof(float);
  if (hipMalloc(&M->p, bytes) != hipSuccess || hipMalloc(&M->m1, bytes) != hipSuccess ||
      hipMalloc(&M->m2, bytes) != hipSuccess || hipMalloc(&M->mu, MLP_IN * 4) != hipSuccess ||
      hipMalloc(&M->sd, MLP_IN * 4) != hipSuccess) {
    hawk_model_free(M);
    return set_error(ctx, HAWK_E_OOM, "model allocation failed");
  }
  // He initialisation of the weights, zero biases; identity standardisation
  std::vector<float> h(MLP_NPARAMS, 0.f);
  uint64_t s = seed ^ 0xC0575EEDull;
  const int o_b1 = MLP_HIDDEN * MLP_IN, o_w2 = o_b1 + MLP_HIDDEN, o_b2 = o_w2 + MLP_HIDDEN * MLP_HIDDEN;
  const int o_w3 = o_b2 + MLP_HIDDEN;
  for (int i = 0; i < o_b1; ++i) h[i] = static_cast<float>(normal(s) * std::sqrt(2.0 / MLP_IN));
  for (int i = o_w2; i < o_b2; ++i) h[i] = static_cast<float>(normal(s) * std::sqrt(2.0 / MLP_HIDDEN));
  for (int i = o_w3; i < o_w3 + MLP_HIDDEN; ++i) h[i] = static_cast<float>(normal(s) * std::sqrt(1.0 / MLP_HIDDEN));
  std::vector<float> mu(MLP_IN, 0.f), sd(MLP_IN, 1.f);
  hawk_status st = hawk_model_set_params(M, h.data(), mu.data(), sd.data());
  if (st) {
    hawk_model_free(M);
    return st;
  }
  *out = M;
  return HAWK_OK;
}

void model_release_device(hawk_model* M) {
  if (!M->ctx) return;
  (void)hipStreamSynchronize(M->ctx->stream);
  for (float* p : {M->p, M->m1, M->m2, M->mu, M->sd})
    if (p) (void)hipFree(p);
  M->p = M->m1 = M->m2 = M->mu = M->sd = nullptr;
  M->ctx = nullptr;
}

extern "C" void hawk_model_free(hawk_model* M) {
  if (!M) return;
  if (M->ctx) {
    M->ctx->models.erase(M);
    model_release_device(M);
  }
  delete M;
}

extern "C" hawk_status hawk_model_set_params(hawk_model* M, const float* params, const float* mu, const float* sd) {
  if (!M || !M->ctx || !params || !mu || !sd) return HAWK_E_ARG;
  for (int k = 0; k < MLP_IN; ++k)
    if (!(sd[k] > 0.f)) return set_error(M->ctx, HAWK_E_ARG, "feature scale must be positive");
  CK(hipMemcpy(M->p, params, MLP_NPARAMS * 4, hipMemcpyHostToDevice), "upload params");
  CK(hipMemcpy(M->mu, mu, MLP_IN * 4, hipMemcpyHostToDevice), "upload mu");
  CK(hipMemcpy(M->sd, sd, MLP_IN * 4, hipMemcpyHostToDevice), "upload sd");
  CK(hipMemset(M->m1, 0, MLP_NPARAMS * 4), "reset moments");
  CK(hipMemset(M->m2, 0, MLP_NPARAMS * 4), "reset moments");
  M->step = 0;
  return HAWK_OK;
}

extern "C" hawk_status hawk_model_get_params(hawk_model* M, float* params, float* mu, float* sd) {
  if (!M || !M->ctx) return HAWK_E_ARG;
  CK(hipStreamSynchronize(M->ctx->stream), "synchronize");
  if (params) CK(hipMemcpy(params, M->p, MLP_NPARAMS * 4, hipMemcpyDeviceToHost), "read params");
  if (mu) CK(hipMemcpy(mu, M->mu, MLP_IN * 4, hipMemcpyDeviceToHost), "read mu");
  if (sd) CK(hipMemcpy(sd, M->sd, MLP_IN * 4, hipMemcpyDeviceToHost), "read sd");
  return HAWK_OK;
}

extern "C" hawk_status hawk_mlp_forward_dev(hawk_model* M, const float* dX, int64_t m, float* dout) {
  if (!M || !M->ctx || m < 0 || (m > 0 && (!dX || !dout))) return HAWK_E_ARG;
  CK(hk_mlp_forward(M->ctx->stream, M->p, M->mu, M->sd, dX, m, dout), "forward");
  return HAWK_OK;
}

extern "C" hawk_status hawk_mlp_grad_dev(hawk_model* M, const float* dX, const float* dy, int64_t m, float* dgrad,
                                         float* dloss) {
  if (!M || !M->ctx || m < 1 || !dX || !dy || !dgrad) return HAWK_E_ARG;
  DevBuf B(M->ctx);
  const int64_t rows = hk_mlp_grad_rows(m);
  float* partial = static_cast<float*>(B.get(static_cast<size_t>(rows) * MLP_NPARAMS * 4));
  float* ploss = static_cast<float*>(B.get(static_cast<size_t>(rows) * 4));
  if (!partial || !ploss) return set_error(M->ctx, HAWK_E_OOM, "gradient scratch");
  CK(hk_mlp_grad(M->ctx->stream, M->p, M->mu, M->sd, dX, dy, nullptr, m, partial, ploss, rows, dgrad, dloss),
     "gradient");
  return HAWK_OK;
}

extern "C" hawk_status hawk_model_train(hawk_model* M, const float* X, const float* y, int64_t m,
                                        const hawk_train_opts* o, float* final_loss) {
  if (!M || !M->ctx) return HAWK_E_ARG;
  if (!X || !y || m < 1 || !o || o->epochs < 1 || o->batch < 1 || !(o->lr > 0.f))
    return set_error(M->ctx, HAWK_E_ARG, "bad training arguments");
  hawk_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  // feature standardisation from the training set
  std::vector<float> mu(MLP_IN, 0.f), sd(MLP_IN, 0.f);
  for (int k = 0; k < MLP_IN; ++k) {
    double s = 0, s2 = 0;
    for (int64_t i = 0; i < m; ++i) {
      const double v = X[i * MLP_IN + k];
      s += v;
      s2 += v * v;
    }
    const double mean = s / m, var = std::max(0.0, s2 / m - mean * mean);
    mu[k] = static_cast<float>(mean);
    sd[k] = static_cast<float>(var > 1e-12 ? std::sqrt(var) : 1.0);
  }
  CK(hipMemcpy(M->mu, mu.data(), MLP_IN * 4, hipMemcpyHostToDevice), "upload mu");
  CK(hipMemcpy(M->sd, sd.data(), MLP_IN * 4, hipMemcpyHostToDevice), "upload sd");
  DevBuf B(ctx);
  const int64_t batch = std::min<int64_t>(o->batch, m);
  // partial rows for the largest gradient launch: the batches and the final full pass
  const int64_t rows = std::max(hk_mlp_grad_rows(batch), hk_mlp_grad_rows(m));
  float* dX = static_cast<float*>(B.get(static_cast<size_t>(m) * MLP_IN * 4));
  float* dy = static_cast<float*>(B.get(static_cast<size_t>(m) * 4));
  int32_t* didx = static_cast<int32_t*>(B.get(static_cast<size_t>(m) * 4 * o->epochs));
  float* partial = static_cast<float*>(B.get(static_cast<size_t>(rows) * MLP_NPARAMS * 4));
  float* ploss = static_cast<float*>(B.get(static_cast<size_t>(rows) * 4));
  float* grad = static_cast<float*>(B.get(MLP_NPARAMS * 4));
  float* dloss = static_cast<float*>(B.get(16));
  if (!dX || !dy || !didx || !partial || !ploss || !grad || !dloss) return set_error(ctx, HAWK_E_OOM, "training buffers");
  CK(hipMemcpyAsync(dX, X, static_cast<size_t>(m) * MLP_IN * 4, hipMemcpyHostToDevice, st), "upload X");
  CK(hipMemcpyAsync(dy, y, static_cast<size_t>(m) * 4, hipMemcpyHostToDevice, st), "upload y");
  // one seeded shuffle per epoch (Fisher-Yates), all uploaded at once
  std::vector<int32_t> perm(static_cast<size_t>(m) * o->epochs);
  uint64_t s = o->seed ^ 0x5EED5EEDull;
  for (int32_t e = 0; e < o->epochs; ++e) {
    int32_t* p = perm.data() + static_cast<size_t>(e) * m;
    for (int64_t i = 0; i < m; ++i) p[i] = static_cast<int32_t>(i);
    for (int64_t i = m - 1; i > 0; --i) std::swap(p[i], p[static_cast<int64_t>(sm64(s) % static_cast<uint64_t>(i + 1))]);
  }
  CK(hipMemcpyAsync(didx, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, st), "upload order");
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int32_t e = 0; e < o->epochs; ++e) {
    for (int64_t b0 = 0; b0 < m; b0 += batch) {
      const int64_t nb = std::min(batch, m - b0);
      CK(hk_mlp_grad(st, M->p, M->mu, M->sd, dX, dy, didx + static_cast<size_t>(e) * m + b0, nb, partial, ploss, rows,
                     grad, dloss), "gradient");
      ++M->step;
      const float c1 = 1.f - std::pow(b1, static_cast<float>(M->step));
      const float c2 = 1.f - std::pow(b2, static_cast<float>(M->step));
      CK(hk_adam(st, M->p, grad, M->m1, M->m2, MLP_NPARAMS, o->lr, b1, b2, eps, c1, c2), "adam");
    }
  }
  if (final_loss) {
    CK(hk_mlp_grad(st, M->p, M->mu, M->sd, dX, dy, nullptr, m, partial, ploss, rows, grad, dloss), "final loss");
    CK(hipMemcpyAsync(final_loss, dloss, 4, hipMemcpyDeviceToHost, st), "read loss");
  }
  CK(hipStreamSynchronize(st), "synchronize");
  return HAWK_OK;
}

extern "C" hawk_status hawk_model_predict(hawk_model* M, const float* X, int64_t m, float* out) {
  if (!M || !M->ctx || m < 0 || (m > 0 && (!X || !out))) return HAWK_E_ARG;
  if (m == 0) return HAWK_OK;
  DevBuf B(M->ctx);
  float* dX = static_cast<float*>(B.get(static_cast<size_t>(m) * MLP_IN * 4));
  float* dO = static_cast<float*>(B.get(static_cast<size_t>(m) * 4));
  if (!dX || !dO) return set_error(M->ctx, HAWK_E_OOM, "predict buffers");
  hipStream_t st = M->ctx->stream;
  CK(hipMemcpyAsync(dX, X, static_cast<size_t>(m) * MLP_IN * 4, hipMemcpyHostToDevice, st), "upload X");
  CK(hk_mlp_forward(st, M->p, M->mu, M->sd, dX, m, dO), "forward");
  CK(hipMemcpyAsync(out, dO, static_cast<size_t>(m) * 4, hipMemcpyDeviceToHost, st), "read predictions");
  CK(hipStreamSynchronize(st), "synchronize");
  return HAWK_OK;
}

extern "C" hawk_status hawk_model_pick_ensemble(hawk_model* const* ms, int32_t nm, float penalty,
                                                hawk_query* const* qs, int32_t n, hawk_variant* out,
                                                float* predicted_ms) {
  if (!ms || nm < 1 || !ms[0] || !ms[0]->ctx || !qs || n < 1 || !out || !(penalty >= 0.f)) return HAWK_E_ARG;
  hawk_model* M = ms[0];  // errors are reported on its context
  hawk_ctx* ctx = M->ctx;
  for (int32_t k = 1; k < nm; ++k)
    if (!ms[k] || ms[k]->ctx != ctx) return set_error(ctx, HAWK_E_ARG, "models of different contexts");
  std::vector<std::vector<hawk_variant>> spaces;
  int64_t cols = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!qs[i] || qs[i]->ctx != ctx) return set_error(ctx, HAWK_E_ARG, "query of another context");
    spaces.push_back(variant_space(qs[i]));
    cols = std::max<int64_t>(cols, static_cast<int64_t>(spaces.back().size()));
  }
  const int64_t m = n * cols;
  std::vector<float> X(static_cast<size_t>(m) * MLP_IN, 0.f);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < cols; ++c) {
      const hawk_variant& v = spaces[i][std::min<int64_t>(c, static_cast<int64_t>(spaces[i].size()) - 1)];
      query_features(qs[i], &v, ctx->num_cus, &X[static_cast<size_t>(i * cols + c) * MLP_IN]);
    }
  DevBuf B(ctx);
  float* dX = static_cast<float*>(B.get(X.size() * 4));
  float* dO = static_cast<float*>(B.get(static_cast<size_t>(m) * nm * 4));
  if (!dX || !dO) return set_error(ctx, HAWK_E_OOM, "pick buffers");
  hipStream_t st = ctx->stream;
  CK(hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, st), "upload features");
  for (int32_t k = 0; k < nm; ++k)
    CK(hk_mlp_forward(st, ms[k]->p, ms[k]->mu, ms[k]->sd, dX, m, dO + k * m), "forward");
  std::vector<float> pred(static_cast<size_t>(m) * nm);
  CK(hipMemcpyAsync(pred.data(), dO, pred.size() * 4, hipMemcpyDeviceToHost, st), "read predictions");
  CK(hipStreamSynchronize(st), "synchronize");
  // score = mean + penalty * standard deviation of the members' ln(ms)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t nv = static_cast<int64_t>(spaces[i].size());
    int64_t best = 0;
    double best_score = 0, best_mean = 0;
    for (int64_t c = 0; c < nv; ++c) {
      double s1 = 0, s2 = 0;
      for (int32_t k = 0; k < nm; ++k) {
        const double y = pred[static_cast<size_t>(k * m + i * cols + c)];
        s1 += y;
        s2 += y * y;
      }
      const double mean = s1 / nm;
      const double sd = std::sqrt(std::max(0.0, s2 / nm - mean * mean));
      const double score = mean + penalty * sd;
      if (c == 0 || score < best_score) {
        best = c;
        best_score = score;
        best_mean = mean;
      }
    }
    out[i] = spaces[i][best];
    if (predicted_ms) predicted_ms[i] = static_cast<float>(std::exp(best_mean));
  }
  return HAWK_OK;
}

extern "C" hawk_status hawk_model_pick(hawk_model* M, hawk_query* const* qs, int32_t n, hawk_variant* out,
                                       float* predicted_ms) {
  if (!M || !M->ctx || !qs || n < 1 || !out) return HAWK_E_ARG;
  // every query's variant space, featurised on the host (plan metadata), scored on the device
  std::vector<std::vector<hawk_variant>> spaces;
  int64_t cols = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!qs[i] || qs[i]->ctx != M->ctx) return set_error(M->ctx, HAWK_E_ARG, "query of another context");
    spaces.push_back(variant_space(qs[i]));
    cols = std::max<int64_t>(cols, static_cast<int64_t>(spaces.back().size()));
  }
  const int64_t rows = n;
  std::vector<float> X(static_cast<size_t>(rows * cols) * MLP_IN, 0.f);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < cols; ++c) {
      const hawk_variant& v = spaces[i][std::min<int64_t>(c, static_cast<int64_t>(spaces[i].size()) - 1)];
      query_features(qs[i], &v, M->ctx->num_cus, &X[static_cast<size_t>(i * cols + c) * MLP_IN]);
    }
  DevBuf B(M->ctx);
  float* dX = static_cast<float*>(B.get(X.size() * 4));
  float* dO = static_cast<float*>(B.get(static_cast<size_t>(rows * cols) * 4));
  int32_t* dI = static_cast<int32_t*>(B.get(static_cast<size_t>(rows) * 4));
  if (!dX || !dO || !dI) return set_error(M->ctx, HAWK_E_OOM, "pick buffers");
  hipStream_t st = M->ctx->stream;
  CK(hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, st), "upload features");
  CK(hk_mlp_forward(st, M->p, M->mu, M->sd, dX, rows * cols, dO), "forward");
  CK(hk_argmin_rows(st, dO, rows, cols, dI), "argmin");
  std::vector<int32_t> idx(static_cast<size_t>(rows));
  std::vector<float> pred(static_cast<size_t>(rows * cols));
  CK(hipMemcpyAsync(idx.data(), dI, idx.size() * 4, hipMemcpyDeviceToHost, st), "read picks");
  CK(hipMemcpyAsync(pred.data(), dO, pred.size() * 4, hipMemcpyDeviceToHost, st), "read predictions");
  CK(hipStreamSynchronize(st), "synchronize");
  for (int32_t i = 0; i < n; ++i) {
    out[i] = spaces[i][idx[i]];
    if (predicted_ms) predicted_ms[i] = std::exp(pred[static_cast<size_t>(i * cols + idx[i])]);
  }
  return HAWK_OK;
}
