// Surrogate network object (see mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace hom {

constexpr int MLP_IN = 32;      // padded input width
constexpr int MLP_W = 256;      // hidden width
constexpr int MLP_OUT = 16;     // padded output width
constexpr int MLP_LAYERS = 5;   // 4 hidden layers + output layer
constexpr int MLP_GATES = 10;   // 1 + 3 gate variables x (linear, square, cube)

struct Mlp {
  int n_in, n_out;
  size_t woff[MLP_LAYERS], boff[MLP_LAYERS];  // offsets in the padded parameter arrays
  size_t npad = 0;
  // device parameters (padded): master FP32, gradient, Adam moments,
  // bf16 hi / lo copies, effective FP32 weights of the bf16 / precise forward
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *eff_bf = nullptr, *eff_pr = nullptr;
  __bf16 *hi = nullptr, *lo = nullptr;
  float* scal = nullptr;  // xmean[32] xinv[32] ymean[16] ystd[16] lossw[16]
  // fixed gated-polynomial skip on the normalized inputs xhat:
  //   y_j += c_j + sum_g s_g(xhat) sum_k G[j][g][k] xhat_k,
  //   s = (1, v_a, v_a^2, v_a^3, v_b, ..., v_c^3), v = xhat at three gate indices
  float* skip = nullptr;  // G [16][MLP_GATES][32], c [16]
  int gate[3] = {0, 0, 0};
  std::vector<double> hskip;                   // host copy of G and c
  std::vector<float> hx_mean, hx_inv;          // host copy of the input scaling
  std::vector<float> hy_mean, hy_std;          // host copy of the output scaling
  // Training targets of physical rows T [n][n_out]: what the skip leaves,
  // normalized, padded to MLP_OUT columns
  void normalized_targets(const float* X, const float* T, long long n, float* out) const;
  // xhat of one raw input row and the skip value of output j
  void normalize_row(const float* x, double* xn) const;
  double skip_value(const double* xn, int j) const;
  // Least-squares fit of the skip on (X, Y), then input / residual scaling
  // from the same rows (lw: loss weights of the outputs)
  void fit_skip(const float* X, const float* Y, long long n, const int* gates, const float* lw, const float* rw);
  std::vector<void*> allocs;
  // training work space
  long long work_rows = 0;
  std::vector<void*> work;
  float *xs = nullptr, *zs[MLP_LAYERS - 1] = {}, *as[MLP_LAYERS - 1] = {}, *yhat = nullptr, *dy = nullptr;
  float *da = nullptr, *dz = nullptr, *xb = nullptr, *tb = nullptr, *rwb = nullptr, *lpart = nullptr;
  // split-K partials of the weight-gradient products and FP64 column-sum
  // partials of the bias gradients (grown on demand, one set per network so
  // that networks can train concurrently)
  float* splitk = nullptr;
  size_t splitk_n = 0;
  double* csum = nullptr;
  size_t csum_n = 0;

  Mlp(int n_in, int n_out, uint64_t seed);
  ~Mlp();
  Mlp(const Mlp&) = delete;
  Mlp& operator=(const Mlp&) = delete;

  void set_scaling(const float* xmean, const float* xstd, const float* ymean, const float* ystd, const float* lw);
  // G [n_out][MLP_GATES][n_in], c [n_out], gates: three input indices
  void set_skip(const int* gates, const float* G, const float* c);
  void refresh(hipStream_t s);
  void ensure_work(long long rows);
  void free_work();
  // x: device [n][n_in]; y: device [n][n_out] (physical units) or null
  void forward(const float* x, float* y, long long n, bool precise, bool save, hipStream_t s);
  // x: device raw inputs, t: device normalized targets [B][16], rw: device
  // row weights [B] or null; fills g
  double loss_grad(const float* x, const float* tnorm, long long B, bool precise, hipStream_t s,
                   const float* rw = nullptr);
  // the gradient of loss_grad without reading the loss back; returns the
  // number of loss partials left in lpart
  int grad_only(const float* x, const float* tnorm, long long B, bool precise, hipStream_t s,
                const float* rw = nullptr);
  void train(const float* X, const float* T, long long n, int epochs, int batch, double lr, uint64_t seed,
             const float* row_weight, float* loss_out);
  // zero the Adam moments (a later train call starts its optimizer afresh)
  void reset_optimizer();
  void get_params(float* out) const;
  void get_grads(float* out) const;
  void set_params(const float* in);
  size_t param_count() const;
};

// ys: scratch [M][n][n_out]
void ensemble_accept(const Mlp* const* nets, int M, const float* x, float* y, float* ys, float* spread,
                     uint8_t* accept, long long n, float thr, float floor_scale, hipStream_t s);
// the same with ys in the library's static device array (no device
// allocation); n * M * n_out above HOM_STATIC_SCRATCH_FLOATS fails with HOM_E_ARG
void ensemble_accept_static(const Mlp* const* nets, int M, const float* x, float* y, float* spread, uint8_t* accept,
                            long long n, float thr, float floor_scale, hipStream_t s);

}  // namespace hom
