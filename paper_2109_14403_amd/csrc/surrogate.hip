// Surrogate with FFT fallback (declared in include/hom.h).
//
// Host orchestration around two device engines: the network ensemble
// (mlp.hip: bf16 MFMA forward of every network, then the mean / spread /
// acceptance kernel) and the batched FFT solver (runtime.hip). Input rows are
// built on the host from each point's macroscopic summary: one row is 32
// floats, far below the cost of either engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <random>
#include <thread>

#include "surrogate.h"

namespace hom {

namespace {

const double kSq2 = std::sqrt(2.0);

inline void to_mandel(const double* c, double* m) {
  for (int a = 0; a < 3; ++a) m[a] = c[a];
  for (int a = 3; a < 6; ++a) m[a] = kSq2 * c[a];
}

inline double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// row (h, k) of history arrays
struct Hist {
  int count, steps;
  const double *strain, *theta, *grad, *dt;
  const double* e(int h, int k) const { return strain + ((size_t)h * steps + k) * 6; }
  double th(int h, int k) const { return theta[(size_t)h * steps + k]; }
  const double* g(int h, int k) const { return grad + ((size_t)h * steps + k) * 3; }
  double d(int h, int k) const { return dt[(size_t)h * steps + k]; }
};

void check_hist(const Hist& H) {
  if (H.count < 1 || H.steps < 1) fail(HOM_E_ARG, "need at least one history of one increment");
  if (!H.strain || !H.theta || !H.grad || !H.dt) fail(HOM_E_ARG, "null history array");
  const size_t n = (size_t)H.count * H.steps;
  for (size_t i = 0; i < n; ++i) {
    if (!(H.dt[i] > 0.0) || !std::isfinite(H.dt[i])) fail(HOM_E_ARG, "time steps must be positive");
    if (!(H.theta[i] > 0.0) || !std::isfinite(H.theta[i])) fail(HOM_E_ARG, "temperatures must be positive");
  }
}

void fill_load(hom_load& L, const double* strain, double theta, const double* grad, double dt) {
  std::memset(&L, 0, sizeof(L));
  std::memcpy(L.strain, strain, sizeof(L.strain));
  L.temp.theta = theta;
  for (int d = 0; d < 3; ++d) L.temp.grad[d] = grad[d];
  L.dt = dt;
}

// Mandel norm of an answer's stress
double stress_norm(const hom_result& r) {
  double m[6];
  to_mandel(r.stress, m);
  double s = 0.0;
  for (double v : m) s += v * v;
  return std::sqrt(s);
}

// teacher-forced rows of the histories in `ids`: summaries from the FFT answers
void forced_rows(const Hist& H, const hom_result* fft, double theta_init, const std::vector<int>& ids, float* X,
                 float* Y, double* denom) {
  size_t r = 0;
  for (int h : ids) {
    double dn = 0.0;
    for (int k = 0; k < H.steps; ++k) dn = std::max(dn, stress_norm(fft[(size_t)h * H.steps + k]));
    SurSummary s;
    sur_summary_init(s, theta_init);
    for (int k = 0; k < H.steps; ++k, ++r) {
      const hom_result& f = fft[(size_t)h * H.steps + k];
      double sig[6];
      to_mandel(f.stress, sig);
      sur_features(s, H.e(h, k), H.th(h, k), H.g(h, k), H.d(h, k), X + r * SUR_IN);
      if (Y) {
        for (int a = 0; a < 6; ++a) Y[r * SUR_OUT + a] = (float)sig[a];
        for (int a = 0; a < 3; ++a) Y[r * SUR_OUT + 6 + a] = (float)f.heat_flux[a];
        Y[r * SUR_OUT + 9] = (float)f.dissipation;
      }
      if (denom) denom[r] = dn;
      sur_commit(s, H.e(h, k), H.th(h, k), H.d(h, k), sig, f.dissipation);
    }
  }
}

double quantile_of(std::vector<double> v, double q) {
  if (v.empty()) return std::numeric_limits<double>::quiet_NaN();
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

void sur_history_rows(int count, int steps, const double* strain, const double* theta, const double* grad,
                      const double* dt, const hom_result* fft, double theta_init, float* X, float* Y, double* denom) {
  const Hist H{count, steps, strain, theta, grad, dt};
  check_hist(H);
  if (!fft || !X) fail(HOM_E_ARG, "null argument");
  if (!(theta_init > 0.0)) fail(HOM_E_ARG, "theta_init must be positive");
  std::vector<int> ids(count);
  std::iota(ids.begin(), ids.end(), 0);
  forced_rows(H, fft, theta_init, ids, X, Y, denom);
}

void sur_summary_init(SurSummary& s, double theta_init) {
  std::memset(&s, 0, sizeof(s));
  s.theta_n = theta_init;
}

void sur_features(const SurSummary& s, const double* strain, double theta, const double* grad, double dt, float* x) {
  double E[6];
  to_mandel(strain, E);
  for (int a = 0; a < 6; ++a) {
    x[a] = (float)E[a];
    x[8 + a] = (float)s.E_n[a];
    x[14 + a] = (float)s.sig_n[a];
    x[20 + a] = (float)s.E_nm1[a];
  }
  x[6] = (float)theta;
  x[7] = (float)std::log10(dt);
  x[26] = (float)s.theta_n;
  x[27] = (float)s.diss_n;
  x[28] = (float)s.diss_int;
  for (int d = 0; d < 3; ++d) x[29 + d] = (float)grad[d];
}

void sur_commit(SurSummary& s, const double* strain, double theta, double dt, const double* sig, double diss) {
  double E[6];
  to_mandel(strain, E);
  for (int a = 0; a < 6; ++a) {
    s.E_nm1[a] = s.E_n[a];
    s.E_n[a] = E[a];
    s.sig_n[a] = sig[a];
  }
  s.theta_n = theta;
  s.diss_n = diss;
  s.diss_int += diss * dt;
}

// ---------------------------------------------------------------------------
// Surrogate
// ---------------------------------------------------------------------------
Surrogate::Surrogate(const hom_grid& g, const uint8_t* ph, const hom_law* lw, int nl, const hom_options& o,
                     const hom_surrogate_config& c)
    : grid(g), laws(lw, lw + nl), opts(o), cfg(c) {
  if (cfg.n_nets < 2 || cfg.n_nets > HOM_ENSEMBLE_MAX_NETS) fail(HOM_E_ARG, "ensemble size must be 2 .. 16");
  if (cfg.epochs < 1 || cfg.batch < 1 || !(cfg.lr > 0.0)) fail(HOM_E_ARG, "training settings out of range");
  if (!(cfg.target > 0.0) || !(cfg.quantile > 0.0 && cfg.quantile <= 1.0))
    fail(HOM_E_ARG, "target must be positive and quantile in (0, 1]");
  if (!(cfg.holdout > 0.0 && cfg.holdout < 1.0)) fail(HOM_E_ARG, "holdout must lie in (0, 1)");
  if (!(cfg.floor_scale > 0.0) || !(cfg.theta_init > 0.0)) fail(HOM_E_ARG, "floor_scale and theta_init must be > 0");
  if (cfg.chunk < 1 || cfg.max_resident < 0) fail(HOM_E_ARG, "chunk must be >= 1 and max_resident >= 0");
  if (opts.stream) fail(HOM_E_ARG, "the surrogate's cells own their streams: opts.stream must be NULL");
  const size_t nv = (size_t)g.n[0] * g.n[1] * g.n[2];
  if (!ph || g.n[0] < 1 || g.n[1] < 1 || g.n[2] < 1) fail(HOM_E_ARG, "null phases or empty grid");
  phases.assign(ph, ph + nv);
  // one cell checks grid, laws and options the way every later one sees them
  new_cells(1);
  for (int m = 0; m < cfg.n_nets; ++m) nets.emplace_back(new Mlp(SUR_IN, SUR_OUT, cfg.seed + 1000003ull * m));
  HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
}

Surrogate::~Surrogate() {
  if (stream) (void)hipStreamSynchronize(stream);
  for (void* p : {(void*)dx, (void*)dy, (void*)dys, (void*)dspread, (void*)dacc, (void*)scratch})
    if (p) (void)hipFree(p);
  if (stream) (void)hipStreamDestroy(stream);
}

void Surrogate::clamp_summary(float* x) const {
  if (!have_range) return;
  for (int j = 8; j < 29; ++j) x[j] = std::min(std::max(x[j], sum_lo[j]), sum_hi[j]);
}

std::unique_ptr<BatchImpl> Surrogate::new_cells(int count) const {
  std::vector<hom_grid> grids(count, grid);
  std::vector<const uint8_t*> ph(count, phases.data());
  return make_batch(count, grids.data(), ph.data(), laws.data(), (int)laws.size(), opts);
}

void Surrogate::solve_histories(int count, int steps, const double* strain, const double* theta, const double* grad,
                                const double* dt, hom_result* out, double* seconds) {
  const Hist H{count, steps, strain, theta, grad, dt};
  check_hist(H);
  if (!out) fail(HOM_E_ARG, "null output");
  double t_solve = 0.0, t_setup = 0.0;
  for (int c0 = 0; c0 < count; c0 += cfg.chunk) {
    const int m = std::min(count, c0 + cfg.chunk) - c0;
    double t0 = now_ms();
    auto cells = new_cells(m);
    t_setup += now_ms() - t0;
    std::vector<hom_load> loads(m);
    std::vector<hom_result> res(m);
    for (int k = 0; k < steps; ++k) {
      for (int i = 0; i < m; ++i) fill_load(loads[i], H.e(c0 + i, k), H.th(c0 + i, k), H.g(c0 + i, k), H.d(c0 + i, k));
      t0 = now_ms();
      cells->solve(loads.data(), res.data());
      t_solve += now_ms() - t0;
      for (int i = 0; i < m; ++i) out[(size_t)(c0 + i) * steps + k] = res[i];
    }
  }
  if (seconds) {
    seconds[0] = t_solve * 1e-3;
    seconds[1] = t_setup * 1e-3;
  }
}

void Surrogate::ensure_rows(long long n) {
  if (n <= cap_rows) return;
  HIPCHK(hipStreamSynchronize(stream));
  for (void* p : {(void*)dx, (void*)dy, (void*)dys, (void*)dspread, (void*)dacc})
    if (p) HIPCHK(hipFree(p));
  dx = dy = dys = dspread = nullptr;
  dacc = nullptr;
  HIPCHK(hipMalloc((void**)&dx, (size_t)n * SUR_IN * 4));
  HIPCHK(hipMalloc((void**)&dy, (size_t)n * SUR_OUT * 4));
  HIPCHK(hipMalloc((void**)&dys, (size_t)n * nets.size() * SUR_OUT * 4));
  HIPCHK(hipMalloc((void**)&dspread, (size_t)n * 4));
  HIPCHK(hipMalloc((void**)&dacc, (size_t)n));
  cap_rows = n;
}

void Surrogate::infer_host(const float* X, long long n, float* y, float* spread) {
  if (n <= 0) return;
  ensure_rows(n);
  std::vector<const Mlp*> nv;
  for (auto& p : nets) nv.push_back(p.get());
  HIPCHK(hipMemcpyAsync(dx, X, (size_t)n * SUR_IN * 4, hipMemcpyHostToDevice, stream));
  ensemble_accept(nv.data(), (int)nv.size(), dx, dy, dys, dspread, dacc, n, (float)threshold,
                  (float)cfg.floor_scale, stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(y, dy, (size_t)n * SUR_OUT * 4, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(spread, dspread, (size_t)n * 4, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
}

void Surrogate::infer_device(const float* x, float* y, uint8_t* acc, long long n, hipStream_t s) {
  if (n <= 0) return;
  const long long need = n * ((long long)nets.size() * SUR_OUT + 1);
  if (need > scratch_rows) {
    HIPCHK(hipDeviceSynchronize());
    if (scratch) HIPCHK(hipFree(scratch));
    scratch = nullptr;
    HIPCHK(hipMalloc((void**)&scratch, (size_t)need * 4));
    scratch_rows = need;
  }
  std::vector<const Mlp*> nv;
  for (auto& p : nets) nv.push_back(p.get());
  float* ys = scratch;
  float* sp = scratch + (size_t)n * nets.size() * SUR_OUT;
  ensemble_accept(nv.data(), (int)nv.size(), x, y, ys, sp, acc, n, (float)threshold, (float)cfg.floor_scale, s);
  HIPCHK(hipGetLastError());
}

void Surrogate::train(int count, int steps, const double* strain, const double* theta, const double* grad,
                      const double* dt, const hom_result* fft, hom_surrogate_report* rep) {
  const Hist H{count, steps, strain, theta, grad, dt};
  check_hist(H);
  if (count < 2) fail(HOM_E_ARG, "need two histories at least (training and calibration)");
  std::vector<hom_result> own;
  if (!fft) {
    own.resize((size_t)count * steps);
    solve_histories(count, steps, strain, theta, grad, dt, own.data(), nullptr);
    fft = own.data();
  }
  // hold-out split by history (seeded)
  std::vector<int> ids(count);
  std::iota(ids.begin(), ids.end(), 0);
  std::mt19937_64 gen(cfg.seed ^ 0x9e3779b97f4a7c15ull);
  std::shuffle(ids.begin(), ids.end(), gen);
  const int nh = std::min(count - 1, std::max(1, (int)std::lround(cfg.holdout * count)));
  std::vector<int> hold(ids.begin(), ids.begin() + nh), tr(ids.begin() + nh, ids.end());
  std::sort(hold.begin(), hold.end());
  std::sort(tr.begin(), tr.end());
  const long long rows = (long long)tr.size() * steps;
  if (rows < cfg.batch) fail(HOM_E_ARG, "fewer training rows than one minibatch");
  std::vector<float> X((size_t)rows * SUR_IN), Y((size_t)rows * SUR_OUT);
  forced_rows(H, fft, cfg.theta_init, tr, X.data(), Y.data(), nullptr);
  for (int j = 0; j < SUR_IN; ++j) {
    sum_lo[j] = std::numeric_limits<float>::max();
    sum_hi[j] = -std::numeric_limits<float>::max();
  }
  for (long long r = 0; r < rows; ++r)
    for (int j = 0; j < SUR_IN; ++j) {
      sum_lo[j] = std::min(sum_lo[j], X[(size_t)r * SUR_IN + j]);
      sum_hi[j] = std::max(sum_hi[j], X[(size_t)r * SUR_IN + j]);
    }
  have_range = true;

  // the fixed skip and scaling, then the network on the remainder: one host
  // thread (and device stream) per network
  const int gates[3] = {7, 6, 26};  // log10 dt, theta^{n+1}, theta^n
  float lw[SUR_OUT];
  for (int j = 0; j < SUR_OUT; ++j) lw[j] = j < 6 ? 4.f : 1.f;  // the stress is the accuracy target
  const int M = (int)nets.size();
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  // every network from its own host thread (and device stream)
  auto each_net = [&](auto&& work) {
    std::vector<std::string> errs(M);
    std::vector<int> codes(M, HOM_OK);
    std::vector<std::thread> pool;
    for (int m = 0; m < M; ++m) {
      pool.emplace_back([&, m] {
        try {
          HIPCHK(hipSetDevice(dev));
          work(m);
        } catch (const Error& e) {
          codes[m] = e.code;
          errs[m] = e.msg;
        } catch (const std::exception& e) {
          codes[m] = HOM_E_DEVICE;
          errs[m] = e.what();
        }
      });
    }
    for (auto& t : pool) t.join();
    for (int m = 0; m < M; ++m)
      if (codes[m] != HOM_OK) fail(codes[m], "network " + std::to_string(m) + ": " + errs[m]);
  };
  const double t0 = now_ms();
  std::vector<float> losses((size_t)M * cfg.epochs, 0.f);
  for (auto& net : nets) net->reset_optimizer();
  each_net([&](int m) {
    nets[m]->fit_skip(X.data(), Y.data(), rows, gates, lw, nullptr);
    nets[m]->train(X.data(), Y.data(), rows, cfg.epochs, cfg.batch, cfg.lr, cfg.seed + 17ull * m, nullptr,
                   losses.data() + (size_t)m * cfg.epochs);
  });
  const double fit_s = (now_ms() - t0) * 1e-3;

  // calibration on the held-out histories
  std::vector<double> hs((size_t)nh * steps * 6), hth((size_t)nh * steps), hg((size_t)nh * steps * 3),
      hdt((size_t)nh * steps);
  std::vector<hom_result> hf((size_t)nh * steps);
  for (int j = 0; j < nh; ++j)
    for (int k = 0; k < steps; ++k) {
      const size_t a = (size_t)j * steps + k, b = (size_t)hold[j] * steps + k;
      std::memcpy(&hs[a * 6], H.e(hold[j], k), 6 * sizeof(double));
      std::memcpy(&hg[a * 3], H.g(hold[j], k), 3 * sizeof(double));
      hth[a] = H.th(hold[j], k);
      hdt[a] = H.d(hold[j], k);
      hf[a] = fft[b];
    }
  hom_surrogate_report r;
  std::memset(&r, 0, sizeof(r));
  calibrate(nh, steps, hs.data(), hth.data(), hg.data(), hdt.data(), hf.data(), cfg.target, cfg.quantile, &r);
  r.train_rows = rows;
  r.fit_seconds = fit_s;
  for (int m = 0; m < HOM_ENSEMBLE_MAX_NETS; ++m)
    r.final_loss[m] = m < M ? (double)losses[(size_t)m * cfg.epochs + cfg.epochs - 1]
                            : std::numeric_limits<double>::quiet_NaN();
  if (rep) *rep = r;
}

void Surrogate::calibrate(int count, int steps, const double* strain, const double* theta, const double* grad,
                          const double* dt, const hom_result* fft, double target, double quantile,
                          hom_surrogate_report* rep) {
  const Hist H{count, steps, strain, theta, grad, dt};
  check_hist(H);
  if (!fft) fail(HOM_E_ARG, "calibration needs the FFT answers");
  if (!(target > 0.0) || !(quantile > 0.0 && quantile <= 1.0)) fail(HOM_E_ARG, "target or quantile out of range");
  std::vector<double> denom(count, 0.0);
  for (int h = 0; h < count; ++h)
    for (int k = 0; k < steps; ++k) denom[h] = std::max(denom[h], stress_norm(fft[(size_t)h * steps + k]));
  // network rollout: every summary from the ensemble's own answers
  std::vector<SurSummary> S(count);
  for (auto& s : S) sur_summary_init(s, cfg.theta_init);
  std::vector<float> X((size_t)count * SUR_IN), y((size_t)count * SUR_OUT), sp(count);
  const size_t N = (size_t)count * steps;
  std::vector<double> err(N), spread(N);
  for (int k = 0; k < steps; ++k) {
    for (int h = 0; h < count; ++h) {
      sur_features(S[h], H.e(h, k), H.th(h, k), H.g(h, k), H.d(h, k), &X[(size_t)h * SUR_IN]);
      clamp_summary(&X[(size_t)h * SUR_IN]);
    }
    infer_host(X.data(), count, y.data(), sp.data());
    for (int h = 0; h < count; ++h) {
      double sig[6], ref[6], d2 = 0.0;
      to_mandel(fft[(size_t)h * steps + k].stress, ref);
      for (int a = 0; a < 6; ++a) {
        sig[a] = y[(size_t)h * SUR_OUT + a];
        d2 += (sig[a] - ref[a]) * (sig[a] - ref[a]);
      }
      err[(size_t)h * steps + k] = std::sqrt(d2) / std::max(denom[h], 1e-12);
      spread[(size_t)h * steps + k] = sp[h];
      sur_commit(S[h], H.e(h, k), H.th(h, k), H.d(h, k), sig, y[(size_t)h * SUR_OUT + 9]);
    }
  }
  // the largest threshold whose accepted rows meet the target at the quantile
  std::vector<size_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return spread[a] < spread[b]; });
  size_t cut = 0, bad = 0;
  for (size_t i = 0; i < N; ++i) {
    bad += err[order[i]] > target ? 1 : 0;
    if ((double)bad <= (1.0 - quantile) * (double)(i + 1) + 1e-12) cut = i + 1;
    else if (quantile >= 1.0) break;
  }
  threshold = cut > 0 ? spread[order[cut - 1]] : -1.0;
  if (!rep) return;
  std::vector<double> acc_err, all(err.begin(), err.end());
  for (size_t i = 0; i < N; ++i)
    if (spread[i] <= threshold) acc_err.push_back(err[i]);
  rep->holdout_rows = (long long)N;
  rep->threshold = threshold;
  rep->holdout_accepted = (double)acc_err.size() / (double)N;
  rep->holdout_accepted_max_error =
      acc_err.empty() ? std::numeric_limits<double>::quiet_NaN() : *std::max_element(acc_err.begin(), acc_err.end());
  rep->holdout_accepted_p99_error = quantile_of(acc_err, 0.99);
  rep->holdout_median_error = quantile_of(all, 0.5);
  // the same rows with the FFT history as summary, and the skip alone
  std::vector<int> ids(count);
  std::iota(ids.begin(), ids.end(), 0);
  std::vector<float> XF(N * SUR_IN), yf(N * SUR_OUT), sf(N);
  std::vector<double> den(N);
  forced_rows(H, fft, cfg.theta_init, ids, XF.data(), nullptr, den.data());
  infer_host(XF.data(), (long long)N, yf.data(), sf.data());
  std::vector<double> ef(N), es(N), xn(SUR_IN);
  const Mlp& net0 = *nets[0];
  for (size_t r = 0; r < N; ++r) {
    double ref[6], d2 = 0.0, s2 = 0.0;
    to_mandel(fft[r].stress, ref);
    net0.normalize_row(&XF[r * SUR_IN], xn.data());
    for (int a = 0; a < 6; ++a) {
      const double v = yf[r * SUR_OUT + a] - ref[a];
      d2 += v * v;
      const double w = net0.skip_value(xn.data(), a) + net0.hy_mean[a] - ref[a];
      s2 += w * w;
    }
    ef[r] = std::sqrt(d2) / std::max(den[r], 1e-12);
    es[r] = std::sqrt(s2) / std::max(den[r], 1e-12);
  }
  rep->holdout_median_error_forced = quantile_of(ef, 0.5);
  rep->skip_median_error = quantile_of(es, 0.5);
}

// ---------------------------------------------------------------------------
// point sets
// ---------------------------------------------------------------------------
SurrogatePoints::SurrogatePoints(Surrogate* s, int count) : sur(s), n(count) {
  if (count < 1) fail(HOM_E_ARG, "need at least one point");
  summary.resize(count);
  for (auto& x : summary) sur_summary_init(x, s->cfg.theta_init);
  mode.assign(count, -1);
}

void SurrogatePoints::step_all(const double* strain, const double* theta, const double* grad, const double* dt,
                               hom_result* out, uint8_t* accepted, hom_surrogate_step_info* info) {
  if (!strain || !theta || !grad || !dt || !out || !accepted) fail(HOM_E_ARG, "null argument");
  const Hist H{n, 1, strain, theta, grad, dt};
  check_hist(H);
  hom_surrogate_step_info inf;
  std::memset(&inf, 0, sizeof(inf));
  // the macroscopic heat capacity <c0> of the microstructure
  double c0 = 0.0;
  {
    std::vector<long long> cnt(256, 0);
    for (uint8_t p : sur->phases) ++cnt[p];
    for (size_t l = 0; l < sur->laws.size(); ++l) c0 += sur->laws[l].c0 * (double)cnt[l] / (double)sur->phases.size();
  }
  const double nan = std::numeric_limits<double>::quiet_NaN();

  // 1. the ensemble for every point not handed to the FFT solver
  double t0 = now_ms();
  std::vector<int> net_pts;
  for (int i = 0; i < n; ++i)
    if (mode[i] < 0) net_pts.push_back(i);
  const long long m = (long long)net_pts.size();
  std::vector<float> X((size_t)m * SUR_IN), y((size_t)m * SUR_OUT), sp(m);
  for (long long j = 0; j < m; ++j) {
    const int i = net_pts[j];
    sur_features(summary[i], strain + 6 * (size_t)i, theta[i], grad + 3 * (size_t)i, dt[i], &X[(size_t)j * SUR_IN]);
    sur->clamp_summary(&X[(size_t)j * SUR_IN]);
  }
  sur->infer_host(X.data(), m, y.data(), sp.data());
  std::vector<int> rejected;
  for (long long j = 0; j < m; ++j) {
    const int i = net_pts[j];
    if (sp[j] <= sur->threshold) {
      hom_result& r = out[i];
      std::memset(&r, 0, sizeof(r));
      for (int a = 0; a < 6; ++a) r.stress[a] = y[(size_t)j * SUR_OUT + a] / (a < 3 ? 1.0 : kSq2);
      for (int a = 0; a < 3; ++a) r.heat_flux[a] = y[(size_t)j * SUR_OUT + 6 + a];
      r.dissipation = y[(size_t)j * SUR_OUT + 9];
      r.coupling = nan;
      r.heat_capacity = c0;
      r.residual = nan;
      r.status = HOM_OK;
      std::memcpy(r.strain, strain + 6 * (size_t)i, sizeof(r.strain));
      r.theta = theta[i];
      r.stagger_iters = 0;
      accepted[i] = 1;
      ++inf.network_points;
    } else {
      rejected.push_back(i);
    }
  }
  inf.rejected_points = (int)rejected.size();
  const double t1 = now_ms();

  auto answer = [&](int i, const hom_result& r) {
    out[i] = r;
    accepted[i] = 0;
  };
  // 2. points with resident cells: one increment each
  for (auto& grp : resident) {
    const int g = (int)grp.points.size();
    std::vector<hom_load> loads(g);
    std::vector<hom_result> res(g);
    for (int j = 0; j < g; ++j) {
      const int i = grp.points[j];
      fill_load(loads[j], strain + 6 * (size_t)i, theta[i], grad + 3 * (size_t)i, dt[i]);
    }
    grp.cells->solve(loads.data(), res.data());
    for (int j = 0; j < g; ++j) answer(grp.points[j], res[j]);
    inf.resident_points += g;
  }
  // 3. newly rejected points: fresh cells replay the macroscopic history, then
  //    answer this increment
  for (size_t c0i = 0; c0i < rejected.size(); c0i += (size_t)sur->cfg.chunk) {
    const int g = (int)std::min(rejected.size() - c0i, (size_t)sur->cfg.chunk);
    std::vector<int> pts(rejected.begin() + c0i, rejected.begin() + c0i + g);
    auto cells = sur->new_cells(g);
    std::vector<hom_load> loads(g);
    std::vector<hom_result> res(g);
    bool ok = true;
    for (int k = 0; k < step; ++k) {
      const std::vector<double>& hk = history[k];
      for (int j = 0; j < g; ++j) {
        const double* row = &hk[(size_t)pts[j] * 11];
        fill_load(loads[j], row, row[6], row + 7, row[10]);
      }
      cells->solve(loads.data(), res.data());
      for (int j = 0; j < g; ++j) ok = ok && res[j].status == HOM_OK;
      inf.replayed_increments += g;
    }
    for (int j = 0; j < g; ++j) {
      const int i = pts[j];
      fill_load(loads[j], strain + 6 * (size_t)i, theta[i], grad + 3 * (size_t)i, dt[i]);
    }
    cells->solve(loads.data(), res.data());
    for (int j = 0; j < g; ++j) {
      ok = ok && res[j].status == HOM_OK;
      answer(pts[j], res[j]);
    }
    // keep the cells while they are in step with their points and there is room
    if (ok && resident_count + g <= sur->cfg.max_resident) {
      for (int i : pts) mode[i] = (int)resident.size();
      resident.push_back(Cells{std::move(cells), pts});
      resident_count += g;
    }
  }
  const double t2 = now_ms();
  inf.network_ms = t1 - t0;
  inf.fallback_ms = t2 - t1;

  // 4. commit: summaries and the macroscopic history
  std::vector<double> row((size_t)n * 11);
  for (int i = 0; i < n; ++i) {
    double* r = &row[(size_t)i * 11];
    std::memcpy(r, strain + 6 * (size_t)i, 6 * sizeof(double));
    r[6] = theta[i];
    std::memcpy(r + 7, grad + 3 * (size_t)i, 3 * sizeof(double));
    r[10] = dt[i];
    double sig[6];
    to_mandel(out[i].stress, sig);
    sur_commit(summary[i], strain + 6 * (size_t)i, theta[i], dt[i], sig, out[i].dissipation);
  }
  history.push_back(std::move(row));
  ++step;
  if (info) *info = inf;
}

}  // namespace hom
