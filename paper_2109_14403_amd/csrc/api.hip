// extern "C" entry points of libhom.so (declared in include/hom.h).
#include <cstring>
#include <new>
#include <vector>

#include "dmn.h"
#include "mlp.h"
#include "runtime.h"
#include "surrogate.h"

struct hom_ctx {
  std::unique_ptr<hom::BatchImpl> impl;
  std::string err;
};
struct hom_batch {
  std::unique_ptr<hom::BatchImpl> impl;
  std::string err;
};
struct hom_dmn {
  std::unique_ptr<hom::Dmn> net;
  std::string err;
};
struct hom_dmn_online {
  hom::DmnOnline* impl = nullptr;
  std::string err;
  ~hom_dmn_online() {
    if (impl) hom::dmn_online_destroy(impl);
  }
};
struct hom_mlp {
  std::unique_ptr<hom::Mlp> net;
  std::string err;
  float* scratch = nullptr;  // per-network outputs of hom_mlp_ensemble_infer
  size_t scratch_floats = 0;
  ~hom_mlp() {
    if (scratch) (void)hipFree(scratch);
  }
};

struct hom_surrogate {
  std::unique_ptr<hom::Surrogate> impl;
};
struct hom_surrogate_points {
  std::unique_ptr<hom::SurrogatePoints> impl;
};

namespace {
thread_local std::string g_setup_error;

template <typename F>
int guarded(std::string* err, F&& f) {
  try {
    f();
    if (err) err->clear();
    return HOM_OK;
  } catch (const hom::Error& e) {
    if (err) *err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (err) *err = "host allocation failed";
    return HOM_E_OOM;
  } catch (const std::exception& e) {
    if (err) *err = e.what();
    return HOM_E_DEVICE;
  }
}

int worst(const hom_result* r, int n) {
  int code = HOM_OK;
  for (int i = 0; i < n; ++i)
    if (r[i].status != HOM_OK && (code == HOM_OK || r[i].status == HOM_E_NAN)) code = r[i].status;
  return code;
}

int stats(const hom::BatchImpl* b, const char** names, int64_t* launches, double* ms, int32_t cap) {
  if (!b) return HOM_E_ARG;
  const hom::Profiler& p = b->profiler();
  const int n = cap < 2 * hom::K_COUNT ? cap : 2 * hom::K_COUNT;
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = hom::kKernelNames[i];
    if (launches) launches[i] = p.launches[i];
    if (ms) ms[i] = p.ms[i];
  }
  return n;
}
}  // namespace

namespace {
hom::DmnSchedule schedule_of(const hom_dmn_train_opts* o) {
  hom::DmnSchedule s;
  if (o) {
    s.lr_max = o->lr_max;
    s.lr_min = o->lr_min;
    s.half_period = o->half_period;
    s.decay = o->decay;
    s.q = o->q;
    s.penalty = o->penalty;
  }
  if (!(s.lr_max > 0.0) || !(s.lr_min >= 0.0) || s.half_period < 1 || !(s.decay > 0.0) || !(s.q >= 1.0) ||
      !(s.penalty >= 0.0))
    hom::fail(HOM_E_ARG, "invalid training options");
  return s;
}
}  // namespace

namespace {
// the first network's scratch holds the per-network outputs of an inference
void grow_scratch(hom_mlp* a, size_t floats) {
  if (floats <= a->scratch_floats) return;
  if (a->scratch) HIPCHK(hipFree(a->scratch));
  a->scratch = nullptr;
  a->scratch_floats = 0;
  HIPCHK(hipMalloc((void**)&a->scratch, floats * 4));
  a->scratch_floats = floats;
}
}  // namespace

extern "C" {

void hom_default_options(hom_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->scheme = HOM_SCHEME_NEWTON_CG;
  o->precision = HOM_FP32;
  o->tol = 1e-6;
  o->thermal_tol = 0.0;
  o->use_graph = 1;
}

int hom_setup(const hom_grid* grid, const uint8_t* phases, const hom_law* laws, int32_t n_laws,
              const hom_options* opts, hom_ctx** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  hom_ctx* c = new (std::nothrow) hom_ctx();
  if (!c) return HOM_E_OOM;
  int rc = guarded(&g_setup_error, [&] {
    if (!grid || !phases || !laws || !opts) hom::fail(HOM_E_ARG, "null argument");
    const uint8_t* ph[1] = {phases};
    c->impl = hom::make_batch(1, grid, ph, laws, n_laws, *opts);
  });
  if (rc != HOM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return HOM_OK;
}

int hom_solve_increment(hom_ctx* c, const double macro_strain[6], const hom_macro_temp* temp, double dt,
                        hom_result* out) {
  if (!c || !c->impl || !macro_strain || !temp || !out) return HOM_E_ARG;
  hom_load L;
  std::memset(&L, 0, sizeof(L));
  std::memcpy(L.strain, macro_strain, sizeof(L.strain));
  L.temp = *temp;
  L.dt = dt;
  return hom_solve_load(c, &L, out);
}

int hom_solve_load(hom_ctx* c, const hom_load* load, hom_result* out) {
  if (!c || !c->impl || !load || !out) return HOM_E_ARG;
  int rc = guarded(&c->err, [&] { c->impl->solve(load, out); });
  if (rc != HOM_OK) return rc;
  rc = worst(out, 1);
  if (rc != HOM_OK) c->err = "increment did not converge (state not committed)";
  return rc;
}

size_t hom_state_size(const hom_ctx* c) { return (c && c->impl) ? c->impl->state_size() : 0; }

int hom_get_state(hom_ctx* c, void* buf, size_t bytes) {
  if (!c || !c->impl || !buf) return HOM_E_ARG;
  return guarded(&c->err, [&] {
    if (bytes != c->impl->state_size()) hom::fail(HOM_E_ARG, "state buffer size mismatch");
    c->impl->get_state(buf);
  });
}

int hom_set_state(hom_ctx* c, const void* buf, size_t bytes) {
  if (!c || !c->impl || !buf) return HOM_E_ARG;
  return guarded(&c->err, [&] {
    if (bytes != c->impl->state_size()) hom::fail(HOM_E_ARG, "state buffer size mismatch");
    c->impl->set_state(buf);
  });
}

int hom_get_field(hom_ctx* c, int32_t which, double* buf, size_t count) {
  if (!c || !c->impl || !buf) return HOM_E_ARG;
  return guarded(&c->err, [&] { c->impl->get_field(which, buf, count); });
}

int hom_kernel_stats(const hom_ctx* c, const char** names, int64_t* launches, double* ms, int32_t cap) {
  return stats(c ? c->impl.get() : nullptr, names, launches, ms, cap);
}

int hom_set_profiling(hom_ctx* c, int32_t on) {
  if (!c || !c->impl) return HOM_E_ARG;
  return guarded(&c->err, [&] { c->impl->set_profiling(on != 0); });
}

int hom_set_laws(hom_ctx* c, const hom_law* laws, int32_t n) {
  if (!c || !c->impl) return HOM_E_ARG;
  return guarded(&c->err, [&] { c->impl->set_laws(laws, n); });
}

int hom_batch_set_laws(hom_batch* b, const hom_law* laws, int32_t n) {
  if (!b || !b->impl) return HOM_E_ARG;
  return guarded(&b->err, [&] { b->impl->set_laws(laws, n); });
}

int hom_algorithmic_tangent(hom_ctx* c, int32_t what, hom_tangent* out) {
  if (!c || !c->impl || !out) return HOM_E_ARG;
  return guarded(&c->err, [&] { c->impl->tangent(what, out); });
}

size_t hom_device_bytes(const hom_ctx* c) { return (c && c->impl) ? c->impl->device_bytes() : 0; }

const char* hom_last_error(const hom_ctx* c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

void hom_destroy(hom_ctx* c) { delete c; }

int hom_batch_setup(int32_t n_prob, const hom_grid* grids, const uint8_t* const* phases, const hom_law* laws,
                    int32_t n_laws, const hom_options* opts, hom_batch** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  hom_batch* b = new (std::nothrow) hom_batch();
  if (!b) return HOM_E_OOM;
  int rc = guarded(&g_setup_error, [&] {
    if (!opts) hom::fail(HOM_E_ARG, "null options");
    b->impl = hom::make_batch(n_prob, grids, phases, laws, n_laws, *opts);
  });
  if (rc != HOM_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return HOM_OK;
}

int hom_batch_solve_increment(hom_batch* b, const double* strain, const hom_macro_temp* temp, const double* dt,
                              hom_result* out) {
  if (!b || !b->impl || !strain || !temp || !dt || !out) return HOM_E_ARG;
  return guarded(&b->err, [&] {
    std::vector<hom_load> loads(b->impl->problems());
    for (size_t i = 0; i < loads.size(); ++i) {
      std::memset(&loads[i], 0, sizeof(hom_load));
      std::memcpy(loads[i].strain, strain + 6 * i, sizeof(loads[i].strain));
      loads[i].temp = temp[i];
      loads[i].dt = dt[i];
    }
    b->impl->solve(loads.data(), out);
  });  // per-problem status is in out[i].status
}

int hom_batch_solve_load(hom_batch* b, const hom_load* loads, hom_result* out) {
  if (!b || !b->impl || !loads || !out) return HOM_E_ARG;
  return guarded(&b->err, [&] { b->impl->solve(loads, out); });
}

int hom_batch_kernel_stats(const hom_batch* b, const char** names, int64_t* launches, double* ms, int32_t cap) {
  return stats(b ? b->impl.get() : nullptr, names, launches, ms, cap);
}

int hom_batch_schedules(const hom_batch* b, int32_t* out, int32_t cap) {
  if (!b || !b->impl || !out || cap < 0) return HOM_E_ARG;
  return b->impl->schedules(out, cap);
}

int hom_schedules(const hom_ctx* c, int32_t* out, int32_t cap) {
  if (!c || !c->impl || !out || cap < 0) return HOM_E_ARG;
  return c->impl->schedules(out, cap);
}

int hom_batch_algorithmic_tangent(hom_batch* b, int32_t what, hom_tangent* out) {
  if (!b || !b->impl || !out) return HOM_E_ARG;
  return guarded(&b->err, [&] { b->impl->tangent(what, out); });
}

const char* hom_batch_last_error(const hom_batch* b) { return b ? b->err.c_str() : g_setup_error.c_str(); }

void hom_batch_destroy(hom_batch* b) { delete b; }


void hom_dmn_default_train_opts(hom_dmn_train_opts* o) {
  if (!o) return;
  const hom::DmnSchedule s;
  o->lr_max = s.lr_max;
  o->lr_min = s.lr_min;
  o->half_period = s.half_period;
  o->decay = s.decay;
  o->q = s.q;
  o->penalty = s.penalty;
}

int hom_dmn_create(int32_t K, uint64_t seed, hom_dmn** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  hom_dmn* d = new (std::nothrow) hom_dmn();
  if (!d) return HOM_E_OOM;
  int rc = guarded(&g_setup_error, [&] { d->net = std::make_unique<hom::Dmn>(K, seed); });
  if (rc != HOM_OK) {
    delete d;
    return rc;
  }
  *out = d;
  return HOM_OK;
}

int hom_dmn_get_params(const hom_dmn* d, double* m, double* v) {
  if (!d || !d->net) return HOM_E_ARG;
  return guarded(nullptr, [&] { d->net->get(m, v); });
}

int hom_dmn_set_params(hom_dmn* d, const double* m, const double* v) {
  if (!d || !d->net) return HOM_E_ARG;
  return guarded(&d->err, [&] { d->net->set(m, v); });
}

int hom_dmn_homogenize(hom_dmn* d, int64_t n, const double* C1, const double* C2, double* C_out) {
  if (!d || !d->net) return HOM_E_ARG;
  return guarded(&d->err, [&] { d->net->homogenize(n, C1, C2, C_out); });
}

int hom_dmn_loss_grad(hom_dmn* d, int64_t n, const double* C1, const double* C2, const double* C_eff,
                      const hom_dmn_train_opts* opts, double* loss, double* gm, double* gv) {
  if (!d || !d->net) return HOM_E_ARG;
  return guarded(&d->err, [&] {
    const double J = d->net->loss_grad(n, C1, C2, C_eff, gm, gv, schedule_of(opts));
    if (loss) *loss = J;
  });
}

int hom_dmn_train(hom_dmn* d, int64_t n, const double* C1, const double* C2, const double* C_eff, int32_t epochs,
                  int32_t batch, uint64_t seed, const hom_dmn_train_opts* opts, double* epoch_loss) {
  if (!d || !d->net) return HOM_E_ARG;
  return guarded(&d->err, [&] { d->net->train(n, C1, C2, C_eff, epochs, batch, seed, epoch_loss, schedule_of(opts)); });
}

const char* hom_dmn_last_error(const hom_dmn* d) { return d ? d->err.c_str() : g_setup_error.c_str(); }

void hom_dmn_destroy(hom_dmn* d) { delete d; }

int hom_dmn_online_create(const hom_dmn* d, const hom_law laws[2], int32_t n_points, double tol, int32_t maxit,
                          hom_dmn_online** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  if (!d || !d->net) return HOM_E_ARG;
  hom_dmn_online* o = new (std::nothrow) hom_dmn_online();
  if (!o) return HOM_E_OOM;
  int rc = guarded(&g_setup_error, [&] { o->impl = hom::dmn_online_create(*d->net, laws, n_points, tol, maxit); });
  if (rc != HOM_OK) {
    delete o;
    return rc;
  }
  *out = o;
  return HOM_OK;
}

int hom_dmn_online_step(hom_dmn_online* o, const double* strain, const double* theta, const double* dt,
                        int32_t what, int32_t trial, hom_dmn_result* out) {
  if (!o || !o->impl || !strain || !theta || !dt || !out) return HOM_E_ARG;
  return guarded(&o->err, [&] { hom::dmn_online_step(o->impl, strain, theta, dt, what, trial, out); });
}

int hom_dmn_online_set_predictor(hom_dmn_online* o, int32_t on) {
  if (!o || !o->impl) return HOM_E_ARG;
  return guarded(&o->err, [&] { hom::dmn_online_set_predictor(o->impl, on); });
}

const char* hom_dmn_online_last_error(const hom_dmn_online* o) { return o ? o->err.c_str() : g_setup_error.c_str(); }

void hom_dmn_online_destroy(hom_dmn_online* o) { delete o; }

int hom_mlp_create(int32_t n_in, int32_t n_out, uint64_t seed, hom_mlp** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  hom_mlp* m = new (std::nothrow) hom_mlp();
  if (!m) return HOM_E_OOM;
  int rc = guarded(&g_setup_error, [&] { m->net = std::make_unique<hom::Mlp>(n_in, n_out, seed); });
  if (rc != HOM_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return HOM_OK;
}

size_t hom_mlp_param_count(const hom_mlp* m) { return (m && m->net) ? m->net->param_count() : 0; }

int hom_mlp_set_scaling(hom_mlp* m, const float* xm, const float* xs, const float* ym, const float* ys,
                        const float* lw) {
  if (!m || !m->net || !xm || !xs || !ym || !ys) return HOM_E_ARG;
  return guarded(&m->err, [&] { m->net->set_scaling(xm, xs, ym, ys, lw); });
}

int hom_mlp_set_skip(hom_mlp* m, const int32_t gates[3], const float* G, const float* c) {
  if (!m || !m->net || !gates || !G || !c) return HOM_E_ARG;
  return guarded(&m->err, [&] {
    const int g[3] = {gates[0], gates[1], gates[2]};
    m->net->set_skip(g, G, c);
  });
}

int hom_mlp_fit_skip(hom_mlp* m, const float* x, const float* y, int64_t n, const int32_t gates[3],
                     const float* lw, const float* rw) {
  if (!m || !m->net || !x || !y || !gates || n < 2) return HOM_E_ARG;
  return guarded(&m->err, [&] {
    const int g[3] = {gates[0], gates[1], gates[2]};
    std::vector<float> w(m->net->n_out, 1.f);
    if (lw) w.assign(lw, lw + m->net->n_out);
    m->net->fit_skip(x, y, n, g, w.data(), rw);
  });
}

int hom_mlp_get_params(const hom_mlp* m, float* host, size_t count) {
  if (!m || !m->net || !host || count != m->net->param_count()) return HOM_E_ARG;
  return guarded(nullptr, [&] { m->net->get_params(host); });
}

int hom_mlp_set_params(hom_mlp* m, const float* host, size_t count) {
  if (!m || !m->net || !host || count != m->net->param_count()) return HOM_E_ARG;
  return guarded(&m->err, [&] { m->net->set_params(host); });
}

int hom_mlp_train(hom_mlp* m, const float* x, const float* y, int64_t n, int32_t epochs, int32_t batch, double lr,
                  uint64_t seed, const float* row_weight, float* epoch_loss) {
  if (!m || !m->net || !x || !y || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0)) return HOM_E_ARG;
  if (row_weight)
    for (int64_t r = 0; r < n; ++r)
      if (!(row_weight[r] >= 0.f) || !std::isfinite(row_weight[r])) return HOM_E_ARG;
  return guarded(&m->err, [&] { m->net->train(x, y, n, epochs, batch, lr, seed, row_weight, epoch_loss); });
}

int hom_mlp_forward(hom_mlp* m, const float* x_dev, float* y_dev, int64_t n, int32_t precise, void* stream) {
  if (!m || !m->net || n < 0) return HOM_E_ARG;
  if (n == 0) return HOM_OK;  // nothing to do (the arrays may be empty)
  if (!x_dev || !y_dev) return HOM_E_ARG;
  return guarded(&m->err, [&] {
    m->net->forward(x_dev, y_dev, n, precise != 0, false, static_cast<hipStream_t>(stream));
    hom::hip_check(hipGetLastError(), "mlp forward launch");
  });
}

int hom_mlp_loss_grad(hom_mlp* m, const float* x, const float* y, int64_t n, int32_t precise, double* loss,
                      float* grad) {
  if (!m || !m->net || !x || !y || n < 1) return HOM_E_ARG;
  return guarded(&m->err, [&] {
    hom::Mlp& net = *m->net;
    std::vector<float> tn((size_t)n * hom::MLP_OUT);
    net.normalized_targets(x, y, n, tn.data());
    float *dx = nullptr, *dt = nullptr;
    HIPCHK(hipMalloc((void**)&dx, n * net.n_in * 4));
    HIPCHK(hipMalloc((void**)&dt, tn.size() * 4));
    struct G {
      float *a, *b;
      ~G() {
        (void)hipFree(a);
        (void)hipFree(b);
      }
    } g{dx, dt};
    HIPCHK(hipMemcpy(dx, x, n * net.n_in * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dt, tn.data(), tn.size() * 4, hipMemcpyHostToDevice));
    const double L = net.loss_grad(dx, dt, n, precise != 0, nullptr);
    hom::hip_check(hipDeviceSynchronize(), "mlp gradient");
    if (loss) *loss = L;
    if (grad) net.get_grads(grad);
  });
}


int hom_mlp_ensemble_infer(hom_mlp* const* nets, int32_t count, const float* x_dev, float* y_dev, float* spread_dev,
                           uint8_t* accept_dev, int64_t n, double threshold, double floor_scale, void* stream) {
  if (!nets || count < 2 || count > HOM_ENSEMBLE_MAX_NETS || n < 0) return HOM_E_ARG;
  for (int m = 0; m < count; ++m)
    if (!nets[m] || !nets[m]->net) return HOM_E_ARG;
  if (n == 0) return HOM_OK;  // nothing to do (the arrays may be empty)
  if (!x_dev || !y_dev || !spread_dev || !accept_dev) return HOM_E_ARG;
  hom_mlp* a = nets[0];
  return guarded(&a->err, [&] {
    const hom::Mlp* nv[HOM_ENSEMBLE_MAX_NETS];
    for (int m = 0; m < count; ++m) {
      nv[m] = nets[m]->net.get();
      if (nv[m]->n_in != nv[0]->n_in || nv[m]->n_out != nv[0]->n_out) hom::fail(HOM_E_ARG, "network shapes differ");
    }
    grow_scratch(a, (size_t)n * count * nv[0]->n_out);
    hom::ensemble_accept(nv, count, x_dev, y_dev, a->scratch, spread_dev, accept_dev, n, (float)threshold,
                            (float)floor_scale, static_cast<hipStream_t>(stream));
    hom::hip_check(hipGetLastError(), "ensemble launch");
  });
}

int hom_mlp_ensemble_infer_static(hom_mlp* const* nets, int32_t count, const float* x_dev, float* y_dev,
                                  float* spread_dev, uint8_t* accept_dev, int64_t n, double threshold,
                                  double floor_scale, void* stream) {
  if (!nets || count < 2 || count > HOM_ENSEMBLE_MAX_NETS || n < 0) return HOM_E_ARG;
  for (int m = 0; m < count; ++m)
    if (!nets[m] || !nets[m]->net) return HOM_E_ARG;
  if (n == 0) return HOM_OK;  // nothing to do (the arrays may be empty)
  if (!x_dev || !y_dev || !spread_dev || !accept_dev) return HOM_E_ARG;
  hom_mlp* a = nets[0];
  return guarded(&a->err, [&] {
    const hom::Mlp* nv[HOM_ENSEMBLE_MAX_NETS];
    for (int m = 0; m < count; ++m) {
      nv[m] = nets[m]->net.get();
      if (nv[m]->n_in != nv[0]->n_in || nv[m]->n_out != nv[0]->n_out) hom::fail(HOM_E_ARG, "network shapes differ");
    }
    hom::ensemble_accept_static(nv, count, x_dev, y_dev, spread_dev, accept_dev, n, (float)threshold,
                                (float)floor_scale, static_cast<hipStream_t>(stream));
    hom::hip_check(hipGetLastError(), "ensemble launch");
  });
}

const char* hom_mlp_last_error(const hom_mlp* m) { return m ? m->err.c_str() : g_setup_error.c_str(); }

void hom_mlp_destroy(hom_mlp* m) { delete m; }

void hom_surrogate_default_config(hom_surrogate_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->n_nets = 8;
  c->epochs = 100;
  c->batch = 4096;
  c->lr = 8e-3;
  c->seed = 0;
  c->target = 1e-3;
  c->quantile = 1.0;
  c->holdout = 0.1;
  c->floor_scale = 0.01;
  c->theta_init = 293.15;
  c->chunk = 1024;
  c->max_resident = 2048;
}

int hom_surrogate_create(const hom_grid* grid, const uint8_t* phases, const hom_law* laws, int32_t n_laws,
                         const hom_options* opts, const hom_surrogate_config* cfg, hom_surrogate** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  if (!grid || !phases || !laws || !opts || !cfg) return HOM_E_ARG;
  hom_surrogate* s = new (std::nothrow) hom_surrogate();
  if (!s) return HOM_E_OOM;
  const int rc = guarded(&g_setup_error, [&] {
    s->impl.reset(new hom::Surrogate(*grid, phases, laws, n_laws, *opts, *cfg));
  });
  if (rc != HOM_OK) {
    delete s;
    return rc;
  }
  *out = s;
  return HOM_OK;
}

int hom_surrogate_solve_histories(hom_surrogate* s, int32_t count, int32_t steps, const double* strain,
                                  const double* theta, const double* grad, const double* dt, hom_result* out,
                                  double* seconds) {
  if (!s || !s->impl) return HOM_E_ARG;
  return guarded(&s->impl->err, [&] {
    s->impl->solve_histories(count, steps, strain, theta, grad, dt, out, seconds);
  });
}

int hom_surrogate_features(int32_t count, int32_t steps, const double* strain, const double* theta,
                           const double* grad, const double* dt, const hom_result* fft, double theta_init, float* X,
                           float* Y, double* denom) {
  return guarded(&g_setup_error, [&] {
    hom::sur_history_rows(count, steps, strain, theta, grad, dt, fft, theta_init, X, Y, denom);
  });
}

int hom_surrogate_train(hom_surrogate* s, int32_t count, int32_t steps, const double* strain, const double* theta,
                        const double* grad, const double* dt, const hom_result* fft, hom_surrogate_report* rep) {
  if (!s || !s->impl) return HOM_E_ARG;
  return guarded(&s->impl->err, [&] { s->impl->train(count, steps, strain, theta, grad, dt, fft, rep); });
}

int hom_surrogate_calibrate(hom_surrogate* s, int32_t count, int32_t steps, const double* strain,
                            const double* theta, const double* grad, const double* dt, const hom_result* fft,
                            double target, double quantile, hom_surrogate_report* rep) {
  if (!s || !s->impl) return HOM_E_ARG;
  return guarded(&s->impl->err, [&] {
    if (rep) std::memset(rep, 0, sizeof(*rep));
    s->impl->calibrate(count, steps, strain, theta, grad, dt, fft, target, quantile, rep);
  });
}

int hom_surrogate_set_threshold(hom_surrogate* s, double threshold) {
  if (!s || !s->impl || std::isnan(threshold)) return HOM_E_ARG;
  s->impl->threshold = threshold;
  return HOM_OK;
}

double hom_surrogate_threshold(const hom_surrogate* s) {
  return s && s->impl ? s->impl->threshold : std::numeric_limits<double>::quiet_NaN();
}

int hom_surrogate_infer(hom_surrogate* s, const float* x_dev, float* y_dev, uint8_t* accepted_dev, int64_t n,
                        void* stream) {
  if (!s || !s->impl || n < 0) return HOM_E_ARG;
  if (n == 0) return HOM_OK;  // nothing to do (the arrays may be empty)
  if (!x_dev || !y_dev || !accepted_dev) return HOM_E_ARG;
  return guarded(&s->impl->err, [&] {
    s->impl->infer_device(x_dev, y_dev, accepted_dev, n, static_cast<hipStream_t>(stream));
  });
}

int hom_surrogate_points_create(hom_surrogate* s, int32_t n_points, hom_surrogate_points** out) {
  if (!out) return HOM_E_ARG;
  *out = nullptr;
  if (!s || !s->impl) return HOM_E_ARG;
  hom_surrogate_points* p = new (std::nothrow) hom_surrogate_points();
  if (!p) return HOM_E_OOM;
  const int rc = guarded(&s->impl->err, [&] { p->impl.reset(new hom::SurrogatePoints(s->impl.get(), n_points)); });
  if (rc != HOM_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return HOM_OK;
}

int hom_surrogate_points_step(hom_surrogate_points* p, const double* strain, const double* theta, const double* grad,
                              const double* dt, hom_result* out, uint8_t* accepted, hom_surrogate_step_info* info) {
  if (!p || !p->impl) return HOM_E_ARG;
  const int rc = guarded(&p->impl->err, [&] { p->impl->step_all(strain, theta, grad, dt, out, accepted, info); });
  return rc != HOM_OK ? rc : worst(out, p->impl->n);
}

const char* hom_surrogate_points_last_error(const hom_surrogate_points* p) {
  return p && p->impl ? p->impl->err.c_str() : g_setup_error.c_str();
}

void hom_surrogate_points_destroy(hom_surrogate_points* p) { delete p; }

const char* hom_surrogate_last_error(const hom_surrogate* s) {
  return s && s->impl ? s->impl->err.c_str() : g_setup_error.c_str();
}

void hom_surrogate_destroy(hom_surrogate* s) { delete s; }

int hom_apply_operator(const hom_grid* grid, int32_t ncomp, int32_t op, double p0, double p1, int32_t precision,
                       const double* in, double* out) {
  if (!grid || !in || !out) return HOM_E_ARG;
  return guarded(&g_setup_error, [&] { hom::apply_operator(*grid, ncomp, op, p0, p1, precision, in, out); });
}

int hom_apply_operator_schedule(const hom_grid* grid, int32_t ncomp, int32_t op, double p0, double p1,
                                int32_t precision, int32_t schedule, const double* in, double* out) {
  if (!grid || !in || !out) return HOM_E_ARG;
  return guarded(&g_setup_error,
                 [&] { hom::apply_operator(*grid, ncomp, op, p0, p1, precision, in, out, schedule); });
}

int hom_eval_law(const hom_law* law, int64_t count, const double* eps, const double* eps_n, const double* state,
                 double theta, double dt, int32_t commit, double* sigma, double* ab, double* nd, double* state_out,
                 double* dissipation, double* coupling) {
  if (!law || !eps || !sigma) return HOM_E_ARG;
  return guarded(&g_setup_error, [&] {
    hom::eval_law(*law, count, eps, eps_n, state, theta, dt, commit, sigma, ab, nd, state_out, dissipation,
                  coupling);
  });
}

}  // extern "C"
