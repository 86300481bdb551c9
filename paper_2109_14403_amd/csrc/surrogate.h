// Surrogate with FFT fallback: an ensemble of networks for one
// microstructure, the batched FFT solver that generates its data and answers
// where it is not trusted, and point sets rolled forward increment by
// increment (see surrogate.hip and include/hom.h).
#pragma once
#include <memory>
#include <vector>

#include "mlp.h"
#include "runtime.h"

namespace hom {

constexpr int SUR_IN = HOM_SURROGATE_IN;
constexpr int SUR_OUT = HOM_SURROGATE_OUT;

// What a point's next input row is built from: its committed macroscopic
// history (Mandel vectors)
struct SurSummary {
  double E_n[6], E_nm1[6], sig_n[6];
  double theta_n, diss_n, diss_int;
};

void sur_summary_init(SurSummary& s, double theta_init);
// the input row of an increment (strain in tensor components)
void sur_features(const SurSummary& s, const double* strain, double theta, const double* grad, double dt, float* x);
// step n -> n+1 with the increment's answer (sig in Mandel)
void sur_commit(SurSummary& s, const double* strain, double theta, double dt, const double* sig, double diss);
// rows of whole histories whose summaries come from their FFT answers
void sur_history_rows(int count, int steps, const double* strain, const double* theta, const double* grad,
                      const double* dt, const hom_result* fft, double theta_init, float* X, float* Y, double* denom);

struct Surrogate {
  hom_grid grid{};
  std::vector<uint8_t> phases;
  std::vector<hom_law> laws;
  hom_options opts{};
  hom_surrogate_config cfg{};
  std::vector<std::unique_ptr<Mlp>> nets;
  double threshold = -1.0;  // rejects every row until trained, calibrated or set
  // range of the summary inputs (8 .. 28) over the training rows: a summary
  // rolled forward from the ensemble's own answers is clamped to it, so the
  // networks never see a summary outside the region they were trained on
  float sum_lo[SUR_IN], sum_hi[SUR_IN];
  bool have_range = false;
  void clamp_summary(float* x) const;
  std::string err;
  hipStream_t stream = nullptr;
  // device rows of host-side inference and the per-network outputs
  float *dx = nullptr, *dy = nullptr, *dys = nullptr, *dspread = nullptr;
  uint8_t* dacc = nullptr;
  long long cap_rows = 0;
  float* scratch = nullptr;  // per-network outputs of hom_surrogate_infer
  long long scratch_rows = 0;

  Surrogate(const hom_grid& g, const uint8_t* ph, const hom_law* lw, int nl, const hom_options& o,
            const hom_surrogate_config& c);
  ~Surrogate();
  Surrogate(const Surrogate&) = delete;
  Surrogate& operator=(const Surrogate&) = delete;

  // `count` fresh FFT cells of the microstructure
  std::unique_ptr<BatchImpl> new_cells(int count) const;
  void solve_histories(int count, int steps, const double* strain, const double* theta, const double* grad,
                       const double* dt, hom_result* out, double* seconds);
  // ensemble on host rows: y [n][10] (mean) and spread [n]
  void infer_host(const float* X, long long n, float* y, float* spread);
  void infer_device(const float* x, float* y, uint8_t* acc, long long n, hipStream_t s);
  void train(int count, int steps, const double* strain, const double* theta, const double* grad, const double* dt,
             const hom_result* fft, hom_surrogate_report* rep);
  void calibrate(int count, int steps, const double* strain, const double* theta, const double* grad,
                 const double* dt, const hom_result* fft, double target, double quantile,
                 hom_surrogate_report* rep);

 private:
  void ensure_rows(long long n);
};

struct SurrogatePoints {
  Surrogate* sur;
  int n = 0;
  int step = 0;  // committed increments
  std::vector<SurSummary> summary;
  // macroscopic history of every point: per committed increment, [n][11]
  // (strain components 6, theta, grad 3, dt)
  std::vector<std::vector<double>> history;
  // points answered by the FFT solver for good: cell group and index in it
  struct Cells {
    std::unique_ptr<BatchImpl> cells;
    std::vector<int> points;
  };
  std::vector<Cells> resident;
  std::vector<int> mode;  // -1: ensemble; >= 0: index into `resident`
  int resident_count = 0;
  std::string err;

  SurrogatePoints(Surrogate* s, int count);
  void step_all(const double* strain, const double* theta, const double* grad, const double* dt, hom_result* out,
                uint8_t* accepted, hom_surrogate_step_info* info);
};

}  // namespace hom
