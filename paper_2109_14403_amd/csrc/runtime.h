// Solver runtime: device memory of a group of equally sized problems, the
// per-increment host preparation, the device-driven iteration loop (eager or
// replayed from captured hipGraphs), tile autotuning and kernel timing.
#pragma once
#include <array>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hom.h"
#include "common.h"
#include "pipe_launch.h"
#include "pointwise.h"

namespace hom {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPCHK(x) ::hom::hip_check((x), #x)

enum KernelKind {
  K_INIT = 0,
  K_EVAL,
  K_XFWD,
  K_YFWD,
  K_ZGREEN,
  K_YINV,
  K_XINV,
  K_REDA,
  K_HIST,
  K_COMMIT,
  K_REDOUT,
  K_COUNT
};
extern const char* const kKernelNames[2 * K_COUNT];

struct Profiler {
  bool on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  int offset = 0;  // K_COUNT for the conduction solve
  int64_t launches[2 * K_COUNT] = {};
  double ms[2 * K_COUNT] = {};
  void begin(int kind, hipStream_t s);
  void end(hipStream_t s);
  void collect();
  ~Profiler();

 private:
  int cur = -1;
  hipEvent_t ev0 = nullptr;
  hipEvent_t get();
};

// Host preparation of the per-increment scalars of one problem.
void fill_inc(ProbInc& in, const std::vector<hom_law>& laws, double theta, double dt);
void validate_laws(const hom_law* laws, int n);

class BatchImpl {
 public:
  virtual ~BatchImpl() = default;
  virtual void solve(const hom_load* loads, hom_result* out) = 0;  // one load per problem
  virtual size_t device_bytes() const = 0;
  virtual int problems() const = 0;
  virtual size_t state_size() const = 0;
  virtual void get_state(void* buf) = 0;
  virtual void set_state(const void* buf) = 0;
  virtual void get_field(int which, double* out, size_t count) = 0;
  virtual void tangent(int what, hom_tangent* out) = 0;  // out: one entry per problem
  virtual void set_laws(const hom_law* laws, int n) = 0;
  virtual const Profiler& profiler() const = 0;
  virtual void set_profiling(bool on) = 0;
  // per grid group: nx, ny, nz and the schedules of the y and z passes of the
  // mechanics and the conduction; returns the number of groups
  virtual int schedules(int32_t* out, int cap) const = 0;
  std::string err;
};

std::unique_ptr<BatchImpl> make_batch(int nprob, const hom_grid* grids, const uint8_t* const* phases,
                                      const hom_law* laws, int nlaws, const hom_options& opts);

// sched < 0: the default schedule (tile width 4, plan 0, else width 2)
void apply_operator(const hom_grid& g, int ncomp, int op, double p0, double p1, int precision, const double* in,
                    double* out, int sched = -1);
void eval_law(const hom_law& law, int64_t count, const double* eps, const double* eps_n, const double* state,
              double theta, double dt, int commit, double* sigma, double* ab, double* nd, double* state_out,
              double* diss, double* coup);

}  // namespace hom
