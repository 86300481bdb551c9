// Solver runtime (see runtime.h).
#include "runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>
#include <numeric>
#include <tuple>

namespace hom {

const char* const kKernelNames[2 * K_COUNT] = {
    "init",     "eval",   "xfwd",   "yfwd",       "zgreen",   "yinv",    "xinv",   "reduce_a", "history",
    "commit",   "reduce_out", "t.init", "t.eval",  "t.xfwd",   "t.yfwd",  "t.zgreen", "t.yinv", "t.xinv",
    "t.reduce_a", "t.history", "t.commit", "t.reduce_out"};

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HOM_E_OOM : HOM_E_DEVICE;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// profiler
// ---------------------------------------------------------------------------
hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}
void Profiler::begin(int kind, hipStream_t s) {
  if (!on) return;
  cur = kind + offset;
  ev0 = get();
  HIPCHK(hipEventRecord(ev0, s));
}
void Profiler::end(hipStream_t s) {
  if (!on) return;
  hipEvent_t e1 = get();
  HIPCHK(hipEventRecord(e1, s));
  pending.push_back({cur, {ev0, e1}});
}
void Profiler::collect() {
  for (auto& p : pending) {
    float t = 0.f;
    HIPCHK(hipEventSynchronize(p.second.second));
    HIPCHK(hipEventElapsedTime(&t, p.second.first, p.second.second));
    ms[p.first] += t;
    launches[p.first] += 1;
    pool.push_back(p.second.first);
    pool.push_back(p.second.second);
  }
  pending.clear();
}
Profiler::~Profiler() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// laws
// ---------------------------------------------------------------------------
void validate_laws(const hom_law* laws, int n) {
  if (n < 1 || n > HOM_MAX_LAWS) fail(HOM_E_ARG, "n_laws must be in [1, 8]");
  int npa = 0;
  for (int i = 0; i < n; ++i) {
    const hom_law& L = laws[i];
    auto bad = [&](const char* w) { fail(HOM_E_ARG, "law " + std::to_string(i) + ": " + w); };
    if (L.kind != HOM_LAW_THERMOELASTIC && L.kind != HOM_LAW_PA66) bad("unknown kind");
    if (!(L.E > 0.0) || !(L.nu > -1.0 && L.nu < 0.5)) bad("need E > 0 and -1 < nu < 0.5");
    if (!(L.kappa0 > 0.0) || !(L.c0 >= 0.0) || !(L.theta0 > 0.0)) bad("need kappa0 > 0, c0 >= 0, theta0 > 0");
    if (!std::isfinite(L.alpha0)) bad("alpha0 must be finite");
    if (L.kind == HOM_LAW_PA66) {
      ++npa;
      if (L.n_maxwell < 0 || L.n_maxwell > HOM_MAX_MAXWELL) bad("n_maxwell out of range");
      for (int j = 0; j < L.n_maxwell; ++j)
        if (!(L.E_i[j] >= 0.0) || !std::isfinite(L.log10_tau_i[j])) bad("invalid Maxwell branch");
      if (!(L.sigma_y0 > 0.0) || !(L.eta0 > 0.0) || !(L.m >= 1.0) || !(L.k_h >= 0.0)) bad("invalid plasticity");
      if (!(L.n_h > 0.0 && L.n_h <= 1.0)) bad("n_h must be in (0, 1]");
      if (!std::isfinite(L.C1) || !std::isfinite(L.C2) || !std::isfinite(L.beta1) || !std::isfinite(L.beta2))
        bad("invalid temperature parameters");
    }
  }
  if (npa > 1) fail(HOM_E_UNSUPPORTED, "at most one PA66 law per setup");
}

void fill_inc(ProbInc& in, const std::vector<hom_law>& laws, double theta, double dt) {
  std::memset(&in, 0, sizeof(in));
  in.theta = theta;
  in.dt = dt;
  in.pa_phase = -1;
  double lmin = 1e300, lmax = -1e300, mmin = 1e300, mmax = -1e300, kmin = 1e300, kmax = -1e300;
  for (size_t i = 0; i < laws.size(); ++i) {
    const hom_law& L = laws[i];
    PhaseInc& ph = in.ph[i];
    ph.kind = L.kind;
    ph.alpha0 = L.alpha0;
    ph.alpha_dth = L.alpha0 * (theta - L.theta0);
    ph.kappa = L.kappa0;
    double K, G;
    if (L.kind == HOM_LAW_THERMOELASTIC) {
      K = L.E / (3.0 * (1.0 - 2.0 * L.nu));
      G = L.E / (2.0 * (1.0 + L.nu));
    } else {
      in.pa_phase = (int)i;
      const double d = theta - L.theta_ref;
      const double a = std::pow(10.0, -L.C1 * d / (L.C2 + d));  // WLF shift
      const double g1 = std::exp(-L.beta1 * d);                   // softening Gamma(theta, beta1)
      const double g2 = std::exp(-L.beta2 * d);
      in.sY = g1 * L.sigma_y0;
      in.ccoef = dt * in.sY / (g2 * L.eta0);
      in.hk = g1 * L.k_h;
      in.nh = L.n_h;
      in.mexp = L.m;
      in.beta1 = L.beta1;
      in.alpha0 = L.alpha0;
      in.dth = theta - L.theta0;
      const double Kinf = L.E / (3.0 * (1.0 - 2.0 * L.nu));
      const double Ginf = L.E / (2.0 * (1.0 + L.nu));
      K = Kinf;
      G = Ginf;
      int nm = 0;
      for (int j = 0; j < L.n_maxwell; ++j) {
        const double Ej = L.E_i[j];
        if (!(Ej > 0.0)) continue;
        const double tau = std::pow(10.0, L.log10_tau_i[j]);
        const double Kj = Ej / (3.0 * (1.0 - 2.0 * L.nu));
        const double Gj = Ej / (2.0 * (1.0 + L.nu));
        const double tauK = tau * Ej / Kj, tauG = tau * Ej / Gj;
        const double rK = dt / (a * tauK), rG = dt / (a * tauG);
        in.K3i[nm] = 3.0 * Kj;
        in.G2i[nm] = 2.0 * Gj;
        in.rK[nm] = rK;
        in.rG[nm] = rG;
        in.fK[nm] = 1.0 / (1.0 + rK);
        in.fG[nm] = 1.0 / (1.0 + rG);
        K += Kj * in.fK[nm];
        G += Gj * in.fG[nm];
        ++nm;
      }
      in.nm = nm;
      in.Kinf3 = 3.0 * Kinf;
      in.Ginf2 = 2.0 * Ginf;
      in.Kbar3 = 3.0 * K;
      in.Gbar2 = 2.0 * G;
    }
    ph.K3 = 3.0 * K;
    ph.G2 = 2.0 * G;
    const double lam = K - 2.0 * G / 3.0;
    lmin = std::min(lmin, lam);
    lmax = std::max(lmax, lam);
    mmin = std::min(mmin, G);
    mmax = std::max(mmax, G);
    kmin = std::min(kmin, L.kappa0);
    kmax = std::max(kmax, L.kappa0);
  }
  in.lam0 = 0.5 * (lmin + lmax);
  in.mu0 = 0.5 * (mmin + mmax);
  in.kappa0 = 0.5 * (kmin + kmax);
}

static int pa66_nstate(const std::vector<hom_law>& laws) {
  for (auto& L : laws)
    if (L.kind == HOM_LAW_PA66) {
      int nm = 0;
      for (int j = 0; j < L.n_maxwell; ++j)
        if (L.E_i[j] > 0.0) ++nm;
      return 7 + 6 * nm;
    }
  return 0;
}

// ---------------------------------------------------------------------------
// twiddles
// ---------------------------------------------------------------------------
template <typename T>
static std::vector<c2<T>> twiddles(int n) {
  std::vector<c2<T>> w(n);
  for (int j = 0; j < n; ++j) {
    // exp(-2 pi i j / n) from an exactly reduced angle
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)n;
    w[j].x = (T)std::cos(ang);
    w[j].y = (T)std::sin(ang);
  }
  return w;
}

// ---------------------------------------------------------------------------
// dispatch of the pipeline launchers by transform length
// ---------------------------------------------------------------------------
#define HOM_DISPATCH(n, call)                 \
  switch (n) {                                \
    case 16: { constexpr int NN = 16; return call; }  \
    case 24: { constexpr int NN = 24; return call; }  \
    case 32: { constexpr int NN = 32; return call; }  \
    case 48: { constexpr int NN = 48; return call; }  \
    case 64: { constexpr int NN = 64; return call; }  \
    case 96: { constexpr int NN = 96; return call; }  \
    case 128: { constexpr int NN = 128; return call; } \
    case 256: { constexpr int NN = 256; return call; } \
  }                                           \
  fail(HOM_E_UNSUPPORTED, "unsupported transform length " + std::to_string(n));

template <typename T>
LaunchInfo run_xfwd(const Pipe<T>& a, hipStream_t s, bool dry) {
  HOM_DISPATCH(a.nx, (xfwd_launch<T, NN>(a, s, dry)))
}
template <typename T>
LaunchInfo run_xinv(const Pipe<T>& a, hipStream_t s, bool dry) {
  HOM_DISPATCH(a.nx, (xinv_launch<T, NN>(a, s, dry)))
}
template <typename T>
LaunchInfo run_ypass(const Pipe<T>& a, int sched, int inverse, hipStream_t s, bool dry) {
  HOM_DISPATCH(a.ny, (ypass_launch<T, NN>(a, sched, inverse, s, dry)))
}
template <typename T>
LaunchInfo run_zgreen(const Pipe<T>& a, int sched, hipStream_t s, bool dry) {
  HOM_DISPATCH(a.nz, (zgreen_launch<T, NN>(a, sched, s, dry)))
}

static bool launch_ok(const LaunchInfo& li) { return li.threads <= 1024 && li.lds <= 160 * 1024; }

// ---------------------------------------------------------------------------
// a group of problems sharing one grid
// ---------------------------------------------------------------------------
template <typename T>
struct Group {
  int nx = 0, ny = 0, nz = 0, P = 0;
  int ps[2] = {0, 0};      // spectral row pitch in kx entries [mech, thermal]
  size_t spec_count = 0;   // complex values of the spectral buffer
  long long nvox = 0;
  // stride of the per-voxel arrays, [prob][comp][vs]: nvox rounded up to 64
  // plus 1024, so that the components and problems a pass streams together
  // start at different offsets from the HBM channel boundaries (measured: 10 %
  // more bandwidth for an x-forward-like pass with 6-component fields)
  long long vs = 0;
  int nprob = 0;
  double len[3] = {1, 1, 1};
  int nstate = 0;
  std::vector<int> members;
  std::vector<void*> allocs;
  size_t bytes = 0;

  uint8_t* phase = nullptr;
  T *xm = nullptr, *xnm = nullptr, *f = nullptr, *r = nullptr, *p = nullptr;
  double* hist = nullptr;
  T *tab = nullptr, *tn = nullptr, *xt = nullptr;
  T* ft = nullptr;  // heat flux of the conduction solve (the stress field stays in f)
  c2<T>* spec = nullptr;
  double* state = nullptr;
  Ctl *ctl_m = nullptr, *ctl_t = nullptr;
  ProbInc* inc_d = nullptr;
  ProbInc* inc_h = nullptr;
  Ctl* ctl_h = nullptr;
  double* part = nullptr;
  int maxblk = 0;
  double* part2 = nullptr;  // first-stage sums of a reduction over many blocks [prob][NPART][nout]
  c2<T>* tw[3] = {nullptr, nullptr, nullptr};
  // schedules of the y and z passes, [mech, thermal]: tile width + 16 x plan
  // variant (pipe_launch.h)
  int txy[2] = {schedule(4, 0), schedule(4, 0)}, txz[2] = {schedule(4, 0), schedule(4, 0)};
  int pt_bpp = 1;
  int cm_bpp = 1;  // blocks per problem of the once-per-increment history sums
  // internal variables and increment slots of the PA66 voxels only, compacted
  // in voxel order: stride ss (the most PA66 voxels of one problem), the PA66
  // voxels before every 64-voxel chunk and the count of every problem
  long long ss = 0;
  int* cbase = nullptr;
  int* npa_d = nullptr;
  std::vector<int> npa;
  int xfblocks = 1, xiblocks = 1;  // x-forward / x-inverse work-groups per problem
  // captured chunks: [0] mechanics, [1] conduction, [2] linearized mechanics
  // (tangent strain columns), [3] linearized mechanics with a source (tangent
  // temperature column)
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  int graph_k[4] = {0, 0, 0, 0};
  // effective algorithmic tangents: per-voxel partials kept at each commit
  // (set up with the tangent option), the stress field saved across the
  // linearized solves, and whether the last increment can be linearized
  T *dsdt = nullptr, *dDde = nullptr, *dDdt = nullptr, *fsave = nullptr;
  // predictor option: the strain change of each problem's last committed
  // increment (field and mean), and whether it belongs to the current state
  T* dx = nullptr;
  std::vector<std::array<double, 6>> dEp;
  std::vector<char> pred_ok;
  // ... and the solutions of the last tangent call, one field per column,
  // which start the next call's linearized solves
  T* tcol = nullptr;
  bool tcol_ok[7] = {false, false, false, false, false, false, false};
  ProbInc* inc_pm_d = nullptr;
  ProbInc* inc_pm_h = nullptr;
  bool tan_ok = false;
  std::vector<std::array<double, 6>> En;
  std::vector<std::array<double, 3>> Gp;
  std::vector<double> c0mean;
  std::vector<std::vector<long long>> phase_count;  // [problem][law]: voxels of each phase

  // Device arrays start at staggered offsets (a different multiple of 4 KiB
  // inside a 2 MiB window for each array of the group): the many arrays a
  // pass streams at once would otherwise advance through the HBM channels in
  // lockstep from equal, 2 MiB-aligned bases (measured: 8 % more bandwidth
  // for an x-forward-like pass over 5 arrays).
  template <typename U>
  U* dalloc(size_t count) {
    const size_t off = count * sizeof(U) >= (1u << 20) ? (allocs.size() * 69 * 4096) % (2u << 20) : 0;
    void* ptr = nullptr;
    HIPCHK(hipMalloc(&ptr, count * sizeof(U) + off + 256));
    allocs.push_back(ptr);
    bytes += count * sizeof(U);
    char* p = static_cast<char*>(ptr) + off;
    HIPCHK(hipMemset(p, 0, count * sizeof(U)));
    return reinterpret_cast<U*>(p);
  }

  // streams of this group's work (the batch's own, or a lane of its own that
  // lets groups of different grids run at the same time)
  hipStream_t stream = nullptr;

  ~Group() {
    for (int i = 0; i < 4; ++i)
      if (graph[i]) (void)hipGraphExecDestroy(graph[i]);
    for (void* ptr : allocs) (void)hipFree(ptr);
    if (inc_h) (void)hipHostFree(inc_h);
    if (inc_pm_h) (void)hipHostFree(inc_pm_h);
    if (ctl_h) (void)hipHostFree(ctl_h);
  }

  void alloc(bool with_state, bool partials = false, bool predictor = false) {
    P = nx / 2 + 1;
    nvox = (long long)nx * ny * nz;
    vs = (nvox + 63) / 64 * 64 + 1024;
    const long long nm = (long long)nprob * vs;
    phase = dalloc<uint8_t>(nm);
    xm = dalloc<T>(6 * nm);
    xnm = dalloc<T>(6 * nm);
    f = dalloc<T>(6 * nm);
    ft = dalloc<T>(3 * nm);
    r = dalloc<T>(6 * nm);
    p = dalloc<T>(6 * nm);
    tab = dalloc<T>(2 * nm);
    tn = dalloc<T>(6 * nm);
    xt = dalloc<T>(3 * nm);
    for (int phys = 0; phys < 2; ++phys) {
      // smallest kx multiple that makes a row a whole number of 128-byte lines
      const int row_bytes = (phys == 0 ? 6 : 3) * (int)sizeof(c2<T>);
      const int step = 128 / std::gcd(128, row_bytes);
      ps[phys] = (P + step - 1) / step * step;
    }
    spec_count = (size_t)nprob * nz * ny * std::max(ps[0] * 6, ps[1] * 3);
    spec = dalloc<c2<T>>(spec_count);
    if (with_state && nstate > 0) {
      const size_t ns = (size_t)nprob * std::max<long long>(ss, 1);
      state = dalloc<double>((size_t)nstate * ns);
      hist = dalloc<double>((size_t)HIST_SLOTS * ns);
      cbase = dalloc<int>((size_t)nprob * ((nvox + 63) / 64));
      npa_d = dalloc<int>(nprob);
    }
    ctl_m = dalloc<Ctl>(nprob);
    ctl_t = dalloc<Ctl>(nprob);
    inc_d = dalloc<ProbInc>(nprob);
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&inc_h), sizeof(ProbInc) * nprob));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&ctl_h), sizeof(Ctl) * nprob));
    std::memset(inc_h, 0, sizeof(ProbInc) * nprob);
    // blocks per problem of the pointwise kernels
    pt_bpp = (int)std::min<long long>((nvox + 255) / 256, std::max<long long>(1, 8192 / nprob));
    pt_bpp = std::max(pt_bpp, 1);
    // the history sums stream the branch strains of the compacted PA66 voxels
    // once per increment and write no partial sums: one voxel per thread
    // (many short work-groups) up to 65536 groups.
    cm_bpp = (int)std::min<long long>((nvox + 255) / 256, std::max<long long>(1, 65536 / nprob));
    cm_bpp = std::max(cm_bpp, pt_bpp);
    const int nlf = x_lines(nx, sizeof(T) == 8, true), nli = x_lines(nx, sizeof(T) == 8, false);
    xfblocks = (ny * nz + nlf - 1) / nlf;
    xiblocks = (ny * nz + nli - 1) / nli;
    maxblk = std::max(pt_bpp, std::max(xfblocks, xiblocks));
    // the commit of the internal variables: one partial a block of 256 voxels
    if (with_state && nstate > 0) maxblk = std::max(maxblk, commit_voxel_blocks(nvox));
    part = dalloc<double>((size_t)nprob * maxblk * NPART);
    part2 = dalloc<double>((size_t)nprob * ((maxblk + RED_CHUNK - 1) / RED_CHUNK) * NPART);
    for (int d = 0; d < 3; ++d) {
      const int n = d == 0 ? nx : (d == 1 ? ny : nz);
      auto w = twiddles<T>(n);
      tw[d] = dalloc<c2<T>>(n);
      HIPCHK(hipMemcpy(tw[d], w.data(), n * sizeof(c2<T>), hipMemcpyHostToDevice));
    }
    En.assign(nprob, {0, 0, 0, 0, 0, 0});
    Gp.assign(nprob, {0, 0, 0});
    dEp.assign(nprob, {0, 0, 0, 0, 0, 0});
    pred_ok.assign(nprob, 0);
    if (predictor) dx = dalloc<T>(6 * nm);
    if (partials) {
      dsdt = dalloc<T>(6 * nm);
      dDde = dalloc<T>(6 * nm);
      dDdt = dalloc<T>(nm);
      inc_pm_d = dalloc<ProbInc>(2 * nprob);
      HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&inc_pm_h), sizeof(ProbInc) * 2 * nprob));
      std::memset(inc_pm_h, 0, sizeof(ProbInc) * 2 * nprob);
    }
  }

  Pipe<T> pipe(int phys, int green) const {
    Pipe<T> a;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.P = P;
    a.PS = ps[phys];
    a.nvox = nvox;
    a.vs = vs;
    a.nprob = nprob;
    a.C = phys == 0 ? 6 : 3;
    a.phase = phase;
    a.x = phys == 0 ? xm : xt;
    a.f = phys == 0 ? f : ft;
    a.r = r;
    a.p = p;
    a.tab = tab;
    a.tn = tn;
    a.spec = spec;
    a.ctl = phys == 0 ? ctl_m : ctl_t;
    a.inc = inc_d;
    a.part = part;
    a.maxblk = maxblk;
    a.twx = tw[0];
    a.twy = tw[1];
    a.twz = tw[2];
    for (int d = 0; d < 3; ++d) {
      a.len[d] = len[d];
      a.ilen[d] = 1.0 / len[d];
    }
    a.green = green;
    a.alpha_blocks = 0;
    return a;
  }

  Pt<T> pt(int phys) const {
    Pt<T> a;
    a.nvox = nvox;
    a.vs = vs;
    a.nprob = nprob;
    a.bpp = pt_bpp;
    a.phase = phase;
    a.x = phys == 0 ? xm : xt;
    a.xn = xnm;
    a.f = phys == 0 ? f : ft;
    a.r = r;
    a.p = p;
    a.tab = tab;
    a.tn = tn;
    a.state = state;
    a.nstate = nstate;
    a.hist = hist;
    a.cbase = cbase;
    a.npa = npa_d;
    a.ss = ss;
    a.ctl = phys == 0 ? ctl_m : ctl_t;
    a.inc = inc_d;
    a.part = part;
    a.maxblk = maxblk;
    a.pv_diss = nullptr;
    a.pv_coup = nullptr;
    a.dsdt = dsdt;
    a.dDde = dDde;
    a.dDdt = dDdt;
    a.inc_pm = inc_pm_d;
    a.s0 = nullptr;
    a.commit = 1;
    a.dp_known = 0;
    a.dx = dx;
    a.x0 = nullptr;
    return a;
  }
};

// ---------------------------------------------------------------------------
// batch of groups
// ---------------------------------------------------------------------------
template <typename T>
class BatchT : public BatchImpl {
 public:
  std::vector<std::unique_ptr<Group<T>>> groups;
  std::vector<std::pair<int, int>> where;
  std::vector<hom_law> laws;
  hom_options opts;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Profiler prof;
  bool linear_mech = true;
  int device = 0;
  // lanes created for groups after the first (library-owned streams only)
  std::vector<hipStream_t> lane_streams;

  ~BatchT() override {
    groups.clear();
    for (hipStream_t q : lane_streams) (void)hipStreamDestroy(q);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  const Profiler& profiler() const override { return prof; }

  void set_profiling(bool on) override {
    prof.collect();
    prof.on = on;
    for (int k = 0; k < 2 * K_COUNT; ++k) {
      prof.launches[k] = 0;
      prof.ms[k] = 0.0;
    }
  }

  int problems() const override { return (int)where.size(); }

  int schedules(int32_t* out, int cap) const override {
    int n = 0;
    for (auto& gp : groups) {
      if (n >= cap) break;
      const auto& G = *gp;
      const int32_t row[7] = {G.nx, G.ny, G.nz, G.txy[0], G.txz[0], G.txy[1], G.txz[1]};
      std::memcpy(out + 7 * n, row, sizeof(row));
      ++n;
    }
    return (int)groups.size();
  }

  size_t device_bytes() const override {
    size_t b = 0;
    for (auto& g : groups) b += g->bytes;
    return b;
  }

  void init(int nprob, const hom_grid* grids, const uint8_t* const* phases, const hom_law* lw, int nlaws,
            const hom_options& o) {
    opts = o;
    laws.assign(lw, lw + nlaws);
    for (auto& L : laws)
      if (L.kind == HOM_LAW_PA66) linear_mech = false;
    prof.on = o.profile != 0;
    if (o.stream) {
      stream = static_cast<hipStream_t>(o.stream);
    } else {
      HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      own_stream = true;
    }
    // group problems by grid
    std::map<std::tuple<int, int, int, double, double, double>, int> key;
    where.resize(nprob);
    for (int i = 0; i < nprob; ++i) {
      const hom_grid& g = grids[i];
      for (int d = 0; d < 3; ++d) {
        if (!supported_n(g.n[d]))
          fail(HOM_E_UNSUPPORTED, "grid size " + std::to_string(g.n[d]) +
                                      " not supported (16, 24, 32, 48, 64, 96, 128, 256)");
        if (!(g.len[d] > 0.0)) fail(HOM_E_ARG, "cell lengths must be positive");
      }
      auto k = std::make_tuple(g.n[0], g.n[1], g.n[2], g.len[0], g.len[1], g.len[2]);
      auto it = key.find(k);
      int gi;
      if (it == key.end()) {
        gi = (int)groups.size();
        key[k] = gi;
        groups.emplace_back(new Group<T>());
        auto& G = *groups.back();
        G.nx = g.n[0];
        G.ny = g.n[1];
        G.nz = g.n[2];
        for (int d = 0; d < 3; ++d) G.len[d] = g.len[d];
      } else {
        gi = it->second;
      }
      where[i] = {gi, (int)groups[gi]->members.size()};
      groups[gi]->members.push_back(i);
    }
    HIPCHK(hipGetDevice(&device));
    // group 0 runs on the batch's streams; with library-owned streams every
    // further group gets a lane of its own (default priority, like all others)
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      Group<T>& G = *groups[gi];
      if (gi == 0 || !own_stream) {
        G.stream = stream;
        continue;
      }
      HIPCHK(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
      lane_streams.push_back(G.stream);
    }
    const int nst = pa66_nstate(laws);
    int pa = -1;  // phase id of the PA66 law
    for (size_t l = 0; l < laws.size(); ++l)
      if (laws[l].kind == HOM_LAW_PA66) pa = (int)l;
    for (auto& gp : groups) {
      auto& G = *gp;
      G.nprob = (int)G.members.size();
      G.nstate = nst;
      const long long nv = (long long)G.nx * G.ny * G.nz;
      std::vector<uint8_t> buf((size_t)G.nprob * nv);
      const long long nch = (nv + 63) / 64;
      std::vector<int> cbase(nst > 0 ? (size_t)G.nprob * nch : 0);
      G.c0mean.assign(G.nprob, 0.0);
      G.npa.assign(G.nprob, 0);
      for (int j = 0; j < G.nprob; ++j) {
        const uint8_t* src = phases[G.members[j]];
        if (!src) fail(HOM_E_ARG, "null phase array");
        std::vector<long long> cnt(256, 0);
        for (long long v = 0; v < nv; ++v) {
          if (src[v] >= laws.size()) fail(HOM_E_ARG, "phase id " + std::to_string(src[v]) + " has no law");
          ++cnt[src[v]];
        }
        G.phase_count.emplace_back(cnt.begin(), cnt.begin() + laws.size());
        double c0 = 0.0;
        for (size_t l = 0; l < laws.size(); ++l) c0 += laws[l].c0 * (double)cnt[l] / (double)nv;
        G.c0mean[j] = c0;
        std::memcpy(buf.data() + (size_t)j * nv, src, nv);
        if (nst > 0) {
          int q = 0;
          for (long long v = 0; v < nv; ++v) {
            if ((v & 63) == 0) cbase[(size_t)j * nch + (v >> 6)] = q;
            if ((int)src[v] == pa) ++q;
          }
          G.npa[j] = q;
          G.ss = std::max<long long>(G.ss, q);
        }
      }
      // every component array of state and hist starts on a 256-byte boundary:
      // a wave's 512-byte accesses then touch 4 cache lines, not 5
      G.ss = (G.ss + 31) / 32 * 32;
      G.alloc(nst > 0, opts.tangent != 0, opts.predictor != 0);
      for (int j = 0; j < G.nprob; ++j)  // the phase array has the padded voxel stride too
        HIPCHK(hipMemcpy(G.phase + (size_t)j * G.vs, buf.data() + (size_t)j * nv, nv, hipMemcpyHostToDevice));
      if (G.state) {
        HIPCHK(hipMemcpy(G.cbase, cbase.data(), cbase.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(G.npa_d, G.npa.data(), G.nprob * sizeof(int), hipMemcpyHostToDevice));
      }
      if (opts.autotune) autotune(G);
    }
    HIPCHK(hipDeviceSynchronize());
  }

  // time the y / z schedules (tile width and FFT plan) on this group's data
  // and keep the fastest
  void autotune(Group<T>& G) {
    hipStream_t stream = G.stream;  // this group's lane
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::vector<Ctl> c(G.nprob);
    for (auto& x : c) {
      std::memset(&x, 0, sizeof(Ctl));
      x.mode = M_EVAL;
    }
    for (int phys = 0; phys < 2; ++phys) {
      Ctl* ctl = phys == 0 ? G.ctl_m : G.ctl_t;
      HIPCHK(hipMemcpy(ctl, c.data(), sizeof(Ctl) * G.nprob, hipMemcpyHostToDevice));
      Pipe<T> a = G.pipe(phys, phys == 0 ? G_PROJ : G_GRADPROJ);
      for (int pass = 0; pass < 2; ++pass) {
        auto run = [&](int sc) { pass == 0 ? run_ypass<T>(a, sc, 0, stream) : run_zgreen<T>(a, sc, stream); };
        std::vector<int> cand;
        for (int sc : kScheduleChoices) {
          LaunchInfo li = pass == 0 ? run_ypass<T>(a, sc, 0, stream, true) : run_zgreen<T>(a, sc, stream, true);
          if (!launch_ok(li)) continue;
          cand.push_back(sc);
          for (int w = 0; w < 2; ++w) run(sc);
        }
        // the candidates take turns over several rounds (in alternating
        // order, so clock ramps and neighbours favour none), each keeping its
        // fastest round: one noisy timing does not decide the schedule
        std::vector<float> best(cand.size(), 1e30f);
        for (int round = 0; round < 5; ++round)
          for (size_t j = 0; j < cand.size(); ++j) {
            const size_t i = (round & 1) ? cand.size() - 1 - j : j;
            HIPCHK(hipEventRecord(e0, stream));
            for (int w = 0; w < 3; ++w) run(cand[i]);
            HIPCHK(hipEventRecord(e1, stream));
            HIPCHK(hipEventSynchronize(e1));
            float t;
            HIPCHK(hipEventElapsedTime(&t, e0, e1));
            best[i] = std::min(best[i], t);
          }
        int bt = schedule(4, 0);
        float bmin = 1e30f;
        for (size_t i = 0; i < cand.size(); ++i)
          if (best[i] < bmin) {
            bmin = best[i];
            bt = cand[i];
          }
        (pass == 0 ? G.txy : G.txz)[phys] = bt;
      }
      std::memset(c.data(), 0, sizeof(Ctl) * G.nprob);
      HIPCHK(hipMemcpy(ctl, c.data(), sizeof(Ctl) * G.nprob, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemset(G.spec, 0, sizeof(c2<T>) * G.spec_count));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }

  void check_tiles(Group<T>& G, int phys) {
    hipStream_t stream = G.stream;  // this group's lane
    Pipe<T> a = G.pipe(phys, 0);
    for (int pass = 0; pass < 2; ++pass) {
      int& sc = (pass == 0 ? G.txy : G.txz)[phys];
      LaunchInfo li = pass == 0 ? run_ypass<T>(a, sc, 0, stream, true) : run_zgreen<T>(a, sc, stream, true);
      if (!launch_ok(li)) sc = schedule(2, 0);
      li = pass == 0 ? run_ypass<T>(a, sc, 0, stream, true) : run_zgreen<T>(a, sc, stream, true);
      if (!launch_ok(li)) fail(HOM_E_UNSUPPORTED, "no valid tile for this grid");
    }
    LaunchInfo lx = run_xfwd<T>(a, stream, true);
    LaunchInfo li = run_xinv<T>(a, stream, true);
    if (!launch_ok(lx) || !launch_ok(li)) fail(HOM_E_UNSUPPORTED, "x-pass does not fit the work-group limits");
  }

  Limits limits(int phys) const {
    Limits lim;
    const bool basic = opts.scheme == HOM_SCHEME_BASIC;
    lim.tol = phys == 0 ? opts.tol : (opts.thermal_tol > 0 ? opts.thermal_tol : opts.tol);
    lim.max_newton = opts.max_iter > 0 ? opts.max_iter : (basic ? 5000 : 40);
    lim.max_krylov = opts.max_krylov > 0 ? opts.max_krylov : 500;
    lim.linear = (phys == 1 || linear_mech) ? 1 : 0;
    return lim;
  }

  // One solver iteration. variant: 0 mechanics, 1 conduction, 2 linearized
  // mechanics (sigma = C_algo x), 3 linearized mechanics with the source
  // d sigma / d theta.
  void iteration(Group<T>& G, int variant, bool basic) {
    hipStream_t stream = G.stream;  // this group's lane
    const int phys = variant == 1 ? 1 : 0;
    const bool rot = opts.discretization == HOM_DISC_ROTATED;
    const int green = phys == 0 ? (basic ? G_GAMMA0 : (rot ? G_PROJ_ROT : G_PROJ))
                                : (basic ? G_GAMMA_TH : (rot ? G_GRADPROJ_ROT : G_GRADPROJ));
    Pipe<T> a = G.pipe(phys, green);
    if (!basic) a.alpha_blocks = G.xfblocks;  // the z pass forms the CG step length
    Pt<T> q = G.pt(phys);
    const int C = phys == 0 ? 6 : 3;
    Limits lim = limits(phys);
    if (variant >= 2) lim.linear = 1;
    Ctl* ctl = phys == 0 ? G.ctl_m : G.ctl_t;
    prof.begin(K_EVAL, stream);
    if (variant >= 2) {
      q.s0 = variant == 3 ? G.dsdt : nullptr;
      launch_eval_linear<T>(q, stream);
    } else {
      launch_eval<T>(q, C, stream);
    }
    prof.end(stream);
    prof.begin(K_XFWD, stream);
    run_xfwd<T>(a, stream);
    prof.end(stream);
    prof.begin(K_YFWD, stream);
    run_ypass<T>(a, G.txy[phys], 0, stream);
    prof.end(stream);
    prof.begin(K_ZGREEN, stream);
    run_zgreen<T>(a, G.txz[phys], stream);
    prof.end(stream);
    prof.begin(K_YINV, stream);
    run_ypass<T>(a, G.txy[phys], 1, stream);
    prof.end(stream);
    prof.begin(K_XINV, stream);
    run_xinv<T>(a, stream);
    prof.end(stream);
    prof.begin(K_REDA, stream);
    launch_reduce_a(ctl, G.part, G.maxblk, G.xiblocks, G.nprob, lim, stream);
    prof.end(stream);
  }

  static long long iteration_cap(const Limits& lim, bool basic) {
    return basic ? (long long)lim.max_newton + 2 : (long long)(lim.max_newton + 1) * (lim.max_krylov + 2);
  }

  int chunk_size(const Group<T>& G) const {
    if (opts.chunk > 0) return opts.chunk;
    // large grids: four iterations per host check (each check is a host round
    // trip of ~1 % of an iteration; after convergence the rest of a chunk's
    // launches return at once); small ones: 16
    return (G.nvox * G.nprob >= (1LL << 22)) ? 4 : 16;
  }

  void run_chunk(Group<T>& G, int variant, bool basic, int k) {
    hipStream_t stream = G.stream;  // this group's lane
    const bool graph = opts.use_graph && !prof.on;
    if (!graph) {
      for (int i = 0; i < k; ++i) iteration(G, variant, basic);
      return;
    }
    if (!G.graph[variant] || G.graph_k[variant] != k) {
      if (G.graph[variant]) HIPCHK(hipGraphExecDestroy(G.graph[variant]));
      hipGraph_t gr;
      HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < k; ++i) iteration(G, variant, basic);
      HIPCHK(hipStreamEndCapture(stream, &gr));
      HIPCHK(hipGraphInstantiate(&G.graph[variant], gr, nullptr, nullptr, 0));
      HIPCHK(hipGraphDestroy(gr));
      G.graph_k[variant] = k;
    }
    HIPCHK(hipGraphLaunch(G.graph[variant], stream));
  }

  // Iterate until no problem of the group is in a pipeline mode (or the cap).
  void iterate(Group<T>& G, int variant, bool basic, long long cap) {
    hipStream_t stream = G.stream;  // this group's lane
    // timed per kernel (profiling): one iteration per check, so that no launch
    // follows convergence and every timed launch did work
    const int k = prof.on ? 1 : chunk_size(G);
    Ctl* ctl = variant == 1 ? G.ctl_t : G.ctl_m;
    long long done_its = 0;
    for (;;) {
      run_chunk(G, variant, basic, k);
      done_its += k;
      HIPCHK(hipMemcpyAsync(G.ctl_h, ctl, sizeof(Ctl) * G.nprob, hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      prof.collect();
      int active = 0;
      for (int j = 0; j < G.nprob; ++j) active += pipeline_mode_host(G.ctl_h[j].mode);
      if (!active || done_its > cap) break;
    }
  }

  // Mechanics of one increment up to convergence; restart keeps the current
  // strain field (a later staggered solve at a new temperature).
  void mech_iterate(Group<T>& G, bool restart) {
    hipStream_t stream = G.stream;  // this group's lane
    const bool basic = opts.scheme == HOM_SCHEME_BASIC;
    Pt<T> q = G.pt(0);
    check_tiles(G, 0);
    prof.offset = 0;
    prof.begin(K_INIT, stream);
    launch_init_mech<T>(q, opts.scheme, stream, restart ? 1 : 0);
    prof.end(stream);
    if (G.state) {
      Pt<T> qh = q;
      qh.bpp = G.cm_bpp;
      prof.begin(K_HIST, stream);
      launch_history<T>(qh, stream);
      prof.end(stream);
    }
    iterate(G, 0, basic, iteration_cap(limits(0), basic));
  }

  // Per-problem means of the first nk partial-sum quantities over nb blocks into
  // ctl.out; many blocks (one voxel per thread) are summed in two stages.
  static void reduce_out(Group<T>& G, Ctl* ctl, int nb, int nk, hipStream_t stream) {
    if (nb > 2 * RED_CHUNK) {
      const int nout = (nb + RED_CHUNK - 1) / RED_CHUNK;
      launch_reduce_stage(G.part, G.maxblk, nb, G.part2, nout, G.nprob, stream);
      launch_reduce_out(ctl, G.part2, nout, nout, G.nprob, nk, 1.0 / (double)G.nvox, stream);
    } else {
      launch_reduce_out(ctl, G.part, G.maxblk, nb, G.nprob, nk, 1.0 / (double)G.nvox, stream);
    }
  }

  // Effective sums of the converged mechanics into ctl.out (copied to ctl_h);
  // commit: also commit the increment of every converged problem; partials:
  // the point partials of the tangent option (before a commit: state n).
  void mech_finish(Group<T>& G, bool commit, bool partials) {
    hipStream_t stream = G.stream;  // this group's lane
    Pt<T> q = G.pt(0);
    q.commit = commit ? 1 : 0;
    // Newton-CG converges on a residual evaluation at the final strain
    q.dp_known = opts.scheme == HOM_SCHEME_NEWTON_CG ? 1 : 0;
    if (partials && G.dsdt) launch_partials<T>(q, stream);
    prof.begin(K_COMMIT, stream);
    const int nb = launch_commit<T>(q, 6, stream);
    prof.end(stream);
    prof.begin(K_REDOUT, stream);
    reduce_out(G, G.ctl_m, nb, MECH_SUMS, stream);
    prof.end(stream);
    HIPCHK(hipMemcpyAsync(G.ctl_h, G.ctl_m, sizeof(Ctl) * G.nprob, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    prof.collect();
  }

  void thermal_solve(Group<T>& G) {
    hipStream_t stream = G.stream;  // this group's lane
    const bool basic = opts.scheme == HOM_SCHEME_BASIC;
    Pt<T> q = G.pt(1);
    check_tiles(G, 1);
    prof.offset = K_COUNT;
    prof.begin(K_INIT, stream);
    launch_init_th<T>(q, opts.scheme, stream);
    prof.end(stream);
    iterate(G, 1, basic, iteration_cap(limits(1), basic));
    prof.begin(K_COMMIT, stream);
    const int nb = launch_commit<T>(q, 3, stream);
    prof.end(stream);
    prof.begin(K_REDOUT, stream);
    reduce_out(G, G.ctl_t, nb, 3, stream);
    prof.end(stream);
    HIPCHK(hipMemcpyAsync(G.ctl_h, G.ctl_t, sizeof(Ctl) * G.nprob, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    prof.collect();
  }

  static int pipeline_mode_host(int m) { return (m == M_EVAL || m == M_CG || m == M_BASIC) ? 1 : 0; }

  static constexpr int kMaxStagger = 30;

  void solve(const hom_load* loads, hom_result* out) override {
    const int n = (int)where.size();
    for (int i = 0; i < n; ++i) {
      const hom_load& L = loads[i];
      if (!(L.dt > 0.0) || !std::isfinite(L.dt)) fail(HOM_E_ARG, "dt must be positive and finite");
      if (!(L.temp.theta > 0.0) || !std::isfinite(L.temp.theta)) fail(HOM_E_ARG, "theta must be positive");
      for (int c = 0; c < 6; ++c)
        if (!std::isfinite(L.strain[c]) || !std::isfinite(L.stress[c]))
          fail(HOM_E_ARG, "macro strain and stress must be finite");
      for (int c = 0; c < 3; ++c)
        if (!std::isfinite(L.temp.grad[c])) fail(HOM_E_ARG, "temperature gradient must be finite");
      if (L.stress_mask > 63u) fail(HOM_E_ARG, "stress_mask has bits above 5");
      if (L.adiabatic != 0 && L.adiabatic != 1) fail(HOM_E_ARG, "adiabatic must be 0 or 1");
      if (L.stress_mask && opts.scheme != HOM_SCHEME_NEWTON_CG)
        fail(HOM_E_UNSUPPORTED, "mixed boundary conditions need the Newton-CG scheme");
      if (L.trial != 0 && L.trial != 1) fail(HOM_E_ARG, "trial must be 0 or 1");
      if (L.trial != loads[0].trial) fail(HOM_E_ARG, "trial must be the same for every problem of a batch");
    }
    const bool trial = loads[0].trial != 0;
    const double sq2 = std::sqrt(2.0);
    const double w[6] = {1, 1, 1, sq2, sq2, sq2};
    auto solve_group = [&](Group<T>& G) {
      hipStream_t stream = G.stream;  // this group's lane
      const int np = G.nprob;
      std::vector<double> th(np), thn(np), pipes(np, 0.0), thprev(np, 0.0), gprev(np, 0.0);
      std::vector<int> newton(np, 0), krylov(np, 0), stag(np, 0);
      bool any_adi = false;
      for (int j = 0; j < np; ++j) {
        const hom_load& L = loads[G.members[j]];
        th[j] = thn[j] = L.temp.theta;
        any_adi = any_adi || L.adiabatic;
      }
      G.tan_ok = false;
      // implicit staggering (adiabatic problems): mechanics at fixed theta,
      // then theta^{n+1} = theta^n + dt <D> / <c0>, until theta is stationary;
      // every later mechanical solve restarts from the last strain field
      for (int s = 0;; ++s) {
        for (int j = 0; j < np; ++j) {
          const hom_load& L = loads[G.members[j]];
          ProbInc& in = G.inc_h[j];
          fill_inc(in, laws, th[j], L.dt);
          in.smask = (int)L.stress_mask;
          for (int c = 0; c < 6; ++c) {
            const bool sc = (L.stress_mask >> c) & 1u;
            in.dE[c] = sc ? 0.0 : w[c] * L.strain[c] - G.En[j][c];
            in.S[c] = sc ? w[c] * L.stress[c] : 0.0;
          }
          for (int c = 0; c < 3; ++c) in.dG[c] = L.temp.grad[c] - G.Gp[j][c];
          // predictor weight: projection of this macro increment on the last
          // one over the strain-controlled components
          in.pred_s = 0.0;
          if (G.dx && G.pred_ok[j]) {
            double ee = 0.0, ep = 0.0;
            for (int c = 0; c < 6; ++c) {
              if ((L.stress_mask >> c) & 1u) continue;
              ee += in.dE[c] * G.dEp[j][c];
              ep += G.dEp[j][c] * G.dEp[j][c];
            }
            if (ep > 0.0 && std::isfinite(ee)) in.pred_s = std::min(2.0, std::max(0.0, ee / ep));
          }
          for (int c = 0; c < 6; ++c) in.dEp[c] = G.dEp[j][c];
          if (G.inc_pm_h) {  // the increment data at theta +- h_theta for the point partials
            fill_inc(G.inc_pm_h[2 * j], laws, th[j] + FD_H_THETA, L.dt);
            fill_inc(G.inc_pm_h[2 * j + 1], laws, th[j] - FD_H_THETA, L.dt);
          }
        }
        HIPCHK(hipMemcpyAsync(G.inc_d, G.inc_h, sizeof(ProbInc) * np, hipMemcpyHostToDevice, stream));
        if (G.inc_pm_h)
          HIPCHK(hipMemcpyAsync(G.inc_pm_d, G.inc_pm_h, sizeof(ProbInc) * 2 * np, hipMemcpyHostToDevice, stream));
        mech_iterate(G, s > 0);
        mech_finish(G, !any_adi && !trial, !any_adi);
        for (int j = 0; j < np; ++j) {
          pipes[j] += G.ctl_h[j].pipelines;
          newton[j] += G.ctl_h[j].newton_it;
          krylov[j] += G.ctl_h[j].krylov;
          stag[j] += 1;
        }
        if (!any_adi) break;
        // the temperature each adiabatic problem moves to. The staggering has
        // converged where the heat equation's image of theta,
        // t = theta^n + dt <D>(theta) / <c0>, stays within tol times the
        // change of theta; otherwise the next theta is the secant root of
        // g(theta) = t - theta through the last two iterates (the first step
        // is the plain fixed-point step theta = t).
        std::vector<double> next(th);
        bool moved = false;
        for (int j = 0; j < np; ++j) {
          const hom_load& L = loads[G.members[j]];
          const Ctl& c = G.ctl_h[j];
          if (!L.adiabatic || c.status != 1) continue;
          const double t = thn[j] + L.dt * c.out[7] / G.c0mean[j];
          if (!std::isfinite(t) || !(t > 0.0)) {
            G.ctl_h[j].status = HOM_E_NAN;
            G.ctl_h[j].mode = M_FAIL;
            continue;
          }
          const double g = t - th[j];
          if (std::fabs(g) <= 10.0 * opts.tol * std::fabs(t - thn[j]) + 1e-12 * thn[j]) continue;
          double tn = t;
          if (s > 0 && g != gprev[j]) {
            const double sec = th[j] - g * (th[j] - thprev[j]) / (g - gprev[j]);
            if (std::isfinite(sec) && sec > 0.0) tn = sec;
          }
          thprev[j] = th[j];
          gprev[j] = g;
          next[j] = tn;
          moved = true;
        }
        if (moved && s + 1 < kMaxStagger) {
          th = next;
          continue;
        }
        // final: commit at the temperatures of the last solve; a problem whose
        // temperature still moves after the last staggered solve does not commit
        for (int j = 0; j < np; ++j)
          if (next[j] != th[j]) {
            G.ctl_h[j].status = HOM_E_NOT_CONVERGED;
            G.ctl_h[j].mode = M_FAIL;
          }
        HIPCHK(hipMemcpyAsync(G.ctl_m, G.ctl_h, sizeof(Ctl) * np, hipMemcpyHostToDevice, stream));
        mech_finish(G, !trial, true);
        break;
      }
      std::vector<Ctl> mech(G.ctl_h, G.ctl_h + np);
      // the conduction field now holds the new mean gradient
      for (int j = 0; j < np; ++j)
        for (int c = 0; c < 3; ++c) G.Gp[j][c] = loads[G.members[j]].temp.grad[c];
      thermal_solve(G);
      bool all = opts.scheme == HOM_SCHEME_NEWTON_CG;
      for (int j = 0; j < np; ++j) {
        const int i = G.members[j];
        const hom_load& L = loads[i];
        const Ctl& cm = mech[j];
        const Ctl& ct = G.ctl_h[j];
        hom_result& r = out[i];
        std::memset(&r, 0, sizeof(r));
        for (int c = 0; c < 6; ++c) {
          r.stress[c] = cm.out[c] / w[c];
          r.strain[c] = ((L.stress_mask >> c) & 1u) ? cm.out[8 + c] / w[c] : L.strain[c];
        }
        for (int c = 0; c < 3; ++c) r.heat_flux[c] = ct.out[c];
        r.dissipation = cm.out[6];
        r.coupling = cm.out[7];
        r.heat_capacity = G.c0mean[j];
        r.residual = cm.res;
        r.newton_iters = newton[j];
        r.krylov_iters = krylov[j];
        r.thermal_iters = ct.krylov > 0 ? ct.krylov : ct.newton_it;
        r.pipelines = pipes[j];
        r.thermal_pipelines = ct.pipelines;
        r.theta = th[j];
        r.stagger_iters = stag[j];
        int st = HOM_OK;
        if (cm.status != 1) st = cm.status < 0 ? cm.status : HOM_E_NOT_CONVERGED;
        if (st == HOM_OK && ct.status != 1) st = ct.status < 0 ? ct.status : HOM_E_NOT_CONVERGED;
        r.status = st;
        if (cm.status == 1 && !trial) {
          for (int c = 0; c < 6; ++c) {
            const double e = ((L.stress_mask >> c) & 1u) ? cm.out[8 + c] : w[c] * L.strain[c];
            G.dEp[j][c] = e - G.En[j][c];
            G.En[j][c] = e;
          }
          G.pred_ok[j] = 1;  // the commit wrote the field of this change
        }
        all = all && cm.status == 1;
      }
      G.tan_ok = all;
    };
    // groups of different grids are independent: with library-owned lanes
    // they run at the same time, one host thread each (the per-kernel
    // profiler times launches one by one, so it keeps them in turn)
    if (groups.size() > 1 && own_stream && !prof.on) {
      std::vector<std::thread> pool;
      std::vector<int> codes(groups.size(), HOM_OK);
      std::vector<std::string> msgs(groups.size());
      for (size_t gi = 0; gi < groups.size(); ++gi)
        pool.emplace_back([&, gi] {
          try {
            HIPCHK(hipSetDevice(device));
            solve_group(*groups[gi]);
          } catch (const Error& e) {
            codes[gi] = e.code;
            msgs[gi] = e.msg;
          } catch (const std::exception& e) {
            codes[gi] = HOM_E_DEVICE;
            msgs[gi] = e.what();
          }
        });
      for (auto& t : pool) t.join();
      for (size_t gi = 0; gi < groups.size(); ++gi)
        if (codes[gi] != HOM_OK) fail(codes[gi], msgs[gi]);
    } else {
      for (auto& gp : groups) solve_group(*gp);
    }
  }

  // New parameters for the phase laws (same kinds; for the PA66 law the same
  // number of Maxwell branches, so the internal variables keep their layout).
  void set_laws(const hom_law* lw, int n) override {
    if (!lw || n != (int)laws.size()) fail(HOM_E_ARG, "need one law per phase of the setup");
    validate_laws(lw, n);
    auto branches = [](const hom_law& L) {
      int nm = 0;
      for (int j = 0; j < L.n_maxwell; ++j) nm += L.E_i[j] > 0.0 ? 1 : 0;
      return nm;
    };
    for (int i = 0; i < n; ++i) {
      if (lw[i].kind != laws[i].kind) fail(HOM_E_ARG, "law " + std::to_string(i) + " changes its kind");
      if (lw[i].kind == HOM_LAW_PA66 && branches(lw[i]) != branches(laws[i]))
        fail(HOM_E_ARG, "law " + std::to_string(i) + " changes its number of Maxwell branches");
    }
    laws.assign(lw, lw + n);
    for (auto& gp : groups) {
      Group<T>& G = *gp;
      for (int j = 0; j < G.nprob; ++j) {
        double c0 = 0.0;
        for (int l = 0; l < n; ++l) c0 += laws[l].c0 * (double)G.phase_count[j][l] / (double)G.nvox;
        G.c0mean[j] = c0;
      }
      G.tan_ok = false;  // the tangent fields belong to the old parameters
      std::fill(G.pred_ok.begin(), G.pred_ok.end(), 0);
      std::fill(G.tcol_ok, G.tcol_ok + 7, false);
    }
  }

  // ---- effective algorithmic tangents of the last increment ---------------
  // Linearized solves with the algorithmic tangent of the converged Newton
  // evaluation: one per unit macro strain (Mandel), and for what = 1 one with
  // mean zero and the source d sigma / d theta. The strain and stress fields
  // of the increment are restored afterwards.
  void tangent(int what, hom_tangent* out) override {
    if (opts.scheme != HOM_SCHEME_NEWTON_CG)
      fail(HOM_E_UNSUPPORTED, "algorithmic tangents need the Newton-CG scheme (its evaluations keep the tangent)");
    if (what != 0 && what != 1) fail(HOM_E_ARG, "what must be 0 (d sigma / dE) or 1 (all four tangents)");
    for (auto& gp : groups) {
      if (!gp->tan_ok)
        fail(HOM_E_ARG, "no converged increment to linearize (every problem's last increment must have converged)");
      if (what == 1 && !gp->dsdt)
        fail(HOM_E_ARG, "temperature and coupling tangents need a setup with the tangent option");
    }
    const double sq2 = std::sqrt(2.0);
    const double w[6] = {1, 1, 1, sq2, sq2, sq2};
    const bool prof_on = prof.on;
    prof.on = false;
    for (auto& gp : groups) {
      Group<T>& G = *gp;
      hipStream_t stream = G.stream;  // this group's lane
      const size_t nm = (size_t)G.nprob * G.vs;
      if (!G.fsave) G.fsave = G.template dalloc<T>(6 * nm);
      HIPCHK(hipMemcpyAsync(G.fsave, G.f, 6 * nm * sizeof(T), hipMemcpyDeviceToDevice, stream));
      auto restore = [&] {
        (void)hipMemcpyAsync(G.xm, G.xnm, 6 * nm * sizeof(T), hipMemcpyDeviceToDevice, stream);
        (void)hipMemcpyAsync(G.f, G.fsave, 6 * nm * sizeof(T), hipMemcpyDeviceToDevice, stream);
        (void)hipStreamSynchronize(stream);
      };
      try {
        const int ncol = what == 1 ? 7 : 6;
        Limits lim = limits(0);
        lim.linear = 1;
        const long long cap = iteration_cap(lim, false);
        Pt<T> q = G.pt(0);
        if (G.dx && !G.tcol) G.tcol = G.template dalloc<T>(7 * 6 * nm);  // predictor: warm starts
        for (int j = 0; j < G.nprob; ++j) {
          hom_tangent& t = out[G.members[j]];
          std::memset(&t, 0, sizeof(t));
          if (what == 0) {
            for (int c = 0; c < 6; ++c) t.dsdt[c] = t.dDde[c] = NAN;
            t.dDdt = NAN;
          }
        }
        for (int col = 0; col < ncol; ++col) {
          for (int j = 0; j < G.nprob; ++j) {
            G.inc_h[j].smask = 0;  // the tangents are derivatives at prescribed strain
            for (int c = 0; c < 6; ++c) G.inc_h[j].dE[c] = (c == col) ? 1.0 : 0.0;
          }
          HIPCHK(hipMemcpyAsync(G.inc_d, G.inc_h, sizeof(ProbInc) * G.nprob, hipMemcpyHostToDevice, stream));
          T* start = G.tcol ? G.tcol + (size_t)col * 6 * nm : nullptr;
          q.x0 = (start && G.tcol_ok[col]) ? start : nullptr;
          launch_init_linear<T>(q, stream);
          iterate(G, col < 6 ? 2 : 3, false, cap);
          launch_tangent_sum<T>(q, stream);
          launch_reduce_out(G.ctl_m, G.part, G.maxblk, G.pt_bpp, G.nprob, 8, 1.0 / (double)G.nvox, stream);
          HIPCHK(hipMemcpyAsync(G.ctl_h, G.ctl_m, sizeof(Ctl) * G.nprob, hipMemcpyDeviceToHost, stream));
          HIPCHK(hipStreamSynchronize(stream));
          for (int j = 0; j < G.nprob; ++j) {
            const Ctl& c = G.ctl_h[j];
            if (c.status != 1)
              fail(c.status < 0 ? c.status : HOM_E_NOT_CONVERGED,
                   "linearized solve " + std::to_string(col) + " of problem " + std::to_string(G.members[j]) +
                       " did not converge");
            hom_tangent& t = out[G.members[j]];
            if (col < 6) {
              for (int I = 0; I < 6; ++I) t.dsde[6 * I + col] = c.out[I] * w[col] / w[I];
              if (what == 1) t.dDde[col] = c.out[6] * w[col];
            } else {
              for (int I = 0; I < 6; ++I) t.dsdt[I] = c.out[I] / w[I];
              t.dDdt = c.out[6] + c.out[7];
            }
            t.solves += 1;
            t.krylov_iters += c.krylov;
            t.pipelines += c.pipelines;
          }
          if (start) {  // converged everywhere: the next call starts from this solution
            HIPCHK(hipMemcpyAsync(start, G.xm, 6 * nm * sizeof(T), hipMemcpyDeviceToDevice, stream));
            G.tcol_ok[col] = true;
          }
        }
      } catch (...) {
        restore();
        prof.on = prof_on;
        throw;
      }
      restore();
      HIPCHK(hipGetLastError());
    }
    prof.on = prof_on;
  }

  // ---- checkpoint: xn, xt, state, macro history -------------------------
  size_t state_size() const override {
    size_t s = 16;
    for (auto& gp : groups) {
      const auto& G = *gp;
      const size_t nm = (size_t)G.nprob * G.nvox;  // fields without the stride padding
      const size_t ns = (size_t)G.nprob * std::max<long long>(G.ss, 1);
      s += nm * 9 * sizeof(T) + (G.state ? ns * G.nstate * sizeof(double) : 0) + G.nprob * 9 * sizeof(double);
    }
    return s;
  }
  void get_state(void* buf) override {
    char* p = static_cast<char*>(buf);
    const uint64_t magic = 0x484f4d5354415445ull, tsz = sizeof(T);
    std::memcpy(p, &magic, 8);
    std::memcpy(p + 8, &tsz, 8);
    p += 16;
    for (auto& gp : groups) {
      auto& G = *gp;
      // fields as [prob][comp][nvox]: the checkpoint does not depend on the
      // device stride padding
      const size_t row = G.nvox * sizeof(T), pitch = G.vs * sizeof(T);
      HIPCHK(hipMemcpy2D(p, row, G.xnm, pitch, row, (size_t)G.nprob * 6, hipMemcpyDeviceToHost));
      p += row * G.nprob * 6;
      HIPCHK(hipMemcpy2D(p, row, G.xt, pitch, row, (size_t)G.nprob * 3, hipMemcpyDeviceToHost));
      p += row * G.nprob * 3;
      if (G.state) {
        const size_t ns = (size_t)G.nprob * std::max<long long>(G.ss, 1);
        HIPCHK(hipMemcpy(p, G.state, ns * G.nstate * sizeof(double), hipMemcpyDeviceToHost));
        p += ns * G.nstate * sizeof(double);
      }
      for (int j = 0; j < G.nprob; ++j) {
        std::memcpy(p, G.En[j].data(), 6 * sizeof(double));
        std::memcpy(p + 6 * sizeof(double), G.Gp[j].data(), 3 * sizeof(double));
        p += 9 * sizeof(double);
      }
    }
  }
  void set_state(const void* buf) override {
    for (auto& gp : groups) {
      gp->tan_ok = false;  // the tangent fields belong to the replaced state
      std::fill(gp->pred_ok.begin(), gp->pred_ok.end(), 0);  // so does the predictor's last change
      std::fill(gp->tcol_ok, gp->tcol_ok + 7, false);
    }
    const char* p = static_cast<const char*>(buf);
    uint64_t magic, tsz;
    std::memcpy(&magic, p, 8);
    std::memcpy(&tsz, p + 8, 8);
    if (magic != 0x484f4d5354415445ull || tsz != sizeof(T)) fail(HOM_E_ARG, "state buffer does not match context");
    p += 16;
    for (auto& gp : groups) {
      auto& G = *gp;
      const size_t row = G.nvox * sizeof(T), pitch = G.vs * sizeof(T);
      HIPCHK(hipMemcpy2D(G.xnm, pitch, p, row, row, (size_t)G.nprob * 6, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy2D(G.xm, pitch, p, row, row, (size_t)G.nprob * 6, hipMemcpyHostToDevice));
      p += row * G.nprob * 6;
      HIPCHK(hipMemcpy2D(G.xt, pitch, p, row, row, (size_t)G.nprob * 3, hipMemcpyHostToDevice));
      p += row * G.nprob * 3;
      if (G.state) {
        const size_t ns = (size_t)G.nprob * std::max<long long>(G.ss, 1);
        HIPCHK(hipMemcpy(G.state, p, ns * G.nstate * sizeof(double), hipMemcpyHostToDevice));
        p += ns * G.nstate * sizeof(double);
      }
      for (int j = 0; j < G.nprob; ++j) {
        std::memcpy(G.En[j].data(), p, 6 * sizeof(double));
        std::memcpy(G.Gp[j].data(), p + 6 * sizeof(double), 3 * sizeof(double));
        p += 9 * sizeof(double);
      }
    }
  }

  void get_field(int which, double* out, size_t count) override {
    if (groups.size() != 1 || groups[0]->nprob != 1) fail(HOM_E_ARG, "fields are per single-problem context");
    auto& G = *groups[0];
    const size_t nv = G.nvox;
    int nc;
    const void* src;
    bool dbl = false;
    switch (which) {
      case HOM_FIELD_STRAIN: nc = 6; src = G.xm; break;
      case HOM_FIELD_STRESS: nc = 6; src = G.f; break;
      case HOM_FIELD_GRADIENT: nc = 3; src = G.xt; break;
      case HOM_FIELD_STATE:
        if (!G.state) fail(HOM_E_ARG, "no internal variables (no PA66 law)");
        nc = G.nstate;
        src = G.state;
        dbl = true;
        break;
      default: fail(HOM_E_ARG, "unknown field");
    }
    if (count != nv * nc) fail(HOM_E_ARG, "field buffer size mismatch: need " + std::to_string(nv * nc));
    HIPCHK(hipStreamSynchronize(stream));
    if (dbl) {
      // internal variables: the compacted PA66 voxels scattered to voxel
      // arrays, zero in the other phases
      const size_t ss = (size_t)G.ss;
      std::vector<double> cmp((size_t)nc * ss);
      std::vector<uint8_t> ph(nv);
      HIPCHK(hipMemcpy(cmp.data(), src, cmp.size() * sizeof(double), hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(ph.data(), G.phase, nv, hipMemcpyDeviceToHost));
      int pa = -1;
      for (size_t l = 0; l < laws.size(); ++l)
        if (laws[l].kind == HOM_LAW_PA66) pa = (int)l;
      size_t q = 0;
      for (size_t v = 0; v < nv; ++v) {
        const bool isp = (int)ph[v] == pa;
        for (int k = 0; k < nc; ++k) out[k * nv + v] = isp ? cmp[k * ss + q] : 0.0;
        if (isp) ++q;
      }
    } else {
      std::vector<T> tmp(count);
      for (int k = 0; k < nc; ++k)  // components vs apart on the device
        HIPCHK(hipMemcpy(tmp.data() + k * nv, static_cast<const T*>(src) + k * G.vs, nv * sizeof(T),
                         hipMemcpyDeviceToHost));
      for (size_t i = 0; i < count; ++i) out[i] = (double)tmp[i];
    }
  }
};

std::unique_ptr<BatchImpl> make_batch(int nprob, const hom_grid* grids, const uint8_t* const* phases,
                                      const hom_law* laws, int nlaws, const hom_options& opts) {
  if (nprob < 1) fail(HOM_E_ARG, "need at least one problem");
  if (!grids || !phases || !laws) fail(HOM_E_ARG, "null argument");
  validate_laws(laws, nlaws);
  if (!(opts.tol > 0.0)) fail(HOM_E_ARG, "tol must be positive");
  if (opts.scheme != HOM_SCHEME_BASIC && opts.scheme != HOM_SCHEME_NEWTON_CG) fail(HOM_E_ARG, "unknown scheme");
  if (opts.discretization != HOM_DISC_COLLOCATION && opts.discretization != HOM_DISC_ROTATED)
    fail(HOM_E_ARG, "unknown discretization");
  if (opts.discretization == HOM_DISC_ROTATED && opts.scheme != HOM_SCHEME_NEWTON_CG)
    fail(HOM_E_UNSUPPORTED, "the rotated discretization is built for the Newton-CG scheme");
  if (opts.predictor != 0 && opts.predictor != 1) fail(HOM_E_ARG, "predictor must be 0 or 1");
  if (opts.precision == HOM_FP64) {
    auto b = std::make_unique<BatchT<double>>();
    b->init(nprob, grids, phases, laws, nlaws, opts);
    return b;
  }
  if (opts.precision == HOM_FP32) {
    auto b = std::make_unique<BatchT<float>>();
    b->init(nprob, grids, phases, laws, nlaws, opts);
    return b;
  }
  fail(HOM_E_ARG, "unknown precision");
}

// ---------------------------------------------------------------------------
// kernel-level entry points
// ---------------------------------------------------------------------------
template <typename T>
static void apply_operator_t(const hom_grid& g, int ncomp, int op, double p0, double p1, const double* in,
                             double* out, int sched) {
  Group<T> G;
  G.nx = g.n[0];
  G.ny = g.n[1];
  G.nz = g.n[2];
  for (int d = 0; d < 3; ++d) G.len[d] = g.len[d];
  G.nprob = 1;
  G.alloc(false);
  const size_t nv = G.nvox;
  std::vector<T> tmp(nv * ncomp);
  for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (T)in[i];
  for (int k = 0; k < ncomp; ++k)  // components G.vs apart on the device
    HIPCHK(hipMemcpy(G.f + k * G.vs, tmp.data() + k * nv, nv * sizeof(T), hipMemcpyHostToDevice));
  Ctl c;
  std::memset(&c, 0, sizeof(c));
  c.mode = M_EVAL;
  HIPCHK(hipMemcpy(G.ctl_m, &c, sizeof(c), hipMemcpyHostToDevice));
  ProbInc inc;
  std::memset(&inc, 0, sizeof(inc));
  inc.lam0 = p0;
  inc.mu0 = p1;
  inc.kappa0 = p0;
  HIPCHK(hipMemcpy(G.inc_d, &inc, sizeof(inc), hipMemcpyHostToDevice));
  const int green = op;
  Pipe<T> a = G.pipe(0, green);
  a.C = ncomp;
  a.ctl = G.ctl_m;
  hipStream_t s = nullptr;
  int tx = sched;
  if (sched < 0) {
    tx = schedule(4, 0);
    if (!launch_ok(run_zgreen<T>(a, tx, s, true))) tx = schedule(2, 0);
  } else if (!launch_ok(run_zgreen<T>(a, tx, s, true)) || !launch_ok(run_ypass<T>(a, tx, 0, s, true))) {
    fail(HOM_E_UNSUPPORTED, "schedule does not fit the work-group limits on this grid");
  }
  (void)hipGetLastError();
  run_xfwd<T>(a, s);
  hip_check(hipGetLastError(), "xfwd launch");
  run_ypass<T>(a, tx, 0, s);
  hip_check(hipGetLastError(), "ypass launch");
  run_zgreen<T>(a, tx, s);
  hip_check(hipGetLastError(), "zgreen launch");
  run_ypass<T>(a, tx, 1, s);
  run_xinv<T>(a, s);
  hip_check(hipGetLastError(), "xinv launch");
  HIPCHK(hipDeviceSynchronize());
  for (int k = 0; k < ncomp; ++k)
    HIPCHK(hipMemcpy(tmp.data() + k * nv, G.r + k * G.vs, nv * sizeof(T), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < tmp.size(); ++i) out[i] = -(double)tmp[i];
}

void apply_operator(const hom_grid& g, int ncomp, int op, double p0, double p1, int precision, const double* in,
                    double* out, int sched) {
  if (sched >= 0) {
    bool known = false;
    for (int sc : kScheduleChoices) known = known || sc == sched;
    if (!known) fail(HOM_E_ARG, "unknown schedule");
  }
  for (int d = 0; d < 3; ++d)
    if (!supported_n(g.n[d])) fail(HOM_E_UNSUPPORTED, "unsupported grid size");
  if (!((ncomp == 6 && (op == G_PROJ || op == G_GAMMA0 || op == G_PROJ_ROT)) ||
        (ncomp == 3 && (op == G_GRADPROJ || op == G_GAMMA_TH || op == G_GRADPROJ_ROT))))
    fail(HOM_E_ARG, "operator / component count mismatch");
  if (op == G_GAMMA0 && !(p1 > 0.0 && p0 + 2.0 * p1 > 0.0)) fail(HOM_E_ARG, "invalid reference medium");
  if (op == G_GAMMA_TH && !(p0 > 0.0)) fail(HOM_E_ARG, "invalid reference conductivity");
  if (precision == HOM_FP64)
    apply_operator_t<double>(g, ncomp, op, p0, p1, in, out, sched);
  else if (precision == HOM_FP32)
    apply_operator_t<float>(g, ncomp, op, p0, p1, in, out, sched);
  else
    fail(HOM_E_ARG, "unknown precision");
}

void eval_law(const hom_law& law, int64_t count, const double* eps, const double* eps_n, const double* state,
              double theta, double dt, int commit, double* sigma, double* ab, double* nd, double* state_out,
              double* diss, double* coup) {
  validate_laws(&law, 1);
  if (count < 1) fail(HOM_E_ARG, "count must be positive");
  if (!(dt > 0.0) || !(theta > 0.0)) fail(HOM_E_ARG, "need dt > 0 and theta > 0");
  std::vector<hom_law> laws(1, law);
  Group<double> G;
  G.nx = (int)count;
  G.ny = 1;
  G.nz = 1;
  G.nprob = 1;
  G.nstate = pa66_nstate(laws);
  // pointwise buffers only (unpadded: the host arrays' layout)
  G.nvox = count;
  G.vs = count;
  G.phase = G.dalloc<uint8_t>(count);
  G.xm = G.dalloc<double>(6 * count);
  G.xnm = G.dalloc<double>(6 * count);
  G.f = G.dalloc<double>(6 * count);
  G.tab = G.dalloc<double>(2 * count);
  G.tn = G.dalloc<double>(6 * count);
  if (G.nstate) {  // every point is a PA66 point: the compact index is the point's
    G.state = G.dalloc<double>(G.nstate * count);
    G.hist = G.dalloc<double>(HIST_SLOTS * count);
    G.ss = count;
    G.npa.assign(1, (int)count);
    std::vector<int> cb((size_t)(count + 63) / 64);
    for (size_t k = 0; k < cb.size(); ++k) cb[k] = (int)(64 * k);
    G.cbase = G.dalloc<int>(cb.size());
    G.npa_d = G.dalloc<int>(1);
    HIPCHK(hipMemcpy(G.cbase, cb.data(), cb.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(G.npa_d, G.npa.data(), sizeof(int), hipMemcpyHostToDevice));
  }
  G.ctl_m = G.dalloc<Ctl>(1);
  G.inc_d = G.dalloc<ProbInc>(1);
  G.pt_bpp = (int)std::min<int64_t>((count + 255) / 256, 4096);
  G.maxblk = std::max(G.pt_bpp, commit_voxel_blocks(count));  // the commit below: a partial a block of 256
  G.part = G.dalloc<double>((size_t)G.maxblk * NPART);
  double* pvd = G.dalloc<double>(count);
  double* pvc = G.dalloc<double>(count);
  HIPCHK(hipMemcpy(G.xm, eps, 6 * count * sizeof(double), hipMemcpyHostToDevice));
  if (eps_n) HIPCHK(hipMemcpy(G.xnm, eps_n, 6 * count * sizeof(double), hipMemcpyHostToDevice));
  if (G.nstate) {
    if (!state) fail(HOM_E_ARG, "PA66 evaluation needs the internal variables");
    HIPCHK(hipMemcpy(G.state, state, G.nstate * count * sizeof(double), hipMemcpyHostToDevice));
  }
  ProbInc inc;
  fill_inc(inc, laws, theta, dt);
  HIPCHK(hipMemcpy(G.inc_d, &inc, sizeof(inc), hipMemcpyHostToDevice));
  Ctl c;
  std::memset(&c, 0, sizeof(c));
  c.mode = M_EVAL;
  HIPCHK(hipMemcpy(G.ctl_m, &c, sizeof(c), hipMemcpyHostToDevice));
  Pt<double> q = G.pt(0);
  q.pv_diss = pvd;
  q.pv_coup = pvc;
  if (G.nstate) launch_history<double>(q, nullptr);
  launch_eval<double>(q, 6, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(sigma, G.f, 6 * count * sizeof(double), hipMemcpyDeviceToHost));
  if (ab) HIPCHK(hipMemcpy(ab, G.tab, 2 * count * sizeof(double), hipMemcpyDeviceToHost));
  if (nd) HIPCHK(hipMemcpy(nd, G.tn, 6 * count * sizeof(double), hipMemcpyDeviceToHost));
  if (commit) {
    c.status = 1;
    c.mode = M_DONE;
    HIPCHK(hipMemcpy(G.ctl_m, &c, sizeof(c), hipMemcpyHostToDevice));
    q.dp_known = 1;  // the evaluation above was at this strain
    launch_commit<double>(q, 6, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    if (state_out && G.nstate)
      HIPCHK(hipMemcpy(state_out, G.state, G.nstate * count * sizeof(double), hipMemcpyDeviceToHost));
    if (diss) HIPCHK(hipMemcpy(diss, pvd, count * sizeof(double), hipMemcpyDeviceToHost));
    if (coup) HIPCHK(hipMemcpy(coup, pvc, count * sizeof(double), hipMemcpyDeviceToHost));
  }
}

}  // namespace hom
