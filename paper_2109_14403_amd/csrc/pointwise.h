// Per-voxel kernels: constitutive evaluation, CG vector updates, commit of
// the internal variables, and the per-problem reductions that drive the
// Newton-CG / basic-scheme state machine on the device.
#pragma once
#include "common.h"

namespace hom {

// Per-voxel slots of the PA66 increment data: deviatoric branch history sum
// (6), spherical history sum, plastic increment of the latest evaluation.
constexpr int HIST_SLOTS = 8;

// Arguments of the pointwise kernels of one group.
template <typename T>
struct Pt {
  long long nvox;
  long long vs;             // stride of the per-voxel arrays: [prob][comp][vs], vs >= nvox
  int nprob;
  int bpp;                  // blocks per problem
  const uint8_t* phase;
  T* x;
  T* xn;                    // committed strain (mechanics)
  T* f;
  T* r;
  T* p;
  T* tab;
  T* tn;
  // Internal variables and increment slots of the PA66 voxels only, compacted
  // in voxel order (a pass over them reads whole cache lines): PA66 voxel v of
  // problem p sits at q = cbase[p][v / 64] + (PA66 voxels before v in its
  // 64-voxel chunk)
  double* state;            // [prob][nstate][ss] (mechanics with a PA66 phase)
  int nstate;
  double* hist;             // [prob][HIST_SLOTS][ss] PA66 branch history sums of the increment, last dp
  const int* cbase;         // [prob][ceil(nvox / 64)] PA66 voxels before each chunk
  const int* npa;           // [prob] PA66 voxels of each problem
  long long ss;             // stride of state and hist (>= every npa)
  Ctl* ctl;
  const ProbInc* inc;
  double* part;
  int maxblk;
  double* pv_diss;          // optional per-voxel dissipation at commit
  double* pv_coup;          // optional per-voxel coupling term at commit
  // effective algorithmic tangents: per-voxel partials at the converged
  // strain of an increment (state n), written by the partials kernel
  T* dsdt;                  // d sigma / d theta   [prob][6][nvox] (Mandel), or null
  T* dDde;                  // d D / d eps         [prob][6][nvox] (Mandel)
  T* dDdt;                  // d D / d theta       [prob][nvox]
  const ProbInc* inc_pm;    // [prob][2]: increment data at theta + h_theta, theta - h_theta
  const T* s0;              // source of a linearized evaluation (sigma = C x + s0), or null
  int commit;               // commit kernel: 1 commit, 0 only the effective sums (a trial)
  int dp_known;             // commit: the last evaluation was at the converged strain (its
                            // plastic increments are in the increment slots)
  T* dx;                    // strain change of the last committed increment [prob][6][nvox], or null
  const T* x0;              // start of a linearized solve [prob][6][nvox], or null (uniform dE)
};

// Effective sums of the commit kernel (mechanics): <sigma> (6), dissipation,
// coupling term, <eps> (6).
constexpr int MECH_SUMS = 14;

// Central-difference steps of the PA66 point partials: Mandel strain and
// temperature [K].
constexpr double FD_H_EPS = 1e-6;
constexpr double FD_H_THETA = 1e-3;

struct Limits {
  double tol;
  int max_newton;   // Newton: residual evaluations; basic: iterations
  int max_krylov;
  int linear;       // 1: CG solves to the tolerance at once
};

}  // namespace hom

// host launchers (pointwise.hip)
namespace hom {
template <typename T>
void launch_init_mech(const Pt<T>& a, int scheme, hipStream_t s, int keep_x = 0);
template <typename T>
void launch_init_th(const Pt<T>& a, int scheme, hipStream_t s);
template <typename T>
void launch_eval(const Pt<T>& a, int C, hipStream_t s);
// sigma = C_algo x (+ s0) with the algorithmic tangent of the last Newton
// evaluation; the tangent fields are read, not written (mechanics only)
template <typename T>
void launch_eval_linear(const Pt<T>& a, hipStream_t s);
// x = dE (uniform) and a fresh Newton state: the start of a linearized solve
template <typename T>
void launch_init_linear(const Pt<T>& a, hipStream_t s);
template <typename T>
void launch_partials(const Pt<T>& a, hipStream_t s);
// per-block sums of the stress (6), dD/deps . x and dD/dtheta of converged problems
template <typename T>
void launch_tangent_sum(const Pt<T>& a, hipStream_t s);
template <typename T>
void launch_history(const Pt<T>& a, hipStream_t s);
void launch_reduce_a(Ctl* ctl, const double* part, int maxblk, int nblk, int nprob, Limits lim, hipStream_t s);
// Whether a commit with these arguments takes the one-voxel-per-thread path
// (internal variables, plastic increments of the last evaluation known), and
// the blocks per problem (partial sums) it then writes.
template <typename T>
inline bool commit_per_voxel(const Pt<T>& a, int C) {
  return C == 6 && a.dp_known && a.state && a.hist;
}
inline int commit_voxel_blocks(long long nvox) { return (int)((nvox + 255) / 256); }
// Returns the blocks per problem whose partial sums it wrote (a.bpp, or
// commit_voxel_blocks(a.nvox) on the one-voxel-per-thread path; a.maxblk must
// hold them).
template <typename T>
int launch_commit(const Pt<T>& a, int C, hipStream_t s);
void launch_reduce_out(Ctl* ctl, const double* part, int maxblk, int nblk, int nprob, int nk, double scale,
                       hipStream_t s);
// First stage of a reduction over many blocks: block (prob, j) sums the
// partials [j * RED_CHUNK, (j + 1) * RED_CHUNK) of every quantity in a fixed
// order into out[prob][NPART][nout], nout = ceil(nblk / RED_CHUNK).
constexpr int RED_CHUNK = 512;
void launch_reduce_stage(const double* part, int maxblk, int nblk, double* out, int nout, int nprob, hipStream_t s);
}  // namespace hom
