// Direct deep material network (paper Sec. 3): a perfect binary tree of
// two-phase laminates. Offline: the linear homogenization function, the loss
// and its gradients in hand-written FP64 kernels (one work-group per stiffness
// sample), AMSGrad with the paper's learning-rate modulation. Online: the
// Newton iteration on the displacement jumps of many macroscopic points at
// once (one wave per point).
//
// Tree indexing on the device (heap order): node h = 1 is the root, the
// children of h are 2h and 2h + 1, the leaves are h = 2^K .. 2^(K+1) - 1
// (leaf l = h - 2^K; phase 1 for even l, phase 2 for odd l). The parameter
// vector of directions is ordered by level, the deepest first: the node j of
// level k (heap h = 2^(k-1) + j) has the parameter index 2^K - 2^k + j.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/hom.h"

namespace hom {

constexpr int DMN_MAX_K = 10;

struct DmnSchedule {
  double lr_max = 1.5e-2, lr_min = 1.5e-3;  // learning-rate modulation of the paper
  int half_period = 50;                      // M
  double decay = 0.999;                      // gamma
  double q = 10.0, penalty = 1e3;            // loss exponent and mixing penalty
  double beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
};

struct Dmn {
  int K, nleaf, nnode;
  int nparam;  // 3 nnode + nleaf
  double* p = nullptr;  // device parameters: m [nnode][3] then v [nleaf]
  double *a1 = nullptr, *a2 = nullptr, *a2max = nullptr;  // AMSGrad moments
  long long steps = 0;
  std::vector<void*> allocs;

  Dmn(int K, uint64_t seed);
  ~Dmn();
  Dmn(const Dmn&) = delete;
  Dmn& operator=(const Dmn&) = delete;

  void get(double* m, double* v) const;
  void set(const double* m, const double* v);
  // C1, C2, Cout: host [n][36] (Mandel, row-major)
  void homogenize(long long n, const double* C1, const double* C2, double* Cout);
  // loss of all n samples as one batch and its gradients (host gm [nnode][3], gv [nleaf])
  double loss_grad(long long n, const double* C1, const double* C2, const double* Cb, double* gm, double* gv,
                   const DmnSchedule& sc);
  void train(long long n, const double* C1, const double* C2, const double* Cb, int epochs, int batch,
             uint64_t seed, double* loss_hist, const DmnSchedule& sc);
};

// Online evaluation over many macroscopic points with the two phase laws.
struct DmnOnline;
DmnOnline* dmn_online_create(const Dmn& net, const hom_law* laws, int npoints, double tol, int maxit);
void dmn_online_destroy(DmnOnline* o);
void dmn_online_set_predictor(DmnOnline* o, int on);
void dmn_online_step(DmnOnline* o, const double* strain, const double* theta, const double* dt, int what,
                     int trial, hom_dmn_result* out);

}  // namespace hom
