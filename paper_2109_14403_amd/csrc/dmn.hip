// Direct deep material network (see dmn.h): offline training kernels and
// the online evaluation of many macroscopic points.
//
// Laminate of two phases with stiffnesses C1, C2, fractions c1, c2 = 1 - c1
// and normal n (the exact laminate rule; the paper writes it with the
// auxiliary parameter lambda of Sec. 3.2, which gives the same stiffness):
// the phase strains are eps1 = eps + c2 N a, eps2 = eps - c1 N a with
// N a = sym(a (x) n) (Mandel, 6 x 3), the jump a makes the traction
// continuous, N^T (sigma1 - sigma2) = 0, so
//   M = N^T (c2 C1 + c1 C2) N,  a = -M^-1 N^T (C1 - C2) eps,
//   C = c1 C1 + c2 C2 - c1 c2 (C1 - C2) N M^-1 N^T (C1 - C2).
// The online Newton step eliminates the jumps of the whole tree the same way,
// from the leaves to the root, with each subtree's condensed tangent and
// stress offset: one 3 x 3 solve per laminate instead of the dense system.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <random>
#include <string>

#include "dmn.h"
#include "pa66.h"
#include "pipeline.h"
#include "runtime.h"

namespace hom {

namespace {

constexpr double SQ2H = 0.70710678118654752440;  // sqrt(2) / 2

// N (6 x 3, Mandel) of a -> sym(a (x) n)
__device__ __forceinline__ void nmat(const double* n, double N[6][3]) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) N[i][k] = 0.0;
  N[0][0] = n[0];
  N[1][1] = n[1];
  N[2][2] = n[2];
  N[3][1] = SQ2H * n[2];
  N[3][2] = SQ2H * n[1];
  N[4][0] = SQ2H * n[2];
  N[4][2] = SQ2H * n[0];
  N[5][0] = SQ2H * n[1];
  N[5][1] = SQ2H * n[0];
}

// adjoint of N with respect to n
__device__ __forceinline__ void nmat_adj(const double Nb[6][3], double* nb) {
  nb[0] = Nb[0][0] + SQ2H * (Nb[4][2] + Nb[5][1]);
  nb[1] = Nb[1][1] + SQ2H * (Nb[3][2] + Nb[5][0]);
  nb[2] = Nb[2][2] + SQ2H * (Nb[3][1] + Nb[4][0]);
}

// inverse of a 3 x 3 matrix by the adjugate; false if singular
__device__ __forceinline__ bool inv3(const double M[3][3], double R[3][3]) {
  const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) scale = fmax(scale, fabs(M[i][j]));
  if (!(fabs(det) > 1e-13 * scale * scale * scale)) return false;
  const double id = 1.0 / det;
  R[0][0] = c00 * id;
  R[1][0] = c01 * id;
  R[2][0] = c02 * id;
  R[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
  R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
  R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
  R[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
  R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
  R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
  return true;
}

__device__ __forceinline__ void unit(const double* m, double* n, double& len) {
  len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  const double il = len > 0.0 ? 1.0 / len : 0.0;
  n[0] = m[0] * il;
  n[1] = m[1] * il;
  n[2] = m[2] * il;
}

// parameter index of the direction of heap node h at depth level k (2^(k-1) <= h < 2^k)
__device__ __forceinline__ int param_of(int h, int nleaf) {
  const int cnt = 1 << (31 - __clz(h));  // 2^(k-1)
  return nleaf - 2 * cnt + (h - cnt);
}

// ---------------------------------------------------------------------------
// offline: laminate forward and backward
// ---------------------------------------------------------------------------
__device__ void lam_fwd(const double* C1, const double* C2, double c1, const double* n, double* C) {
  const double c2 = 1.0 - c1;
  double N[6][3];
  nmat(n, N);
  double G[6][3], HN[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double g = 0.0, h = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const double a = C1[6 * i + j], b = C2[6 * i + j];
        g += (a - b) * N[j][k];
        h += (c2 * a + c1 * b) * N[j][k];
      }
      G[i][k] = g;
      HN[i][k] = h;
    }
  double M[3][3], Mi[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) s += N[i][k] * HN[i][l];
      M[k][l] = s;
    }
  if (!inv3(M, Mi)) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) Mi[k][l] = 0.0;
  }
  double GM[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) GM[i][k] = G[i][0] * Mi[0][k] + G[i][1] * Mi[1][k] + G[i][2] * Mi[2][k];
  const double cc = c1 * c2;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      C[6 * i + j] = c1 * C1[6 * i + j] + c2 * C2[6 * i + j] -
                     cc * (GM[i][0] * G[j][0] + GM[i][1] * G[j][1] + GM[i][2] * G[j][2]);
}

// Reverse mode of lam_fwd: given Cb = dJ/dC, writes dJ/dC1, dJ/dC2 (if the
// pointers are non-null), dJ/dc1 and dJ/dn.
__device__ void lam_bwd(const double* C1, const double* C2, double c1, const double* n, const double* Cb,
                        double* C1b, double* C2b, double& c1b, double* nb) {
  const double c2 = 1.0 - c1;
  const double cc = c1 * c2;
  double N[6][3];
  nmat(n, N);
  double G[6][3], HN[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double g = 0.0, h = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const double a = C1[6 * i + j], b = C2[6 * i + j];
        g += (a - b) * N[j][k];
        h += (c2 * a + c1 * b) * N[j][k];
      }
      G[i][k] = g;
      HN[i][k] = h;
    }
  double M[3][3], Mi[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) s += N[i][k] * HN[i][l];
      M[k][l] = s;
    }
  if (!inv3(M, Mi)) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) Mi[k][l] = 0.0;
  }
  double GM[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) GM[i][k] = G[i][0] * Mi[0][k] + G[i][1] * Mi[1][k] + G[i][2] * Mi[2][k];
  // C = c1 C1 + c2 C2 - cc X, X = G Mi G^T
  double dx = 0.0, dd = 0.0;  // <Cb, X>, <Cb, C1 - C2>
  double Gb[6][3];            // dJ/dG = -cc (Cb + Cb^T) G Mi
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Gb[i][k] = 0.0;
  double Mib[3][3];           // dJ/dMi = -cc G^T Cb G
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Mib[k][l] = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      const double cb = Cb[6 * i + j];
      const double cbs = cb + Cb[6 * j + i];
      dx += cb * (GM[i][0] * G[j][0] + GM[i][1] * G[j][1] + GM[i][2] * G[j][2]);
      dd += cb * (C1[6 * i + j] - C2[6 * i + j]);
#pragma unroll
      for (int k = 0; k < 3; ++k) Gb[i][k] -= cc * cbs * GM[j][k];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) Mib[k][l] -= cc * G[i][k] * cb * G[j][l];
    }
  // Mi = M^-1: Mb = -Mi Mib Mi (Mi symmetric)
  double T[3][3], Mb[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) T[k][l] = Mib[k][0] * Mi[0][l] + Mib[k][1] * Mi[1][l] + Mib[k][2] * Mi[2][l];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Mb[k][l] = -(Mi[k][0] * T[0][l] + Mi[k][1] * T[1][l] + Mi[k][2] * T[2][l]);
  // M = N^T H N, H = c2 C1 + c1 C2: Hb = N Mb N^T, Nb = HN (Mb + Mb^T)
  double Nb[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) s += HN[i][l] * (Mb[k][l] + Mb[l][k]);
      Nb[i][k] = s;
    }
  // G = (C1 - C2) N: Nb += (C1 - C2)^T Gb, (C1 - C2)b = Gb N^T
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int i = 0; i < 6; ++i) s += (C1[6 * i + j] - C2[6 * i + j]) * Gb[i][k];
      Nb[j][k] += s;
    }
  double dh = 0.0;  // <Hb, C2 - C1>
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double hb = 0.0, db = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        db += Gb[i][k] * N[j][k];
#pragma unroll
        for (int l = 0; l < 3; ++l) hb += N[i][k] * Mb[k][l] * N[j][l];
      }
      dh += hb * (C2[6 * i + j] - C1[6 * i + j]);
      const double cb = Cb[6 * i + j];
      if (C1b) C1b[6 * i + j] = c1 * cb + c2 * hb + db;
      if (C2b) C2b[6 * i + j] = c2 * cb + c1 * hb - db;
    }
  c1b = dd - (1.0 - 2.0 * c1) * dx + dh;
  nmat_adj(Nb, nb);
}

struct OffArgs {
  int K, nleaf;
  const double* p;     // m [nnode][3], v [nleaf]
  const double* C1;    // [S][36]
  const double* C2;
  const double* Cb;    // [S][36] targets, or null
  const int* idx;      // [B] sample of each block, or null (block = sample)
  double* Cnode;       // [B][nleaf][36] (heap index 1 .. nleaf - 1)
  double* D;           // [B][36] prediction, or null
  double* err;         // [B] relative l1 errors, or null
  double* Cadj;        // [B][nleaf][36] adjoints (backward)
  double* grad;        // [B][nparam] per-sample gradients (backward)
  int B;
  double q;
};

// subtree weights, heap order, in LDS
__device__ void subtree_weights(const OffArgs& a, double* wsub) {
  const int nleaf = a.nleaf;
  const double* v = a.p + 3 * (nleaf - 1);
  for (int l = threadIdx.x; l < nleaf; l += blockDim.x) wsub[nleaf + l] = fmax(v[l], 0.0);
  __syncthreads();
  for (int cnt = nleaf >> 1; cnt >= 1; cnt >>= 1) {
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) wsub[cnt + j] = wsub[2 * (cnt + j)] + wsub[2 * (cnt + j) + 1];
    __syncthreads();
  }
}

__device__ __forceinline__ const double* child_C(const OffArgs& a, int s, int sample, int h) {
  if (h >= a.nleaf) {
    const int l = h - a.nleaf;
    return ((l & 1) ? a.C2 : a.C1) + (long long)sample * 36;
  }
  return a.Cnode + ((long long)s * a.nleaf + h) * 36;
}

__global__ void __launch_bounds__(512) k_dmn_fwd(OffArgs a) {
  __shared__ double wsub[2 * (1 << DMN_MAX_K)];
  const int s = blockIdx.x;
  const int sample = a.idx ? a.idx[s] : s;
  subtree_weights(a, wsub);
  for (int cnt = a.nleaf >> 1; cnt >= 1; cnt >>= 1) {
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      const double wl = wsub[2 * h], wr = wsub[2 * h + 1], sw = wl + wr;
      const double c1 = sw > 0.0 ? wl / sw : 0.5;
      double n[3], len;
      unit(a.p + 3 * param_of(h, a.nleaf), n, len);
      lam_fwd(child_C(a, s, sample, 2 * h), child_C(a, s, sample, 2 * h + 1), c1, n,
              a.Cnode + ((long long)s * a.nleaf + h) * 36);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* C = a.Cnode + ((long long)s * a.nleaf + 1) * 36;
    if (a.D)
      for (int i = 0; i < 36; ++i) a.D[(long long)s * 36 + i] = C[i];
    if (a.err && a.Cb) {
      const double* T = a.Cb + (long long)sample * 36;
      double num = 0.0, den = 0.0;
      for (int i = 0; i < 36; ++i) {
        num += fabs(T[i] - C[i]);
        den += fabs(T[i]);
      }
      a.err[s] = num / den;
    }
  }
}

// per-sample gradient of J1 = (1/B) (sum_s e_s^q)^(1/q) with respect to all parameters
__global__ void __launch_bounds__(512) k_dmn_bwd(OffArgs a) {
  __shared__ double wsub[2 * (1 << DMN_MAX_K)];
  __shared__ double wbar[2 * (1 << DMN_MAX_K)];
  const int s = blockIdx.x;
  const int sample = a.idx ? a.idx[s] : s;
  const int nleaf = a.nleaf;
  subtree_weights(a, wsub);
  double* grad = a.grad + (long long)s * (3 * (nleaf - 1) + nleaf);
  if (threadIdx.x == 0) {
    double sq = 0.0;
    for (int b = 0; b < a.B; ++b) sq += pow(a.err[b], a.q);
    const double e = a.err[s];
    // dJ1/de_s = (1/B) (sum e^q)^(1/q - 1) e_s^(q - 1)
    const double f = sq > 0.0 ? pow(sq, 1.0 / a.q - 1.0) * pow(e, a.q - 1.0) / a.B : 0.0;
    const double* T = a.Cb + (long long)sample * 36;
    const double* C = a.Cnode + ((long long)s * nleaf + 1) * 36;
    double den = 0.0;
    for (int i = 0; i < 36; ++i) den += fabs(T[i]);
    double* R = a.Cadj + ((long long)s * nleaf + 1) * 36;
    for (int i = 0; i < 36; ++i) {
      const double d = T[i] - C[i];
      R[i] = d > 0.0 ? -f / den : (d < 0.0 ? f / den : 0.0);
    }
    wbar[1] = 0.0;  // the mixing penalty is added once per batch by the update kernel
  }
  __syncthreads();
  for (int cnt = 1; cnt < nleaf; cnt <<= 1) {
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      const double wl = wsub[2 * h], wr = wsub[2 * h + 1], sw = wl + wr;
      const double c1 = sw > 0.0 ? wl / sw : 0.5;
      const int pi = param_of(h, nleaf);
      double n[3], len;
      unit(a.p + 3 * pi, n, len);
      const bool inner = 2 * h < nleaf;
      double c1b, nb[3];
      lam_bwd(child_C(a, s, sample, 2 * h), child_C(a, s, sample, 2 * h + 1), c1, n,
              a.Cadj + ((long long)s * nleaf + h) * 36,
              inner ? a.Cadj + ((long long)s * nleaf + 2 * h) * 36 : nullptr,
              inner ? a.Cadj + ((long long)s * nleaf + 2 * h + 1) * 36 : nullptr, c1b, nb);
      // n = m / |m|
      const double dn = nb[0] * n[0] + nb[1] * n[1] + nb[2] * n[2];
      const double il = len > 0.0 ? 1.0 / len : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) grad[3 * pi + k] = (nb[k] - dn * n[k]) * il;
      // c1 = wl / (wl + wr); the node weight wl + wr passes its adjoint down
      double gl = wbar[h], gr = wbar[h];
      if (sw > 0.0) {
        gl += c1b * wr / (sw * sw);
        gr -= c1b * wl / (sw * sw);
      }
      wbar[2 * h] = gl;
      wbar[2 * h + 1] = gr;
    }
    __syncthreads();
  }
  const double* v = a.p + 3 * (nleaf - 1);
  for (int l = threadIdx.x; l < nleaf; l += blockDim.x)
    grad[3 * (nleaf - 1) + l] = v[l] > 0.0 ? wbar[nleaf + l] : 0.0;
}

struct StepArgs {
  int nparam, nnode, nleaf, B;
  double* p;
  double *a1, *a2, *a2max;
  const double* grad;   // [B][nparam]
  const double* err;    // [B]
  double* gout;         // [nparam] summed gradient (or null)
  double* loss;         // loss of this batch (or null)
  double* loss_acc;     // accumulated batch losses (or null)
  double lr, q, penalty, beta1, beta2, eps;
  long long t;          // step number (1-based), for the bias corrections
  int update;
};

// sum of the per-sample gradients (fixed order) plus the mixing penalty,
// loss value, AMSGrad update
__global__ void __launch_bounds__(1024) k_dmn_step(StepArgs a) {
  __shared__ double red[32];
  __shared__ double wsum;
  const double* v = a.p + 3 * a.nnode;
  double part = 0.0;
  for (int l = threadIdx.x; l < a.nleaf; l += blockDim.x) part += fmax(v[l], 0.0);
  double r[1] = {part};
  block_sum<1>(r, red);
  if (threadIdx.x == 0) {
    wsum = r[0];
    if (a.loss || a.loss_acc) {
      double sq = 0.0;
      for (int b = 0; b < a.B; ++b) sq += pow(a.err[b], a.q);
      const double J = pow(sq, 1.0 / a.q) / a.B + a.penalty * (r[0] - 1.0) * (r[0] - 1.0);
      if (a.loss) *a.loss = J;
      if (a.loss_acc) *a.loss_acc += J;
    }
  }
  __syncthreads();
  const double pen = 2.0 * a.penalty * (wsum - 1.0);
  const double bc1 = 1.0 - pow(a.beta1, (double)a.t), bc2 = 1.0 - pow(a.beta2, (double)a.t);
  for (int i = threadIdx.x; i < a.nparam; i += blockDim.x) {
    double g = 0.0;
    for (int b = 0; b < a.B; ++b) g += a.grad[(long long)b * a.nparam + i];
    if (i >= 3 * a.nnode && v[i - 3 * a.nnode] > 0.0) g += pen;
    if (a.gout) a.gout[i] = g;
    if (!a.update) continue;
    const double m1 = a.beta1 * a.a1[i] + (1.0 - a.beta1) * g;
    const double m2 = a.beta2 * a.a2[i] + (1.0 - a.beta2) * g * g;
    const double mx = fmax(a.a2max[i], m2);
    a.a1[i] = m1;
    a.a2[i] = m2;
    a.a2max[i] = mx;
    a.p[i] -= a.lr * (m1 / bc1) / (sqrt(mx / bc2) + a.eps);
  }
}

template <typename U>
U* dalloc_into(std::vector<void*>& allocs, size_t count) {
  void* ptr = nullptr;
  hip_check(hipMalloc(&ptr, count * sizeof(U) + 256), "hipMalloc");
  allocs.push_back(ptr);
  hip_check(hipMemset(ptr, 0, count * sizeof(U)), "hipMemset");
  return static_cast<U*>(ptr);
}

int threads_for(int nleaf) { return std::min(512, std::max(64, nleaf / 2)); }

}  // namespace

// ---------------------------------------------------------------------------
// Dmn host object
// ---------------------------------------------------------------------------
Dmn::Dmn(int K_, uint64_t seed) : K(K_) {
  if (K < 1 || K > DMN_MAX_K) fail(HOM_E_ARG, "DMN depth must be in [1, 10]");
  nleaf = 1 << K;
  nnode = nleaf - 1;
  nparam = 3 * nnode + nleaf;
  p = dalloc_into<double>(allocs, nparam);
  a1 = dalloc_into<double>(allocs, nparam);
  a2 = dalloc_into<double>(allocs, nparam);
  a2max = dalloc_into<double>(allocs, nparam);
  // directions uniform on the unit sphere, weights uniform on [0, 1] rescaled
  // to sum to one (the paper's initialization)
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::uniform_real_distribution<double> ud(0.0, 1.0);
  std::vector<double> h(nparam);
  for (int i = 0; i < nnode; ++i) {
    double x, y, z, r;
    do {
      x = nd(rng);
      y = nd(rng);
      z = nd(rng);
      r = std::sqrt(x * x + y * y + z * z);
    } while (r < 1e-12);
    h[3 * i] = x / r;
    h[3 * i + 1] = y / r;
    h[3 * i + 2] = z / r;
  }
  double sw = 0.0;
  for (int l = 0; l < nleaf; ++l) sw += (h[3 * nnode + l] = ud(rng));
  for (int l = 0; l < nleaf; ++l) h[3 * nnode + l] /= sw;
  hip_check(hipMemcpy(p, h.data(), nparam * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
}

Dmn::~Dmn() {
  for (void* ptr : allocs) (void)hipFree(ptr);
}

void Dmn::get(double* m, double* v) const {
  std::vector<double> h(nparam);
  hip_check(hipMemcpy(h.data(), p, nparam * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  if (m) std::memcpy(m, h.data(), 3 * nnode * sizeof(double));
  if (v) std::memcpy(v, h.data() + 3 * nnode, nleaf * sizeof(double));
}

void Dmn::set(const double* m, const double* v) {
  std::vector<double> h(nparam);
  get(h.data(), h.data() + 3 * nnode);
  if (m) std::memcpy(h.data(), m, 3 * nnode * sizeof(double));
  if (v) std::memcpy(h.data() + 3 * nnode, v, nleaf * sizeof(double));
  for (int i = 0; i < nnode; ++i)
    if (!(h[3 * i] * h[3 * i] + h[3 * i + 1] * h[3 * i + 1] + h[3 * i + 2] * h[3 * i + 2] > 0.0))
      fail(HOM_E_ARG, "direction " + std::to_string(i) + " is zero");
  for (double x : h)
    if (!std::isfinite(x)) fail(HOM_E_ARG, "parameters must be finite");
  hip_check(hipMemcpy(p, h.data(), nparam * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
  steps = 0;
  hip_check(hipMemset(a1, 0, nparam * sizeof(double)), "hipMemset");
  hip_check(hipMemset(a2, 0, nparam * sizeof(double)), "hipMemset");
  hip_check(hipMemset(a2max, 0, nparam * sizeof(double)), "hipMemset");
}

namespace {
void check_samples(long long n, const double* C1, const double* C2) {
  if (n < 1) fail(HOM_E_ARG, "need at least one sample");
  if (!C1 || !C2) fail(HOM_E_ARG, "null stiffness array");
  for (long long i = 0; i < 36 * n; ++i)
    if (!std::isfinite(C1[i]) || !std::isfinite(C2[i])) fail(HOM_E_ARG, "stiffnesses must be finite");
}

struct DevSamples {
  std::vector<void*> allocs;
  double *C1 = nullptr, *C2 = nullptr, *Cb = nullptr;
  DevSamples(long long n, const double* c1, const double* c2, const double* cb) {
    C1 = dalloc_into<double>(allocs, 36 * n);
    C2 = dalloc_into<double>(allocs, 36 * n);
    hip_check(hipMemcpy(C1, c1, 36 * n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    hip_check(hipMemcpy(C2, c2, 36 * n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    if (cb) {
      Cb = dalloc_into<double>(allocs, 36 * n);
      hip_check(hipMemcpy(Cb, cb, 36 * n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    }
  }
  ~DevSamples() {
    for (void* p : allocs) (void)hipFree(p);
  }
};
}  // namespace

void Dmn::homogenize(long long n, const double* C1, const double* C2, double* Cout) {
  check_samples(n, C1, C2);
  if (!Cout) fail(HOM_E_ARG, "null output");
  DevSamples d(n, C1, C2, nullptr);
  std::vector<void*> tmp;
  OffArgs a{};
  a.K = K;
  a.nleaf = nleaf;
  a.p = p;
  a.C1 = d.C1;
  a.C2 = d.C2;
  a.Cnode = dalloc_into<double>(tmp, (size_t)n * nleaf * 36);
  a.D = dalloc_into<double>(tmp, (size_t)n * 36);
  a.B = (int)n;
  hipLaunchKernelGGL(k_dmn_fwd, dim3((unsigned)n), dim3(threads_for(nleaf)), 0, nullptr, a);
  hip_check(hipGetLastError(), "k_dmn_fwd");
  hip_check(hipMemcpy(Cout, a.D, 36 * n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  for (void* ptr : tmp) (void)hipFree(ptr);
}

double Dmn::loss_grad(long long n, const double* C1, const double* C2, const double* Cb, double* gm, double* gv,
                      const DmnSchedule& sc) {
  check_samples(n, C1, C2);
  if (!Cb) fail(HOM_E_ARG, "null targets");
  DevSamples d(n, C1, C2, Cb);
  std::vector<void*> tmp;
  OffArgs a{};
  a.K = K;
  a.nleaf = nleaf;
  a.p = p;
  a.C1 = d.C1;
  a.C2 = d.C2;
  a.Cb = d.Cb;
  a.Cnode = dalloc_into<double>(tmp, (size_t)n * nleaf * 36);
  a.Cadj = dalloc_into<double>(tmp, (size_t)n * nleaf * 36);
  a.err = dalloc_into<double>(tmp, n);
  a.grad = dalloc_into<double>(tmp, (size_t)n * nparam);
  a.B = (int)n;
  a.q = sc.q;
  hipLaunchKernelGGL(k_dmn_fwd, dim3((unsigned)n), dim3(threads_for(nleaf)), 0, nullptr, a);
  hipLaunchKernelGGL(k_dmn_bwd, dim3((unsigned)n), dim3(threads_for(nleaf)), 0, nullptr, a);
  StepArgs s{};
  s.nparam = nparam;
  s.nnode = nnode;
  s.nleaf = nleaf;
  s.B = (int)n;
  s.p = p;
  s.grad = a.grad;
  s.err = a.err;
  s.gout = dalloc_into<double>(tmp, nparam);
  s.loss = dalloc_into<double>(tmp, 1);
  s.q = sc.q;
  s.penalty = sc.penalty;
  s.t = 1;
  s.update = 0;
  s.beta1 = sc.beta1;
  s.beta2 = sc.beta2;
  hipLaunchKernelGGL(k_dmn_step, dim3(1), dim3(1024), 0, nullptr, s);
  hip_check(hipGetLastError(), "dmn kernels");
  std::vector<double> g(nparam);
  double J = 0.0;
  hip_check(hipMemcpy(g.data(), s.gout, nparam * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  hip_check(hipMemcpy(&J, s.loss, sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  if (gm) std::memcpy(gm, g.data(), 3 * nnode * sizeof(double));
  if (gv) std::memcpy(gv, g.data() + 3 * nnode, nleaf * sizeof(double));
  for (void* ptr : tmp) (void)hipFree(ptr);
  return J;
}

void Dmn::train(long long n, const double* C1, const double* C2, const double* Cb, int epochs, int batch,
                uint64_t seed, double* loss_hist, const DmnSchedule& sc) {
  check_samples(n, C1, C2);
  if (!Cb) fail(HOM_E_ARG, "null targets");
  if (batch < 1 || batch > n) fail(HOM_E_ARG, "batch must be in [1, n]");
  if (epochs < 0) fail(HOM_E_ARG, "epochs must be >= 0");
  DevSamples d(n, C1, C2, Cb);
  std::vector<void*> tmp;
  OffArgs a{};
  a.K = K;
  a.nleaf = nleaf;
  a.p = p;
  a.C1 = d.C1;
  a.C2 = d.C2;
  a.Cb = d.Cb;
  a.Cnode = dalloc_into<double>(tmp, (size_t)batch * nleaf * 36);
  a.Cadj = dalloc_into<double>(tmp, (size_t)batch * nleaf * 36);
  a.err = dalloc_into<double>(tmp, batch);
  a.grad = dalloc_into<double>(tmp, (size_t)batch * nparam);
  a.B = batch;
  a.q = sc.q;
  const long long nb = n / batch;  // incomplete batches are dropped
  int* idx = dalloc_into<int>(tmp, (size_t)nb * batch);
  double* lacc = dalloc_into<double>(tmp, std::max(epochs, 1));
  std::vector<int> perm(n);
  std::mt19937_64 rng(seed);
  StepArgs s{};
  s.nparam = nparam;
  s.nnode = nnode;
  s.nleaf = nleaf;
  s.B = batch;
  s.p = p;
  s.a1 = a1;
  s.a2 = a2;
  s.a2max = a2max;
  s.grad = a.grad;
  s.err = a.err;
  s.q = sc.q;
  s.penalty = sc.penalty;
  s.beta1 = sc.beta1;
  s.beta2 = sc.beta2;
  s.eps = sc.eps;
  s.update = 1;
  const double pi = 3.14159265358979323846;
  for (int e = 0; e < epochs; ++e) {
    for (long long i = 0; i < n; ++i) perm[i] = (int)i;
    std::shuffle(perm.begin(), perm.end(), rng);
    hip_check(hipMemcpy(idx, perm.data(), nb * batch * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
    // harmonic modulation with geometric decay (the paper's warm restarts)
    s.lr = std::pow(sc.decay, e) *
           (sc.lr_min + 0.5 * (sc.lr_max - sc.lr_min) * (1.0 + std::cos(pi * e / sc.half_period)));
    s.loss_acc = lacc + e;
    for (long long b = 0; b < nb; ++b) {
      a.idx = idx + b * batch;
      hipLaunchKernelGGL(k_dmn_fwd, dim3(batch), dim3(threads_for(nleaf)), 0, nullptr, a);
      hipLaunchKernelGGL(k_dmn_bwd, dim3(batch), dim3(threads_for(nleaf)), 0, nullptr, a);
      s.t = ++steps;
      hipLaunchKernelGGL(k_dmn_step, dim3(1), dim3(1024), 0, nullptr, s);
    }
    hip_check(hipGetLastError(), "dmn training kernels");
  }
  hip_check(hipDeviceSynchronize(), "dmn training");
  if (loss_hist && epochs > 0) {
    hip_check(hipMemcpy(loss_hist, lacc, epochs * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
    for (int e = 0; e < epochs; ++e) loss_hist[e] /= (double)nb;
  }
  for (void* ptr : tmp) (void)hipFree(ptr);
}

// ---------------------------------------------------------------------------
// online evaluation
// ---------------------------------------------------------------------------
namespace {

constexpr int ON_MAX_K = 8;
// per point: sigma 6, coupling, dissipation, dsde 36, dsdt 6, dDde 6, dDdt,
// residual, iterations, status
constexpr int ON_OUT = 64;
constexpr int O_DSDT = 44, O_DDDE = 50, O_DDDT = 56, O_RES = 57, O_IT = 58, O_ST = 59;
constexpr int ON_SCR = 24;  // per internal node: G (18), da0 (3)

struct OnArgs {
  int K, nleaf;
  const double* p;
  const ProbInc* inc;   // [point]
  const ProbInc* inc_pm;  // [point][2]: theta + h_theta, theta - h_theta (all four tangents)
  int what;             // 1: also the temperature and coupling tangents
  int trial;            // 1: never commit
  int pa_phase;         // phase (0: even leaves, 1: odd leaves) with the PA66 law, -1 if none
  double* state;        // [point][nstate][nleaf / 2]
  int nstate;
  double* hist;         // [point][HIST_SLOTS][nleaf / 2]
  double* epsn;         // [point][nleaf][6]
  double* a;            // [point][nleaf][3] jumps (heap index)
  double* scr;          // [point][nleaf][ON_SCR]
  const double* E;      // [point][6] Mandel
  double* out;          // [point][ON_OUT]
  double tol, gamma;
  int maxit, maxbt;
};

struct OnShared {
  double wsub[2 << ON_MAX_K];
  double nv[(1 << ON_MAX_K) * 3];  // unit directions, heap index
  double V[(2 << ON_MAX_K) * 6];   // strains (top-down) / weighted stress sums (bottom-up)
  double KA[(1 << ON_MAX_K) * 36]; // condensed tangents, children level
  double KB[(1 << (ON_MAX_K - 1)) * 36];
  double da[(1 << ON_MAX_K) * 3];  // Newton step of the jumps (heap index)
  double red[16 * 2];
  double res;
};

// leaf law: stress and compressed tangent 3K P1 + ca P2 + cb N N
__device__ void leaf_eval(const OnArgs& g, const ProbInc& in, int pt, int l, const double* e, double* sg,
                          double& K3, double& ca, double& cb, double* nd) {
  const int phase = l & 1;
  const PhaseInc& pi = in.ph[phase];
  if (phase == g.pa_phase) {
    const int q = l >> 1;
    const long long ss = g.nleaf >> 1;
    const double* st = g.state + (long long)pt * g.nstate * ss + q;
    double* hs = g.hist + (long long)pt * HIST_SLOTS * ss + q;
    PaOut o;
    pa66_point(in, e, st, ss, nullptr, nullptr, o, nullptr, nullptr, hs, hs + 7 * ss);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      sg[c] = o.sig[c];
      nd[c] = o.nd[c];
    }
    K3 = pi.K3;
    ca = o.a;
    cb = o.b;
  } else {
    const double tr3 = (e[0] + e[1] + e[2]) * (1.0 / 3.0);
    const double sph = pi.K3 * (tr3 - pi.alpha_dth) - pi.G2 * tr3;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      sg[c] = pi.G2 * e[c] + (c < 3 ? sph : 0.0);
      nd[c] = 0.0;
    }
    K3 = pi.K3;
    ca = pi.G2;
    cb = 0.0;
  }
}

// w C of a leaf into KA: C_IJ = ca d_IJ + (K3 - ca) / 3 [I, J < 3] + cb N_I N_J
__device__ __forceinline__ void put_leaf_tangent(OnShared& S, int l, double w, double K3, double ca, double cb,
                                                 const double* nd) {
  double* Kl = S.KA + 36 * l;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      Kl[6 * i + j] = w * ((i == j ? ca : 0.0) + (i < 3 && j < 3 ? (K3 - ca) * (1.0 / 3.0) : 0.0) + cb * nd[i] * nd[j]);
}

__device__ __forceinline__ double node_c1(const OnShared& S, int h) {
  const double wl = S.wsub[2 * h], wr = S.wsub[2 * h + 1], sw = wl + wr;
  return sw > 0.0 ? wl / sw : 0.5;
}

// Residual at the jumps a (block-wide): leaf strains top-down, leaf laws,
// weighted stress sums bottom-up, |A^T W sigma| / ((2^K - 1) |sigma_bar|).
// Leaves keep their strain, stress and w C (in KA) for the Newton step.
__device__ double residual(const OnArgs& g, OnShared& S, const ProbInc& in, int pt, const double* a, double* e,
                           double* sg) {
  const int nleaf = g.nleaf;
  const int tid = threadIdx.x;
  if (tid == 0)
    for (int c = 0; c < 6; ++c) S.V[6 + c] = g.E[6 * pt + c];
  __syncthreads();
  for (int cnt = 1; cnt < nleaf; cnt <<= 1) {
    for (int j = tid; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      const double c1 = node_c1(S, h), c2 = 1.0 - c1;
      double N[6][3];
      nmat(S.nv + 3 * h, N);
      const double* ah = a + 3 * h;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double j6 = N[c][0] * ah[0] + N[c][1] * ah[1] + N[c][2] * ah[2];
        S.V[6 * (2 * h) + c] = S.V[6 * h + c] + c2 * j6;
        S.V[6 * (2 * h + 1) + c] = S.V[6 * h + c] - c1 * j6;
      }
    }
    __syncthreads();
  }
  const int l = tid;
  const double w = S.wsub[nleaf + l];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = S.V[6 * (nleaf + l) + c];
  double K3, ca, cb, nd[6];
  leaf_eval(g, in, pt, l, e, sg, K3, ca, cb, nd);
  put_leaf_tangent(S, l, w, K3, ca, cb, nd);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 6; ++c) S.V[6 * (nleaf + l) + c] = w * sg[c];
  __syncthreads();
  double gg = 0.0;
  for (int cnt = nleaf >> 1; cnt >= 1; cnt >>= 1) {
    for (int j = tid; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      const double c1 = node_c1(S, h), c2 = 1.0 - c1;
      double N[6][3];
      nmat(S.nv + 3 * h, N);
      const double* s1 = S.V + 6 * (2 * h);
      const double* s2 = S.V + 6 * (2 * h + 1);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double r = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) r += N[c][k] * (c2 * s1[c] - c1 * s2[c]);
        gg += r * r;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) S.V[6 * h + c] = s1[c] + s2[c];
    }
    __syncthreads();
  }
  double r2[1] = {gg};
  block_sum<1>(r2, S.red);
  if (tid == 0) {
    double sb = 0.0;
    for (int c = 0; c < 6; ++c) sb += S.V[6 + c] * S.V[6 + c];
    S.res = sqrt(r2[0]) / ((double)(nleaf - 1) * fmax(sqrt(sb), 1e-300));
  }
  __syncthreads();
  return S.res;
}

// Condensation from the leaves to the root with the leaf tangents in KA and
// the weighted leaf stresses in V: per node G and da0 (scratch) with
// da = da0 + G deps; returns with the root's condensed tangent in the buffer
// it names (KA or KB).
__device__ double* condense(const OnArgs& g, OnShared& S, int pt) {
  const int nleaf = g.nleaf;
  const int tid = threadIdx.x;
  double* src = S.KA;
  double* dst = S.KB;
  double* scr = g.scr + (long long)pt * nleaf * ON_SCR;
  for (int cnt = nleaf >> 1; cnt >= 1; cnt >>= 1) {
    for (int j = tid; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      const double c1 = node_c1(S, h), c2 = 1.0 - c1;
      double N[6][3];
      nmat(S.nv + 3 * h, N);
      const double* K1 = src + 36 * (2 * j);
      const double* K2 = src + 36 * (2 * j + 1);
      const double* s1 = S.V + 6 * (2 * h);
      const double* s2 = S.V + 6 * (2 * h + 1);
      // X = (c2 K1 - c1 K2) N (6 x 3), M = N^T (c2^2 K1 + c1^2 K2) N, r = N^T (c2 s1 - c1 s2)
      double X[6][3], HN[6][3];
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double x = 0.0, hh = 0.0;
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const double k1 = K1[6 * i + q], k2 = K2[6 * i + q];
            x += (c2 * k1 - c1 * k2) * N[q][k];
            hh += (c2 * c2 * k1 + c1 * c1 * k2) * N[q][k];
          }
          X[i][k] = x;
          HN[i][k] = hh;
        }
      double M[3][3], Mi[3][3], r[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double rr = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) rr += N[c][k] * (c2 * s1[c] - c1 * s2[c]);
        r[k] = rr;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          double m = 0.0;
#pragma unroll
          for (int i = 0; i < 6; ++i) m += N[i][k] * HN[i][q];
          M[k][q] = m;
        }
      }
      // a subtree without weight on one side has no say in its jump: it stays
      const bool ok = (c1 * c2 * S.wsub[h] > 0.0) && inv3(M, Mi);
      double Gm[3][6], d0[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        d0[k] = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) Gm[k][i] = 0.0;
      }
      if (ok) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          d0[k] = -(Mi[k][0] * r[0] + Mi[k][1] * r[1] + Mi[k][2] * r[2]);
#pragma unroll
          for (int i = 0; i < 6; ++i) Gm[k][i] = -(Mi[k][0] * X[i][0] + Mi[k][1] * X[i][1] + Mi[k][2] * X[i][2]);
        }
      }
      double* sc = scr + (long long)h * ON_SCR;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sc[18 + k] = d0[k];
#pragma unroll
        for (int i = 0; i < 6; ++i) sc[6 * k + i] = Gm[k][i];
      }
      // parent: s = s1 + s2 + X d0, K = K1 + K2 + X G
      double sp[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) sp[i] = s1[i] + s2[i] + X[i][0] * d0[0] + X[i][1] * d0[1] + X[i][2] * d0[2];
      double* Kp = dst + 36 * j;
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int q = 0; q < 6; ++q)
          Kp[6 * i + q] = K1[6 * i + q] + K2[6 * i + q] + X[i][0] * Gm[0][q] + X[i][1] * Gm[1][q] + X[i][2] * Gm[2][q];
#pragma unroll
      for (int i = 0; i < 6; ++i) S.V[6 * h + i] = sp[i];
    }
    __syncthreads();
    double* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// da from the root down (deps_root = 0), into S.da (heap index); the strain
// changes of every node and leaf into V
__device__ void expand(const OnArgs& g, OnShared& S, int pt) {
  const int nleaf = g.nleaf;
  const int tid = threadIdx.x;
  const double* scr = g.scr + (long long)pt * nleaf * ON_SCR;
  if (tid == 0)
    for (int c = 0; c < 6; ++c) S.V[6 + c] = 0.0;
  __syncthreads();
  for (int cnt = 1; cnt < nleaf; cnt <<= 1) {
    for (int j = tid; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      const double c1 = node_c1(S, h), c2 = 1.0 - c1;
      const double* sc = scr + (long long)h * ON_SCR;
      const double* de = S.V + 6 * h;
      double d[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double x = sc[18 + k];
#pragma unroll
        for (int i = 0; i < 6; ++i) x += sc[6 * k + i] * de[i];
        d[k] = x;
        S.da[3 * h + k] = x;
      }
      double N[6][3];
      nmat(S.nv + 3 * h, N);
#pragma unroll
      for (int c = 0; c < 6; ++c) {  // children, the leaves included
        const double j6 = N[c][0] * d[0] + N[c][1] * d[1] + N[c][2] * d[2];
        S.V[6 * (2 * h) + c] = de[c] + c2 * j6;
        S.V[6 * (2 * h + 1) + c] = de[c] - c1 * j6;
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1 << ON_MAX_K) k_dmn_online(OnArgs g) {
  __shared__ OnShared S;
  const int pt = blockIdx.x;
  const int nleaf = g.nleaf;
  const int tid = threadIdx.x;
  const ProbInc& in = g.inc[pt];
  // weights and directions
  const double* v = g.p + 3 * (nleaf - 1);
  S.wsub[nleaf + tid] = fmax(v[tid], 0.0);
  __syncthreads();
  for (int cnt = nleaf >> 1; cnt >= 1; cnt >>= 1) {
    for (int j = tid; j < cnt; j += blockDim.x) {
      const int h = cnt + j;
      S.wsub[h] = S.wsub[2 * h] + S.wsub[2 * h + 1];
      double len;
      unit(g.p + 3 * param_of(h, nleaf), S.nv + 3 * h, len);
    }
    __syncthreads();
  }
  // branch history sums of the PA66 leaves for this increment
  if ((tid & 1) == g.pa_phase) {
    const long long ss = nleaf >> 1;
    const int q = tid >> 1;
    double hd[6], hs;
    pa66_history(in, g.state + (long long)pt * g.nstate * ss + q, ss, hd, hs);
    double* h = g.hist + (long long)pt * HIST_SLOTS * ss + q;
#pragma unroll
    for (int c = 0; c < 6; ++c) h[c * ss] = hd[c];
    h[6 * ss] = hs;
    h[7 * ss] = -1.0;
  }
  __syncthreads();
  double* a = g.a + (long long)pt * nleaf * 3;  // heap index, jumps of the last increment
  double e[6], sg[6];
  double res = residual(g, S, in, pt, a, e, sg);
  int it = 0;
  for (it = 1; it <= g.maxit; ++it) {
    condense(g, S, pt);
    expand(g, S, pt);
    const double res_old = res;
    for (int h = tid + 1; h < nleaf; h += blockDim.x)
#pragma unroll
      for (int k = 0; k < 3; ++k) a[3 * h + k] += S.da[3 * h + k];
    __syncthreads();
    res = residual(g, S, in, pt, a, e, sg);
    for (int i = 0; i < g.maxbt; ++i) {  // backtracking: steps 1, gamma, gamma^2, ...
      if (res < res_old) break;
      const double cut = pow(g.gamma, (double)i) * (1.0 - g.gamma);
      for (int h = tid + 1; h < nleaf; h += blockDim.x)
#pragma unroll
        for (int k = 0; k < 3; ++k) a[3 * h + k] -= cut * S.da[3 * h + k];
      __syncthreads();
      res = residual(g, S, in, pt, a, e, sg);
    }
    if (res < g.tol) break;
  }
  const bool conv = res < g.tol;
  const bool commit = conv && !g.trial;
  if (it > g.maxit) it = g.maxit;
  // effective stress (V[1] after the last residual), tangent by a final
  // condensation at the converged state
  double* o = g.out + (long long)pt * ON_OUT;
  if (tid == 0)
    for (int c = 0; c < 6; ++c) o[c] = S.V[6 + c];
  __syncthreads();
  double* Kroot = condense(g, S, pt);
  for (int i = tid; i < 36; i += blockDim.x) o[8 + i] = Kroot[i];
  __syncthreads();
  if (g.what) {
    // point partials of every leaf at its converged strain, from state n:
    // d sigma / d theta, d D / d eps, d D / d theta (closed form for the
    // thermoelastic phase, central differences of the PA66 update)
    const int l = tid;
    const int phase = l & 1;
    const double* enp = g.epsn + ((long long)pt * nleaf + l) * 6;
    double en[6], st_[6], gd[6], hd;
#pragma unroll
    for (int c = 0; c < 6; ++c) en[c] = enp[c];
    if (phase == g.pa_phase) {
      const long long ss = nleaf >> 1;
      const int q = l >> 1;
      const double* st = g.state + (long long)pt * g.nstate * ss + q;
      const double* hs = g.hist + (long long)pt * HIST_SLOTS * ss + q;
      double sp[6], Dp = 0.0;
      for (int k = 0; k < 14; ++k) {
        const bool th = k < 2;
        const ProbInc& ik = th ? g.inc_pm[2 * pt + k] : in;
        double ek[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) ek[c] = e[c];
        const int dir = (k - 2) >> 1;
        if (!th) ek[dir] += (k & 1) ? -FD_H_EPS : FD_H_EPS;
        PaOut po;
        double dis, cpl;
        pa66_point(ik, ek, st, ss, nullptr, en, po, &dis, &cpl, th ? nullptr : hs, nullptr);
        if (!(k & 1)) {
#pragma unroll
          for (int c = 0; c < 6; ++c) sp[c] = po.sig[c];
          Dp = cpl;
        } else if (th) {
#pragma unroll
          for (int c = 0; c < 6; ++c) st_[c] = (sp[c] - po.sig[c]) * (0.5 / FD_H_THETA);
          hd = (Dp - cpl) * (0.5 / FD_H_THETA);
        } else {
          gd[dir] = (Dp - cpl) * (0.5 / FD_H_EPS);
        }
      }
    } else {
      const PhaseInc& pi = in.ph[phase];
      const double ca = pi.K3 * pi.alpha0;
      const double trd = (e[0] - en[0]) + (e[1] - en[1]) + (e[2] - en[2]);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        st_[c] = c < 3 ? -ca : 0.0;
        gd[c] = c < 3 ? -in.theta * ca / in.dt : 0.0;
      }
      hd = -ca * trd / in.dt;
    }
    const double wl = S.wsub[nleaf + l];
    double K3, ca, cb, nd[6], sgl[6];
    leaf_eval(g, in, pt, l, e, sgl, K3, ca, cb, nd);
    // d<sigma>/dtheta: the jumps equilibrate the leaf sources w dsigma/dtheta
    put_leaf_tangent(S, l, wl, K3, ca, cb, nd);
#pragma unroll
    for (int c = 0; c < 6; ++c) S.V[6 * (nleaf + l) + c] = wl * st_[c];
    __syncthreads();
    condense(g, S, pt);
    if (tid == 0)
      for (int c = 0; c < 6; ++c) o[O_DSDT + c] = S.V[6 + c];
    __syncthreads();
    expand(g, S, pt);  // the leaf strains' derivatives d eps / d theta
    double dT = wl * hd;
#pragma unroll
    for (int c = 0; c < 6; ++c) dT += wl * gd[c] * S.V[6 * (nleaf + l) + c];
    double r1[1] = {dT};
    block_sum<1>(r1, S.red);
    if (tid == 0) o[O_DDDT] = r1[0];
    __syncthreads();
    // d<D>/dE = sum_l w_l (d eps_l / dE)^T dD/deps_l: the condensed value of
    // the leaf sources w dD/deps (the localization is symmetric in this sense)
    put_leaf_tangent(S, l, wl, K3, ca, cb, nd);
#pragma unroll
    for (int c = 0; c < 6; ++c) S.V[6 * (nleaf + l) + c] = wl * gd[c];
    __syncthreads();
    condense(g, S, pt);
    if (tid == 0)
      for (int c = 0; c < 6; ++c) o[O_DDDE + c] = S.V[6 + c];
    __syncthreads();
  }
  // coupling term and dissipation of every leaf; commit if converged
  double D = 0.0, Dd = 0.0;
  {
    const int l = tid;
    const int phase = l & 1;
    const double* en = g.epsn + ((long long)pt * nleaf + l) * 6;
    if (phase == g.pa_phase) {
      const long long ss = nleaf >> 1;
      const int q = l >> 1;
      double* st = g.state + (long long)pt * g.nstate * ss + q;
      double* hs = g.hist + (long long)pt * HIST_SLOTS * ss + q;
      double enl[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) enl[c] = en[c];
      PaOut po;
      pa66_point(in, e, st, ss, commit ? st : nullptr, enl, po, &Dd, &D, hs, nullptr);
    } else {
      const PhaseInc& pi = in.ph[phase];
      const double trd = (e[0] - en[0]) + (e[1] - en[1]) + (e[2] - en[2]);
      D = -in.theta * pi.K3 * pi.alpha0 * trd / in.dt;
    }
  }
  const double w = S.wsub[nleaf + tid];
  double r2[2] = {w * D, w * Dd};
  block_sum<2>(r2, S.red);
  if (commit) {
    double* en = g.epsn + ((long long)pt * nleaf + tid) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) en[c] = e[c];
  }
  if (tid == 0) {
    o[6] = r2[0];
    o[7] = r2[1];
    o[O_RES] = res;
    o[O_IT] = it;
    o[O_ST] = conv ? 1.0 : 0.0;
  }
}

}  // namespace

struct DmnOnline {
  int K, nleaf, npoints, nstate = 0, pa_phase = -1;
  double tol;
  int maxit;
  std::vector<hom_law> laws;
  std::vector<void*> allocs;
  double *p = nullptr, *state = nullptr, *hist = nullptr, *epsn = nullptr, *a = nullptr, *scr = nullptr;
  double *E = nullptr, *out = nullptr;
  ProbInc *inc = nullptr, *inc_pm = nullptr;
  std::vector<ProbInc> inc_h, inc_pm_h;
  ~DmnOnline() {
    for (void* ptr : allocs) (void)hipFree(ptr);
  }
};

DmnOnline* dmn_online_create(const Dmn& net, const hom_law* laws, int npoints, double tol, int maxit) {
  if (net.K > ON_MAX_K) fail(HOM_E_UNSUPPORTED, "online evaluation supports depths up to 8");
  if (npoints < 1) fail(HOM_E_ARG, "need at least one point");
  if (!(tol > 0.0) || maxit < 1) fail(HOM_E_ARG, "need tol > 0 and maxit >= 1");
  if (!laws) fail(HOM_E_ARG, "null laws");
  validate_laws(laws, 2);
  auto o = std::make_unique<DmnOnline>();
  o->K = net.K;
  o->nleaf = net.nleaf;
  o->npoints = npoints;
  o->tol = tol;
  o->maxit = maxit;
  o->laws.assign(laws, laws + 2);
  for (int i = 0; i < 2; ++i)
    if (laws[i].kind == HOM_LAW_PA66) {
      o->pa_phase = i;
      int nm = 0;
      for (int j = 0; j < laws[i].n_maxwell; ++j) nm += laws[i].E_i[j] > 0.0 ? 1 : 0;
      o->nstate = 7 + 6 * nm;
    }
  const size_t half = (size_t)o->nleaf / 2;
  o->p = dalloc_into<double>(o->allocs, net.nparam);
  hip_check(hipMemcpy(o->p, net.p, net.nparam * sizeof(double), hipMemcpyDeviceToDevice), "hipMemcpy");
  if (o->nstate) {
    o->state = dalloc_into<double>(o->allocs, (size_t)npoints * o->nstate * half);
    o->hist = dalloc_into<double>(o->allocs, (size_t)npoints * HIST_SLOTS * half);
  }
  o->epsn = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * 6);
  o->a = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * 3);
  o->scr = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * ON_SCR);
  o->E = dalloc_into<double>(o->allocs, (size_t)npoints * 6);
  o->out = dalloc_into<double>(o->allocs, (size_t)npoints * ON_OUT);
  o->inc = dalloc_into<ProbInc>(o->allocs, npoints);
  o->inc_pm = dalloc_into<ProbInc>(o->allocs, 2 * (size_t)npoints);
  o->inc_h.resize(npoints);
  o->inc_pm_h.resize(2 * (size_t)npoints);
  return o.release();
}

void dmn_online_destroy(DmnOnline* o) { delete o; }

void dmn_online_step(DmnOnline* o, const double* strain, const double* theta, const double* dt, int what,
                     int trial, hom_dmn_result* res) {
  if (what != 0 && what != 1) fail(HOM_E_ARG, "what must be 0 (d sigma / dE) or 1 (all four tangents)");
  if (trial != 0 && trial != 1) fail(HOM_E_ARG, "trial must be 0 or 1");
  const int n = o->npoints;
  const double sq2 = std::sqrt(2.0);
  const double w[6] = {1, 1, 1, sq2, sq2, sq2};
  std::vector<double> E(6 * n);
  for (int i = 0; i < n; ++i) {
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) fail(HOM_E_ARG, "dt must be positive and finite");
    if (!(theta[i] > 0.0) || !std::isfinite(theta[i])) fail(HOM_E_ARG, "theta must be positive");
    for (int c = 0; c < 6; ++c) {
      if (!std::isfinite(strain[6 * i + c])) fail(HOM_E_ARG, "macro strain must be finite");
      E[6 * i + c] = w[c] * strain[6 * i + c];
    }
    fill_inc(o->inc_h[i], o->laws, theta[i], dt[i]);
    if (what) {
      fill_inc(o->inc_pm_h[2 * i], o->laws, theta[i] + FD_H_THETA, dt[i]);
      fill_inc(o->inc_pm_h[2 * i + 1], o->laws, theta[i] - FD_H_THETA, dt[i]);
    }
  }
  if (what)
    hip_check(hipMemcpy(o->inc_pm, o->inc_pm_h.data(), 2 * n * sizeof(ProbInc), hipMemcpyHostToDevice),
              "hipMemcpy");
  hip_check(hipMemcpy(o->E, E.data(), 6 * n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
  hip_check(hipMemcpy(o->inc, o->inc_h.data(), n * sizeof(ProbInc), hipMemcpyHostToDevice), "hipMemcpy");
  OnArgs g{};
  g.K = o->K;
  g.nleaf = o->nleaf;
  g.p = o->p;
  g.inc = o->inc;
  g.inc_pm = o->inc_pm;
  g.what = what;
  g.trial = trial;
  g.pa_phase = o->pa_phase;
  g.state = o->state;
  g.nstate = o->nstate;
  g.hist = o->hist;
  g.epsn = o->epsn;
  g.a = o->a;
  g.scr = o->scr;
  g.E = o->E;
  g.out = o->out;
  g.tol = o->tol;
  g.gamma = 0.5;
  g.maxit = o->maxit;
  g.maxbt = 8;
  static_assert(sizeof(OnShared) <= 160 * 1024, "online DMN work-group does not fit the LDS");
  hipLaunchKernelGGL(k_dmn_online, dim3(n), dim3(o->nleaf), 0, nullptr, g);
  hip_check(hipGetLastError(), "k_dmn_online");
  std::vector<double> out((size_t)ON_OUT * n);
  hip_check(hipMemcpy(out.data(), o->out, out.size() * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  for (int i = 0; i < n; ++i) {
    const double* r = out.data() + (size_t)ON_OUT * i;
    hom_dmn_result& t = res[i];
    std::memset(&t, 0, sizeof(t));
    for (int c = 0; c < 6; ++c) t.stress[c] = r[c] / w[c];
    t.coupling = r[6];
    t.dissipation = r[7];
    for (int I = 0; I < 6; ++I)
      for (int J = 0; J < 6; ++J) t.dsde[6 * I + J] = r[8 + 6 * I + J] * w[J] / w[I];
    for (int c = 0; c < 6; ++c) {
      t.dsdt[c] = what ? r[O_DSDT + c] / w[c] : NAN;
      t.dDde[c] = what ? r[O_DDDE + c] * w[c] : NAN;
    }
    t.dDdt = what ? r[O_DDDT] : NAN;
    t.residual = r[O_RES];
    t.newton_iters = (int)r[O_IT];
    t.status = r[O_ST] == 1.0 ? HOM_OK : HOM_E_NOT_CONVERGED;
  }
}

}  // namespace hom
