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
#include <unordered_map>
#include <utility>

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
  // C = c1 C1 + c2 C2 - cc X, X = G Mi G^T = GM G^T. With T = Cb G:
  //   <Cb, X> = <GM, T>, dJ/dMi = -cc G^T T, dJ/dG = -cc (Cb + Cb^T) GM,
  // one row of Cb at a time
  double dx = 0.0, dd = 0.0;  // <Cb, X>, <Cb, C1 - C2>
  double Gb[6][3], T[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Gb[i][k] = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double cr[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      cr[j] = Cb[6 * i + j];
      dd += cr[j] * (C1[6 * i + j] - C2[6 * i + j]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double t = 0.0, u = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        t += cr[j] * G[j][k];
        u += cr[j] * GM[j][k];
        Gb[j][k] -= cc * cr[j] * GM[i][k];  // (Cb^T GM)[j][k]
      }
      T[i][k] = t;
      Gb[i][k] -= cc * u;  // (Cb GM)[i][k]
      dx += GM[i][k] * t;
    }
  }
  double Mib[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double m = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) m += G[i][k] * T[i][l];
      Mib[k][l] = -cc * m;
    }
  // Mi = M^-1: Mb = -Mi Mib Mi (Mi symmetric)
  double W[3][3], Mb[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) W[k][l] = Mib[k][0] * Mi[0][l] + Mib[k][1] * Mi[1][l] + Mib[k][2] * Mi[2][l];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Mb[k][l] = -(Mi[k][0] * W[0][l] + Mi[k][1] * W[1][l] + Mi[k][2] * W[2][l]);
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
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) s += (C1[6 * i + j] - C2[6 * i + j]) * Gb[i][k];
      Nb[j][k] += s;
    }
  // Hb = N Mb N^T = NM N^T
  double NM[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l) NM[i][l] = N[i][0] * Mb[0][l] + N[i][1] * Mb[1][l] + N[i][2] * Mb[2][l];
  double dh = 0.0;  // <Hb, C2 - C1>
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double hb = 0.0, db = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        db += Gb[i][k] * N[j][k];
        hb += NM[i][k] * N[j][k];
      }
      dh += hb * (C2[6 * i + j] - C1[6 * i + j]);
      const double cb = Cb[6 * i + j];
      if (C1b) C1b[6 * i + j] = c1 * cb + c2 * hb + db;
      if (C2b) C2b[6 * i + j] = c2 * cb + c1 * hb - db;
    }
  c1b = dd - (1.0 - 2.0 * c1) * dx + dh;
  nmat_adj(Nb, nb);
}

// threads of an offline work-group (one sample): the bottom level of a depth-8
// tree has 128 laminates; deeper trees loop. Small groups leave the reverse
// mode of a laminate its full register budget.
constexpr int OFF_THREADS = 128;

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

__global__ void __launch_bounds__(OFF_THREADS) k_dmn_fwd(OffArgs a) {
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
__global__ void __launch_bounds__(OFF_THREADS) k_dmn_bwd(OffArgs a) {
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

int threads_for(int nleaf) { return std::min(OFF_THREADS, std::max(64, nleaf / 2)); }

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
// online evaluation (paper Sec. 3.3): Newton's method on the jumps of the
// whole tree for many macroscopic points, one wave per point.
//
// Lane t of a point owns the subtree of R = K - S levels below the depth-S
// node 2^S + t (S = min(K, 6)), i.e. 2^R leaves whose data stay in its
// registers. The S levels above are combined across lanes with shuffles: the
// depth-d node j (heap 2^d + j) belongs to lane j 2^(S-d), its right child to
// lane j 2^(S-d) + 2^(S-d-1). Per-node data in global memory (the jumps, the
// elimination factors G, d0 and the last Newton step) are touched only by the
// owning lane, so a point needs neither LDS nor a barrier and many points
// share a CU.
//
// One bottom-up sweep forms the residual (weighted stress sums and the
// traction mismatch N^T (c2 s1 - c1 s2) of every laminate) and, in the same
// pass, eliminates the jumps: with the children's condensed tangents K1, K2
// and condensed stresses, X = (c2 K1 - c1 K2) N, M = N^T (c2^2 K1 + c1^2 K2) N,
// G = -M^-1 X^T, d0 = -M^-1 N^T (c2 s1' - c1 s2'), and the parent gets
// K = K1 + K2 + X G (the symmetric Schur complement) and s' = s1' + s2' + X d0.
// The top-down sweep turns a root strain change into the jumps' Newton steps
// da = d0 + G deps. The converged root tangent is the effective algorithmic
// tangent d<sigma>/dE.
// ---------------------------------------------------------------------------
namespace {

constexpr int ON_MAX_K = 8;
constexpr int ON_LANES = 64;  // one wave per point
constexpr int ON_SHUF = 6;    // levels combined across the lanes (2^6 = 64)
// per point: sigma 6, coupling, dissipation, dsde 36, dsdt 6, dDde 6, dDdt,
// residual, iterations, status
constexpr int ON_OUT = 64;
constexpr int O_DSDT = 44, O_DDDE = 50, O_DDDT = 56, O_RES = 57, O_IT = 58, O_ST = 59;
constexpr int ON_SCR = 24;  // per internal node: G (18), d0 (3), last Newton step (3)
constexpr int ON_NODE = 8;  // per heap node: unit direction (3), c1, subtree weight
constexpr int ON_LP = 16;   // per leaf: d sigma / d theta (6), d D / d eps (6), d D / d theta

struct OnArgs {
  int K, nleaf, S;
  const double* node;     // [2 nleaf][ON_NODE], heap index (leaves: weight in slot 4)
  const ProbInc* inc;     // [distinct (theta, dt) of the call]
  const ProbInc* inc_pm;  // [distinct][2]: theta + h_theta, theta - h_theta (all four tangents)
  const int* inc_ix;      // [point] index into inc
  int what;               // 1: also the temperature and coupling tangents
  int trial;              // 1: never commit
  int pa_phase;           // phase (0: even leaves, 1: odd leaves) with the PA66 law, -1 if none
  double* state;          // [point][nstate][nleaf / 2]
  int nstate;
  double* hist;           // [point][HIST_SLOTS][nleaf / 2]
  double* epsn;           // [point][nleaf][6]
  double* a;              // [point][nleaf][3] jumps (heap index)
  double* scr;            // [point][nleaf][ON_SCR]
  double* lp;             // [point][nleaf][ON_LP] leaf partials (what = 1)
  // predictor (pred = 1): jump change of the last committed increment, the
  // jumps at the start of this call and whether the point's last call
  // committed; the last committed macro strain and its change (kept with the
  // predictor off too)
  int pred;
  double* dah;            // [point][nleaf][3]
  double* a0;             // [point][nleaf][3]
  double* Ep;             // [point][12]: E of the last commit (6), its change (6)
  int* committed;         // [point]
  const double* E;        // [point][6] Mandel
  double* out;            // [point][ON_OUT]
  double tol, gamma;
  int maxit, maxbt;
};

// node table of a network: unit directions, c1 and subtree weights (heap index)
__global__ void k_dmn_node_table(const double* p, int nleaf, double* node) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double* v = p + 3 * (nleaf - 1);
  for (int l = 0; l < nleaf; ++l) node[ON_NODE * (nleaf + l) + 4] = fmax(v[l], 0.0);
  for (int h = nleaf - 1; h >= 1; --h) {
    double* nh = node + ON_NODE * h;
    const double wl = node[ON_NODE * (2 * h) + 4], wr = node[ON_NODE * (2 * h + 1) + 4], sw = wl + wr;
    double len;
    unit(p + 3 * param_of(h, nleaf), nh, len);
    nh[3] = sw > 0.0 ? wl / sw : 0.5;
    nh[4] = sw;
  }
}

// packed index of the symmetric 6 x 6 entry (i, j)
__host__ __device__ constexpr int sx(int i, int j) {
  return i <= j ? i * 6 - (i * (i - 1)) / 2 + (j - i) : j * 6 - (j * (j - 1)) / 2 + (i - j);
}

// a leaf: weight, compressed tangent 3K P1 + ca P2 + cb N N, weighted stress (or source)
struct LeafV {
  double w, K3, ca, cb, nd[6];
  double s[6];
};
// a condensed subtree: tangent (packed symmetric, in the lane's LDS slot:
// entry e at K[e * ON_LANES]), plain and condensed stress sums
struct NodeV {
  double* K;
  double s[6], sp[6];
};

__device__ __forceinline__ double kent(const LeafV& a, int i, int q) {
  return a.w * ((i == q ? a.ca : 0.0) + (i < 3 && q < 3 ? (a.K3 - a.ca) * (1.0 / 3.0) : 0.0) + a.cb * a.nd[i] * a.nd[q]);
}
__device__ __forceinline__ double kent(const NodeV& a, int i, int q) { return a.K[sx(i, q) * ON_LANES]; }
__device__ __forceinline__ const double* plain(const LeafV& a) { return a.s; }
__device__ __forceinline__ const double* plain(const NodeV& a) { return a.s; }
__device__ __forceinline__ const double* cond(const LeafV& a) { return a.s; }
__device__ __forceinline__ const double* cond(const NodeV& a) { return a.sp; }

__device__ __forceinline__ void to_node(const LeafV& L, NodeV& v) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int q = i; q < 6; ++q) v.K[sx(i, q) * ON_LANES] = kent(L, i, q);
#pragma unroll
  for (int c = 0; c < 6; ++c) v.s[c] = v.sp[c] = L.s[c];
}

// N a = sym(a (x) n) (Mandel) for the unit direction n
__device__ __forceinline__ void n_apply(const double* n, const double* a, double* v) {
  v[0] = n[0] * a[0];
  v[1] = n[1] * a[1];
  v[2] = n[2] * a[2];
  v[3] = SQ2H * (n[2] * a[1] + n[1] * a[2]);
  v[4] = SQ2H * (n[2] * a[0] + n[0] * a[2]);
  v[5] = SQ2H * (n[1] * a[0] + n[0] * a[1]);
}
// N^T v
__device__ __forceinline__ void nt_apply(const double* n, const double* v, double* r) {
  r[0] = n[0] * v[0] + SQ2H * (n[2] * v[4] + n[1] * v[5]);
  r[1] = n[1] * v[1] + SQ2H * (n[2] * v[3] + n[0] * v[5]);
  r[2] = n[2] * v[2] + SQ2H * (n[1] * v[3] + n[0] * v[4]);
}
__device__ __forceinline__ double* node_scr(const OnArgs& g, int pt, int h) {
  return g.scr + ((long long)pt * g.nleaf + h) * ON_SCR;
}
__device__ __forceinline__ double* node_jump(const OnArgs& g, int pt, int h) {
  return g.a + ((long long)pt * g.nleaf + h) * 3;
}

// Laminate h from its children A (phase 1 side) and B: residual contribution
// (PLAIN: from the plain sums), elimination factors into the node's scratch,
// condensed tangent and stresses into P. P may be A itself: every entry of P
// is written after the last read of the same entry of A.
template <bool PLAIN, class CA, class CB>
__device__ __forceinline__ void combine(const OnArgs& g, int pt, int h, const CA& A, const CB& B, NodeV& P,
                                        double& gg) {
  const double* nt = g.node + ON_NODE * h;
  const double n[3] = {nt[0], nt[1], nt[2]};
  const double c1 = nt[3], c2 = 1.0 - c1, wsub = nt[4];
  const double s0 = SQ2H * n[0], s1 = SQ2H * n[1], s2 = SQ2H * n[2];
  // X = (c2 K1 - c1 K2) N and M = N^T (c2^2 K1 + c1^2 K2) N, column by column
  double X[6][3], M[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double hc[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double a1, a2;
      if (k == 0) {
        a1 = kent(A, i, 0) * n[0] + kent(A, i, 4) * s2 + kent(A, i, 5) * s1;
        a2 = kent(B, i, 0) * n[0] + kent(B, i, 4) * s2 + kent(B, i, 5) * s1;
      } else if (k == 1) {
        a1 = kent(A, i, 1) * n[1] + kent(A, i, 3) * s2 + kent(A, i, 5) * s0;
        a2 = kent(B, i, 1) * n[1] + kent(B, i, 3) * s2 + kent(B, i, 5) * s0;
      } else {
        a1 = kent(A, i, 2) * n[2] + kent(A, i, 3) * s1 + kent(A, i, 4) * s0;
        a2 = kent(B, i, 2) * n[2] + kent(B, i, 3) * s1 + kent(B, i, 4) * s0;
      }
      X[i][k] = c2 * a1 - c1 * a2;
      hc[i] = c2 * c2 * a1 + c1 * c1 * a2;
    }
    double mc[3];
    nt_apply(n, hc, mc);
#pragma unroll
    for (int q = 0; q < 3; ++q) M[q][k] = mc[q];
  }
  const double* p1 = cond(A);
  const double* p2 = cond(B);
  double dv[6], r[3];
#pragma unroll
  for (int c = 0; c < 6; ++c) dv[c] = c2 * p1[c] - c1 * p2[c];
  nt_apply(n, dv, r);
  if constexpr (PLAIN) {
    const double* q1 = plain(A);
    const double* q2 = plain(B);
    double pv[6], rp[3];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      pv[c] = c2 * q1[c] - c1 * q2[c];
      P.s[c] = q1[c] + q2[c];
    }
    nt_apply(n, pv, rp);
    gg += rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2];
  }
  // a subtree without weight on one side has no say in its jump: it stays
  double Mi[3][3];
  const bool ok = (c1 * c2 * wsub > 0.0) && inv3(M, Mi);
  double* sc = node_scr(g, pt, h);
  double d0[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d0[k] = ok ? -(Mi[k][0] * r[0] + Mi[k][1] * r[1] + Mi[k][2] * r[2]) : 0.0;
    sc[18 + k] = d0[k];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) P.sp[i] = p1[i] + p2[i] + X[i][0] * d0[0] + X[i][1] * d0[1] + X[i][2] * d0[2];
  // G = -M^-1 X^T one column at a time; K = K1 + K2 + X G
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double gq[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gq[k] = ok ? -(Mi[k][0] * X[q][0] + Mi[k][1] * X[q][1] + Mi[k][2] * X[q][2]) : 0.0;
      sc[6 * k + q] = gq[k];
    }
#pragma unroll
    for (int i = 0; i <= q; ++i)
      P.K[sx(i, q) * ON_LANES] =
          kent(A, i, q) + kent(B, i, q) + X[i][0] * gq[0] + X[i][1] * gq[1] + X[i][2] * gq[2];
  }
}

// children strains of laminate h: eps1 = eps + c2 N a, eps2 = eps - c1 N a
__device__ __forceinline__ void split(const OnArgs& g, int h, const double* jump, const double* e, double* el,
                                      double* er) {
  const double* nt = g.node + ON_NODE * h;
  const double c1 = nt[3], c2 = 1.0 - c1;
  double jn[6];
  n_apply(nt, jump, jn);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    el[c] = e[c] + c2 * jn[c];
    er[c] = e[c] - c1 * jn[c];
  }
}

// Newton step of node h from the strain change of the node: da = d0 + G deps
// (kept in the scratch; added to the jump if `update`), and the children's
// strain changes
__device__ __forceinline__ void node_step(const OnArgs& g, int pt, int h, const double* de, bool update, double* dl,
                                          double* dr) {
  double* sc = node_scr(g, pt, h);
  double da[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double x = sc[18 + k];
#pragma unroll
    for (int i = 0; i < 6; ++i) x += sc[6 * k + i] * de[i];
    da[k] = x;
    sc[21 + k] = x;
  }
  if (update) {
    double* ah = node_jump(g, pt, h);
#pragma unroll
    for (int k = 0; k < 3; ++k) ah[k] += da[k];
  }
  split(g, h, da, de, dl, dr);
}

// the register levels of a lane: the subtree of LV levels below node h
template <int LV>
struct RegTree {
  // strains from the jumps, leaves by leaf(l, eps, LeafV&), combination upwards
  template <bool PLAIN, class LeafFn>
  static __device__ __forceinline__ void up(const OnArgs& g, int pt, int h, const double* e, NodeV& out, double& gg,
                                            LeafFn& leaf) {
    double el[6], er[6];
    split(g, h, node_jump(g, pt, h), e, el, er);
    if constexpr (LV == 1) {
      LeafV A, B;
      leaf(2 * h - g.nleaf, el, A);
      leaf(2 * h + 1 - g.nleaf, er, B);
      combine<PLAIN>(g, pt, h, A, B, out, gg);
    } else {
      NodeV B;
      B.K = out.K + 21 * ON_LANES;  // the next slot
      RegTree<LV - 1>::template up<PLAIN>(g, pt, 2 * h, el, out, gg, leaf);
      RegTree<LV - 1>::template up<PLAIN>(g, pt, 2 * h + 1, er, B, gg, leaf);
      combine<PLAIN>(g, pt, h, out, B, out, gg);
    }
  }
  // leaf strains from the jumps: fn(l, eps)
  template <class Fn>
  static __device__ __forceinline__ void down(const OnArgs& g, int pt, int h, const double* e, Fn& fn) {
    double el[6], er[6];
    split(g, h, node_jump(g, pt, h), e, el, er);
    if constexpr (LV == 1) {
      fn(2 * h - g.nleaf, el);
      fn(2 * h + 1 - g.nleaf, er);
    } else {
      RegTree<LV - 1>::down(g, pt, 2 * h, el, fn);
      RegTree<LV - 1>::down(g, pt, 2 * h + 1, er, fn);
    }
  }
  // Newton steps from the node's strain change; leaf strain changes: fn(l, deps)
  template <class Fn>
  static __device__ __forceinline__ void expand(const OnArgs& g, int pt, int h, const double* de, bool update,
                                                Fn& fn) {
    double dl[6], dr[6];
    node_step(g, pt, h, de, update, dl, dr);
    if constexpr (LV == 1) {
      fn(2 * h - g.nleaf, dl);
      fn(2 * h + 1 - g.nleaf, dr);
    } else {
      RegTree<LV - 1>::expand(g, pt, 2 * h, dl, update, fn);
      RegTree<LV - 1>::expand(g, pt, 2 * h + 1, dr, update, fn);
    }
  }
};

__device__ __forceinline__ double shdown(double v, int d) { return __shfl_down(v, d, ON_LANES); }
__device__ __forceinline__ double shup(double v, int d) { return __shfl_up(v, d, ON_LANES); }

// sum over the wave, the same value on every lane
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = ON_LANES / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, ON_LANES);
  return __shfl(v, 0, ON_LANES);
}

// root strain (E, or 0 for a change) to the lane's depth-S node: shuffle levels,
// each owner splits its node with `jump(h, jn)`
template <class JumpFn>
__device__ __forceinline__ void shuffle_down(const OnArgs& g, int lane, double* e, JumpFn& jump) {
  const bool act = lane < (1 << g.S);
  for (int d = 0; d < g.S; ++d) {
    const int sh = g.S - d, half = 1 << (sh - 1);
    const int pos = lane & ((1 << sh) - 1);
    double er[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (act && pos == 0) jump((1 << d) + (lane >> sh), e, er);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double t = shup(er[c], half);
      if (act && pos == half) e[c] = t;
    }
  }
}

// the lane's depth-S node value up to the root (lane 0), combining at every
// shuffle level: stress sums by shuffles, tangents read from the right
// child's LDS slot
template <bool PLAIN>
__device__ __forceinline__ void shuffle_up(const OnArgs& g, int pt, int lane, NodeV& cur, double& gg) {
  const bool act = lane < (1 << g.S);
  for (int d = g.S - 1; d >= 0; --d) {
    const int sh = g.S - d, half = 1 << (sh - 1);
    __syncthreads();  // the children's tangents are in their lanes' slots
    NodeV rb;
    rb.K = cur.K + half;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      rb.s[c] = PLAIN ? shdown(cur.s[c], half) : 0.0;
      rb.sp[c] = shdown(cur.sp[c], half);
    }
    if (act && (lane & ((1 << sh) - 1)) == 0) combine<PLAIN>(g, pt, (1 << d) + (lane >> sh), cur, rb, cur, gg);
  }
}

// Strains of every leaf at the current jumps (leaves by `leaf`), residual
// and elimination of the whole tree; root values on lane 0. root.K names the
// lane's first LDS slot.
template <int R, bool PLAIN, class LeafFn>
__device__ __forceinline__ void eval_pass(const OnArgs& g, int pt, int lane, LeafFn& leaf, NodeV& root,
                                          double& gg) {
  __syncthreads();  // the slots of the previous sweep have been read
  double e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = lane == 0 ? g.E[6 * pt + c] : 0.0;
  auto jump = [&](int h, double* ev, double* er) {
    double el[6];
    split(g, h, node_jump(g, pt, h), ev, el, er);
#pragma unroll
    for (int c = 0; c < 6; ++c) ev[c] = el[c];
  };
  shuffle_down(g, lane, e, jump);
  if constexpr (R == 0) {
    LeafV L{};
    if (lane < g.nleaf) leaf(lane, e, L);
    to_node(L, root);
  } else {
    RegTree<R>::template up<PLAIN>(g, pt, (1 << g.S) + lane, e, root, gg, leaf);
  }
  shuffle_up<PLAIN>(g, pt, lane, root, gg);
}

// leaf strains at the current jumps: fn(l, eps)
template <int R, class Fn>
__device__ __forceinline__ void strains_pass(const OnArgs& g, int pt, int lane, Fn& fn) {
  double e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = lane == 0 ? g.E[6 * pt + c] : 0.0;
  auto jump = [&](int h, double* ev, double* er) {
    double el[6];
    split(g, h, node_jump(g, pt, h), ev, el, er);
#pragma unroll
    for (int c = 0; c < 6; ++c) ev[c] = el[c];
  };
  shuffle_down(g, lane, e, jump);
  if constexpr (R == 0) {
    if (lane < g.nleaf) fn(lane, e);
  } else {
    RegTree<R>::down(g, pt, (1 << g.S) + lane, e, fn);
  }
}

// Newton steps of all jumps for a zero root strain change (after eval_pass);
// the leaf strain changes: fn(l, deps)
template <int R, class Fn>
__device__ __forceinline__ void expand_pass(const OnArgs& g, int pt, int lane, bool update, Fn& fn) {
  double de[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  auto step = [&](int h, double* dv, double* dr) {
    double dl[6];
    node_step(g, pt, h, dv, update, dl, dr);
#pragma unroll
    for (int c = 0; c < 6; ++c) dv[c] = dl[c];
  };
  shuffle_down(g, lane, de, step);
  if constexpr (R == 0) {
    if (lane < g.nleaf) fn(lane, de);
  } else {
    RegTree<R>::expand(g, pt, (1 << g.S) + lane, de, update, fn);
  }
}

// every internal node the lane owns: fn(h)
template <int R, class Fn>
__device__ __forceinline__ void for_owned(const OnArgs& g, int lane, Fn& fn) {
  if (lane >= (1 << g.S)) return;
  for (int d = 0; d < g.S; ++d) {
    const int sh = g.S - d;
    if ((lane & ((1 << sh) - 1)) == 0) fn((1 << d) + (lane >> sh));
  }
  const int h0 = (1 << g.S) + lane;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < (1 << r); ++k) fn((h0 << r) + k);
}

// effective stress and the full 6 x 6 tangent of the root
__device__ __forceinline__ void put_root(double* o, const NodeV& root) {
#pragma unroll
  for (int c = 0; c < 6; ++c) o[c] = root.s[c];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) o[8 + 6 * i + j] = root.K[sx(i, j) * ON_LANES];
}

// |A^T W sigma| / ((2^K - 1) |sigma_bar|) from the lanes' sums and the root on lane 0
__device__ __forceinline__ double residual_norm(const OnArgs& g, int lane, const NodeV& root, double gg) {
  gg = wave_sum(gg);
  double sb = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) sb += root.s[c] * root.s[c];
  const double r = sqrt(gg) / ((double)(g.nleaf - 1) * fmax(sqrt(sb), 1e-300));
  return __shfl(r, 0, ON_LANES);
}

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

// point partials of leaf l at its converged strain e, from state n:
// d sigma / d theta, d D / d eps, d D / d theta (closed form for the
// thermoelastic phase, central differences of the PA66 update)
__device__ void leaf_partials(const OnArgs& g, const ProbInc& in, int pt, int l, const double* e, double* st_,
                              double* gd, double& hd) {
  const int phase = l & 1;
  const double* enp = g.epsn + ((long long)g.nleaf * pt + l) * 6;
  double en[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) en[c] = enp[c];
  if (phase == g.pa_phase) {
    const long long ss = g.nleaf >> 1;
    const int q = l >> 1;
    const double* st = g.state + (long long)pt * g.nstate * ss + q;
    const double* hs = g.hist + (long long)pt * HIST_SLOTS * ss + q;
    double sp[6], Dp = 0.0;
    for (int k = 0; k < 14; ++k) {
      const bool th = k < 2;
      const ProbInc& ik = th ? g.inc_pm[2 * g.inc_ix[pt] + k] : in;
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
}

template <int R>
__global__ void __launch_bounds__(ON_LANES) k_dmn_online(OnArgs g) {
  // condensed tangents: one slot per register level (at least one), lane-interleaved
  __shared__ double kslot[(R > 0 ? R : 1) * 21 * ON_LANES];
  const int pt = blockIdx.x;
  const int lane = threadIdx.x;
  const int nleaf = g.nleaf;
  constexpr int LPT = 1 << R;  // leaves per lane
  const int ix = g.inc_ix[pt];
  const ProbInc& in = g.inc[ix];
  const bool leaves = lane * LPT < nleaf;
  // branch history sums of this lane's PA66 leaves for this increment
  if (leaves && g.pa_phase >= 0) {
    const long long ss = nleaf >> 1;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int l = lane * LPT + i;
      if ((l & 1) != g.pa_phase) continue;
      const int q = l >> 1;
      double hd[6], hs;
      pa66_history(in, g.state + (long long)pt * g.nstate * ss + q, ss, hd, hs);
      double* h = g.hist + (long long)pt * HIST_SLOTS * ss + q;
#pragma unroll
      for (int c = 0; c < 6; ++c) h[c * ss] = hd[c];
      h[6 * ss] = hs;
      h[7 * ss] = -1.0;
    }
  }
  // predictor: start from the committed jumps plus s times their last change,
  // s = projection of this macro increment on the last committed one
  double pred_s = 0.0;
  if (g.pred) {
    const double* ep = g.Ep + 12 * pt;
    double ee = 0.0, pp = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      ee += (g.E[6 * pt + c] - ep[c]) * ep[6 + c];
      pp += ep[6 + c] * ep[6 + c];
    }
    if (g.committed[pt] && pp > 0.0 && isfinite(ee)) pred_s = fmin(2.0, fmax(0.0, ee / pp));
    auto start = [&](int h) {
      double* ah = node_jump(g, pt, h);
      double* a0 = g.a0 + ((long long)pt * nleaf + h) * 3;
      const double* dh = g.dah + ((long long)pt * nleaf + h) * 3;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a0[k] = ah[k];
        ah[k] += pred_s * dh[k];
      }
    };
    for_owned<R>(g, lane, start);
  }
  auto wleaf = [&](int l) { return g.node[ON_NODE * (nleaf + l) + 4]; };
  auto law = [&](int l, const double* e, LeafV& L) {
    double sg[6];
    leaf_eval(g, in, pt, l, e, sg, L.K3, L.ca, L.cb, L.nd);
    L.w = wleaf(l);
#pragma unroll
    for (int c = 0; c < 6; ++c) L.s[c] = L.w * sg[c];
  };
  NodeV root;
  root.K = kslot + lane;
  double gg = 0.0;
  eval_pass<R, true>(g, pt, lane, law, root, gg);
  double res = residual_norm(g, lane, root, gg);
  auto nothing = [](int, const double*) {};
  int it = 0;
  for (it = 1; it <= g.maxit; ++it) {
    expand_pass<R>(g, pt, lane, true, nothing);
    const double res_old = res;
    gg = 0.0;
    eval_pass<R, true>(g, pt, lane, law, root, gg);
    res = residual_norm(g, lane, root, gg);
    for (int i = 0; i < g.maxbt; ++i) {  // backtracking: steps 1, gamma, gamma^2, ...
      if (res < res_old) break;
      const double cut = pow(g.gamma, (double)i) * (1.0 - g.gamma);
      auto back = [&](int h) {
        double* ah = node_jump(g, pt, h);
        const double* sc = node_scr(g, pt, h);
#pragma unroll
        for (int k = 0; k < 3; ++k) ah[k] -= cut * sc[21 + k];
      };
      for_owned<R>(g, lane, back);
      gg = 0.0;
      eval_pass<R, true>(g, pt, lane, law, root, gg);
      res = residual_norm(g, lane, root, gg);
    }
    if (res < g.tol) break;
  }
  const bool conv = res < g.tol;
  const bool commit = conv && !g.trial;
  if (it > g.maxit) it = g.maxit;
  // effective stress and tangent: the root of the last sweep
  double* o = g.out + (long long)pt * ON_OUT;
  if (lane == 0) put_root(o, root);
  if (g.what) {
    auto partials = [&](int l, const double* e) {
      double st_[6], gd[6], hd;
      leaf_partials(g, in, pt, l, e, st_, gd, hd);
      double* lp = g.lp + ((long long)pt * nleaf + l) * ON_LP;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        lp[c] = st_[c];
        lp[6 + c] = gd[c];
      }
      lp[12] = hd;
    };
    strains_pass<R>(g, pt, lane, partials);
    // d<sigma>/dtheta: the jumps equilibrate the leaf sources w dsigma/dtheta
    auto src_theta = [&](int l, const double* e, LeafV& L) {
      const double* lp = g.lp + ((long long)pt * nleaf + l) * ON_LP;
      double sg[6];
      leaf_eval(g, in, pt, l, e, sg, L.K3, L.ca, L.cb, L.nd);
      L.w = wleaf(l);
#pragma unroll
      for (int c = 0; c < 6; ++c) L.s[c] = L.w * lp[c];
    };
    NodeV rt;
    rt.K = kslot + lane;
    double unused = 0.0;
    eval_pass<R, false>(g, pt, lane, src_theta, rt, unused);
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) o[O_DSDT + c] = rt.sp[c];
    // d<D>/dtheta = sum_l w_l (dD/dtheta_l + dD/deps_l . d eps_l / d theta)
    double dT = 0.0;
    auto heat = [&](int l, const double* de) {
      const double* lp = g.lp + ((long long)pt * nleaf + l) * ON_LP;
      double x = lp[12];
#pragma unroll
      for (int c = 0; c < 6; ++c) x += lp[6 + c] * de[c];
      dT += wleaf(l) * x;
    };
    expand_pass<R>(g, pt, lane, false, heat);
    dT = wave_sum(dT);
    if (lane == 0) o[O_DDDT] = dT;
    // d<D>/dE = sum_l w_l (d eps_l / dE)^T dD/deps_l: the condensed value of
    // the leaf sources w dD/deps (the localization is symmetric in this sense)
    auto src_coup = [&](int l, const double* e, LeafV& L) {
      const double* lp = g.lp + ((long long)pt * nleaf + l) * ON_LP;
      double sg[6];
      leaf_eval(g, in, pt, l, e, sg, L.K3, L.ca, L.cb, L.nd);
      L.w = wleaf(l);
#pragma unroll
      for (int c = 0; c < 6; ++c) L.s[c] = L.w * lp[6 + c];
    };
    eval_pass<R, false>(g, pt, lane, src_coup, rt, unused);
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) o[O_DDDE + c] = rt.sp[c];
  }
  // coupling term and dissipation of every leaf; commit if converged
  double D = 0.0, Dd = 0.0;
  auto fin = [&](int l, const double* e) {
    const int phase = l & 1;
    double* en = g.epsn + ((long long)pt * nleaf + l) * 6;
    double Dl = 0.0, Ddl = 0.0;
    if (phase == g.pa_phase) {
      const long long ss = nleaf >> 1;
      const int q = l >> 1;
      double* st = g.state + (long long)pt * g.nstate * ss + q;
      double* hs = g.hist + (long long)pt * HIST_SLOTS * ss + q;
      double enl[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) enl[c] = en[c];
      PaOut po;
      pa66_point(in, e, st, ss, commit ? st : nullptr, enl, po, &Ddl, &Dl, hs, nullptr);
    } else {
      const PhaseInc& pi = in.ph[phase];
      const double trd = (e[0] - en[0]) + (e[1] - en[1]) + (e[2] - en[2]);
      Dl = -in.theta * pi.K3 * pi.alpha0 * trd / in.dt;
    }
    const double w = wleaf(l);
    D += w * Dl;
    Dd += w * Ddl;
    if (commit)
#pragma unroll
      for (int c = 0; c < 6; ++c) en[c] = e[c];
  };
  strains_pass<R>(g, pt, lane, fin);
  if (g.pred) {
    if (commit) {
      auto change = [&](int h) {
        const double* ah = node_jump(g, pt, h);
        const double* a0 = g.a0 + ((long long)pt * nleaf + h) * 3;
        double* dh = g.dah + ((long long)pt * nleaf + h) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) dh[k] = ah[k] - a0[k];
      };
      for_owned<R>(g, lane, change);
    }
    if (lane == 0) g.committed[pt] = commit ? 1 : 0;
  }
  // the committed macro strain and its last change are kept with the
  // predictor off too, so that switching it on measures the next increment
  // from the right base
  if (lane == 0 && commit) {
    double* ep = g.Ep + 12 * pt;
    for (int c = 0; c < 6; ++c) {
      ep[6 + c] = g.E[6 * pt + c] - ep[c];
      ep[c] = g.E[6 * pt + c];
    }
  }
  D = wave_sum(D);
  Dd = wave_sum(Dd);
  if (lane == 0) {
    o[6] = D;
    o[7] = Dd;
    o[O_RES] = res;
    o[O_IT] = it;
    o[O_ST] = conv ? 1.0 : 0.0;
  }
}

}  // namespace

struct PairHash {
  size_t operator()(const std::pair<uint64_t, uint64_t>& k) const {
    return std::hash<uint64_t>()(k.first * 0x9E3779B97F4A7C15ull ^ k.second);
  }
};

struct DmnOnline {
  int K, nleaf, npoints, nstate = 0, pa_phase = -1;
  double tol;
  int maxit;
  std::vector<hom_law> laws;
  std::vector<void*> allocs;
  double *p = nullptr, *node = nullptr, *state = nullptr, *hist = nullptr, *epsn = nullptr, *a = nullptr;
  double *scr = nullptr, *lp = nullptr, *E = nullptr, *out = nullptr;
  double *dah = nullptr, *a0 = nullptr, *Ep = nullptr;
  int* committed = nullptr;
  int pred = 0;
  ProbInc *inc = nullptr, *inc_pm = nullptr;
  int* inc_ix = nullptr;
  std::vector<ProbInc> inc_h, inc_pm_h;
  // pinned staging of the per-point inputs and outputs
  double *E_h = nullptr, *out_h = nullptr;
  int* ix_h = nullptr;
  ~DmnOnline() {
    for (void* ptr : allocs) (void)hipFree(ptr);
    for (void* ptr : {(void*)E_h, (void*)out_h, (void*)ix_h})
      if (ptr) (void)hipHostFree(ptr);
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
  o->node = dalloc_into<double>(o->allocs, (size_t)2 * o->nleaf * ON_NODE);
  hipLaunchKernelGGL(k_dmn_node_table, dim3(1), dim3(1), 0, nullptr, o->p, o->nleaf, o->node);
  hip_check(hipGetLastError(), "k_dmn_node_table");
  if (o->nstate) {
    o->state = dalloc_into<double>(o->allocs, (size_t)npoints * o->nstate * half);
    o->hist = dalloc_into<double>(o->allocs, (size_t)npoints * HIST_SLOTS * half);
  }
  o->epsn = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * 6);
  o->a = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * 3);
  o->scr = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * ON_SCR);
  o->lp = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * ON_LP);
  o->dah = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * 3);
  o->a0 = dalloc_into<double>(o->allocs, (size_t)npoints * o->nleaf * 3);
  o->Ep = dalloc_into<double>(o->allocs, (size_t)npoints * 12);
  o->committed = dalloc_into<int>(o->allocs, npoints);
  o->E = dalloc_into<double>(o->allocs, (size_t)npoints * 6);
  o->out = dalloc_into<double>(o->allocs, (size_t)npoints * ON_OUT);
  o->inc = dalloc_into<ProbInc>(o->allocs, npoints);
  o->inc_pm = dalloc_into<ProbInc>(o->allocs, 2 * (size_t)npoints);
  o->inc_ix = dalloc_into<int>(o->allocs, npoints);
  o->inc_h.reserve(npoints);
  o->inc_pm_h.reserve(2 * (size_t)npoints);
  hip_check(hipHostMalloc((void**)&o->E_h, (size_t)npoints * 6 * sizeof(double)), "hipHostMalloc");
  hip_check(hipHostMalloc((void**)&o->out_h, (size_t)npoints * ON_OUT * sizeof(double)), "hipHostMalloc");
  hip_check(hipHostMalloc((void**)&o->ix_h, (size_t)npoints * sizeof(int)), "hipHostMalloc");
  return o.release();
}

void dmn_online_destroy(DmnOnline* o) { delete o; }

void dmn_online_set_predictor(DmnOnline* o, int on) {
  if (on != 0 && on != 1) fail(HOM_E_ARG, "predictor must be 0 or 1");
  // jump changes are recorded only while the predictor is on: switching it
  // on forgets what an earlier on-period left, so the first call starts from
  // the current jumps
  if (on && !o->pred)
    hip_check(hipMemset(o->committed, 0, (size_t)o->npoints * sizeof(int)), "hipMemset");
  o->pred = on;
}

void dmn_online_step(DmnOnline* o, const double* strain, const double* theta, const double* dt, int what,
                     int trial, hom_dmn_result* res) {
  if (what != 0 && what != 1) fail(HOM_E_ARG, "what must be 0 (d sigma / dE) or 1 (all four tangents)");
  if (trial != 0 && trial != 1) fail(HOM_E_ARG, "trial must be 0 or 1");
  const int n = o->npoints;
  const double sq2 = std::sqrt(2.0);
  const double w[6] = {1, 1, 1, sq2, sq2, sq2};
  // one increment record per distinct (theta, dt): points of one macroscopic
  // step usually share both
  o->inc_h.clear();
  o->inc_pm_h.clear();
  std::unordered_map<std::pair<uint64_t, uint64_t>, int, PairHash> seen;
  double last_t = NAN, last_d = NAN;
  int last_ix = -1;
  for (int i = 0; i < n; ++i) {
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) fail(HOM_E_ARG, "dt must be positive and finite");
    if (!(theta[i] > 0.0) || !std::isfinite(theta[i])) fail(HOM_E_ARG, "theta must be positive");
    for (int c = 0; c < 6; ++c) {
      if (!std::isfinite(strain[6 * i + c])) fail(HOM_E_ARG, "macro strain must be finite");
      o->E_h[6 * i + c] = w[c] * strain[6 * i + c];
    }
    if (theta[i] != last_t || dt[i] != last_d) {
      uint64_t kt, kd;
      std::memcpy(&kt, &theta[i], 8);
      std::memcpy(&kd, &dt[i], 8);
      auto it = seen.find({kt, kd});
      if (it != seen.end()) {
        last_ix = it->second;
      } else {
        last_ix = (int)o->inc_h.size();
        seen.emplace(std::make_pair(kt, kd), last_ix);
        o->inc_h.emplace_back();
        fill_inc(o->inc_h.back(), o->laws, theta[i], dt[i]);
        if (what) {
          o->inc_pm_h.emplace_back();
          fill_inc(o->inc_pm_h.back(), o->laws, theta[i] + FD_H_THETA, dt[i]);
          o->inc_pm_h.emplace_back();
          fill_inc(o->inc_pm_h.back(), o->laws, theta[i] - FD_H_THETA, dt[i]);
        }
      }
      last_t = theta[i];
      last_d = dt[i];
    }
    o->ix_h[i] = last_ix;
  }
  const size_t nu = o->inc_h.size();
  if (what)
    hip_check(hipMemcpy(o->inc_pm, o->inc_pm_h.data(), 2 * nu * sizeof(ProbInc), hipMemcpyHostToDevice),
              "hipMemcpy");
  hip_check(hipMemcpy(o->inc, o->inc_h.data(), nu * sizeof(ProbInc), hipMemcpyHostToDevice), "hipMemcpy");
  hip_check(hipMemcpy(o->inc_ix, o->ix_h, n * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
  hip_check(hipMemcpy(o->E, o->E_h, 6 * n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
  OnArgs g{};
  g.K = o->K;
  g.nleaf = o->nleaf;
  g.S = std::min(o->K, ON_SHUF);
  g.node = o->node;
  g.inc = o->inc;
  g.inc_pm = o->inc_pm;
  g.inc_ix = o->inc_ix;
  g.what = what;
  g.trial = trial;
  g.pa_phase = o->pa_phase;
  g.state = o->state;
  g.nstate = o->nstate;
  g.hist = o->hist;
  g.epsn = o->epsn;
  g.a = o->a;
  g.scr = o->scr;
  g.lp = o->lp;
  g.pred = o->pred;
  g.dah = o->dah;
  g.a0 = o->a0;
  g.Ep = o->Ep;
  g.committed = o->committed;
  g.E = o->E;
  g.out = o->out;
  g.tol = o->tol;
  g.gamma = 0.5;
  g.maxit = o->maxit;
  g.maxbt = 8;
  static_assert(ON_MAX_K - ON_SHUF <= 2, "at most two register levels per lane");
  switch (o->K - g.S) {  // register levels below the shuffle levels
    case 0:
      hipLaunchKernelGGL(k_dmn_online<0>, dim3(n), dim3(ON_LANES), 0, nullptr, g);
      break;
    case 1:
      hipLaunchKernelGGL(k_dmn_online<1>, dim3(n), dim3(ON_LANES), 0, nullptr, g);
      break;
    default:
      hipLaunchKernelGGL(k_dmn_online<2>, dim3(n), dim3(ON_LANES), 0, nullptr, g);
      break;
  }
  hip_check(hipGetLastError(), "k_dmn_online");
  hip_check(hipMemcpy(o->out_h, o->out, (size_t)ON_OUT * n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  for (int i = 0; i < n; ++i) {
    const double* r = o->out_h + (size_t)ON_OUT * i;
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
