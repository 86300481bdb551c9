// Shared device/host structures of the solver runtime.
//
// Layout in HBM (per group of equally sized problems, problem-major):
//   real fields      [prob][comp][z][y][x]            x fastest, SoA components
//   spectra          [prob][kz][ky][kx][comp]         complex, kx = 0..nx/2,
//                                                     components interleaved so
//                                                     that a tile of kx columns
//                                                     is one contiguous segment
//   PA66 state       [prob][var][voxel]               FP64, var = eps_p, eps_vp(6),
//                                                     eps_v_i(6) for i = 1..N
// Strains and stresses are Mandel vectors (11, 22, 33, sqrt2 23, sqrt2 13, sqrt2 12).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"

namespace hom {

constexpr int MAX_PHASES = 8;
constexpr int MAX_MAXWELL = 16;
constexpr int NPART = 16;  // FP64 partial sums per block

// Block partial sums are stored quantity-major per problem,
// [prob][NPART][maxblk], so that a reduction reads each quantity as one
// contiguous run of doubles.
__host__ __device__ inline long long part_index(int prob, int q, int blk, int maxblk) {
  return ((long long)prob * NPART + q) * maxblk + blk;
}

enum Mode : int { M_DONE = 0, M_EVAL = 1, M_CG = 2, M_BASIC = 3, M_FAIL = -1 };
// Green operators: projectors and isotropic reference operators of the
// collocation scheme; *_ROT: the projectors of the rotated finite-difference
// scheme (complex modified wave vectors).
enum Green : int { G_PROJ = 0, G_GAMMA0 = 1, G_GRADPROJ = 2, G_GAMMA_TH = 3, G_PROJ_ROT = 4, G_GRADPROJ_ROT = 5 };
enum LawKind : int { LAW_TE = 1, LAW_PA66 = 2 };

// Per-problem solver control, owned by the device. The reduce kernels are
// the only writers of mode transitions.
struct Ctl {
  int mode;
  int newton_it;    // residual evaluations done (Newton) / iterations (basic)
  int cg_it;        // CG iterations in the current Newton step
  int cg_ready;     // A p of the current CG iteration is available
  int pending;      // x += dx before the next evaluation
  int status;       // 0 running, 1 converged, <0 failure code
  int pipelines;    // FFT pipeline applications so far
  int krylov;       // total CG iterations
  double rr;        // r.r of the current CG residual
  double alpha, beta;
  double res;       // relative residual of the last evaluation
  double fnorm;     // ||f|| of the last evaluation
  double cg_target; // stop CG when r.r <= cg_target
  double out[NPART];
};

// Per-phase data of one increment.
struct PhaseInc {
  int kind;
  double K3;        // 3K (instantaneous bulk for the PA66)
  double G2;        // 2G (instantaneous shear for the PA66)
  double alpha_dth; // alpha0 (theta - theta0)
  double alpha0;
  double kappa;
};

// Per-problem data of one increment, prepared on the host in FP64.
struct ProbInc {
  double theta, dt;
  double dE[6];     // change of the macro strain (Mandel) since the last commit
  double dG[3];     // change of the macro temperature gradient
  double lam0, mu0, kappa0;  // basic-scheme reference media
  int smask;        // mixed conditions: bit c set => Mandel component c of <sigma> is prescribed
  double S[6];      // prescribed effective stress (Mandel) of the masked components
  double pred_s;    // predictor: weight of the last committed strain fluctuation change (0: none)
  double dEp[6];    // mean strain change of the last committed increment (Mandel)
  PhaseInc ph[MAX_PHASES];
  // PA66 (at most one inelastic law per setup)
  int pa_phase;     // phase id of the PA66 law, -1 if none
  int nm;           // number of Maxwell branches
  double Kinf3, Ginf2;
  double K3i[MAX_MAXWELL], G2i[MAX_MAXWELL];
  double rK[MAX_MAXWELL], rG[MAX_MAXWELL];
  double fK[MAX_MAXWELL], fG[MAX_MAXWELL];  // 1 / (1 + r)
  double Kbar3, Gbar2;
  double sY, ccoef;  // yield stress, dt sY / eta
  double hk, nh, mexp, beta1, alpha0, dth;
};

// Arguments shared by the pipeline kernels of one group.
template <typename T>
struct Pipe {
  int nx, ny, nz, P;        // P = nx / 2 + 1
  int PS;                   // row pitch of the spectra in kx entries: P rounded up so that a
                            // row of PS * C complex values is a whole number of 128-byte lines
  long long nvox;
  long long vs;             // stride of the per-voxel arrays: [prob][comp][vs], vs >= nvox
  int nprob;
  int C;
  const uint8_t* phase;     // [prob][nvox]
  T* x;                     // unknown field (strain / temperature gradient)
  T* f;                     // field to transform (stress / flux)
  T* r;
  T* p;
  const T* tab;             // tangent factors [prob][2][nvox] (mechanics)
  const T* tn;              // tangent direction [prob][6][nvox] (mechanics)
  c2<T>* spec;              // [prob][nz][ny][PS][C], kx < P used
  Ctl* ctl;
  const ProbInc* inc;
  double* part;             // [prob][NPART][maxblk]
  int maxblk;
  const c2<T>* twx;         // W_nx^j, j < nx
  const c2<T>* twy;
  const c2<T>* twz;
  double len[3];
  double ilen[3];           // 1 / len
  int green;                // Green enum
  int alpha_blocks;         // > 0: the z pass forms the CG step length from the first
                            // alpha_blocks partial sums of the x-forward pass
};

__device__ __forceinline__ bool pipeline_mode(int m) { return m == M_EVAL || m == M_CG || m == M_BASIC; }

}  // namespace hom
