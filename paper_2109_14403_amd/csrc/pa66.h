// PA66 point law (paper Sec. 4), FP64, shared by the cell solver's per-voxel
// kernels and the DMN's leaves. Header-only: every translation unit that
// includes it compiles its own copy of these device functions.
#pragma once
#include <math.h>

#include "common.h"

namespace hom {

// Streaming per-voxel data (fields, internal variables, increment slots) is
// touched once per kernel: non-temporal accesses in the evaluation and the
// history sums (the in-place commit of the internal variables measured faster
// with cached accesses).
template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void stnt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// p + off elements with a 32-bit offset (off * sizeof(T) < 2^32). The per-voxel
// functions below take uniform array bases and the voxel as `off`, so that
// every access has the scalar-base + 32-bit-offset form (no 64-bit address
// arithmetic per access and per component); off = 0 takes p as the voxel's
// own pointer.
template <typename T>
__device__ __forceinline__ T* pa_at(T* p, unsigned off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T* pa_at(const T* p, unsigned off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off * (unsigned)sizeof(T));
}

// ---------------------------------------------------------------------------
// PA66 law (paper Sec. 4) for one voxel, FP64, implicit Euler.
//
// With e = eps - eps_vp - alpha (theta - theta0) I, the viscous strains of the
// Maxwell branches have the closed-form update
//   sph:  S_i' = (S_i + rK_i tr(e)/3) / (1 + rK_i)
//   dev:  D_i' = (D_i + rG_i dev e) / (1 + rG_i),
// rK_i = dt / (a_theta tau_K,i), rG_i = dt / (a_theta tau_G,i). The deviatoric
// stress is then s = 2 Gbar (dev eps - eps_vp') - sum 2 G_i D_i / (1 + rG_i)
// with Gbar = G_inf + sum G_i / (1 + rG_i), so the viscoplastic flow along
// s / |s| reduces to a radial return: s = s_tr (1 - 3 Gbar dp / seq_tr) and the
// plastic increment dp solves the implicit overstress equation
//   g(dp) = dp - dt (sY / eta) <(seq_tr - 3 Gbar dp - sY - H(eps_p + dp)) / sY>^m = 0,
// solved by a bracketed Newton iteration (g is increasing and concave).
// The algorithmic tangent is 3 Kbar P1 + 2 Gbar [th1 (P2 - N N) + cp N N],
// stored as (a, b, N) = (2 Gbar th1, 2 Gbar (cp - th1), N).
// ---------------------------------------------------------------------------
struct PaOut {
  double sig[6];
  double a, b;
  double nd[6];
  double dp;
};

// x^p for x > 0 by one log and one exp (a few ulp; FP64 pow is several
// times dearer and the root is only needed to ~1e-15 relative)
__device__ __forceinline__ double powpos(double x, double p) { return exp(p * log(x)); }

// <x>^m and <x>^(m-1) for x >= 0 (exact products for m = 2)
__device__ __forceinline__ void pow_m(double x, double m, double& xm, double& xm1) {
  if (x > 0.0) {
    if (m == 2.0) {
      xm = x * x;
      xm1 = x;
    } else {
      xm = powpos(x, m);
      xm1 = xm / x;
    }
  } else {
    xm = 0.0;
    xm1 = m > 1.0 ? 0.0 : (m == 1.0 ? 1.0 : INFINITY);
  }
}

// guess: a previous root for nearby data (warm start), used if inside the bracket
__device__ __forceinline__ double pa66_solve_dp(const ProbInc& in, double seq, double ep, double f, double G3,
                                                double guess, double& dgd) {
  double lo = 0.0, hi = f / G3;
  double d = (guess > lo && guess < hi) ? guess : 0.5 * hi;
  const double c = in.ccoef, sY = in.sY, m = in.mexp, hk = in.hk, nh = in.nh;
  const double isY = 1.0 / sY;
  double A = 0.0, hp = INFINITY;
  // step tolerance: the stress correction 3 Gbar dp moves by < 1e-14 seq_tr
  // (a relative test on dp alone can sit below the rounding noise of g)
  const double dtol = 1e-14 * seq / G3;
  for (int it = 0; it < 80; ++it) {
    const double e = ep + d;
    // H(eps_p + d) = hk e^nh and H' = nh hk e^(nh - 1) from one power
    const double hq = e > 0.0 ? hk * powpos(e, nh - 1.0) : 0.0;
    const double he = hq * e;
    const double x = (seq - G3 * d - sY - he) * isY;
    double xm, xm1;
    pow_m(x, m, xm, xm1);
    const double gv = d - c * xm;
    if (gv < 0.0)
      lo = d;
    else
      hi = d;
    hp = e > 0.0 ? nh * hq : INFINITY;  // H'
    A = c * m * xm1 * isY;
    const double gd = 1.0 + A * (G3 + hp);
    const double dn = d - gv / gd;
    // converged: accept the Newton point (it may sit on the bracket end the
    // step came from, so test before the bracket safeguard)
    if (gv == 0.0 || fabs(dn - d) <= dtol) {
      d = fmin(fmax(dn, lo), hi);
      break;
    }
    d = (dn > lo && dn < hi) ? dn : 0.5 * (lo + hi);
    if (hi - lo <= dtol) break;
  }
  // d dp / d seq_tr at the root (from the last step: d moved by <= 1e-15 relative)
  dgd = A > 0.0 ? A / (1.0 + A * (G3 + hp)) : 0.0;
  return d;
}

// Maxwell branches streamed together by the per-voxel branch loops
constexpr int PA66_GROUP = 2;

// Branch history sums of one voxel, fixed during an increment (they depend on
// the viscous strains of step n and on theta, dt only):
//   hd = sum_i 2 G_i D_i / (1 + rG_i)   (deviatoric, 6 Mandel components)
//   hs = sum_i 3 K_i S_i / (1 + rK_i)   (S_i = tr(eps_v_i) / 3)
// so that the trial stress is s_tr = 2 Gbar (dev eps - eps_vp) - hd and the
// spherical stress 3 Kbar tr(e)/3 - hs.
__device__ __forceinline__ void pa66_history(const ProbInc& in, const double* st, long long ss, double* hd,
                                             double& hs, unsigned off = 0) {
#pragma unroll
  for (int c = 0; c < 6; ++c) hd[c] = 0.0;
  hs = 0.0;
  const int nm = in.nm;
  // PA66_GROUP branches a step: all their loads are issued before the first
  // is used (a load index past the last branch repeats the last one, in
  // bounds, and is not summed)
  for (int i0 = 0; i0 < nm; i0 += PA66_GROUP) {
    double v[PA66_GROUP][6];
#pragma unroll
    for (int j = 0; j < PA66_GROUP; ++j) {
      const int i = min(i0 + j, nm - 1);
#pragma unroll
      for (int c = 0; c < 6; ++c) v[j][c] = ldnt(pa_at(st + (7 + 6 * i + c) * ss, off));
    }
#pragma unroll
    for (int j = 0; j < PA66_GROUP; ++j) {
      const int i = i0 + j;
      if (i >= nm) break;
      const double sn = (v[j][0] + v[j][1] + v[j][2]) * (1.0 / 3.0);
      const double w = in.G2i[i] * in.fG[i];
      hd[0] += w * (v[j][0] - sn);
      hd[1] += w * (v[j][1] - sn);
      hd[2] += w * (v[j][2] - sn);
      hd[3] += w * v[j][3];
      hd[4] += w * v[j][4];
      hd[5] += w * v[j][5];
      hs += in.K3i[i] * in.fK[i] * sn;
    }
  }
}

// What the commit of a voxel needs from its evaluation besides PaOut: the
// deviatoric strain, the internal variables of step n (eps_vp, eps_p) and
// tr(eps)/3 - alpha (theta - theta0).
struct PaPre {
  double d[6], evp[6];
  double ep, em;
};

// Trial state of one voxel at strain eps: the strain split and the internal
// variables of step n (p), the deviatoric trial stress str, the spherical
// stress sph and |str|. If `hist` is non-null the branch history sums are
// read from it ([HIST_SLOTS][ss]: hd, hs), else computed from the state.
__device__ __forceinline__ void pa66_trial(const ProbInc& in, const double* eps, const double* st, long long ss,
                                           const double* hist, PaPre& p, double* str, double& sph, double& snrm,
                                           unsigned off = 0) {
  const double tr3 = (eps[0] + eps[1] + eps[2]) * (1.0 / 3.0);
  p.em = tr3 - in.ph[in.pa_phase].alpha_dth;
#pragma unroll
  for (int c = 0; c < 6; ++c) p.d[c] = eps[c];
  p.d[0] -= tr3;
  p.d[1] -= tr3;
  p.d[2] -= tr3;
  p.ep = ldnt(pa_at(st, off));
#pragma unroll
  for (int c = 0; c < 6; ++c) p.evp[c] = ldnt(pa_at(st + (1 + c) * ss, off));
  double hd[6], hs;
  if (hist) {
#pragma unroll
    for (int c = 0; c < 6; ++c) hd[c] = ldnt(pa_at(hist + c * ss, off));
    hs = ldnt(pa_at(hist + 6 * ss, off));
  } else {
    pa66_history(in, st, ss, hd, hs, off);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) str[c] = in.Gbar2 * (p.d[c] - p.evp[c]) - hd[c];
  sph = in.Kbar3 * p.em - hs;
  double sn2 = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) sn2 += str[c] * str[c];
  snrm = sqrt(sn2);
}

// Stress, flow direction and tangent factors of the return with plastic
// increment dp (th1 = 1 - 3 Gbar dp / seq_tr, cp = 1 - 3 Gbar d dp / d seq_tr)
__device__ __forceinline__ void pa66_out(const ProbInc& in, const double* str, double sph, double snrm, double dp,
                                         double th1, double cp, PaOut& o) {
  const double inv = snrm > 0.0 ? 1.0 / snrm : 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    o.nd[c] = str[c] * inv;
    o.sig[c] = th1 * str[c];
  }
  o.sig[0] += sph;
  o.sig[1] += sph;
  o.sig[2] += sph;
  o.a = in.Gbar2 * th1;
  o.b = in.Gbar2 * (cp - th1);
  o.dp = dp;
}

// Radial return of one voxel at strain eps (history sums as in pa66_trial).
// `guess` is the plastic increment of the voxel's previous evaluation in this
// increment (negative: none), the start of the scalar Newton iteration.
__device__ __forceinline__ void pa66_return(const ProbInc& in, const double* eps, const double* st, long long ss,
                                            const double* hist, double guess, PaOut& o, PaPre& p,
                                            unsigned off = 0) {
  double str[6], sph, snrm;
  pa66_trial(in, eps, st, ss, hist, p, str, sph, snrm, off);
  const double seq = 1.2247448713915890 * snrm;  // sqrt(3/2) |s|
  const double H = p.ep > 0.0 ? in.hk * powpos(p.ep, in.nh) : 0.0;
  const double f = seq - in.sY - H;
  double dp = 0.0, th1 = 1.0, cp = 1.0;
  const double G3 = 1.5 * in.Gbar2;
  if (f > 0.0 && snrm > 0.0) {
    double dgd;
    dp = pa66_solve_dp(in, seq, p.ep, f, G3, guess, dgd);
    th1 = 1.0 - G3 * dp / seq;
    cp = 1.0 - G3 * dgd;
  }
  pa66_out(in, str, sph, snrm, dp, th1, cp, o);
}

// The same return with its plastic increment dp known (an evaluation at this
// strain has solved for it): stress and flow direction without the scalar
// Newton iteration (the tangent factor b is left at zero).
__device__ __forceinline__ void pa66_return_at(const ProbInc& in, const double* eps, const double* st, long long ss,
                                               const double* hist, double dp, PaOut& o, PaPre& p,
                                               unsigned off = 0) {
  double str[6], sph, snrm;
  pa66_trial(in, eps, st, ss, hist, p, str, sph, snrm, off);
  const double seq = 1.2247448713915890 * snrm;
  const bool flow = dp > 0.0 && snrm > 0.0;
  const double th1 = flow ? 1.0 - 1.5 * in.Gbar2 * dp / seq : 1.0;
  pa66_out(in, str, sph, snrm, flow ? dp : 0.0, th1, th1, o);
}

// 3 K_inf + sum_i 3 K_i: the trace share of the coupling term that does not
// depend on the branches' viscous strains
__device__ __forceinline__ double pa66_k3_total(const ProbInc& in) {
  double k = in.Kinf3;
  for (int i = 0; i < in.nm; ++i) k += in.K3i[i];
  return k;
}

// Commit of the Maxwell branches of one voxel, given dn = dev eps - eps_vp'
// and em = tr(eps)/3 - alpha (theta - theta0) of the converged strain: the
// closed-form viscous strain update (written to st_out if non-null; st_out
// may be st), the branches' share of the dissipation times dt
//   wsum = sum_i [3 K_i (em - S_i') 3 (S_i' - S_i) + 2 G_i (dn - D_i') : (D_i' - D_i)]
// and ksum = sum_i 3 K_i (S_i' - S_i), the branches' share of the coupling
// term's trace sum (which is (3 K_inf + sum_i 3 K_i) tr(deps) - 3 ksum).
// PA66_GROUP branches a step: their loads are all issued before the first
// store (a load index past the last branch repeats the last one, in bounds;
// it is neither updated nor summed).
__device__ __forceinline__ void pa66_branches(const ProbInc& in, const double* st, long long ss, double* st_out,
                                              const double* dn, double em, double& wsum, double& ksum,
                                              unsigned off = 0) {
  wsum = 0.0;
  ksum = 0.0;
  const int nm = in.nm;
  for (int i0 = 0; i0 < nm; i0 += PA66_GROUP) {
    double v[PA66_GROUP][6];
#pragma unroll
    for (int j = 0; j < PA66_GROUP; ++j) {
      const int i = min(i0 + j, nm - 1);
#pragma unroll
      for (int c = 0; c < 6; ++c) v[j][c] = *pa_at(st + (7 + 6 * i + c) * ss, off);
    }
#pragma unroll
    for (int j = 0; j < PA66_GROUP; ++j) {
      const int i = i0 + j;
      if (i >= nm) break;
      const double sn = (v[j][0] + v[j][1] + v[j][2]) * (1.0 / 3.0);
      const double s1 = in.fK[i] * (sn + in.rK[i] * em);
      double dnew[6], dold[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        dold[c] = v[j][c] - (c < 3 ? sn : 0.0);
        dnew[c] = in.fG[i] * (dold[c] + in.rG[i] * dn[c]);
      }
      double w = in.K3i[i] * (em - s1) * 3.0 * (s1 - sn);
#pragma unroll
      for (int c = 0; c < 6; ++c) w += in.G2i[i] * (dn[c] - dnew[c]) * (dnew[c] - dold[c]);
      wsum += w;
      ksum += in.K3i[i] * (s1 - sn);
      if (st_out) {
        double* evo = st_out + (7 + 6 * i) * ss;
#pragma unroll
        for (int c = 0; c < 6; ++c) *pa_at(evo + c * ss, off) = dnew[c] + (c < 3 ? s1 : 0.0);
      }
    }
  }
}

// Trial / final evaluation. `hist` and the start of the scalar Newton
// iteration as in pa66_return; `dp_slot`, if non-null, holds the start and a
// trial evaluation stores its result there. If `diss` is non-null the
// dissipation and coupling term are computed, and if `st_out` is non-null too
// the new internal variables are written there.
static __device__ void pa66_point(const ProbInc& in, const double* eps, const double* st, long long ss, double* st_out,
                           const double* eps_n, PaOut& o, double* diss, double* coup,
                           const double* hist = nullptr, double* dp_slot = nullptr, unsigned off = 0) {
  PaPre p;
  pa66_return(in, eps, st, ss, hist, dp_slot ? *pa_at(dp_slot, off) : -1.0, o, p, off);
  const double dp = o.dp;
  const double em = p.em, ep = p.ep;
  const double* d = p.d;
  const double* evp = p.evp;
  if (!diss) {
    if (dp_slot) *pa_at(dp_slot, off) = dp;
    return;
  }

  // ---- commit: new internal variables, dissipation, coupling ------------
  const double dt = in.dt;
  const double k15 = 1.2247448713915890 * dp;
  double evp1[6], dn[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    evp1[c] = evp[c] + k15 * o.nd[c];
    dn[c] = d[c] - evp1[c];
    if (st_out) *pa_at(st_out + (1 + c) * ss, off) = evp1[c];
  }
  const double ep1 = ep + dp;
  if (st_out) *pa_at(st_out, off) = ep1;
  double trd = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) trd += eps[c] - eps_n[c];
  double wsum, ksum;
  pa66_branches(in, st, ss, st_out, dn, em, wsum, ksum, off);
  const double dis = (in.sY * dp + wsum) / dt;
  const double trsum = pa66_k3_total(in) * trd - 3.0 * ksum;
  const double Hn = ep1 > 0.0 ? in.hk * powpos(ep1, in.nh) : 0.0;
  *diss = dis;
  *coup = -in.theta * (in.alpha0 * trsum / dt + in.beta1 * Hn * dp / dt) + dis;
}

}  // namespace hom
