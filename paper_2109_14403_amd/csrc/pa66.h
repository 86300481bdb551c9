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

// Branch history sums of one voxel, fixed during an increment (they depend on
// the viscous strains of step n and on theta, dt only):
//   hd = sum_i 2 G_i D_i / (1 + rG_i)   (deviatoric, 6 Mandel components)
//   hs = sum_i 3 K_i S_i / (1 + rK_i)   (S_i = tr(eps_v_i) / 3)
// so that the trial stress is s_tr = 2 Gbar (dev eps - eps_vp) - hd and the
// spherical stress 3 Kbar tr(e)/3 - hs.
__device__ __forceinline__ void pa66_history(const ProbInc& in, const double* st, long long ss, double* hd,
                                             double& hs) {
#pragma unroll
  for (int c = 0; c < 6; ++c) hd[c] = 0.0;
  hs = 0.0;
  for (int i = 0; i < in.nm; ++i) {
    const double* ev = st + (7 + 6 * i) * ss;
    const double v0 = ldnt(ev), v1 = ldnt(ev + ss), v2 = ldnt(ev + 2 * ss);
    const double sn = (v0 + v1 + v2) * (1.0 / 3.0);
    const double w = in.G2i[i] * in.fG[i];
    hd[0] += w * (v0 - sn);
    hd[1] += w * (v1 - sn);
    hd[2] += w * (v2 - sn);
    hd[3] += w * ldnt(ev + 3 * ss);
    hd[4] += w * ldnt(ev + 4 * ss);
    hd[5] += w * ldnt(ev + 5 * ss);
    hs += in.K3i[i] * in.fK[i] * sn;
  }
}

// Trial / final evaluation. If `hist` is non-null the branch history sums are
// read from it ([HIST_SLOTS][ss]: hd, hs, dp), else computed from the state.
// `dp_slot`, if non-null, holds the plastic increment of the voxel's previous
// evaluation in this increment (negative: none), the start of the scalar
// Newton iteration; a trial evaluation stores its result there. If `diss` is
// non-null the dissipation and coupling term are computed, and if `st_out`
// is non-null too the new internal variables are written there.
static __device__ void pa66_point(const ProbInc& in, const double* eps, const double* st, long long ss, double* st_out,
                           const double* eps_n, PaOut& o, double* diss, double* coup,
                           const double* hist = nullptr, double* dp_slot = nullptr) {
  const double tr3 = (eps[0] + eps[1] + eps[2]) * (1.0 / 3.0);
  const double em = tr3 - in.ph[in.pa_phase].alpha_dth;
  double d[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) d[c] = eps[c];
  d[0] -= tr3;
  d[1] -= tr3;
  d[2] -= tr3;
  const double ep = ldnt(st);
  double evp[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) evp[c] = ldnt(st + (1 + c) * ss);
  double hd[6], hs;
  if (hist) {
#pragma unroll
    for (int c = 0; c < 6; ++c) hd[c] = ldnt(hist + c * ss);
    hs = ldnt(hist + 6 * ss);
  } else {
    pa66_history(in, st, ss, hd, hs);
  }
  double str[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) str[c] = in.Gbar2 * (d[c] - evp[c]) - hd[c];
  const double sph = in.Kbar3 * em - hs;
  double sn2 = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) sn2 += str[c] * str[c];
  const double snrm = sqrt(sn2);
  const double seq = 1.2247448713915890 * snrm;  // sqrt(3/2) |s|
  const double H = ep > 0.0 ? in.hk * powpos(ep, in.nh) : 0.0;
  const double f = seq - in.sY - H;
  double dp = 0.0, th1 = 1.0, cp = 1.0;
  const double G3 = 1.5 * in.Gbar2;
  if (f > 0.0 && snrm > 0.0) {
    double dgd;
    dp = pa66_solve_dp(in, seq, ep, f, G3, dp_slot ? *dp_slot : -1.0, dgd);
    th1 = 1.0 - G3 * dp / seq;
    cp = 1.0 - G3 * dgd;
  }
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
  if (!diss) {
    if (dp_slot) *dp_slot = dp;
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
    if (st_out) st_out[(1 + c) * ss] = evp1[c];
  }
  const double ep1 = ep + dp;
  if (st_out) st_out[0] = ep1;
  double dis = in.sY * dp;
  double trd = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) trd += eps[c] - eps_n[c];
  double trsum = in.Kinf3 * trd;
  for (int i = 0; i < in.nm; ++i) {
    const double* ev = st + (7 + 6 * i) * ss;
    double* evo = st_out ? st_out + (7 + 6 * i) * ss : nullptr;
    double v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = ev[c * ss];
    const double sn = (v[0] + v[1] + v[2]) * (1.0 / 3.0);
    const double s1 = in.fK[i] * (sn + in.rK[i] * em);
    double dnew[6], dold[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      dold[c] = v[c] - (c < 3 ? sn : 0.0);
      dnew[c] = in.fG[i] * (dold[c] + in.rG[i] * dn[c]);
    }
    double w = in.K3i[i] * (em - s1) * 3.0 * (s1 - sn);
#pragma unroll
    for (int c = 0; c < 6; ++c) w += in.G2i[i] * (dn[c] - dnew[c]) * (dnew[c] - dold[c]);
    dis += w;
    trsum += in.K3i[i] * (trd - 3.0 * (s1 - sn));
    if (st_out) {
#pragma unroll
      for (int c = 0; c < 6; ++c) evo[c * ss] = dnew[c] + (c < 3 ? s1 : 0.0);
    }
  }
  dis /= dt;
  const double Hn = ep1 > 0.0 ? in.hk * powpos(ep1, in.nh) : 0.0;
  *diss = dis;
  *coup = -in.theta * (in.alpha0 * trsum / dt + in.beta1 * Hn * dp / dt) + dis;
}

}  // namespace hom
