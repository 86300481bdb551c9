// Per-voxel kernels and per-problem reductions (see pointwise.h).
#include <math.h>

#include "pa66.h"
#include "pipeline.h"
#include "pointwise.h"

namespace hom {

constexpr int PT_THREADS = 256;

// Compact index of this lane's voxel among the PA66 voxels of its problem (pa:
// the voxel is one). Every wave of the per-voxel kernels holds the 64 voxels of
// one aligned chunk (v = 64 k + lane), so the index is the chunk's base plus
// the PA66 lanes below this one; lanes past the last voxel are inactive and
// above every active lane.
__device__ __forceinline__ unsigned pa_index(const int* cbase, long long v, bool pa) {
  const unsigned long long m = __ballot(pa);
  const unsigned lane = threadIdx.x & 63;
  const int chunk = __builtin_amdgcn_readfirstlane((int)(v >> 6));
  return (unsigned)cbase[chunk] + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
}

// ---------------------------------------------------------------------------
// Start of an increment: x = x^n + dE (conduction: x += dG) and a fresh
// solver state; keep_x restarts the iteration from the current x instead.
template <typename T, int C>
__global__ void __launch_bounds__(PT_THREADS) k_init(Pt<T> a, int basic, int keep_x) {
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const ProbInc& in = a.inc[prob];
  if (blk == 0 && threadIdx.x == 0) {
    Ctl& c = a.ctl[prob];
    c.mode = basic ? M_BASIC : M_EVAL;
    c.newton_it = 0;
    c.cg_it = 0;
    c.cg_ready = 0;
    c.pending = 0;
    c.status = 0;
    c.pipelines = 0;
    c.krylov = 0;
    c.rr = c.alpha = c.beta = c.res = c.fnorm = c.cg_target = 0.0;
  }
  if (keep_x) return;
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * C * vs;
  // predictor: add s times the fluctuation that the last committed increment added
  const bool pred = C == 6 && a.dx && in.pred_s != 0.0;
  const T ps = T(in.pred_s);
  for (long long v = (long long)blk * PT_THREADS + threadIdx.x; v < nv; v += (long long)a.bpp * PT_THREADS) {
    if constexpr (C == 6) {
      if (pred) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
          a.x[fo + c * vs + v] =
              a.xn[fo + c * vs + v] + T(in.dE[c]) + ps * (a.dx[fo + c * vs + v] - T(in.dEp[c]));
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) a.x[fo + c * vs + v] = a.xn[fo + c * vs + v] + T(in.dE[c]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.x[fo + c * vs + v] += T(in.dG[c]);
    }
  }
}

template <typename T, int C>
__global__ void __launch_bounds__(PT_THREADS) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_eval(Pt<T> a) {
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const Ctl& ctl = a.ctl[prob];
  const int mode = ctl.mode;
  if (mode != M_EVAL && mode != M_BASIC) return;
  const bool pending = ctl.pending != 0;  // last CG step x += alpha p not yet applied
  const T alpha = T(ctl.alpha);
  const bool want_tan = (mode == M_EVAL);
  const ProbInc& in = a.inc[prob];
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * C * vs;
  const uint8_t* phase = a.phase + (long long)prob * vs;
  const long long step = (long long)a.bpp * PT_THREADS;
  // the next voxel's strain, CG step and phase are loaded while this voxel's
  // internal variables are read and its law is evaluated
  T xn[C], pn[C];
  int phn = 0;
  const auto fetch = [&](long long w) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      xn[c] = ldnt(a.x + fo + c * vs + w);
      pn[c] = pending ? ldnt(a.p + fo + c * vs + w) : T(0);
    }
    phn = phase[w];
  };
  long long v = (long long)blk * PT_THREADS + threadIdx.x;
  if (v < nv) fetch(v);
  for (; v < nv; v += step) {
    T e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T xv = xn[c];
      if (pending) {
        xv += alpha * pn[c];
        stnt(a.x + fo + c * vs + v, xv);
      }
      e[c] = xv;
    }
    const int ph = phn;
    if (v + step < nv) fetch(v + step);
    if constexpr (C == 6) {
      double sg[6];
      double ca, cb = 0.0;
      const long long to = (long long)prob * 2 * vs;
      const bool isp = ph == in.pa_phase;
      const unsigned q = a.state ? pa_index(a.cbase + (long long)prob * ((nv + 63) >> 6), v, isp) : 0u;
      if (isp) {
        double ed[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) ed[c] = (double)e[c];
        const double* st = a.state + (long long)prob * a.nstate * a.ss;
        double* hs = a.hist ? a.hist + (long long)prob * HIST_SLOTS * a.ss : nullptr;
        PaOut o;
        pa66_point(in, ed, st, a.ss, nullptr, nullptr, o, nullptr, nullptr, hs, hs ? hs + 7 * a.ss : nullptr, q);
#pragma unroll
        for (int c = 0; c < 6; ++c) sg[c] = o.sig[c];
        ca = o.a;
        cb = o.b;
        if (want_tan && cb != 0.0) {
          const long long no = (long long)prob * 6 * vs;
#pragma unroll
          for (int c = 0; c < 6; ++c) stnt(a.tn + no + c * vs + v, T(o.nd[c]));
        }
      } else {
        const PhaseInc& pi = in.ph[ph];
        const double tr3 = ((double)e[0] + (double)e[1] + (double)e[2]) * (1.0 / 3.0);
        const double sph = pi.K3 * (tr3 - pi.alpha_dth) - pi.G2 * tr3;
#pragma unroll
        for (int c = 0; c < 6; ++c) sg[c] = pi.G2 * (double)e[c];
        sg[0] += sph;
        sg[1] += sph;
        sg[2] += sph;
        ca = pi.G2;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) stnt(a.f + fo + c * vs + v, T(sg[c]));
      if (want_tan) {
        stnt(a.tab + to + v, T(ca));
        stnt(a.tab + to + vs + v, T(cb));
      }
    } else {
      const T kap = T(in.ph[ph].kappa);
#pragma unroll
      for (int c = 0; c < C; ++c) stnt(a.f + fo + c * vs + v, kap * e[c]);
    }
  }
}

// Branch history sums of the PA66 voxels for the increment about to be solved.
template <typename T>
__global__ void __launch_bounds__(PT_THREADS) k_history(Pt<T> a) {
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const ProbInc& in = a.inc[prob];
  // the compacted PA66 voxels in order: no phase test, whole cache lines
  const long long ss = a.ss, ns = a.npa[prob];
  const double* st = a.state + (long long)prob * a.nstate * ss;
  double* h = a.hist + (long long)prob * HIST_SLOTS * ss;
  for (long long ql = (long long)blk * PT_THREADS + threadIdx.x; ql < ns; ql += (long long)a.bpp * PT_THREADS) {
    const unsigned q = (unsigned)ql;
    double hd[6], hs;
    pa66_history(in, st, ss, hd, hs, q);
#pragma unroll
    for (int c = 0; c < 6; ++c) stnt(pa_at(h + c * ss, q), hd[c]);
    stnt(pa_at(h + 6 * ss, q), hs);
    stnt(pa_at(h + 7 * ss, q), -1.0);  // no plastic increment known yet
  }
}

// One-kernel commit: the effective sums of a converged increment and, with
// a.commit = 1, the new internal variables, the committed strain and the
// stress field (a.commit = 0: the sums of an increment that is not final
// yet). It serves conduction, mechanics without internal variables, and the
// basic scheme, whose last evaluation precedes its last strain update;
// otherwise k_commit_vox below takes the mechanics.
template <typename T, int C>
__global__ void __launch_bounds__(PT_THREADS) k_commit(Pt<T> a) {
  constexpr int NS = C == 6 ? MECH_SUMS : 8;
  __shared__ double red[NS * 16];
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const Ctl& ctl = a.ctl[prob];
  if (ctl.status != 1) return;
  const ProbInc& in = a.inc[prob];
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * C * vs;
  const uint8_t* phase = a.phase + (long long)prob * vs;
  const bool commit = a.commit != 0;
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  for (long long v = (long long)blk * PT_THREADS + threadIdx.x; v < nv; v += (long long)a.bpp * PT_THREADS) {
    const int ph = phase[v];
    if constexpr (C == 6) {
      double e[6], en[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        e[c] = (double)a.x[fo + c * vs + v];
        en[c] = (double)a.xn[fo + c * vs + v];
      }
      double sg[6], dis = 0.0, cpl;
      const bool isp = ph == in.pa_phase;
      const unsigned q = a.state ? pa_index(a.cbase + (long long)prob * ((nv + 63) >> 6), v, isp) : 0u;
      if (isp) {
        double* st = a.state + (long long)prob * a.nstate * a.ss;
        // the branch history sums of this increment are in hist (the state
        // has not changed since they were formed): one pass over the branches
        const double* hs = a.hist ? a.hist + (long long)prob * HIST_SLOTS * a.ss : nullptr;
        double* dps = a.hist ? a.hist + (long long)prob * HIST_SLOTS * a.ss + 7 * a.ss : nullptr;
        PaOut o;
        pa66_point(in, e, st, a.ss, commit ? st : nullptr, en, o, &dis, &cpl, hs, dps, q);
#pragma unroll
        for (int c = 0; c < 6; ++c) sg[c] = o.sig[c];
      } else {
        const PhaseInc& pi = in.ph[ph];
        const double tr3 = (e[0] + e[1] + e[2]) * (1.0 / 3.0);
        const double sph = pi.K3 * (tr3 - pi.alpha_dth) - pi.G2 * tr3;
#pragma unroll
        for (int c = 0; c < 6; ++c) sg[c] = pi.G2 * e[c];
        sg[0] += sph;
        sg[1] += sph;
        sg[2] += sph;
        const double trd = (e[0] - en[0]) + (e[1] - en[1]) + (e[2] - en[2]);
        // Gough-Joule: D = -theta eps_dot : C[alpha] (paper Sec. 4, E-glass)
        cpl = -in.theta * pi.K3 * pi.alpha0 * trd / in.dt;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        acc[c] += sg[c];
        acc[8 + c] += e[c];
      }
      acc[6] += dis;
      acc[7] += cpl;
      if (!commit) continue;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        a.xn[fo + c * vs + v] = T(e[c]);  // the committed strain (exact: e was read from T)
        a.f[fo + c * vs + v] = T(sg[c]);
      }
      if (a.dx)
#pragma unroll
        for (int c = 0; c < 6; ++c) a.dx[fo + c * vs + v] = T(e[c] - en[c]);
      if (a.pv_diss) {
        a.pv_diss[(long long)prob * vs + v] = dis;
        a.pv_coup[(long long)prob * vs + v] = cpl;
      }
    } else {
      const double kap = in.ph[ph].kappa;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] -= kap * (double)a.x[fo + c * vs + v];
    }
  }
  block_sum<NS>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) a.part[part_index(prob, k, blk, a.maxblk)] = acc[k];
  }
}

// Effective sums (and, with a.commit = 1, the commit) of a converged
// increment for mechanics with internal variables whose last evaluation was
// at the converged strain (a.dp_known = 1: its plastic increments are in the
// increment slots): the radial return at that plastic increment without the
// scalar Newton iteration, the new eps_p and eps_vp, the Maxwell branches
// streamed PA66_GROUP at a time, the committed strain and stress fields, and
// the effective sums. One voxel per thread (a.bpp = ceil(nvox / PT_THREADS)):
// without a voxel loop the loop-invariant constants of the FP64 exp/log do
// not hold registers for the whole kernel, and more waves keep loads in
// flight. A trial (a.commit = 0) runs the same arithmetic without the writes,
// so that its sums equal those of the commit bit for bit.
template <typename T>
__global__ void __launch_bounds__(PT_THREADS) k_commit_vox(Pt<T> a) {
  __shared__ double red[MECH_SUMS * 16];
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const Ctl& ctl = a.ctl[prob];
  if (ctl.status != 1) return;
  const ProbInc& in = a.inc[prob];
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * 6 * vs;
  const uint8_t* phase = a.phase + (long long)prob * vs;
  const double k3 = pa66_k3_total(in);
  const bool commit = a.commit != 0;
  // uniform bases; the voxel is a 32-bit offset
  const T* xb = a.x + fo;
  T* xnb = a.xn + fo;
  T* fb = a.f + fo;
  T* dxb = a.dx ? a.dx + fo : nullptr;
  double* st = a.state + (long long)prob * a.nstate * a.ss;
  const double* hs = a.hist + (long long)prob * HIST_SLOTS * a.ss;
  const long long ss = a.ss;
  const int* cbase = a.cbase + (long long)prob * ((nv + 63) >> 6);
  double* pvd = commit && a.pv_diss ? a.pv_diss + (long long)prob * vs : nullptr;
  double* pvc = commit && a.pv_coup ? a.pv_coup + (long long)prob * vs : nullptr;
  double acc[MECH_SUMS];
#pragma unroll
  for (int k = 0; k < MECH_SUMS; ++k) acc[k] = 0.0;
  const long long vl = (long long)blk * PT_THREADS + threadIdx.x;
  if (vl < nv) {
    const unsigned v = (unsigned)vl;
    const int ph = *pa_at(phase, v);
    double e[6], en[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      e[c] = (double)*pa_at(xb + c * vs, v);
      en[c] = (double)*pa_at(xnb + c * vs, v);
    }
    double sg[6], dis = 0.0, cpl;
    const double trd = (e[0] - en[0]) + (e[1] - en[1]) + (e[2] - en[2]);
    const bool isp = ph == in.pa_phase;
    const unsigned q = pa_index(cbase, vl, isp);
    if (isp) {
      PaOut o;
      PaPre p;
      pa66_return_at(in, e, st, ss, hs, ldnt(pa_at(hs + 7 * ss, q)), o, p, q);
      const double k15 = 1.2247448713915890 * o.dp;
      double dn[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double evp1 = p.evp[c] + k15 * o.nd[c];
        dn[c] = p.d[c] - evp1;
        if (commit) *pa_at(st + (1 + c) * ss, q) = evp1;
      }
      const double ep1 = p.ep + o.dp;
      if (commit) *pa_at(st, q) = ep1;
      double wsum, ksum;
      pa66_branches(in, st, ss, commit ? st : nullptr, dn, p.em, wsum, ksum, q);
      const double Hn = ep1 > 0.0 ? in.hk * powpos(ep1, in.nh) : 0.0;
      dis = (in.sY * o.dp + wsum) / in.dt;
      cpl = -in.theta * (in.alpha0 * (k3 * trd - 3.0 * ksum) + in.beta1 * Hn * o.dp) / in.dt + dis;
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = o.sig[c];
    } else {
      const PhaseInc& pi = in.ph[ph];
      const double tr3 = (e[0] + e[1] + e[2]) * (1.0 / 3.0);
      const double sph = pi.K3 * (tr3 - pi.alpha_dth) - pi.G2 * tr3;
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = pi.G2 * e[c];
      sg[0] += sph;
      sg[1] += sph;
      sg[2] += sph;
      // Gough-Joule: D = -theta eps_dot : C[alpha] (paper Sec. 4, E-glass)
      cpl = -in.theta * pi.K3 * pi.alpha0 * trd / in.dt;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      acc[c] = sg[c];
      acc[8 + c] = e[c];
    }
    acc[6] = dis;
    acc[7] = cpl;
    if (commit) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        *pa_at(xnb + c * vs, v) = T(e[c]);  // the committed strain (exact: e was read from T)
        *pa_at(fb + c * vs, v) = T(sg[c]);
      }
      if (dxb)
#pragma unroll
        for (int c = 0; c < 6; ++c) *pa_at(dxb + c * vs, v) = T(e[c] - en[c]);
      if (pvd) {
        *pa_at(pvd, v) = dis;
        *pa_at(pvc, v) = cpl;
      }
    }
  }
  block_sum<MECH_SUMS>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < MECH_SUMS; ++k) a.part[part_index(prob, k, blk, a.maxblk)] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// effective algorithmic tangents (paper Sec. 3.3: derivatives of the effective
// stress and coupling term with respect to the macro strain and temperature,
// taken after Newton's method has converged). The strain-jump derivatives of
// the paper become fluctuation fields of the cell problem linearized at the
// converged strain: x_j with mean E_j, and x_theta with mean zero and source
// d sigma / d theta, both equilibrated with the algorithmic tangent.
// ---------------------------------------------------------------------------

// Start of a linearized solve: x = dE (uniform), Newton state reset.
template <typename T>
__global__ void __launch_bounds__(PT_THREADS) k_init_linear(Pt<T> a) {
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const ProbInc& in = a.inc[prob];
  if (blk == 0 && threadIdx.x == 0) {
    Ctl& c = a.ctl[prob];
    c.mode = M_EVAL;
    c.newton_it = c.cg_it = c.cg_ready = c.pending = c.status = c.pipelines = c.krylov = 0;
    c.rr = c.alpha = c.beta = c.res = c.fnorm = c.cg_target = 0.0;
  }
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * 6 * vs;
  for (long long v = (long long)blk * PT_THREADS + threadIdx.x; v < nv; v += (long long)a.bpp * PT_THREADS) {
    if (a.x0) {  // an earlier solution of the same column: same mean, close fluctuation
#pragma unroll
      for (int c = 0; c < 6; ++c) stnt(a.x + fo + c * vs + v, ldnt(a.x0 + fo + c * vs + v));
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) stnt(a.x + fo + c * vs + v, T(in.dE[c]));
    }
  }
}

// sigma = C x (+ s0), C = 3K P1 + a P2 + b N N with (a, b, N) of the last
// Newton evaluation and 3K of the voxel's phase (the operator of the CG steps).
template <typename T>
__global__ void __launch_bounds__(PT_THREADS) k_eval_linear(Pt<T> a) {
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  const Ctl& ctl = a.ctl[prob];
  if (ctl.mode != M_EVAL) return;
  const bool pending = ctl.pending != 0;
  const T alpha = T(ctl.alpha);
  const ProbInc& in = a.inc[prob];
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * 6 * vs;
  const long long to = (long long)prob * 2 * vs;
  const uint8_t* phase = a.phase + (long long)prob * vs;
  for (long long v = (long long)blk * PT_THREADS + threadIdx.x; v < nv; v += (long long)a.bpp * PT_THREADS) {
    double e[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      T xv = ldnt(a.x + fo + c * vs + v);
      if (pending) {
        xv += alpha * ldnt(a.p + fo + c * vs + v);
        stnt(a.x + fo + c * vs + v, xv);
      }
      e[c] = (double)xv;
    }
    const double ca = (double)ldnt(a.tab + to + v);
    const double cb = (double)ldnt(a.tab + to + vs + v);
    const double K3 = in.ph[phase[v]].K3;
    const double tr3 = (e[0] + e[1] + e[2]) * (1.0 / 3.0);
    const double sph = (K3 - ca) * tr3;
    double sg[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sg[c] = ca * e[c] + (c < 3 ? sph : 0.0);
    if (cb != 0.0) {
      double nd[6], dot = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        nd[c] = (double)ldnt(a.tn + fo + c * vs + v);
        dot += nd[c] * e[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] += cb * dot * nd[c];
    }
    if (a.s0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] += (double)ldnt(a.s0 + fo + c * vs + v);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) stnt(a.f + fo + c * vs + v, T(sg[c]));
  }
}

// Point partials at the converged strain x, from state n (run before the
// commit of a converged increment): d sigma / d theta, d D / d eps and
// d D / d theta of the coupling term D. Thermoelastic phases in closed form
// (sigma = C[eps - alpha (theta - theta0)], D = -theta C[alpha] : eps_dot);
// the PA66 law by central differences of its implicit Euler update: 2
// evaluations at theta +- h_theta (with the branch history sums of those
// temperatures) and 12 at eps +- h_eps along each Mandel direction.
template <typename T>
__global__ void __launch_bounds__(PT_THREADS) k_partials(Pt<T> a) {
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  if (a.ctl[prob].status != 1) return;
  const ProbInc& in = a.inc[prob];
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * 6 * vs;
  const uint8_t* phase = a.phase + (long long)prob * vs;
  for (long long v = (long long)blk * PT_THREADS + threadIdx.x; v < nv; v += (long long)a.bpp * PT_THREADS) {
    const int ph = phase[v];
    double e[6], en[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      e[c] = (double)a.x[fo + c * vs + v];
      en[c] = (double)a.xn[fo + c * vs + v];
    }
    double st_[6], gd[6], hd;
    const bool isp = ph == in.pa_phase;
    const unsigned q = a.state ? pa_index(a.cbase + (long long)prob * ((nv + 63) >> 6), v, isp) : 0u;
    if (isp) {
      const double* st = a.state + (long long)prob * a.nstate * a.ss;
      const double* hs = a.hist ? a.hist + (long long)prob * HIST_SLOTS * a.ss : nullptr;
      double sp[6], Dp = 0.0;
      for (int k = 0; k < 14; ++k) {
        const bool th = k < 2;
        const ProbInc& ik = th ? a.inc_pm[2 * prob + k] : in;
        double ek[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) ek[c] = e[c];
        const int dir = (k - 2) >> 1;
        if (!th) ek[dir] += (k & 1) ? -FD_H_EPS : FD_H_EPS;
        PaOut o;
        double dis, cpl;
        pa66_point(ik, ek, st, a.ss, nullptr, en, o, &dis, &cpl, th ? nullptr : hs, nullptr, q);
        if (!(k & 1)) {  // + side: keep it for the difference with the - side
#pragma unroll
          for (int c = 0; c < 6; ++c) sp[c] = o.sig[c];
          Dp = cpl;
        } else if (th) {
#pragma unroll
          for (int c = 0; c < 6; ++c) st_[c] = (sp[c] - o.sig[c]) * (0.5 / FD_H_THETA);
          hd = (Dp - cpl) * (0.5 / FD_H_THETA);
        } else {
          gd[dir] = (Dp - cpl) * (0.5 / FD_H_EPS);
        }
      }
    } else {
      const PhaseInc& pi = in.ph[ph];
      const double ca = pi.K3 * pi.alpha0;  // C[alpha] = 3K alpha0 on the normal components
      const double trd = (e[0] - en[0]) + (e[1] - en[1]) + (e[2] - en[2]);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        st_[c] = c < 3 ? -ca : 0.0;
        gd[c] = c < 3 ? -in.theta * ca / in.dt : 0.0;
      }
      hd = -ca * trd / in.dt;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      a.dsdt[fo + c * vs + v] = T(st_[c]);
      a.dDde[fo + c * vs + v] = T(gd[c]);
    }
    a.dDdt[(long long)prob * vs + v] = T(hd);
  }
}

// Per-block sums over the voxels of a converged linearized solve: the stress
// (6) and, if the partials are kept, dD/deps . x and dD/dtheta.
template <typename T>
__global__ void __launch_bounds__(PT_THREADS) k_tangent_sum(Pt<T> a) {
  __shared__ double red[8 * 16];
  const int prob = blockIdx.x / a.bpp;
  const int blk = blockIdx.x % a.bpp;
  if (a.ctl[prob].status != 1) return;
  const long long nv = a.nvox;
  const long long vs = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * 6 * vs;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  for (long long v = (long long)blk * PT_THREADS + threadIdx.x; v < nv; v += (long long)a.bpp * PT_THREADS) {
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += (double)ldnt(a.f + fo + c * vs + v);
    if (a.dDde) {
#pragma unroll
      for (int c = 0; c < 6; ++c)
        acc[6] += (double)ldnt(a.dDde + fo + c * vs + v) * (double)ldnt(a.x + fo + c * vs + v);
      acc[7] += (double)ldnt(a.dDdt + (long long)prob * vs + v);
    }
  }
  block_sum<8>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a.part[part_index(prob, k, blk, a.maxblk)] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// per-problem reductions and state transitions (one block per problem)
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 1024;

// Fixed-order sums of the first NK quantities over the blocks' partials: each
// thread takes blocks tid, tid + blockDim, ... of every quantity (contiguous
// runs), then a fixed tree over the threads.
template <int NK>
__device__ __forceinline__ void sum_parts(const double* part, int maxblk, int nblk, int prob, double* out,
                                          double* red /* >= NK * 16 */) {
  double v[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) v[k] = 0.0;
  const double* base = part + part_index(prob, 0, 0, maxblk);
#pragma unroll 4
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NK; ++k) v[k] += base[(long long)k * maxblk + b];
  }
  block_sum<NK>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NK; ++k) out[k] = v[k];
  }
  __syncthreads();
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_a(Ctl* ctl, const double* part, int maxblk, int nblk,
                                                           Limits lim) {
  __shared__ double red[2 * 16];
  __shared__ double s[2];
  const int prob = blockIdx.x;
  Ctl& c = ctl[prob];
  const int mode = c.mode;
  if (!(mode == M_EVAL || mode == M_BASIC || (mode == M_CG && c.cg_ready))) return;
  sum_parts<2>(part, maxblk, nblk, prob, s, red);
  if (threadIdx.x != 0) return;
  c.pipelines += 1;
  if (mode == M_CG) {
    // after the CG update of the x-inverse pass: s[0] = r.r of the new residual
    const double rn = s[0];
    c.beta = c.rr > 0.0 ? rn / c.rr : 0.0;
    c.rr = rn;
    c.cg_it += 1;
    c.krylov += 1;
    c.cg_ready = 0;
    if (!isfinite(rn)) {
      c.mode = M_FAIL;
      c.status = -4;
    } else if (rn <= c.cg_target || c.cg_it >= lim.max_krylov) {
      c.mode = M_EVAL;
      c.pending = 1;
    }
  } else if (mode == M_EVAL) {
    const double rr = s[0], ff = s[1];
    const double res = ff > 0.0 ? sqrt(rr / ff) : 0.0;
    c.res = res;
    c.fnorm = sqrt(ff);
    c.newton_it += 1;
    c.pending = 0;
    if (!isfinite(res)) {
      c.mode = M_FAIL;
      c.status = -4;
    } else if (res <= lim.tol) {
      c.mode = M_DONE;
      c.status = 1;
    } else if (c.newton_it > lim.max_newton) {
      c.mode = M_FAIL;
      c.status = -3;
    } else {
      const double eta = lim.linear ? 0.0 : fmin(0.1, res);
      const double tgt = fmax(eta * sqrt(rr), 0.5 * lim.tol * sqrt(ff));
      c.cg_target = tgt * tgt;
      c.rr = rr;
      c.cg_it = 0;
      c.cg_ready = 0;
      c.beta = 0.0;
      c.mode = M_CG;
    }
  } else {  // basic scheme
    const double dd = s[0], xx = s[1];
    const double err = xx > 0.0 ? sqrt(dd / xx) : 0.0;
    c.res = err;
    c.newton_it += 1;
    if (!isfinite(err)) {
      c.mode = M_FAIL;
      c.status = -4;
    } else if (err <= lim.tol) {
      c.mode = M_DONE;
      c.status = 1;
    } else if (c.newton_it >= lim.max_newton) {
      c.mode = M_FAIL;
      c.status = -3;
    }
  }
}

constexpr int RED_STAGE_THREADS = 256;
__global__ void __launch_bounds__(RED_STAGE_THREADS) k_reduce_stage(const double* part, int maxblk, int nblk,
                                                                    double* out, int nout) {
  __shared__ double red[NPART * 16];
  const int prob = blockIdx.x / nout;
  const int j = blockIdx.x % nout;
  const int b0 = j * RED_CHUNK;
  const int nb = min(RED_CHUNK, nblk - b0);
  double v[NPART];
#pragma unroll
  for (int k = 0; k < NPART; ++k) v[k] = 0.0;
  const double* base = part + part_index(prob, 0, b0, maxblk);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] += base[(long long)k * maxblk + b];
  }
  block_sum<NPART>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) out[part_index(prob, k, j, nout)] = v[k];
  }
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_out(Ctl* ctl, const double* part, int maxblk, int nblk,
                                                             int nk, double scale) {
  __shared__ double red[NPART * 16];
  __shared__ double s[NPART];
  const int prob = blockIdx.x;
  Ctl& c = ctl[prob];
  if (c.status != 1) return;
  sum_parts<NPART>(part, maxblk, nblk, prob, s, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < nk; ++k) c.out[k] = s[k] * scale;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_init_mech(const Pt<T>& a, int scheme, hipStream_t s, int keep_x) {
  hipLaunchKernelGGL((k_init<T, 6>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a, scheme == 0 ? 1 : 0, keep_x);
}
template <typename T>
void launch_init_th(const Pt<T>& a, int scheme, hipStream_t s) {
  hipLaunchKernelGGL((k_init<T, 3>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a, scheme == 0 ? 1 : 0, 0);
}
template <typename T>
void launch_eval(const Pt<T>& a, int C, hipStream_t s) {
  if (C == 6)
    hipLaunchKernelGGL((k_eval<T, 6>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((k_eval<T, 3>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
}
template <typename T>
void launch_history(const Pt<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_history<T>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
}
template <typename T>
int launch_commit(const Pt<T>& a, int C, hipStream_t s) {
  static_assert(PT_THREADS == 256, "commit_voxel_blocks takes 256 voxels a block");
  if (commit_per_voxel(a, C)) {
    Pt<T> b = a;
    b.bpp = commit_voxel_blocks(a.nvox);
    hipLaunchKernelGGL((k_commit_vox<T>), dim3((long long)b.nprob * b.bpp), dim3(PT_THREADS), 0, s, b);
    return b.bpp;
  }
  if (C == 6)
    hipLaunchKernelGGL((k_commit<T, 6>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((k_commit<T, 3>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
  return a.bpp;
}
void launch_reduce_a(Ctl* ctl, const double* part, int maxblk, int nblk, int nprob, Limits lim, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_a, dim3(nprob), dim3(RED_THREADS), 0, s, ctl, part, maxblk, nblk, lim);
}
void launch_reduce_stage(const double* part, int maxblk, int nblk, double* out, int nout, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stage, dim3((long long)nprob * nout), dim3(RED_STAGE_THREADS), 0, s, part, maxblk, nblk,
                     out, nout);
}
void launch_reduce_out(Ctl* ctl, const double* part, int maxblk, int nblk, int nprob, int nk, double scale,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_out, dim3(nprob), dim3(RED_THREADS), 0, s, ctl, part, maxblk, nblk, nk, scale);
}

template <typename T>
void launch_eval_linear(const Pt<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_eval_linear<T>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
}
template <typename T>
void launch_init_linear(const Pt<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_init_linear<T>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
}
template <typename T>
void launch_partials(const Pt<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_partials<T>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
}
template <typename T>
void launch_tangent_sum(const Pt<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_tangent_sum<T>), dim3(a.nprob * a.bpp), dim3(PT_THREADS), 0, s, a);
}

#define HOM_INST_PT(T)                                                  \
  template void launch_eval_linear<T>(const Pt<T>&, hipStream_t);       \
  template void launch_init_linear<T>(const Pt<T>&, hipStream_t);       \
  template void launch_partials<T>(const Pt<T>&, hipStream_t);          \
  template void launch_tangent_sum<T>(const Pt<T>&, hipStream_t);       \
  template void launch_init_mech<T>(const Pt<T>&, int, hipStream_t, int); \
  template void launch_init_th<T>(const Pt<T>&, int, hipStream_t);      \
  template void launch_eval<T>(const Pt<T>&, int, hipStream_t);         \
  template void launch_history<T>(const Pt<T>&, hipStream_t);           \
  template int launch_commit<T>(const Pt<T>&, int, hipStream_t);
HOM_INST_PT(float)
HOM_INST_PT(double)

}  // namespace hom
