// The five-pass FFT / Green-operator pipeline of one solver iteration.
//
//   xfwd   pre-operation per voxel (copy of the stress / flux field, or the
//          algorithmic tangent applied to the CG direction), then real-to-
//          complex transforms along x (two real components packed into one
//          complex line), written as the half spectrum kx = 0..nx/2.
//   ypass  complex transforms along y on tiles of TX contiguous kx columns.
//   zgreen forward transform along z, Green operator per frequency on all
//          components, inverse transform along z.
//   ypass  inverse along y.
//   xinv   complex-to-real inverse along x, scaled by 1/(nx ny nz), then the
//          post-operation per voxel (residual / CG residual update / basic-
//          scheme update) with FP64 partial sums for the reductions.
//
// CG keeps three fields (x, r, p): the step x += alpha p of iteration k is
// deferred to the x-forward pass of iteration k + 1 (or to the next
// constitutive evaluation), which reads the old p anyway.
//
// Every kernel serves all problems of a group in one launch: blockIdx.x runs
// over (problem, tile), and a block whose problem is not iterating exits at
// once.
#pragma once
#include "common.h"

namespace hom {

// Sum of per-thread doubles over the block, deterministic (fixed tree).
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red /* >= K * 16 doubles */) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * 16 + wave] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[k * 16 + w];
      v[k] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Green operators on a Mandel (C = 6) or vector (C = 3) complex array.
// ---------------------------------------------------------------------------
// Signed frequency of index k on an n-point axis over a length with
// reciprocal il; the Nyquist entry of an even axis is nulled.
template <typename T>
__device__ __forceinline__ T frequency_component(int k, int n, T il) {
  int sk = k < (n + 1) / 2 ? k : k - n;
  if ((n & 1) == 0 && k == n / 2) sk = 0;
  return T(sk) * il;
}

// 1 / sqrt(m2) for m2 > 0: the hardware reciprocal square root (1 ulp) in
// FP32, the correctly rounded quotient in FP64
__device__ __forceinline__ float inv_norm(float m2) { return __builtin_amdgcn_rsqf(m2); }
__device__ __forceinline__ double inv_norm(double m2) { return 1.0 / sqrt(m2); }

template <typename T>
__device__ __forceinline__ void green_mech(c2<T>* v, T n0, T n1, T n2, T cs, T hcn) {
  // out = cs (n (x) u + u (x) n) - cn (n . u) n (x) n with u = tau n, applied
  // to real and imaginary parts (projector: cs = 1, cn = 1), as
  //   w = cs u - (cn / 2) (n . u) n,  out_ii = 2 n_i w_i,
  //   out_jk = sqrt2 (n_j w_k + n_k w_j)  (Mandel);  hcn = cn / 2.
  // Mandel off-diagonal entries carry sqrt2: tau_jk = v / sqrt2.
  const T r2 = T(0.70710678118654752);
  const T s2 = T(1.4142135623730951);
  const T m0 = n0 * r2, m1 = n1 * r2, m2 = n2 * r2;
  const c2<T> u0 = cscale(v[0], n0) + cscale(v[5], m1) + cscale(v[4], m2);
  const c2<T> u1 = cscale(v[5], m0) + cscale(v[1], n1) + cscale(v[3], m2);
  const c2<T> u2 = cscale(v[4], m0) + cscale(v[3], m1) + cscale(v[2], n2);
  const c2<T> hq = cscale(cscale(u0, n0) + cscale(u1, n1) + cscale(u2, n2), hcn);
  const c2<T> w0 = cscale(u0, cs) - cscale(hq, n0);
  const c2<T> w1 = cscale(u1, cs) - cscale(hq, n1);
  const c2<T> w2 = cscale(u2, cs) - cscale(hq, n2);
  v[0] = cscale(w0, n0 + n0);
  v[1] = cscale(w1, n1 + n1);
  v[2] = cscale(w2, n2 + n2);
  const T q0 = n0 * s2, q1 = n1 * s2, q2 = n2 * s2;
  v[3] = cscale(w2, q1) + cscale(w1, q2);
  v[4] = cscale(w2, q0) + cscale(w0, q2);
  v[5] = cscale(w1, q0) + cscale(w0, q1);
}

// Rotated finite-difference scheme: with e_j = exp(i 2 pi k_j / n_j) and
// h_j = L_j / n_j, k_j = (e_j - 1) / h_j * prod_{l != j} (1 + e_l) / 2 (the
// difference of a corner displacement along j averaged over the 4 cell edges
// parallel to j); n = k / |k|, zero where |k| < 1e-12 sqrt(sum_j (2 / h_j)^2).
// ex, ey, ez are exp(-i 2 pi k_j / n_j) (forward twiddles).
template <typename T>
__device__ __forceinline__ void rotated_direction(c2<T> ex, c2<T> ey, c2<T> ez, int nx, int ny, int nz,
                                                  const double* len, c2<T>* n, bool& zero) {
  const c2<T> e[3] = {conjg(ex), conjg(ey), conjg(ez)};
  const T ih[3] = {T(nx / len[0]), T(ny / len[1]), T(nz / len[2])};
  c2<T> d[3], av[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    d[j] = cscale(e[j] - mk(T(1), T(0)), ih[j]);
    av[j] = cscale(e[j] + mk(T(1), T(0)), T(0.5));
  }
  n[0] = cmul(d[0], cmul(av[1], av[2]));
  n[1] = cmul(d[1], cmul(av[0], av[2]));
  n[2] = cmul(d[2], cmul(av[0], av[1]));
  T m2 = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) m2 += n[j].x * n[j].x + n[j].y * n[j].y;
  const T kmax2 = T(4) * (ih[0] * ih[0] + ih[1] * ih[1] + ih[2] * ih[2]);
  zero = !(m2 > T(1e-24) * kmax2);
  const T inv = zero ? T(0) : T(1) / sqrt(m2);
#pragma unroll
  for (int j = 0; j < 3; ++j) n[j] = cscale(n[j], inv);
}

// Hermitian orthogonal projector onto sym(n (x) a) for a complex unit n:
// u = tau conj(n), q = conj(n) . u, out = sym(n (x) (2 u - q n)).
template <typename T>
__device__ __forceinline__ void green_mech_herm(c2<T>* v, const c2<T>* n) {
  const T r2 = T(0.70710678118654752);
  const c2<T> t[3][3] = {{v[0], cscale(v[5], r2), cscale(v[4], r2)},
                         {cscale(v[5], r2), v[1], cscale(v[3], r2)},
                         {cscale(v[4], r2), cscale(v[3], r2), v[2]}};
  const c2<T> nb[3] = {conjg(n[0]), conjg(n[1]), conjg(n[2])};
  c2<T> u[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) u[i] = cmul(t[i][0], nb[0]) + cmul(t[i][1], nb[1]) + cmul(t[i][2], nb[2]);
  const c2<T> q = cmul(nb[0], u[0]) + cmul(nb[1], u[1]) + cmul(nb[2], u[2]);
  c2<T> w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = cscale(u[i], T(2)) - cmul(n[i], q);
  v[0] = cmul(n[0], w[0]);
  v[1] = cmul(n[1], w[1]);
  v[2] = cmul(n[2], w[2]);
  v[3] = cscale(cmul(n[1], w[2]) + cmul(n[2], w[1]), r2);  // sqrt2 * (n1 w2 + n2 w1) / 2
  v[4] = cscale(cmul(n[0], w[2]) + cmul(n[2], w[0]), r2);
  v[5] = cscale(cmul(n[0], w[1]) + cmul(n[1], w[0]), r2);
}

// n (conj(n) . g) for a complex unit n.
template <typename T>
__device__ __forceinline__ void green_grad_herm(c2<T>* v, const c2<T>* n) {
  const c2<T> s = cmul(conjg(n[0]), v[0]) + cmul(conjg(n[1]), v[1]) + cmul(conjg(n[2]), v[2]);
  v[0] = cmul(n[0], s);
  v[1] = cmul(n[1], s);
  v[2] = cmul(n[2], s);
}

template <typename T>
__device__ __forceinline__ void green_grad(c2<T>* v, T n0, T n1, T n2, T s) {
  c2<T> q = cscale(cscale(v[0], n0) + cscale(v[1], n1) + cscale(v[2], n2), s);
  v[0] = cscale(q, n0);
  v[1] = cscale(q, n1);
  v[2] = cscale(q, n2);
}

// ---------------------------------------------------------------------------
// 16-byte global accesses: four consecutive reals, a run of complex values
// ---------------------------------------------------------------------------
template <typename T>
struct Q4 {
  T v[4];
};
// Every field and spectrum element is touched once per pass, and a pass moves
// far more data than the caches hold: the contiguous streaming accesses of the
// x passes are non-temporal (on gfx950 a 1 GiB copy runs 5-15 % faster that
// way). The y / z passes keep cached accesses: their tiles fill 128-byte lines
// from neighbouring work-groups, which the L2 merges.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Q4<float> ld4(const float* p) {
  const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return Q4<float>{{t.x, t.y, t.z, t.w}};
}
__device__ __forceinline__ Q4<double> ld4(const double* p) {
  const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  const nt_d2 b = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p) + 1);
  return Q4<double>{{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ void st4(float* p, const float (&v)[4]) {
  const nt_f4 t = {v[0], v[1], v[2], v[3]};
  __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(p));
}
__device__ __forceinline__ void st4(double* p, const double (&v)[4]) {
  const nt_d2 a = {v[0], v[1]}, b = {v[2], v[3]};
  __builtin_nontemporal_store(a, reinterpret_cast<nt_d2*>(p));
  __builtin_nontemporal_store(b, reinterpret_cast<nt_d2*>(p) + 1);
}
// one complex value
__device__ __forceinline__ c2<float> ldc(const c2<float>* p) {
  const nt_f2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
  return mk(t.x, t.y);
}
__device__ __forceinline__ c2<double> ldc(const c2<double>* p) {
  const nt_d2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return mk(t.x, t.y);
}
__device__ __forceinline__ void stc(c2<float>* p, c2<float> v) {
  const nt_f2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<nt_f2*>(p));
}
__device__ __forceinline__ void stc(c2<double>* p, c2<double> v) {
  const nt_d2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<nt_d2*>(p));
}

// Element v of a uniform base, with the byte offset formed in 32-bit unsigned
// arithmetic so the access takes the scalar-base + 32-bit-offset form (needs
// v * sizeof(T) < 2^32 inside one component of one problem: true for every
// supported grid, n <= 256).
template <typename T>
__device__ __forceinline__ const T* at(const T* base, unsigned v) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + v * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T* at(T* base, unsigned v) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + v * (unsigned)sizeof(T));
}

// Staging layout of the x passes between the per-voxel phases and the line
// transforms: one row of SP complex values per transform lane, x fastest. A
// thread's four consecutive voxels are 32 contiguous bytes, and the odd pitch
// puts neighbouring transform lanes on different LDS banks.
constexpr int xstage_pitch(int n) { return n + 1; }

// Dynamic LDS of the pipeline kernels in complex values: N twiddles, then the
// work buffer. The launchers size their launches from these, so kernel and
// launch cannot disagree.
template <int N, int NL, int C>
constexpr int xfwd_lds_elems() {
  return N + NL * ((C + 1) / 2) * xstage_pitch(N);  // staging rows (>= N * L, the exchange)
}
template <int N, int NL, int C>
constexpr int xinv_lds_elems() {
  // staged half spectra, or the staging rows (>= N * L, the exchange)
  return N + (NL * (N / 2 + 1) * C > NL * ((C + 1) / 2) * xstage_pitch(N) ? NL * (N / 2 + 1) * C
                                                                            : NL * ((C + 1) / 2) * xstage_pitch(N));
}
template <int N, int TX, int C>
constexpr int tile_lds_elems() {
  return N + N * TX * C;  // y and z passes: the transform exchange of TX * C lines
}

// ---------------------------------------------------------------------------
// x forward: pre-operation + packed real-to-complex transforms
// ---------------------------------------------------------------------------
// Threads of an x-forward work-group: the G * L of the line transforms, or
// one per four-voxel work item of the per-voxel phase if that is more (the
// extra threads idle through the transforms), so that the per-voxel phase,
// whose loads dominate, takes one memory round trip
template <int N, int NL, int C>
constexpr int xfwd_threads() {
  constexpr int ft = (N / Plan<N>::M) * NL * ((C + 1) / 2);
  constexpr int items = NL * N / 4;
  return items > ft ? items : ft;
}

// FP32: at most 128 VGPRs, four waves per SIMD (a few spilled values are
// cheaper than the third of the occupancy the unbounded build gives up)
template <typename T, int C, int N, int NL>
__global__ void __launch_bounds__((xfwd_threads<N, NL, C>()))
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_xfwd(Pipe<T> a) {
  constexpr int M = Plan<N>::M;
  constexpr int G = N / M;
  constexpr int NP = (C + 1) / 2;
  constexpr int L = NL * NP;
  constexpr int H = N / 2 + 1;
  constexpr int SP = xstage_pitch(N);
  static_assert(xfwd_lds_elems<N, NL, C>() - N >= L * SP && L * SP >= N * L, "x-forward LDS buffer too small");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  c2<T>* tw = reinterpret_cast<c2<T>*>(smem_raw);
  c2<T>* buf = tw + N;

  __shared__ double red[16];
  const int nlines = a.ny * a.nz;
  const int bpp = (nlines + NL - 1) / NL;
  const int prob = blockIdx.x / bpp;
  const int blk = blockIdx.x % bpp;
  const int line0 = blk * NL;
  const Ctl& ctl = a.ctl[prob];
  const int mode = ctl.mode;
  if (!pipeline_mode(mode)) return;
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  for (int i = tid; i < N; i += nth) tw[i] = a.twx[i];
  double pcp = 0.0;  // CG: partial sum of p . C p  (= p . A p, p being compatible)

  const long long nv = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * C * nv;
  const uint8_t* phase = a.phase + (long long)prob * nv;
  const ProbInc& inc = a.inc[prob];
  const bool cg = (mode == M_CG);
  const bool first = (ctl.cg_it == 0);
  const T beta = T(ctl.beta);
  const T alpha_prev = T(ctl.alpha);  // step length of the previous CG iteration
  __shared__ T ptab[MAX_PHASES];  // 3K (mechanics) or kappa (conduction) per phase
  if (tid < MAX_PHASES) ptab[tid] = T(C == 6 ? inc.ph[tid].K3 : inc.ph[tid].kappa);
  __syncthreads();

  // four consecutive voxels of one line per work item, 16-byte accesses
  const int nvl = min(NL, nlines - line0);
  // uniform per-component bases and a 32-bit voxel offset: loads and stores
  // take the scalar-base + 32-bit-offset form
  const unsigned v0 = (unsigned)(line0 * N);
  const T* fb = a.f + fo;
  const T* rb = a.r + fo;
  T* pb = a.p + fo;
  T* xb = a.x + fo;
  const T* tb = a.tab + (long long)prob * 2 * nv;
  const T* nb = a.tn + (long long)prob * 6 * nv;
  for (int w = tid; w < NL * N / 4; w += nth) {
    const int e = 4 * w;
    const int li = e / N;
    const int xv = e - li * N;
    T out[4][2 * NP];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 2 * NP; ++c) out[j][c] = T(0);
    if (li < nvl) {
      const unsigned v = v0 + (unsigned)e;
      if (!cg) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const Q4<T> q = ld4(at(fb + c * nv, v));
#pragma unroll
          for (int j = 0; j < 4; ++j) out[j][c] = q.v[j];
        }
      } else {
        // p = r + beta p; the step x += alpha p of the previous iteration is
        // applied here, where the old direction is read anyway. Every load of
        // the work item is issued before the first store (one memory round
        // trip instead of one per component).
        Q4<T> rq[C], pq[C], xq[C];
#pragma unroll
        for (int c = 0; c < C; ++c) rq[c] = ld4(at(rb + c * nv, v));
        if (!first) {  // uniform over the block
#pragma unroll
          for (int c = 0; c < C; ++c) {
            pq[c] = ld4(at(pb + c * nv, v));
            xq[c] = ld4(at(xb + c * nv, v));
          }
        }
        Q4<T> ca, cb;
        if constexpr (C == 6) {
          ca = ld4(at(tb, v));
          cb = ld4(at(tb + nv, v));
        }
        const uchar4 ph = *reinterpret_cast<const uchar4*>(at(phase, v));
        T pv[C][4];
        if (first) {
#pragma unroll
          for (int c = 0; c < C; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) pv[c][j] = rq[c].v[j];
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            T xn[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              pv[c][j] = rq[c].v[j] + beta * pq[c].v[j];
              xn[j] = xq[c].v[j] + alpha_prev * pq[c].v[j];
            }
            st4(at(xb + c * nv, v), xn);
          }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) st4(at(pb + c * nv, v), pv[c]);
        const int phs[4] = {ph.x, ph.y, ph.z, ph.w};
        if constexpr (C == 6) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const T tr3 = (pv[0][j] + pv[1][j] + pv[2][j]) * T(1.0 / 3.0);
            const T sph = (ptab[phs[j]] - ca.v[j]) * tr3;
#pragma unroll
            for (int c = 0; c < 6; ++c) out[j][c] = ca.v[j] * pv[c][j];
            out[j][0] += sph;
            out[j][1] += sph;
            out[j][2] += sph;
          }
          if (cb.v[0] != T(0) || cb.v[1] != T(0) || cb.v[2] != T(0) || cb.v[3] != T(0)) {
            T nd[6][4];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              const Q4<T> q = ld4(at(nb + c * nv, v));
#pragma unroll
              for (int j = 0; j < 4; ++j) nd[c][j] = q.v[j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (cb.v[j] == T(0)) continue;
              T dot = T(0);
#pragma unroll
              for (int c = 0; c < 6; ++c) dot += nd[c][j] * pv[c][j];
#pragma unroll
              for (int c = 0; c < 6; ++c) out[j][c] += cb.v[j] * dot * nd[c][j];
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const T kap = ptab[phs[j]];
#pragma unroll
            for (int c = 0; c < C; ++c) out[j][c] = kap * pv[c][j];
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int c = 0; c < C; ++c) pcp += (double)pv[c][j] * (double)out[j][c];
      }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) buf[(li * NP + q) * SP + xv + j] = mk(out[j][2 * q], out[j][2 * q + 1]);
  }
  if (cg) {  // uniform per block
    double s[1] = {pcp};
    block_sum<1>(s, red);
    if (tid == 0) a.part[part_index(prob, 0, blk, a.maxblk)] = s[0];
  }
  __syncthreads();

  const bool fw = tid < G * L;  // a thread of the line transforms
  const int l = tid % L;
  const int t = fw ? tid / L : 0;
  c2<T> r[M];
#pragma unroll
  for (int m = 0; m < M; ++m) r[m] = fw ? buf[l * SP + t + G * m] : mk(T(0), T(0));
  Plan<N>::run(r, t, tw, buf, L, l, fw);
  __syncthreads();
  if (fw) {
#pragma unroll
    for (int m = 0; m < M; ++m) buf[(t + G * m) * L + l] = r[m];
  }
  __syncthreads();

  // unpack the two real transforms of each complex line and write the block's
  // contiguous run of half spectra [line][kx][comp] with 16-byte stores
  const int rowp = a.PS * C;
  c2<T>* spec = a.spec + (long long)prob * a.nz * a.ny * rowp + (long long)line0 * rowp;
  constexpr int V = 16 / sizeof(c2<T>);
  const int total = nvl * H * C;
  auto value = [&](int e) -> c2<T> {
    const int c = e % C;
    const int rest = e / C;
    const int k = rest % H;
    const int li = rest / H;
    const int q = c >> 1;
    const c2<T> zk = buf[k * L + li * NP + q];
    const c2<T> zm = conjg(buf[((N - k) % N) * L + li * NP + q]);
    const c2<T> val = (c & 1) ? mul_mi(zk - zm) : (zk + zm);
    return cscale(val, T(0.5));
  };
  // rows are rowp apart; the (kx, comp) entries of one row are contiguous
  if constexpr (V == 2 && C % 2 == 0) {
    // pairs of components of one kx: 16-byte aligned stores (rowp * 8 is a
    // multiple of 128 and the pair starts at an even entry)
    for (int i = tid; i < total / 2; i += nth) {
      const int e = 2 * i;
      const int li = e / (H * C);
      const c2<T> u0 = value(e), u1 = value(e + 1);
      const nt_f4 t = {u0.x, u0.y, u1.x, u1.y};
      __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(spec + li * rowp + (e - li * H * C)));
    }
  } else {
    for (int e = tid; e < total; e += nth) {
      const int li = e / (H * C);
      stc(spec + li * rowp + (e - li * H * C), value(e));
    }
  }
}

// Work-groups are dispatched to the 8 XCDs round-robin (work-group i to XCD
// i mod 8), each XCD with its own L2. This bijection of [0, n) gives every XCD
// a contiguous range of tiles, so neighbouring kx tiles, which share 128-byte
// lines when a tile row is not a whole number of lines, meet in one L2.
__device__ __forceinline__ int xcd_remap(int i, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = i & 7, k = i >> 3;
  return x * q + min(x, rem) + k;
}

// ---------------------------------------------------------------------------
// y pass (forward or inverse) on tiles of TX kx columns
// ---------------------------------------------------------------------------
template <typename T, int C, int N, int TX, int V>
__global__ void __launch_bounds__((N / Plan<N, V>::M) * TX * C) k_ypass(Pipe<T> a, int inverse) {
  constexpr int M = Plan<N, V>::M;
  constexpr int G = N / M;
  constexpr int L = TX * C;
  static_assert(tile_lds_elems<N, TX, C>() - N >= N * L, "tile LDS buffer too small");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  c2<T>* tw = reinterpret_cast<c2<T>*>(smem_raw);
  c2<T>* buf = tw + N;
  const int P = a.P;
  const int nkb = (P + TX - 1) / TX;
  const int bpp = a.nz * nkb;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int prob = bid / bpp;
  const int b = bid % bpp;
  if (!pipeline_mode(a.ctl[prob].mode)) return;
  const int z = b / nkb;
  const int kb = b % nkb;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += blockDim.x) tw[i] = a.twy[i];
  const int l = tid % L;
  const int t = tid / L;
  const int kx = kb * TX + l / C;
  const int c = l % C;
  const bool active = kx < P;
  const long long stride = (long long)a.PS * C;
  c2<T>* base = a.spec + (long long)prob * a.nz * a.ny * a.PS * C + ((long long)z * a.ny * a.PS + kx) * C + c;
  c2<T> r[M];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    c2<T> v = active ? base[(t + G * m) * stride] : mk(T(0), T(0));
    r[m] = inverse ? conjg(v) : v;
  }
  Plan<N, V>::run(r, t, tw, buf, L, l, active);
  if (active) {
#pragma unroll
    for (int m = 0; m < M; ++m) base[(t + G * m) * stride] = inverse ? conjg(r[m]) : r[m];
  }
}

// ---------------------------------------------------------------------------
// z forward + Green operator + z inverse on tiles of TX kx columns
// ---------------------------------------------------------------------------
template <typename T, int C, int N, int TX, int V>
__global__ void __launch_bounds__((N / Plan<N, V>::M) * TX * C)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) k_zgreen(Pipe<T> a) {
  constexpr int M = Plan<N, V>::M;
  constexpr int G = N / M;
  constexpr int L = TX * C;
  static_assert(tile_lds_elems<N, TX, C>() - N >= N * L, "tile LDS buffer too small");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  c2<T>* tw = reinterpret_cast<c2<T>*>(smem_raw);
  c2<T>* buf = tw + N;
  const int P = a.P;
  const int nkb = (P + TX - 1) / TX;
  const int bpp = a.ny * nkb;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int prob = bid / bpp;
  const int b = bid % bpp;
  if (!pipeline_mode(a.ctl[prob].mode)) return;
  const int ky = b / nkb;
  const int kb = b % nkb;
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  if (a.alpha_blocks > 0 && b == 0) {
    // CG step length alpha = r.r / p.C p from the x-forward pass's partials of
    // p.C p (= p.A p: p is compatible and the projector orthogonal). Formed
    // by the first work-group of the problem while the others transform; the
    // x-inverse pass applies it.
    Ctl& cw = a.ctl[prob];
    if (cw.mode == M_CG && !cw.cg_ready) {  // uniform over the work-group
      __shared__ double red[16];
      double s[1] = {0.0};
      const double* pp = a.part + part_index(prob, 0, 0, a.maxblk);
      for (int i = tid; i < a.alpha_blocks; i += nth) s[0] += pp[i];
      block_sum<1>(s, red);
      if (tid == 0) {
        const double pap = s[0];
        if (!(pap > 0.0) || !isfinite(pap)) {
          cw.mode = M_FAIL;
          cw.status = -4;
        } else {
          cw.alpha = cw.rr / pap;
          cw.cg_ready = 1;
        }
      }
    }
  }
  for (int i = tid; i < N; i += nth) tw[i] = a.twz[i];
  const int l = tid % L;
  const int t = tid / L;
  const int kx = kb * TX + l / C;
  const int c = l % C;
  const bool active = kx < P;
  const long long stride = (long long)a.ny * a.PS * C;
  c2<T>* base = a.spec + (long long)prob * a.nz * a.ny * a.PS * C + ((long long)ky * a.PS + kx) * C + c;
  c2<T> r[M];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) r[m] = active ? base[(t + G * m) * stride] : mk(T(0), T(0));
  Plan<N, V>::run(r, t, tw, buf, L, l, active);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) buf[(t + G * m) * L + l] = r[m];
  __syncthreads();

  const ProbInc& inc = a.inc[prob];
  T cs = T(1), hcn = T(0.5);
  if (a.green == G_GAMMA0) {
    cs = T(1.0 / (2.0 * inc.mu0));
    hcn = T(0.5 * (inc.lam0 + inc.mu0) / (inc.mu0 * (inc.lam0 + 2.0 * inc.mu0)));
  } else if (a.green == G_GAMMA_TH) {
    cs = T(1.0 / inc.kappa0);
  }
  const bool rot = (a.green == G_PROJ_ROT || a.green == G_GRADPROJ_ROT);
  // every index of this thread has the same kx (nth is a multiple of TX):
  // the x and y parts of the frequency are fixed, the z part varies
  const int kxx = kb * TX + tid % TX;
  const T fa = frequency_component<T>(kxx, a.nx, T(a.ilen[0]));
  const T fb = frequency_component<T>(ky, a.ny, T(a.ilen[1]));
  const T fab2 = fa * fa + fb * fb;
  const T il2 = T(a.ilen[2]);
  static_assert(((N / Plan<N, V>::M) * TX * C) % TX == 0, "thread count must be a multiple of TX");
  for (int idx = tid; idx < N * TX; idx += nth) {
    const int kz = idx / TX;
    const int kxi = idx - kz * TX;
    if (kxx >= P) break;
    T n0 = T(0), n1 = T(0), n2 = T(0);
    c2<T> nc[3];
    bool zero;
    if (rot) {
      rotated_direction<T>(a.twx[kxx], a.twy[ky], tw[kz], a.nx, a.ny, a.nz, a.len, nc, zero);
    } else {
      const T fc = frequency_component<T>(kz, a.nz, il2);
      const T m2 = fc * fc + fab2;
      zero = !(m2 > T(0));
      const T inv = zero ? T(0) : inv_norm(m2);
      n0 = fa * inv;
      n1 = fb * inv;
      n2 = fc * inv;
    }
    c2<T> v[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) v[cc] = buf[kz * L + kxi * C + cc];
    if (zero) {
      // the mean: removed, except for the stress-controlled components of
      // mixed conditions, whose mean strain is an unknown of the iteration
      // (the projector's zero-frequency block is the mask). A residual
      // evaluation compares the mean stress with the prescribed one (the
      // spectrum is unnormalized: the mean mode holds nvox <sigma>).
      const bool mean = (kxx == 0 && ky == 0 && kz == 0);
      const bool eval = a.ctl[prob].mode == M_EVAL;
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        if (C == 6 && mean && ((inc.smask >> cc) & 1))
          v[cc] = mk(v[cc].x - (eval ? T((double)a.nvox * inc.S[cc]) : T(0)), T(0));
        else
          v[cc] = mk(T(0), T(0));
      }
    } else if (rot) {
      if constexpr (C == 6)
        green_mech_herm<T>(v, nc);
      else
        green_grad_herm<T>(v, nc);
    } else {
      if constexpr (C == 6)
        green_mech<T>(v, n0, n1, n2, cs, hcn);
      else
        green_grad<T>(v, n0, n1, n2, cs);
    }
#pragma unroll
    for (int cc = 0; cc < C; ++cc) buf[kz * L + kxi * C + cc] = v[cc];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) r[m] = conjg(buf[(t + G * m) * L + l]);
  Plan<N, V>::run(r, t, tw, buf, L, l, active);
  if (active) {
#pragma unroll
    for (int m = 0; m < M; ++m) base[(t + G * m) * stride] = conjg(r[m]);
  }
}

// ---------------------------------------------------------------------------
// x inverse: packed complex-to-real transforms + post-operation + partial sums
// ---------------------------------------------------------------------------
template <typename T, int C, int N, int NL>
__global__ void __launch_bounds__((N / Plan<N>::M) * NL * ((C + 1) / 2)) k_xinv(Pipe<T> a) {
  constexpr int M = Plan<N>::M;
  constexpr int G = N / M;
  constexpr int NP = (C + 1) / 2;
  constexpr int L = NL * NP;
  constexpr int H = N / 2 + 1;
  constexpr int SP = xstage_pitch(N);
  static_assert(xinv_lds_elems<N, NL, C>() - N >= L * SP && xinv_lds_elems<N, NL, C>() - N >= NL * H * C &&
                    L * SP >= N * L,
                "x-inverse LDS buffer too small");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  c2<T>* tw = reinterpret_cast<c2<T>*>(smem_raw);
  c2<T>* buf = tw + N;  // holds the staged half spectra first, then the line FFTs
  __shared__ double red[2 * 16];

  const int nlines = a.ny * a.nz;
  const int bpp = (nlines + NL - 1) / NL;
  const int prob = blockIdx.x / bpp;
  const int blk = blockIdx.x % bpp;
  const int line0 = blk * NL;
  const Ctl& ctl = a.ctl[prob];
  const int mode = ctl.mode;
  if (!pipeline_mode(mode)) return;
  const T alpha = T(ctl.alpha);
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  for (int i = tid; i < N; i += nth) tw[i] = a.twx[i];
  // stage the block's half spectra [line][kx][comp] (rows rowp apart in
  // memory, packed in LDS)
  const int nvl = min(NL, nlines - line0);
  const int rowp = a.PS * C;
  const c2<T>* spec = a.spec + (long long)prob * a.nz * a.ny * rowp + (long long)line0 * rowp;
  // all of a thread's loads are issued before the LDS writes (the launch has
  // exactly NTH threads)
  constexpr int NTH = G * L;
  if constexpr (sizeof(c2<T>) == 8 && C % 2 == 0) {
    constexpr int K = (NL * H * C / 2 + NTH - 1) / NTH;
    const int tot = nvl * H * C / 2;
    const nt_f4* s4 = reinterpret_cast<const nt_f4*>(spec);
    nt_f4* d4 = reinterpret_cast<nt_f4*>(buf);
    nt_f4 t4[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {  // unconditional loads (index clamped in range), no branch between them
      const int e = 2 * min(tid + k * NTH, tot - 1);
      const int li = e / (H * C);
      t4[k] = __builtin_nontemporal_load(s4 + (li * rowp + (e - li * H * C)) / 2);
    }
    // unconditional writes too (else the compiler sinks each load into its
    // write's branch): a clamped thread rewrites the last element's own value
#pragma unroll
    for (int k = 0; k < K; ++k) d4[min(tid + k * NTH, tot - 1)] = t4[k];
  } else {
    constexpr int K = (NL * H * C + NTH - 1) / NTH;
    const int tot = nvl * H * C;
    c2<T> t2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = min(tid + k * NTH, tot - 1);
      const int li = e / (H * C);
      t2[k] = ldc(spec + li * rowp + (e - li * H * C));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) buf[min(tid + k * NTH, tot - 1)] = t2[k];
  }
  for (int e = nvl * H * C + tid; e < NL * H * C; e += nth) buf[e] = mk(T(0), T(0));
  __syncthreads();
  const int l = tid % L;
  const int t = tid / L;
  const int li = l / NP;
  const int q = l - li * NP;
  c2<T> r[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int p = t + G * m;
    const bool lo = p <= N / 2;
    const int kk = lo ? p : N - p;
    c2<T> A = buf[(li * H + kk) * C + 2 * q];
    c2<T> B = (2 * q + 1 < C) ? buf[(li * H + kk) * C + 2 * q + 1] : mk(T(0), T(0));
    if (!lo) {
      A = conjg(A);
      B = conjg(B);
    }
    // Z = A + i B, transformed as conj(DFT(conj(Z)))
    r[m] = mk(A.x - B.y, -(A.y + B.x));
  }
  Plan<N>::run(r, t, tw, buf, L, l, true);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) buf[l * SP + t + G * m] = conjg(r[m]);
  __syncthreads();

  const long long nv = a.vs;  // stride of the per-voxel arrays (component, problem)
  const long long fo = (long long)prob * C * nv;
  const T scale = T(1.0 / ((double)a.nx * a.ny * a.nz));
  double s0 = 0.0, s1 = 0.0;
  const unsigned v0 = (unsigned)(line0 * N);
  const T* sb = (mode == M_EVAL ? a.f : (mode == M_CG ? a.r : a.x)) + fo;  // uniform bases
  T* db = (mode == M_BASIC ? a.x : a.r) + fo;
  for (int w = tid; w < nvl * N / 4; w += nth) {
    const int e = 4 * w;
    const int lj = e / N;
    const int xv = e - lj * N;
    const unsigned v = v0 + (unsigned)e;
    // the work item's global operand for every component first (one memory
    // round trip), then the transformed values from LDS, then the stores
    Q4<T> q[C];
#pragma unroll
    for (int c = 0; c < C; ++c) q[c] = ld4(at(sb + c * nv, v));
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T g[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const c2<T> z = buf[(lj * NP + (c >> 1)) * SP + xv + j];
        g[j] = ((c & 1) ? z.y : z.x) * scale;
      }
      T* o = at(db + c * nv, v);
      T out[4];
      if (mode == M_EVAL) {  // residual field r = -Gamma sigma; norms of r and sigma
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          out[j] = -g[j];
          s0 += (double)g[j] * (double)g[j];
          s1 += (double)q[c].v[j] * (double)q[c].v[j];
        }
        st4(o, out);
      } else if (mode == M_CG) {
        // residual update with alpha = r.r / p.C p: r -= alpha A p (the step
        // x += alpha p follows in the next x-forward pass or evaluation)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          out[j] = q[c].v[j] - alpha * g[j];
          s0 += (double)out[j] * (double)out[j];
        }
        st4(o, out);
      } else {  // basic scheme: x -= Gamma0 sigma
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          out[j] = q[c].v[j] - g[j];
          s0 += (double)g[j] * (double)g[j];
          s1 += (double)out[j] * (double)out[j];
        }
        st4(o, out);
      }
    }
  }
  double s[2] = {s0, s1};
  block_sum<2>(s, red);
  if (tid == 0) {
    a.part[part_index(prob, 0, blk, a.maxblk)] = s[0];
    a.part[part_index(prob, 1, blk, a.maxblk)] = s[1];
  }
}

}  // namespace hom
