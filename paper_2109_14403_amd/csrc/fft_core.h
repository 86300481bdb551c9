// Line FFTs for gfx950: register-resident Stockham autosort with one LDS
// exchange between radix passes.
//
// A line of length N is owned by G = N / M threads of a work-group; thread t
// holds the M elements x[t + G m], m = 0..M-1, in registers. Every radix-R
// pass works on butterflies j = t + s G (s = 0..M/R-1), whose inputs are
// exactly x[j + r N/R] -- a subset of the thread's own registers. Outputs go
// to their autosorted positions through LDS; the last pass writes back to
// the same strided positions, so the transform ends in registers in the
// layout it started in. Butterfly-internal twiddles are compile-time
// constants; the inter-pass twiddles come from an FP64-computed table of
// W_N^j = exp(-2 pi i j / N) held in LDS.
//
// The transform computed is the unnormalized forward DFT
//   X[k] = sum_n x[n] exp(-2 pi i n k / N).
// The inverse is obtained by conjugating input and output.
#pragma once
#include <hip/hip_runtime.h>

namespace hom {

template <typename T>
struct c2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ c2<T> mk(T a, T b) {
  c2<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ c2<T> operator+(c2<T> a, c2<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ c2<T> operator-(c2<T> a, c2<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ c2<T> cscale(c2<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ c2<T> conjg(c2<T> a) { return mk(a.x, -a.y); }
// multiply by -i
template <typename T>
__device__ __forceinline__ c2<T> mul_mi(c2<T> a) { return mk(a.y, -a.x); }

// cos(2 pi j / 48), j any integer; exact on the quarter-wave grid.
__host__ __device__ constexpr double cos48(int j) {
  constexpr double q[13] = {1.0,
                            0.99144486137381038,
                            0.96592582628906831,
                            0.92387953251128674,
                            0.86602540378443865,
                            0.79335334029123517,
                            0.70710678118654752,
                            0.60876142900872066,
                            0.5,
                            0.38268343236508977,
                            0.25881904510252074,
                            0.13052619222005159,
                            0.0};
  int k = ((j % 48) + 48) % 48;
  return k <= 12 ? q[k] : (k <= 24 ? -q[24 - k] : (k <= 36 ? -q[k - 24] : q[48 - k]));
}
__host__ __device__ constexpr double sin48(int j) { return cos48(j - 12); }

// exp(-2 pi i j / R) for R dividing 48
template <typename T, int R>
__device__ __forceinline__ c2<T> wconst(int j) {
  static_assert(48 % R == 0, "radix must divide 48");
  return mk(T(cos48(j * (48 / R))), T(-sin48(j * (48 / R))));
}

// a * exp(-2 pi i j / R); the quarter-turn factors 1, -i, -1, i exactly, as
// sign changes and swaps
template <typename T, int R>
__device__ __forceinline__ c2<T> mul_wconst(c2<T> a, int j) {
  const int q = ((j * (48 / R)) % 48 + 48) % 48;
  if (q % 12 == 0) {
    switch (q / 12) {
      case 0:
        return a;
      case 1:
        return mul_mi(a);
      case 2:
        return mk(-a.x, -a.y);
      default:
        return mk(-a.y, a.x);
    }
  }
  return cmul(a, wconst<T, R>(j));
}

template <int R, typename T>
struct DFT;

template <typename T>
struct DFT<1, T> {
  static __device__ __forceinline__ void run(c2<T>*) {}
};

template <typename T>
struct DFT<2, T> {
  static __device__ __forceinline__ void run(c2<T>* v) {
    c2<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T>
struct DFT<3, T> {
  static __device__ __forceinline__ void run(c2<T>* v) {
    const T h = T(0.86602540378443865);  // sin(2 pi / 3)
    c2<T> s = v[1] + v[2];
    c2<T> d = v[1] - v[2];
    c2<T> m = v[0] - cscale(s, T(0.5));
    c2<T> rot = mk(d.y * h, -d.x * h);  // -i h d
    v[0] = v[0] + s;
    v[1] = m + rot;
    v[2] = m - rot;
  }
};

template <typename T>
struct DFT<4, T> {
  static __device__ __forceinline__ void run(c2<T>* v) {
    c2<T> t0 = v[0] + v[2];
    c2<T> t1 = v[0] - v[2];
    c2<T> t2 = v[1] + v[3];
    c2<T> t3 = mul_mi(v[1] - v[3]);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
  }
};

// Cooley-Tukey composition R = R1 R2 with input n = R2 n1 + n2 and output
// k = k1 + R1 k2:  X[k1 + R1 k2] = sum_n2 W_R2^{n2 k2} W_R^{n2 k1} sum_n1 x[R2 n1 + n2] W_R1^{n1 k1}
template <int R1, int R2, typename T>
__device__ __forceinline__ void dft_ct(c2<T>* v) {
  constexpr int R = R1 * R2;
  c2<T> u[R];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    c2<T> t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
    DFT<R1, T>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) u[n2 * R1 + k1] = mul_wconst<T, R>(t[k1], n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    c2<T> t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = u[n2 * R1 + k1];
    DFT<R2, T>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
  }
}

template <typename T>
struct DFT<6, T> {
  static __device__ __forceinline__ void run(c2<T>* v) { dft_ct<2, 3, T>(v); }
};
template <typename T>
struct DFT<8, T> {
  static __device__ __forceinline__ void run(c2<T>* v) { dft_ct<2, 4, T>(v); }
};
template <typename T>
struct DFT<12, T> {
  static __device__ __forceinline__ void run(c2<T>* v) { dft_ct<4, 3, T>(v); }
};
template <typename T>
struct DFT<16, T> {
  static __device__ __forceinline__ void run(c2<T>* v) { dft_ct<4, 4, T>(v); }
};

// One Stockham pass of radix R at span NS over a line of N points, executed by
// the thread at position t of G = N/M. `buf` is the work-group's LDS array
// holding all lines interleaved: element e of line l lives at buf[e * L + l].
// A non-final pass synchronizes before writing into `buf` and again before
// reloading the registers in strided order.
template <int N, int M, int R, int NS, bool LAST, typename T>
__device__ __forceinline__ void stockham_pass(c2<T>* a, int t, const c2<T>* __restrict__ tw, c2<T>* buf,
                                              int L, int l, bool active) {
  constexpr int G = N / M;
  constexpr int S = M / R;
  static_assert(M % R == 0, "radix must divide the per-thread element count");
  if (!LAST) __syncthreads();  // earlier readers of buf are done
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = t + s * G;
    const int k = j % NS;
    c2<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[s + r * S];
    if (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * (N / (NS * R))]);
    }
    DFT<R, T>::run(v);
    if (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[s + r * S] = v[r];
    } else if (active) {
      const int idx = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(idx + r * NS) * L + l] = v[r];
    }
  }
  if (!LAST) {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int m = 0; m < M; ++m) a[m] = buf[(t + G * m) * L + l];
    }
  }
}

// Plans: per-thread element count M (threads per line G = N / M) and the
// sequence of radix passes.
// Plan<N, V>: elements per thread M and the radix passes of a length-N line
// transform. V = 0 is the plan of every pass; the y and z passes also have
// plan V = 1 (another register / pass trade-off), and the autotuner times
// both on the problem's own data.
template <int N, int V = 0>
struct Plan;

#define HOM_PASS(Nv, Mv, R, NS, LAST) stockham_pass<Nv, Mv, R, NS, LAST, T>(a, t, tw, buf, L, l, active)

template <>
struct Plan<16, 0> {
  static constexpr int M = 4;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(16, 4, 4, 1, false);
    HOM_PASS(16, 4, 4, 4, true);
  }
};
template <>
struct Plan<24, 0> {
  static constexpr int M = 12;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(24, 12, 12, 1, false);
    HOM_PASS(24, 12, 2, 12, true);
  }
};
template <>
struct Plan<32, 0> {
  static constexpr int M = 8;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(32, 8, 8, 1, false);
    HOM_PASS(32, 8, 4, 8, true);
  }
};
template <>
struct Plan<48, 0> {
  static constexpr int M = 12;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(48, 12, 12, 1, false);
    HOM_PASS(48, 12, 4, 12, true);
  }
};
template <>
struct Plan<64, 0> {
  static constexpr int M = 8;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(64, 8, 8, 1, false);
    HOM_PASS(64, 8, 8, 8, true);
  }
};
template <>
struct Plan<96, 0> {
  static constexpr int M = 24;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(96, 24, 12, 1, false);
    HOM_PASS(96, 24, 8, 12, true);
  }
};
template <>
struct Plan<128, 0> {
  static constexpr int M = 16;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(128, 16, 16, 1, false);
    HOM_PASS(128, 16, 8, 16, true);
  }
};
template <>
struct Plan<256, 0> {
  static constexpr int M = 16;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(256, 16, 16, 1, false);
    HOM_PASS(256, 16, 16, 16, true);
  }
};
// the alternative plans (V = 1)
template <>
struct Plan<16, 1> {
  static constexpr int M = 8;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(16, 8, 8, 1, false);
    HOM_PASS(16, 8, 2, 8, true);
  }
};
template <>
struct Plan<24, 1> {
  static constexpr int M = 12;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(24, 12, 4, 1, false);
    HOM_PASS(24, 12, 6, 4, true);
  }
};
template <>
struct Plan<32, 1> {
  static constexpr int M = 16;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(32, 16, 16, 1, false);
    HOM_PASS(32, 16, 2, 16, true);
  }
};
template <>
struct Plan<48, 1> {
  static constexpr int M = 12;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(48, 12, 4, 1, false);
    HOM_PASS(48, 12, 12, 4, true);
  }
};
template <>
struct Plan<64, 1> {
  static constexpr int M = 16;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(64, 16, 16, 1, false);
    HOM_PASS(64, 16, 4, 16, true);
  }
};
template <>
struct Plan<96, 1> {
  static constexpr int M = 12;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(96, 12, 12, 1, false);
    HOM_PASS(96, 12, 4, 12, false);
    HOM_PASS(96, 12, 2, 48, true);
  }
};
template <>
struct Plan<128, 1> {
  static constexpr int M = 8;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(128, 8, 8, 1, false);
    HOM_PASS(128, 8, 8, 8, false);
    HOM_PASS(128, 8, 2, 64, true);
  }
};
template <>
struct Plan<256, 1> {
  static constexpr int M = 8;
  template <typename T>
  static __device__ __forceinline__ void run(c2<T>* a, int t, const c2<T>* tw, c2<T>* buf, int L, int l,
                                             bool active) {
    HOM_PASS(256, 8, 8, 1, false);
    HOM_PASS(256, 8, 8, 8, false);
    HOM_PASS(256, 8, 4, 64, true);
  }
};
#undef HOM_PASS

}  // namespace hom
