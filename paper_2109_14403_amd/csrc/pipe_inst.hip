// Instantiation of the pipeline kernels for one transform length HOM_N.
#include "pipe_launch.h"
#include "pipeline.h"

#ifndef HOM_N
#error "compile with -DHOM_N=<transform length>"
#endif

namespace hom {

namespace {

template <typename T, int C, int N, int NL>
LaunchInfo xfwd_c(const Pipe<T>& a, hipStream_t s, bool dry) {
  LaunchInfo li;
  li.threads = xfwd_threads<N, NL, C>();
  li.blocks = a.nprob * ((a.ny * a.nz + NL - 1) / NL);
  li.lds = (size_t)xfwd_lds_elems<N, NL, C>() * sizeof(c2<T>);
  {
    static bool attr = false;
    if (!attr && li.lds > 65536) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xfwd<T, C, N, NL>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
      attr = true;
    }
  }
  if (!dry) {
    hipLaunchKernelGGL((k_xfwd<T, C, N, NL>), dim3(li.blocks), dim3(li.threads), li.lds, s, a);
  }
  return li;
}

template <typename T, int C, int N, int NL>
LaunchInfo xinv_c(const Pipe<T>& a, hipStream_t s, bool dry) {
  constexpr int G = N / Plan<N>::M;
  constexpr int NP = (C + 1) / 2;
  constexpr int L = NL * NP;
  LaunchInfo li;
  li.threads = G * L;
  li.blocks = a.nprob * ((a.ny * a.nz + NL - 1) / NL);
  li.lds = (size_t)xinv_lds_elems<N, NL, C>() * sizeof(c2<T>);
  {
    static bool attr = false;
    if (!attr && li.lds > 65536) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xinv<T, C, N, NL>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
      attr = true;
    }
  }
  if (!dry) {
    hipLaunchKernelGGL((k_xinv<T, C, N, NL>), dim3(li.blocks), dim3(li.threads), li.lds, s, a);
  }
  return li;
}

template <typename T, int C, int N, int TX, int V>
LaunchInfo ypass_c(const Pipe<T>& a, int inverse, hipStream_t s, bool dry) {
  constexpr int G = N / Plan<N, V>::M;
  LaunchInfo li;
  li.threads = G * TX * C;
  li.blocks = a.nprob * a.nz * ((a.P + TX - 1) / TX);
  li.lds = (size_t)tile_lds_elems<N, TX, C>() * sizeof(c2<T>);
  {
    static bool attr = false;
    if (!attr && li.lds > 65536) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ypass<T, C, N, TX, V>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
      attr = true;
    }
  }
  if (!dry) {
    hipLaunchKernelGGL((k_ypass<T, C, N, TX, V>), dim3(li.blocks), dim3(li.threads), li.lds, s, a, inverse);
  }
  return li;
}

template <typename T, int C, int N, int TX, int V>
LaunchInfo zgreen_c(const Pipe<T>& a, hipStream_t s, bool dry) {
  constexpr int G = N / Plan<N, V>::M;
  LaunchInfo li;
  li.threads = G * TX * C;
  li.blocks = a.nprob * a.ny * ((a.P + TX - 1) / TX);
  li.lds = (size_t)tile_lds_elems<N, TX, C>() * sizeof(c2<T>);
  {
    static bool attr = false;
    if (!attr && li.lds > 65536) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zgreen<T, C, N, TX, V>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      (void)hipGetLastError();
      attr = true;
    }
  }
  if (!dry) {
    hipLaunchKernelGGL((k_zgreen<T, C, N, TX, V>), dim3(li.blocks), dim3(li.threads), li.lds, s, a);
  }
  return li;
}

// schedule code -> tile width and plan variant
template <typename T, int C, int N, int V>
LaunchInfo ypass_v(const Pipe<T>& a, int tx, int inverse, hipStream_t s, bool dry) {
  if (tx == 2) return ypass_c<T, C, N, 2, V>(a, inverse, s, dry);
  if (tx == 8) return ypass_c<T, C, N, 8, V>(a, inverse, s, dry);
  return ypass_c<T, C, N, 4, V>(a, inverse, s, dry);
}
template <typename T, int C, int N, int V>
LaunchInfo zgreen_v(const Pipe<T>& a, int tx, hipStream_t s, bool dry) {
  if (tx == 2) return zgreen_c<T, C, N, 2, V>(a, s, dry);
  if (tx == 8) return zgreen_c<T, C, N, 8, V>(a, s, dry);
  return zgreen_c<T, C, N, 4, V>(a, s, dry);
}

}  // namespace

template <typename T, int N>
LaunchInfo xfwd_launch(const Pipe<T>& a, hipStream_t s, bool dry) {
  static_assert(plan_m(N) == Plan<N>::M, "launch plan and transform plan disagree");
  constexpr int NL = x_lines(N, sizeof(T) == 8, true);
  return a.C == 6 ? xfwd_c<T, 6, N, NL>(a, s, dry) : xfwd_c<T, 3, N, NL>(a, s, dry);
}

template <typename T, int N>
LaunchInfo xinv_launch(const Pipe<T>& a, hipStream_t s, bool dry) {
  constexpr int NL = x_lines(N, sizeof(T) == 8, false);
  return a.C == 6 ? xinv_c<T, 6, N, NL>(a, s, dry) : xinv_c<T, 3, N, NL>(a, s, dry);
}

template <typename T, int N>
LaunchInfo ypass_launch(const Pipe<T>& a, int sched, int inverse, hipStream_t s, bool dry) {
  const int tx = schedule_tile(sched);
  if (schedule_plan(sched) == 1)
    return a.C == 6 ? ypass_v<T, 6, N, 1>(a, tx, inverse, s, dry) : ypass_v<T, 3, N, 1>(a, tx, inverse, s, dry);
  return a.C == 6 ? ypass_v<T, 6, N, 0>(a, tx, inverse, s, dry) : ypass_v<T, 3, N, 0>(a, tx, inverse, s, dry);
}

template <typename T, int N>
LaunchInfo zgreen_launch(const Pipe<T>& a, int sched, hipStream_t s, bool dry) {
  const int tx = schedule_tile(sched);
  if (schedule_plan(sched) == 1)
    return a.C == 6 ? zgreen_v<T, 6, N, 1>(a, tx, s, dry) : zgreen_v<T, 3, N, 1>(a, tx, s, dry);
  return a.C == 6 ? zgreen_v<T, 6, N, 0>(a, tx, s, dry) : zgreen_v<T, 3, N, 0>(a, tx, s, dry);
}

#define HOM_INST(T)                                                                         \
  template LaunchInfo xfwd_launch<T, HOM_N>(const Pipe<T>&, hipStream_t, bool);             \
  template LaunchInfo xinv_launch<T, HOM_N>(const Pipe<T>&, hipStream_t, bool);             \
  template LaunchInfo ypass_launch<T, HOM_N>(const Pipe<T>&, int, int, hipStream_t, bool);  \
  template LaunchInfo zgreen_launch<T, HOM_N>(const Pipe<T>&, int, hipStream_t, bool);
HOM_INST(float)
HOM_INST(double)

}  // namespace hom
