// Host launchers of the FFT pipeline kernels. The kernels are templated on
// the line length; one object file per supported length instantiates them
// (pipe_inst.hip compiled with -DHOM_N=<n>), and the dispatchers below pick
// the instantiation at run time.
#pragma once
#include "common.h"

namespace hom {

// Supported transform lengths along every axis.
constexpr int kSupportedN[] = {16, 24, 32, 48, 64, 96, 128, 256};

inline bool supported_n(int n) {
  for (int v : kSupportedN)
    if (v == n) return true;
  return false;
}

// Elements per thread of the line FFT of length n (threads per line = n / M).
constexpr int plan_m(int n) {
  switch (n) {
    case 16: return 4;
    case 24: return 12;
    case 32: return 8;
    case 48: return 12;
    case 64: return 8;
    case 96: return 24;
    case 128: return 16;
    case 256: return 16;
  }
  return 0;
}

// x-pass lines per work-group. The FP32 forward pass holds the three CG
// fields of its voxels in registers, which allows fewer of its work-groups per
// CU: it takes half as many lines, so more, smaller work-groups overlap their
// load and transform phases.
constexpr int x_lines(int n, bool fp64, bool fwd) {
  const int nl = ((fp64 ? 64 : 128) / (n / plan_m(n))) / (fwd && !fp64 ? 2 : 1);
  return nl < 1 ? 1 : nl;
}

// Schedules of the y and z passes: tile width (kx columns per work-group: 2,
// 4 or 8) and FFT plan variant (0 or 1, Plan<N, V>), packed as width + 16 V.
// The autotuner times every one on the problem's own data.
constexpr int schedule(int tile, int plan) { return tile + 16 * plan; }
constexpr int schedule_tile(int s) { return s & 15; }
constexpr int schedule_plan(int s) { return s >> 4; }
constexpr int kScheduleChoices[] = {schedule(2, 0), schedule(4, 0), schedule(8, 0),
                                    schedule(2, 1), schedule(4, 1), schedule(8, 1)};

struct LaunchInfo {
  int blocks;
  int threads;
  size_t lds;
};

template <typename T, int N>
LaunchInfo xfwd_launch(const Pipe<T>& a, hipStream_t s, bool dry);
template <typename T, int N>
LaunchInfo xinv_launch(const Pipe<T>& a, hipStream_t s, bool dry);
template <typename T, int N>
LaunchInfo ypass_launch(const Pipe<T>& a, int sched, int inverse, hipStream_t s, bool dry);
template <typename T, int N>
LaunchInfo zgreen_launch(const Pipe<T>& a, int sched, hipStream_t s, bool dry);

template <typename T>
LaunchInfo run_xfwd(const Pipe<T>& a, hipStream_t s, bool dry = false);
template <typename T>
LaunchInfo run_xinv(const Pipe<T>& a, hipStream_t s, bool dry = false);
template <typename T>
LaunchInfo run_ypass(const Pipe<T>& a, int sched, int inverse, hipStream_t s, bool dry = false);
template <typename T>
LaunchInfo run_zgreen(const Pipe<T>& a, int sched, hipStream_t s, bool dry = false);

}  // namespace hom
