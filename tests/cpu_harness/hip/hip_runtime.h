#pragma once
// Host shim: lets the line-FFT device code compile for the CPU, one std::thread
// per lane, __syncthreads() as a std::barrier (used only by the CPU harness test).
#include <barrier>
#include <cmath>
#define __device__
#define __host__
#define __forceinline__ inline
#define __global__
#define __restrict__
extern thread_local std::barrier<>* g_bar;
inline void __syncthreads() { g_bar->arrive_and_wait(); }

// Wavefront shuffle of the lanes of one simulated line (thread g_lane of the
// block): every lane stores its value, then reads lane - o of its segment.
extern thread_local int g_lane;
extern double* g_shfl;
template <typename T> inline T __shfl_up(T v, unsigned o, int width) {
  g_shfl[g_lane] = (double)v;
  __syncthreads();
  const int l = g_lane % width;
  const T r = l >= (int)o ? (T)g_shfl[g_lane - (int)o] : v;
  __syncthreads();
  return r;
}
