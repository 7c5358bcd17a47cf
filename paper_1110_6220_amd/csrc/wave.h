// Wave-wide reductions for gfx950 (wave64): DPP row exchanges within each row
// of 16 lanes, then the four row results read with readlane.
#pragma once
#include <hip/hip_runtime.h>

namespace eik {
namespace wave {

// IEEE minNum without the compiler's NaN canonicalisation of the operands
// (operands here are never signalling NaNs); a quiet NaN operand yields the
// other operand.  ALU-only inline assembly.
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float vmin(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// DPP controls: swap neighbouring lanes, swap lane pairs, mirror within half
// rows, mirror within rows
constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double min_d(double v) {
  v = vmin(v, dpp_d<kXor1>(v));
  v = vmin(v, dpp_d<kXor2>(v));
  v = vmin(v, dpp_d<kHalfMirror>(v));
  v = vmin(v, dpp_d<kMirror>(v));
  return vmin(vmin(readlane_d(v, 0), readlane_d(v, 16)), vmin(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double max_d(double v) {
  v = vmax(v, dpp_d<kXor1>(v));
  v = vmax(v, dpp_d<kXor2>(v));
  v = vmax(v, dpp_d<kHalfMirror>(v));
  v = vmax(v, dpp_d<kMirror>(v));
  return vmax(vmax(readlane_d(v, 0), readlane_d(v, 16)), vmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ int min_i(int v) {
  v = min(v, dpp_i<kXor1>(v));
  v = min(v, dpp_i<kXor2>(v));
  v = min(v, dpp_i<kHalfMirror>(v));
  v = min(v, dpp_i<kMirror>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Wave-wide minimum of the lanes' (v, c) in lexicographic order (values are
// never NaN; lanes without an entry hold (+inf, INT_MAX)); the winning
// lane's (v, c, slot), wave-uniform.
__device__ __forceinline__ void argmin(double& v, int& c, int& slot, int lane) {
  const double vm = min_d(v);
  const unsigned long long tie = __ballot(v == vm);
  int win = __builtin_ctzll(tie);
  if (tie & (tie - 1)) {  // equal values: the smallest cell index
    const bool in = (tie >> lane) & 1ull;
    const int cm = min_i(in ? c : 0x7fffffff);
    win = __builtin_ctzll(__ballot(in && c == cm));
  }
  v = vm;
  c = __builtin_amdgcn_readlane(c, win);
  slot = __builtin_amdgcn_readlane(slot, win);
}

}  // namespace wave
}  // namespace eik
