// Wavefront (64-lane) reductions and broadcasts for gfx950 without the LDS
// crossbar: DPP within each 16-lane row (quad_perm xor-1/xor-2, half-row and
// row mirrors), v_permlane16_swap across row pairs and v_permlane32_swap
// across wave halves.  Every lane ends with the same value, computed with the
// same operand order (each step combines a value with its partner's, and the
// operations used are commutative), so results are bitwise identical across
// lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rbp {
namespace wave {

constexpr int kXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141; // lane i <-> 7-i within each 8 lanes
constexpr int kMirror = 0x140;     // lane i <-> 15-i within each row

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL>(int(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// exchanges across 16-lane rows (r0<->r1, r2<->r3) and wave halves: each lane
// gets the pair (value of the lower row/half, value of the upper one)
struct PairD { double a, b; };
struct PairI { int a, b; };
__device__ __forceinline__ PairI swap16_i32(int v) {
  auto r = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(v), static_cast<unsigned>(v), false, false);
  return {int(r[0]), int(r[1])};
}
__device__ __forceinline__ PairI swap32_i32(int v) {
  auto r = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(v), static_cast<unsigned>(v), false, false);
  return {int(r[0]), int(r[1])};
}
__device__ __forceinline__ PairD swap_f64(double v, bool s32) {
  const long long b = __double_as_longlong(v);
  const PairI lo = s32 ? swap32_i32(int(b & 0xffffffffll)) : swap16_i32(int(b & 0xffffffffll));
  const PairI hi = s32 ? swap32_i32(int(b >> 32)) : swap16_i32(int(b >> 32));
  auto mk = [](int l, int h) {
    return __longlong_as_double((static_cast<long long>(h) << 32) | static_cast<unsigned int>(l));
  };
  return {mk(lo.a, hi.a), mk(lo.b, hi.b)};
}

template <typename Op>
__device__ __forceinline__ double reduce_f64(double v, Op op) {
  v = op(v, dpp_f64<kXor1>(v));
  v = op(v, dpp_f64<kXor2>(v));
  v = op(v, dpp_f64<kHalfMirror>(v));
  v = op(v, dpp_f64<kMirror>(v));
  PairD p = swap_f64(v, false);
  v = op(p.a, p.b);
  p = swap_f64(v, true);
  return op(p.a, p.b);
}

__device__ __forceinline__ double sum(double v) {
  return reduce_f64(v, [](double a, double b) { return a + b; });
}
// four sums at once (the stages of the four trees interleave)
__device__ __forceinline__ void sum4(double (&v)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = v[u] + dpp_f64<kXor1>(v[u]);
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = v[u] + dpp_f64<kXor2>(v[u]);
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = v[u] + dpp_f64<kHalfMirror>(v[u]);
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = v[u] + dpp_f64<kMirror>(v[u]);
#pragma unroll
  for (int u = 0; u < 4; ++u) { const PairD p = swap_f64(v[u], false); v[u] = p.a + p.b; }
#pragma unroll
  for (int u = 0; u < 4; ++u) { const PairD p = swap_f64(v[u], true); v[u] = p.a + p.b; }
}
__device__ __forceinline__ double max(double v) {
  return reduce_f64(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ double min(double v) {
  return reduce_f64(v, [](double a, double b) { return fmin(a, b); });
}

// (value, id) with the larger value, the lower id on ties
__device__ __forceinline__ void pick_max(double& v, int& id, double ov, int oid) {
  if (ov > v || (ov == v && oid < id)) { v = ov; id = oid; }
}
__device__ __forceinline__ void pick_min(double& v, int& id, double ov, int oid) {
  if (ov < v || (ov == v && oid < id)) { v = ov; id = oid; }
}

template <bool MAX>
__device__ __forceinline__ void arg_reduce(double& v, int& id) {
  auto pick = [](double& a, int& ia, double b, int ib) {
    if (MAX) pick_max(a, ia, b, ib); else pick_min(a, ia, b, ib);
  };
  pick(v, id, dpp_f64<kXor1>(v), dpp_i32<kXor1>(id));
  pick(v, id, dpp_f64<kXor2>(v), dpp_i32<kXor2>(id));
  pick(v, id, dpp_f64<kHalfMirror>(v), dpp_i32<kHalfMirror>(id));
  pick(v, id, dpp_f64<kMirror>(v), dpp_i32<kMirror>(id));
  {
    const PairD p = swap_f64(v, false);
    const PairI q = swap16_i32(id);
    v = p.a; id = q.a;
    pick(v, id, p.b, q.b);
  }
  {
    const PairD p = swap_f64(v, true);
    const PairI q = swap32_i32(id);
    v = p.a; id = q.a;
    pick(v, id, p.b, q.b);
  }
}
__device__ __forceinline__ void argmax(double& v, int& id) { arg_reduce<true>(v, id); }
__device__ __forceinline__ void argmin(double& v, int& id) { arg_reduce<false>(v, id); }

// value of lane k (k uniform across the wave)
__device__ __forceinline__ float bcast(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double bcast(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), k);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

}  // namespace wave
}  // namespace rbp
