// Device helpers shared by the HIP sources: wave64 DPP reductions, block reductions,
// global-address-space views of device pointers, direct global->LDS staging and the
// flat-index walker of the staging loops.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sp_internal.h"

namespace {

constexpr float kB0 = 0.0625f, kB1 = 0.25f, kB2 = 0.375f;   // (1,4,6,4,1)/16, exact in FP32
__device__ __forceinline__ float binom(int i) {              // i in -2..2
  return (i == 0) ? kB2 : ((i == 1 || i == -1) ? kB1 : kB0);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------- wave64 reductions (DPP)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }

// Minimum and maximum of non-negative floats on their bit patterns: for values >= 0 the
// unsigned order of the bits is the float order, so no NaN canonicalisation is needed.
__device__ __forceinline__ float fmin_nn(float a, float b) {
  return __uint_as_float(min(__float_as_uint(a), __float_as_uint(b)));
}
__device__ __forceinline__ float fmax_nn(float a, float b) {
  return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}
// Per 16-lane row (an 8x8 block of 2x2 quads): every lane ends with its row's minimum and
// maximum.  Written as DPP-combined v_min_u32/v_max_u32 (the compiler keeps a separate
// DPP move per step); every lane must be active.  The s_nop 1 before each step gives
// the two wait states a DPP read of a VGPR needs after a VALU write to it.
__device__ __forceinline__ void row16_minmax_nn(float& mn, float& mx) {
  uint32_t a = __float_as_uint(mn), b = __float_as_uint(mx);
  asm volatile(
      "s_nop 1\n"
      "v_min_u32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
      "v_max_u32_dpp %1, %1, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n"
      "s_nop 1\n"
      "v_min_u32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
      "v_max_u32_dpp %1, %1, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n"
      "s_nop 1\n"
      "v_min_u32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n"
      "v_max_u32_dpp %1, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xf\n"
      "s_nop 1\n"
      "v_min_u32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n"
      "v_max_u32_dpp %1, %1, %1 row_mirror row_mask:0xf bank_mask:0xf\n"
      : "+v"(a), "+v"(b));
  mn = __uint_as_float(a);
  mx = __uint_as_float(b);
}

// The four 16-lane rows' results of row16_minmax_nn combined across the wavefront: rows
// whose block is not valid are set aside (min ignores them, max and sum count them as 0:
// the values are >= 0), then two DPP broadcast steps (row 15 into the next row, then lane
// 31 into rows 2 and 3) leave in lane 63 the minimum, the maximum and the sum of the row
// maxima ((b2 + b3) + (b0 + b1)).  Every lane must be active.
__device__ __forceinline__ void rows4_combine_nn(float mn, float mx, bool valid, float& omn, float& omx, float& osum) {
  uint32_t a = valid ? __float_as_uint(mn) : 0xffffffffu, b = valid ? __float_as_uint(mx) : 0u;
  float c = valid ? mx : 0.f;
  asm volatile(
      "s_nop 1\n"
      "v_min_u32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n"
      "v_max_u32_dpp %1, %1, %1 row_bcast:15 row_mask:0xa bank_mask:0xf\n"
      "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n"
      "s_nop 1\n"
      "v_min_u32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n"
      "v_max_u32_dpp %1, %1, %1 row_bcast:31 row_mask:0xc bank_mask:0xf\n"
      "v_add_f32_dpp %2, %2, %2 row_bcast:31 row_mask:0xc bank_mask:0xf\n"
      : "+v"(a), "+v"(b), "+v"(c));
  omn = a == 0xffffffffu ? INFINITY : __uint_as_float(a);
  omx = __uint_as_float(b);
  osum = c;
}

struct OpMax { __device__ static float f(float a, float b) { return fmaxf(a, b); } };
struct OpMin { __device__ static float f(float a, float b) { return fminf(a, b); } };
struct OpSum { __device__ static float f(float a, float b) { return a + b; } };

// Every lane must be active.  Result is wave-uniform.
template <class Op>
__device__ __forceinline__ float wave_reduce(float v) {
  v = Op::f(v, dpp_f<0xB1>(v));    // quad_perm [1,0,3,2]
  v = Op::f(v, dpp_f<0x4E>(v));    // quad_perm [2,3,0,1]
  v = Op::f(v, dpp_f<0x141>(v));   // row_half_mirror
  v = Op::f(v, dpp_f<0x140>(v));   // row_mirror: every lane of a row holds the row result
  const int b = __float_as_int(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(b, 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(b, 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(b, 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(b, 48));
  return Op::f(Op::f(r0, r1), Op::f(r2, r3));
}

__device__ __forceinline__ int wave_min_i(int v) {
  v = min(v, dpp_i<0xB1>(v));
  v = min(v, dpp_i<0x4E>(v));
  v = min(v, dpp_i<0x141>(v));
  v = min(v, dpp_i<0x140>(v));
  const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return min(min(r0, r1), min(r2, r3));
}

__device__ __forceinline__ uint32_t wave_max_u(uint32_t v) {
  int x = (int)v;
  // values are non-negative sums of three bytes, so signed max is the unsigned max
  x = max(x, dpp_i<0xB1>(x));
  x = max(x, dpp_i<0x4E>(x));
  x = max(x, dpp_i<0x141>(x));
  x = max(x, dpp_i<0x140>(x));
  const int r0 = __builtin_amdgcn_readlane(x, 0), r1 = __builtin_amdgcn_readlane(x, 16);
  const int r2 = __builtin_amdgcn_readlane(x, 32), r3 = __builtin_amdgcn_readlane(x, 48);
  return (uint32_t)max(max(r0, r1), max(r2, r3));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL));
  const int hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int LANE>
__device__ __forceinline__ double readlane_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), LANE);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), LANE);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Wave-uniform FP64 sum (every lane active).
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane_d<0>(v) + readlane_d<16>(v)) + (readlane_d<32>(v) + readlane_d<48>(v));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Block-wide (256 threads) reductions; result returned to every thread.
template <class Op>
__device__ float block_reduce(float v, float* sh4) {
  v = wave_reduce<Op>(v);
  __syncthreads();
  if (lane_id() == 0) sh4[wave_id()] = v;
  __syncthreads();
  return Op::f(Op::f(sh4[0], sh4[1]), Op::f(sh4[2], sh4[3]));
}

__device__ double block_sum_d(double v, double* sh256) {
  sh256[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh256[threadIdx.x] += sh256[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh256[0];
  __syncthreads();
  return r;
}

// Exact 64-bit sum over the workgroup: butterfly within each wavefront, then the four
// wavefront sums (two barriers).
__device__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh4) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane_id() == 0) sh4[wave_id()] = v;
  __syncthreads();
  const unsigned long long r = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- LDS staging
// Direct global -> LDS loads (global_load_lds_dword): each active lane fetches one float
// into LDS at the wavefront's uniform base + 4 * lane, without a VGPR round trip and
// without a wait per element, so a staging loop keeps all its loads in flight.  A loop
// over a flat index i = threadIdx.x + k * SP_BLOCK passes the lane's own destination
// (region + i); since i - lane is the same for the whole wavefront, the base is
// region + i - lane.  The copy is complete after lds_wait() and a barrier.  The 16-byte
// form (global_load_lds_dwordx4, lane l writing four floats at the base + 16 * l) is used
// through the wave-uniform helpers below; its source and destination are 16-byte aligned.
typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ void lds_load(float* dst_of_lane, const float* src) {
  __builtin_amdgcn_global_load_lds(src, (lds_void*)(dst_of_lane - lane_id()), 4, 0, 0);
}
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0); }

// Global-memory views of device pointers.  Pointers read from the stream and step
// descriptors are generic to the compiler, which then emits flat memory instructions;
// those count against the LDS counter as well, so each LDS wait would also wait for
// every outstanding global store.  Cast to the global address space they become
// global_load / global_store.
template <class T>
using gp = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gp<T> G(T* p) {
  return (gp<T>)p;
}

// base + a 32-bit byte offset, which the compiler addresses as a scalar base plus one
// vector register (no 64-bit vector add per access).  Frames hold at most 2^28 pixels,
// so byte offsets into a plane stay below 2^30.
template <class T>
__device__ __forceinline__ gp<T> at_bytes(gp<T> base, uint32_t byte_off) {
  typedef __attribute__((address_space(1))) char gchar;
  return (gp<T>)((gchar*)base + byte_off);
}

// Wave-uniform forms of the direct loads: wave_dst is the LDS address of the wavefront's
// lane 0 (one value for the whole wavefront, so M0 is set from scalar registers with no
// read-back from a vector register), and the source is a uniform base plus the lane's
// 32-bit byte offset (the scalar-base form of the instruction).  A loop over k with
// element i = k * SP_BLOCK + threadIdx.x passes region + k * SP_BLOCK + wave_first()
// (times 4 for the 16-byte form).
__device__ __forceinline__ int wave_first() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63); }
__device__ __forceinline__ void lds_load_u(float* wave_dst, gp<const float> base, uint32_t byte_off) {
  __builtin_amdgcn_global_load_lds(at_bytes(base, byte_off), (lds_void*)wave_dst, 4, 0, 0);
}
__device__ __forceinline__ void lds_load4_u(float* wave_dst, gp<const float> base, uint32_t byte_off) {
  __builtin_amdgcn_global_load_lds(at_bytes(base, byte_off), (lds_void*)wave_dst, 16, 0, 0);
}
// Streaming store (nt: not kept in the caches) for per-pixel outputs written once and not
// read again within the step.
__device__ __forceinline__ void st_stream(gp<float> p, float v) { __builtin_nontemporal_store(v, p); }

// Row and column of the flat index i = threadIdx.x + k * SP_BLOCK over rows of length
// w, advanced by SP_BLOCK per step: the quotient and remainder of the start and of the
// stride are taken once, so a staging loop does no integer division per element.
struct Walk2 {
  int r, c, dr, dc, w;
  __device__ __forceinline__ Walk2(int start, int w_) : w(max(w_, 1)) {
    r = start / w;
    c = start - r * w;
    dr = SP_BLOCK / w;
    dc = SP_BLOCK - dr * w;
  }
  __device__ __forceinline__ void next() {
    r += dr;
    c += dc;
    if (c >= w) {
      c -= w;
      ++r;
    }
  }
};

}  // namespace
