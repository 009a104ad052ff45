// Minimum cut of the MRF (Section 4: the MAP labelling is the minimum s-t cut of the graph
// with one vertex per pixel, t-links c(s, v) and c(v, t) from the unary costs and a pair of
// equal directed n-links between 8-neighbours), on integer capacities q(c) =
// rint(c * scale) clamped to [0, 2^24], so the flow is exact.  The source side is the object:
// a pixel on the sink side pays U0, one on the source side U1.
//
// Push-relabel on the grid.  Each t-link pair is saturated up front (min(U0, U1) flows
// source -> pixel -> sink), leaving an excess U0 - min at the pixel and a residual U1 - min to
// the sink.  Then rounds of
//   * a global relabel: every height set to the exact distance to the sink in the residual
//     graph, by Bellman-Ford relaxation over 32x32 tiles in LDS (each pass relaxes its tile to
//     a fixed point against the neighbouring tiles' heights; passes repeat until none lowers a
//     height), and a count of the pixels with excess that can reach the sink;
//   * launches of push / relabel cycles, one thread per pixel: a pixel with excess pushes to
//     its lowest residual neighbour (or the sink) when it is higher, else lifts itself above
//     it.  Excess and residual capacities change only by device-scope atomics and a pixel
//     only takes away what it has just read, so they never go negative whatever the
//     interleaving; stale heights of neighbours only delay work.
// The rounds end when no pixel with excess can reach the sink: the preflow is then maximum,
// and the pixels that can still reach the sink form the smallest sink side of all minimum
// cuts (the same for every maximum flow); the others are the object.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <algorithm>

#include "sp_internal.h"
#include "sp_kernels.h"
#include "sp_device.h"

namespace {

// Offsets of the n-link directions E, W, S, N, SE, NW, SW, NE.
__device__ __forceinline__ int DYf(int d) { return (d == 2 || d == 4 || d == 6) ? 1 : ((d == 3 || d == 5 || d == 7) ? -1 : 0); }
__device__ __forceinline__ int DXf(int d) { return (d == 0 || d == 4 || d == 7) ? 1 : ((d == 1 || d == 5 || d == 6) ? -1 : 0); }

__device__ __forceinline__ int32_t ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t quant(float c, float scale) {
  float v = rintf(c * scale);
  if (!(v > 0.f)) return 0;   // negative and NaN
  return v >= (float)SP_CUT_CAPMAX ? SP_CUT_CAPMAX : (int32_t)v;
}

__global__ __launch_bounds__(SP_BLOCK) void k_cut_init(CutIO io) {
  __shared__ unsigned long long sh4[4];
  const int n = io.H * io.W;
  unsigned long long acc = 0;
  for (int i = blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += gridDim.x * SP_BLOCK) {
    const int y = i / io.W, x = i - (i / io.W) * io.W;
    const int32_t cs = quant(io.unary[i], io.scale), ct = quant(io.unary[n + i], io.scale);
    const int32_t m = min(cs, ct);
    acc += (unsigned long long)m;
    io.e[i] = cs - m;
    io.rt[i] = ct - m;
    io.h[i] = ct - m > 0 ? 1 : SP_CUT_INF;
    // the capacity of a pair sits in the pairwise plane of its upper (or left) pixel
    const float* pw = io.pairwise;
    int32_t c[8];
    c[0] = x + 1 < io.W ? quant(pw[i], io.scale) : 0;                                       // E
    c[1] = x > 0 ? quant(pw[i - 1], io.scale) : 0;                                          // W
    c[2] = y + 1 < io.H ? quant(pw[n + i], io.scale) : 0;                                   // S
    c[3] = y > 0 ? quant(pw[n + i - io.W], io.scale) : 0;                                   // N
    c[4] = (y + 1 < io.H && x + 1 < io.W) ? quant(pw[2 * n + i], io.scale) : 0;             // SE
    c[5] = (y > 0 && x > 0) ? quant(pw[2 * n + i - io.W - 1], io.scale) : 0;                // NW
    c[6] = (y + 1 < io.H && x > 0) ? quant(pw[3 * n + i], io.scale) : 0;                    // SW
    c[7] = (y > 0 && x + 1 < io.W) ? quant(pw[3 * n + i - io.W + 1], io.scale) : 0;         // NE
#pragma unroll
    for (int d = 0; d < 8; ++d) io.r[(size_t)d * n + i] = c[d];
  }
  acc = block_sum_u64(acc, sh4);
  if (threadIdx.x == 0 && acc) atomicAdd(&io.flow[0], acc);
}

// One tile of the global relabel.  Region: the tile and a one-pixel ring; the ring keeps
// the heights its owners had when read (an upper bound, which is all relaxation needs).
__global__ __launch_bounds__(SP_BLOCK) void k_cut_relabel(CutIO io) {
  constexpr int RN = SP_CUT_T + 2;
  constexpr int PER = SP_CUT_T * SP_CUT_T / SP_BLOCK;
  __shared__ int32_t hl[RN * RN];
  __shared__ int act_sh[4];
  const int ntx = (io.W + SP_CUT_T - 1) / SP_CUT_T;
  const int ty0 = (blockIdx.x / ntx) * SP_CUT_T, tx0 = (blockIdx.x % ntx) * SP_CUT_T;
  const int n = io.H * io.W;
  for (int k = threadIdx.x; k < RN * RN; k += SP_BLOCK) {
    const int y = ty0 - 1 + k / RN, x = tx0 - 1 + k % RN;
    int32_t v = SP_CUT_INF;
    if (y >= 0 && y < io.H && x >= 0 && x < io.W) {
      const int i = y * io.W + x;
      v = io.reset ? (io.rt[i] > 0 ? 1 : SP_CUT_INF) : io.h[i];
    }
    hl[k] = v;
  }
  // the residual n-links of the thread's pixels as bit masks (bit d: r(v, d) > 0)
  uint32_t mask[PER];
  int32_t h0[PER];
  int li[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + k * SP_BLOCK;
    const int y = ty0 + t / SP_CUT_T, x = tx0 + t % SP_CUT_T;
    li[k] = (t / SP_CUT_T + 1) * RN + (t % SP_CUT_T) + 1;
    mask[k] = 0;
    if (y < io.H && x < io.W) {
      const int i = y * io.W + x;
#pragma unroll
      for (int d = 0; d < 8; ++d)
        if (io.r[(size_t)d * n + i] > 0) mask[k] |= 1u << d;
      mask[k] |= 1u << 8;   // in the frame
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) h0[k] = hl[li[k]];
  for (int it = 0; it < RN * RN; ++it) {
    bool ch = false;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (!(mask[k] & 0x100)) continue;
      int32_t best = hl[li[k]];
#pragma unroll
      for (int d = 0; d < 8; ++d)
        if (mask[k] & (1u << d)) best = min(best, hl[li[k] + DYf(d) * RN + DXf(d)] + 1);
      if (best < hl[li[k]]) {
        hl[li[k]] = best;
        ch = true;
      }
    }
    if (!__syncthreads_or(ch)) break;
  }
  // write back the lowered heights (all of them in a reset pass); count the pixels with
  // excess that reach the sink
  bool wrote = false;
  int act = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (!(mask[k] & 0x100)) continue;
    const int t = threadIdx.x + k * SP_BLOCK;
    const int i = (ty0 + t / SP_CUT_T) * io.W + tx0 + t % SP_CUT_T;
    const int32_t v = hl[li[k]];
    if (io.reset || v != h0[k]) io.h[i] = v;
    wrote |= v != h0[k];
    if (v < SP_CUT_INF && io.e[i] > 0) ++act;
  }
  for (int o = 32; o > 0; o >>= 1) act += __shfl_xor(act, o);
  if (lane_id() == 0) act_sh[wave_id()] = act;
  const bool any = __syncthreads_or(wrote);
  if (threadIdx.x == 0) {
    const int tot = act_sh[0] + act_sh[1] + act_sh[2] + act_sh[3];
    if (tot) atomicAdd(&io.flags[1], tot);
    if (any) atomicOr(&io.flags[0], 1);
  }
}

// Push / relabel cycles, one thread per pixel.
__global__ __launch_bounds__(SP_BLOCK) void k_cut_push(CutIO io) {
  __shared__ unsigned long long sh4[4];
  const int n = io.H * io.W;
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  unsigned long long sunk = 0;
  if (i < n) {
    const int y = i / io.W, x = i - y * io.W;
    for (int cyc = 0; cyc < io.cycles; ++cyc) {
      const int32_t ev = ld(io.e + i);
      const int32_t hv = ld(io.h + i);
      if (ev <= 0 || hv >= SP_CUT_INF) break;
      const int32_t rtv = io.rt[i];
      int32_t hmin = SP_CUT_INF, cap = 0;
      int dmin = -1;
      if (rtv > 0) {
        hmin = 0;
        dmin = 8;
        cap = rtv;
      }
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int yy = y + DYf(d), xx = x + DXf(d);
        if (yy < 0 || yy >= io.H || xx < 0 || xx >= io.W) continue;
        const int32_t rr = ld(io.r + (size_t)d * n + i);
        if (rr <= 0) continue;
        const int32_t hu = ld(io.h + yy * io.W + xx);
        if (hu < hmin) {
          hmin = hu;
          dmin = d;
          cap = rr;
        }
      }
      if (dmin < 0 || hmin >= SP_CUT_INF) {
        st(io.h + i, SP_CUT_INF);   // no residual path: it cannot reach the sink
        break;
      }
      if (hv > hmin) {
        const int32_t delta = min(ev, cap);
        if (dmin == 8) {
          io.rt[i] = rtv - delta;
          sunk += (unsigned long long)delta;
        } else {
          const int j = (y + DYf(dmin)) * io.W + x + DXf(dmin);
          atomicSub(io.r + (size_t)dmin * n + i, delta);
          atomicAdd(io.r + (size_t)(dmin ^ 1) * n + j, delta);
          atomicAdd(io.e + j, delta);
        }
        atomicSub(io.e + i, delta);
      } else {
        st(io.h + i, hmin + 1);
      }
    }
  }
  sunk = block_sum_u64(sunk, sh4);
  if (threadIdx.x == 0 && sunk) atomicAdd(&io.flow[1], sunk);
}

__global__ __launch_bounds__(SP_BLOCK) void k_cut_labels(CutIO io) {
  const int n = io.H * io.W;
  for (int i = blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += gridDim.x * SP_BLOCK)
    io.labels[i] = io.h[i] >= SP_CUT_INF ? 1 : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && io.flow_out)
    *io.flow_out = (int64_t)(io.flow[0] + io.flow[1]);
}

__global__ void k_cut_zero(CutIO io, int what) {
  if (threadIdx.x == 0) {
    if (what & 1) io.flow[0] = io.flow[1] = 0ull;
    if (what & 2) io.flags[0] = io.flags[1] = 0;
  }
}

}  // namespace

hipError_t sp_launch_cut(int phase, const CutIO& io, hipStream_t st) {
  const int n = io.H * io.W;
  const int grid = (int)std::min(4096, (n + SP_BLOCK - 1) / SP_BLOCK);
  switch (phase) {
    case 0:
      hipLaunchKernelGGL(k_cut_zero, dim3(1), dim3(64), 0, st, io, 3);
      hipLaunchKernelGGL(k_cut_init, dim3(grid), dim3(SP_BLOCK), 0, st, io);
      break;
    case 1: {
      const int tiles = ((io.H + SP_CUT_T - 1) / SP_CUT_T) * ((io.W + SP_CUT_T - 1) / SP_CUT_T);
      hipLaunchKernelGGL(k_cut_zero, dim3(1), dim3(64), 0, st, io, 2);
      hipLaunchKernelGGL(k_cut_relabel, dim3(tiles), dim3(SP_BLOCK), 0, st, io);
      break;
    }
    case 2: hipLaunchKernelGGL(k_cut_push, dim3((n + SP_BLOCK - 1) / SP_BLOCK), dim3(SP_BLOCK), 0, st, io); break;
    case 3: hipLaunchKernelGGL(k_cut_labels, dim3(grid), dim3(SP_BLOCK), 0, st, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
