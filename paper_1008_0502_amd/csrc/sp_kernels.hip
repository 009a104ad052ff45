// HIP kernels (gfx950, wave64) of the saliency -> Kalman prior -> MRF weight path.
//
// One workgroup of 256 threads per job; the job table says which stream and which
// tile.  Maps are row-major FP32.  Reductions inside a wavefront use DPP row
// permutes (quad_perm, row_half_mirror, row_mirror) plus readlane across the four
// rows; across wavefronts they go through LDS in a fixed order, so every result is
// independent of scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "sp_internal.h"
#include "sp_kernels.h"

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

__device__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* sh256) {
  sh256[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh256[threadIdx.x] += sh256[threadIdx.x + s];
    __syncthreads();
  }
  const unsigned long long r = sh256[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- stream helpers
__device__ __forceinline__ const float* base_ptr(const StreamDesc& sd, const float* ckpt, int l) {
  return (l == sd.c_min && ckpt) ? ckpt : sd.base[l];
}

// Channel k (I, RG, BY, O0, O45, O90, O135, M) of level l.
__device__ __forceinline__ const float* chan_ptr(const StreamDesc& sd, const float* ckpt, int k, int l) {
  const size_t plane = (size_t)sd.Hl[l] * sd.Wl[l];
  if (k < 3) return base_ptr(sd, ckpt, l) + k * plane;
  if (k == 7) return base_ptr(sd, ckpt, l) + 3 * plane;
  return sd.gab[l] + (k - 3) * plane;
}

// Sample-aligned bilinear tap set for target index y of a map whose source level is
// d steps coarser and has n samples: position y / 2^d clamped to [0, n-1].
struct Tap { int i0, i1; float w; };
__device__ __forceinline__ Tap bilinear_tap(int y, int d, int n) {
  float f = (float)y * __int_as_float((127 - d) << 23);   // y * 2^-d, exact
  f = fminf(f, (float)(n - 1));
  Tap t;
  t.i0 = (int)f;
  t.w = f - (float)t.i0;
  t.i1 = min(t.i0 + 1, n - 1);
  return t;
}

__device__ __forceinline__ float bilinear(const float* X, int Ws, const Tap& ty, const Tap& tx) {
  const float a = X[(size_t)ty.i0 * Ws + tx.i0], b = X[(size_t)ty.i0 * Ws + tx.i1];
  const float c = X[(size_t)ty.i1 * Ws + tx.i0], e = X[(size_t)ty.i1 * Ws + tx.i1];
  const float top = (1.f - tx.w) * a + tx.w * b;
  const float bot = (1.f - tx.w) * c + tx.w * e;
  return (1.f - ty.w) * top + ty.w * bot;
}

// N(.) parameters of one map from its partial triples (min, max, sum of block maxima).
struct NParams { float mn, inv, scale; int flat; };

__device__ NParams nparams_from_parts(const float* parts, int n, int nb, float flat_tol,
                                      float* sh4, double* sh256) {
  float mn = INFINITY, mx = -INFINITY;
  double sb = 0.0;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) {
    mn = fminf(mn, parts[3 * i]);
    mx = fmaxf(mx, parts[3 * i + 1]);
    sb += (double)parts[3 * i + 2];
  }
  mn = block_reduce<OpMin>(mn, sh4);
  mx = block_reduce<OpMax>(mx, sh4);
  sb = block_sum_d(sb, sh256);
  NParams p;
  p.mn = mn;
  p.flat = (mx - mn <= flat_tol) ? 1 : 0;
  if (p.flat) {
    p.inv = 0.f;
    p.scale = 0.f;
  } else {
    const double range = (double)mx - (double)mn;
    const double mbar = (nb > 1) ? (((sb - (double)nb * (double)mn) / range) - 1.0) / (double)(nb - 1) : 0.0;
    p.inv = (float)(1.0 / range);
    p.scale = (float)((1.0 - mbar) * (1.0 - mbar));
  }
  return p;
}

__device__ __forceinline__ float napply(const NParams& p, float v) {
  return p.flat ? 0.f : ((v - p.mn) * p.inv) * p.scale;
}

__device__ __forceinline__ int nblocks8(int h, int w) { return ((h + 7) >> 3) * ((w + 7) >> 3); }

// Max of S with its first row-major index, from (max, index) partials.
__device__ void smax_from_parts(const float* parts, int n, float* m_out, int* idx_out, float* sh4, int* shi4) {
  float m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) m = fmaxf(m, parts[2 * i]);
  m = block_reduce<OpMax>(m, sh4);
  int idx = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK)
    if (parts[2 * i] == m) idx = min(idx, __float_as_int(parts[2 * i + 1]));
  idx = wave_min_i(idx);
  __syncthreads();
  if (lane_id() == 0) shi4[wave_id()] = idx;
  __syncthreads();
  *m_out = m;
  *idx_out = min(min(shi4[0], shi4[1]), min(shi4[2], shi4[3]));
}

// Observation before clamping: bilinear up-sample of S / m at level-0 pixel (y, x).
__device__ __forceinline__ float observe_u(const float* S, int Hc, int Wc, int c, float m, int y, int x) {
  const Tap ty = bilinear_tap(y, c, Hc), tx = bilinear_tap(x, c, Wc);
  return bilinear(S, Wc, ty, tx) / m;
}

__device__ __forceinline__ bool on_border(int y, int x, int H, int W, int b) {
  return y < b || y >= H - b || x < b || x >= W - b;
}

#define IOF(field) (ios ? ios[J.stream].field : io0.field)

// ---------------------------------------------------------------- colour statistics
// Largest R+G+B over a band of rows; optionally the sum of squared colour
// differences over the 8-neighbour pairs whose first pixel lies in the band.
__global__ __launch_bounds__(SP_BLOCK) void k_rgb(const Job* __restrict__ jobs,
                                                  const StreamDesc* __restrict__ sds,
                                                  const StepIO* __restrict__ ios, StepIO io0, int want_d2) {
  __shared__ unsigned long long sh[SP_BLOCK];
  __shared__ float sh4[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const uint8_t* __restrict__ rgb = IOF(rgb);
  const int W = sd.W, H = sd.H;
  uint32_t mx = 0;
  unsigned long long d2 = 0;
  const int n = J.th * W;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) {
    const int y = J.y0 + i / W, x = i % W;
    const uint8_t* p = rgb + ((size_t)y * W + x) * 3;
    const int r = p[0], g = p[1], b = p[2];
    mx = max(mx, (uint32_t)(r + g + b));
    if (want_d2) {
      if (x + 1 < W) {
        const int dr = r - p[3], dg = g - p[4], db = b - p[5];
        d2 += (unsigned)(dr * dr + dg * dg + db * db);
      }
      if (y + 1 < H) {
        const uint8_t* q = p + (size_t)3 * W;
        int dr = r - q[0], dg = g - q[1], db = b - q[2];
        d2 += (unsigned)(dr * dr + dg * dg + db * db);
        if (x + 1 < W) {
          dr = r - q[3]; dg = g - q[4]; db = b - q[5];
          d2 += (unsigned)(dr * dr + dg * dg + db * db);
        }
        if (x > 0) {
          dr = r - q[-3]; dg = g - q[-2]; db = b - q[-1];
          d2 += (unsigned)(dr * dr + dg * dg + db * db);
        }
      }
    }
  }
  (void)sh4;
  mx = wave_max_u(mx);
  __shared__ uint32_t shm[4];
  if (lane_id() == 0) shm[wave_id()] = mx;
  const unsigned long long tot = want_d2 ? block_sum_u64(d2, sh) : 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    sd.rgb_max_part[J.a] = max(max(shm[0], shm[1]), max(shm[2], shm[3]));
    if (want_d2) sd.rgb_d2_part[J.a] = tot;
  }
}

// ---------------------------------------------------------------- pyramid
// Separable blur + decimation of a (2*TH+3) x (2*TW+3) LDS region into TH x TW.
template <int TH, int TW, int RH, int RW>
__device__ __forceinline__ void down_region(float (*F)[RH][RW], float (*Hb)[RH][TW], int nch) {
  for (int i = threadIdx.x; i < nch * RH * TW; i += SP_BLOCK) {
    const int c = i / (RH * TW), rem = i - c * RH * TW, r = rem / TW, j = rem - r * TW;
    const float* row = &F[c][r][2 * j];
    Hb[c][r][j] = kB0 * row[0] + kB1 * row[1] + kB2 * row[2] + kB1 * row[3] + kB0 * row[4];
  }
}

template <int TH, int TW>
__global__ __launch_bounds__(SP_BLOCK) void k_feat(const Job* __restrict__ jobs,
                                                   const StreamDesc* __restrict__ sds,
                                                   const StepIO* __restrict__ ios, StepIO io0) {
  constexpr int RH = 2 * TH + 3, RW = 2 * TW + 3;
  __shared__ float F[4][RH][RW];
  __shared__ float Hb[4][RH][TW];
  __shared__ uint32_t shm[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const uint8_t* __restrict__ rgb = IOF(rgb);
  const uint8_t* __restrict__ prev = IOF(rgb_prev);
  float* ckpt = IOF(ckpt);
  uint32_t smax = 0;
  for (int i = threadIdx.x; i < sd.n_rgb; i += SP_BLOCK) smax = max(smax, sd.rgb_max_part[i]);
  smax = wave_max_u(smax);
  if (lane_id() == 0) shm[wave_id()] = smax;
  __syncthreads();
  smax = max(max(shm[0], shm[1]), max(shm[2], shm[3]));
  const int H = sd.H, W = sd.W;
  const int Y0 = 2 * J.y0 - 2, X0 = 2 * J.x0 - 2;
  for (int i = threadIdx.x; i < RH * RW; i += SP_BLOCK) {
    const int ry = i / RW, rx = i - ry * RW;
    const int y = clampi(Y0 + ry, 0, H - 1), x = clampi(X0 + rx, 0, W - 1);
    const size_t o = ((size_t)y * W + x) * 3;
    const int R8 = rgb[o], G8 = rgb[o + 1], B8 = rgb[o + 2];
    const int S8 = R8 + G8 + B8;
    const float I = (float)S8 / 765.f;
    float rg = 0.f, by = 0.f;
    if ((uint32_t)(10 * S8) > smax) {
      const float inv = 3.f / (float)S8;
      const float rp = (float)R8 * inv, gp = (float)G8 * inv, bp = (float)B8 * inv;
      const float Rc = fmaxf(0.f, rp - (gp + bp) * 0.5f);
      const float Gc = fmaxf(0.f, gp - (rp + bp) * 0.5f);
      const float Bc = fmaxf(0.f, bp - (rp + gp) * 0.5f);
      const float Yc = fmaxf(0.f, fminf(rp, gp) - bp);
      rg = Rc - Gc;
      by = Bc - Yc;
    }
    float M = 0.f;
    if (prev) {
      const int P8 = prev[o] + prev[o + 1] + prev[o + 2];
      M = fabsf(I - (float)P8 / 765.f);
    }
    F[0][ry][rx] = I;
    F[1][ry][rx] = rg;
    F[2][ry][rx] = by;
    F[3][ry][rx] = M;
  }
  __syncthreads();
  down_region<TH, TW, RH, RW>(F, Hb, 4);
  __syncthreads();
  const int H1 = sd.Hl[1], W1 = sd.Wl[1];
  float* dst = (sd.c_min == 1 && ckpt) ? ckpt : sd.base[1];
  const size_t plane = (size_t)H1 * W1;
  for (int i = threadIdx.x; i < TH * TW; i += SP_BLOCK) {
    const int yy = i / TW, xx = i - yy * TW;
    const int y = J.y0 + yy, x = J.x0 + xx;
    if (yy < J.th && xx < J.tw && y < H1 && x < W1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float v = kB0 * Hb[c][2 * yy][xx] + kB1 * Hb[c][2 * yy + 1][xx] + kB2 * Hb[c][2 * yy + 2][xx] +
                        kB1 * Hb[c][2 * yy + 3][xx] + kB0 * Hb[c][2 * yy + 4][xx];
        dst[c * plane + (size_t)y * W1 + x] = v;
      }
    }
  }
}

template <int TH, int TW>
__global__ __launch_bounds__(SP_BLOCK) void k_down(const Job* __restrict__ jobs,
                                                   const StreamDesc* __restrict__ sds,
                                                   const StepIO* __restrict__ ios, StepIO io0) {
  constexpr int RH = 2 * TH + 3, RW = 2 * TW + 3;
  __shared__ float F[4][RH][RW];
  __shared__ float Hb[4][RH][TW];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  float* ckpt = IOF(ckpt);
  const int l = J.a;
  const int Hs = sd.Hl[l], Ws = sd.Wl[l];
  const float* src = base_ptr(sd, ckpt, l);
  const size_t splane = (size_t)Hs * Ws;
  const int Y0 = 2 * J.y0 - 2, X0 = 2 * J.x0 - 2;
  for (int i = threadIdx.x; i < RH * RW; i += SP_BLOCK) {
    const int ry = i / RW, rx = i - ry * RW;
    const int y = clampi(Y0 + ry, 0, Hs - 1), x = clampi(X0 + rx, 0, Ws - 1);
    const size_t o = (size_t)y * Ws + x;
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c][ry][rx] = src[c * splane + o];
  }
  __syncthreads();
  down_region<TH, TW, RH, RW>(F, Hb, 4);
  __syncthreads();
  const int Hd = sd.Hl[l + 1], Wd = sd.Wl[l + 1];
  float* dst = (l + 1 == sd.c_min && ckpt) ? ckpt : sd.base[l + 1];
  const size_t plane = (size_t)Hd * Wd;
  for (int i = threadIdx.x; i < TH * TW; i += SP_BLOCK) {
    const int yy = i / TW, xx = i - yy * TW;
    const int y = J.y0 + yy, x = J.x0 + xx;
    if (yy < J.th && xx < J.tw && y < Hd && x < Wd) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float v = kB0 * Hb[c][2 * yy][xx] + kB1 * Hb[c][2 * yy + 1][xx] + kB2 * Hb[c][2 * yy + 2][xx] +
                        kB1 * Hb[c][2 * yy + 3][xx] + kB0 * Hb[c][2 * yy + 4][xx];
        dst[c * plane + (size_t)y * Wd + x] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- Gabor orientation maps
// 13x13 (radius R) zero-DC even Gabor kernels applied as separable rank-1 terms:
//   O0 = H[gm] V[g], O90 = H[g] V[gm],
//   O45 = H[gc] V[gc] - H[gs] V[gs] - c45 H[g] V[g], O135 = same with + H[gs] V[gs].
__global__ __launch_bounds__(SP_BLOCK) void k_gabor(const Job* __restrict__ jobs,
                                                    const StreamDesc* __restrict__ sds,
                                                    const StepIO* __restrict__ ios, StepIO io0) {
  constexpr int T = 16, RM = T + 2 * SP_MAXR;
  __shared__ float Ir[RM][RM + 1];
  __shared__ float V[4][T][RM + 1];
  __shared__ float taps[4][2 * SP_MAXR + 1];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  float* ckpt = IOF(ckpt);
  const int l = J.a, R = sd.gr, n = 2 * R + 1, RR = T + 2 * R;
  const int Hs = sd.Hl[l], Ws = sd.Wl[l];
  const float* I = base_ptr(sd, ckpt, l);
  if ((int)threadIdx.x < 4 * n) taps[threadIdx.x / n][threadIdx.x % n] = sd.gf[threadIdx.x / n][threadIdx.x % n];
  for (int i = threadIdx.x; i < RR * RR; i += SP_BLOCK) {
    const int ry = i / RR, rx = i - ry * RR;
    const int y = clampi(J.y0 - R + ry, 0, Hs - 1), x = clampi(J.x0 - R + rx, 0, Ws - 1);
    Ir[ry][rx] = I[(size_t)y * Ws + x];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * T * RR; i += SP_BLOCK) {
    const int f = i / (T * RR), rem = i - f * T * RR, yy = rem / RR, xr = rem - yy * RR;
    float acc = 0.f;
    for (int v = 0; v < n; ++v) acc += taps[f][v] * Ir[yy + v][xr];
    V[f][yy][xr] = acc;
  }
  __syncthreads();
  const int yy = threadIdx.x / T, xx = threadIdx.x % T;
  const int y = J.y0 + yy, x = J.x0 + xx;
  float A = 0.f, B = 0.f, C = 0.f, D = 0.f, E = 0.f;
  for (int u = 0; u < n; ++u) {
    const float vg = V[0][yy][xx + u];
    A += taps[1][u] * vg;
    B += taps[0][u] * vg;
    C += taps[0][u] * V[1][yy][xx + u];
    D += taps[2][u] * V[2][yy][xx + u];
    E += taps[3][u] * V[3][yy][xx + u];
  }
  if (yy < J.th && xx < J.tw && y < Hs && x < Ws) {
    const size_t plane = (size_t)Hs * Ws, o = (size_t)y * Ws + x;
    float* G = sd.gab[l];
    G[o] = A;
    G[plane + o] = D - E - sd.c45 * B;
    G[2 * plane + o] = C;
    G[3 * plane + o] = D + E - sd.c45 * B;
  }
}

// ---------------------------------------------------------------- centre-surround statistics
// Tile of the centre level c; each wavefront takes 8x8 blocks of the tile.
__global__ __launch_bounds__(SP_BLOCK) void k_csstats(const Job* __restrict__ jobs,
                                                      const StreamDesc* __restrict__ sds,
                                                      const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float acc[4][4 * SP_NCH][3];      // [wave][pair-in-centre * 8 + k][min, max, sum]
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* ckpt = IOF(ckpt);
  const int c = J.a, Hc = sd.Hl[c], Wc = sd.Wl[c];
  const int lane = lane_id(), w = wave_id();
  const int nbx = (J.tw + 7) >> 3, nby = (J.th + 7) >> 3, nbk = nbx * nby;
  int npc = 0;
  for (int p = 0; p < sd.n_pairs; ++p) npc += (sd.pc[p] == c);
  for (int i = threadIdx.x; i < 4 * npc * SP_NCH; i += SP_BLOCK) {
    const int ww = i / (npc * SP_NCH), m = i - ww * npc * SP_NCH;
    acc[ww][m][0] = INFINITY;
    acc[ww][m][1] = -INFINITY;
    acc[ww][m][2] = 0.f;
  }
  __syncthreads();
  for (int bk = w; bk < nbk; bk += 4) {
    const int by = bk / nbx, bx = bk - by * nbx;
    const int y = J.y0 + 8 * by + (lane >> 3), x = J.x0 + 8 * bx + (lane & 7);
    const bool exists = (J.y0 + 8 * by < Hc) && (J.x0 + 8 * bx < Wc);
    const bool valid = y < Hc && x < Wc;
    const int yc = min(y, Hc - 1), xc = min(x, Wc - 1);
    int m = 0;
    for (int p = 0; p < sd.n_pairs; ++p) {
      if (sd.pc[p] != c) continue;
      const int s = sd.ps[p], d = s - c;
      const int Hs = sd.Hl[s], Ws = sd.Wl[s];
      const Tap ty = bilinear_tap(yc, d, Hs), tx = bilinear_tap(xc, d, Ws);
      for (int k = 0; k < SP_NCH; ++k, ++m) {
        const float xcv = chan_ptr(sd, ckpt, k, c)[(size_t)yc * Wc + xc];
        const float up = bilinear(chan_ptr(sd, ckpt, k, s), Ws, ty, tx);
        const float F = fabsf(xcv - up);
        const float bmn = wave_reduce<OpMin>(valid ? F : INFINITY);
        const float bmx = wave_reduce<OpMax>(valid ? F : -INFINITY);
        if (lane == 0 && exists) {
          acc[w][m][0] = fminf(acc[w][m][0], bmn);
          acc[w][m][1] = fmaxf(acc[w][m][1], bmx);
          acc[w][m][2] += bmx;
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npc * SP_NCH; i += SP_BLOCK) {
    const int pi = i / SP_NCH, k = i - pi * SP_NCH;
    int p = 0, seen = -1;
    for (; p < sd.n_pairs; ++p)
      if (sd.pc[p] == c && ++seen == pi) break;
    const float mn = fminf(fminf(acc[0][i][0], acc[1][i][0]), fminf(acc[2][i][0], acc[3][i][0]));
    const float mx = fmaxf(fmaxf(acc[0][i][1], acc[1][i][1]), fmaxf(acc[2][i][1], acc[3][i][1]));
    const float sm = (acc[0][i][2] + acc[1][i][2]) + (acc[2][i][2] + acc[3][i][2]);
    float* out = sd.cs_part + 3 * ((size_t)sd.cs_off[p] + (size_t)k * sd.ntiles_lvl[c] + J.tid);
    out[0] = mn;
    out[1] = mx;
    out[2] = sm;
  }
}

// ---------------------------------------------------------------- across-scale sum
// Computes N(F(c,s)) for every pair on the region of level c that the c_max tile
// needs, reduces it (blur + decimate with clamp) up to c_max, and sums it.
constexpr int CA_T = 16;                // c_max tile edge
constexpr int CA_R1 = 2 * CA_T + 3;     // 35: region one level finer
constexpr int CA_R2 = 2 * CA_R1 + 3;    // 73: region two levels finer

struct Range { int lo, n; };            // contiguous valid rows (or columns)

__device__ __forceinline__ Range finer_range(Range r, int n_finer) {
  const int lo = clampi(2 * r.lo - 2, 0, n_finer - 1);
  const int hi = clampi(2 * (r.lo + r.n - 1) + 2, 0, n_finer - 1);
  return Range{lo, hi - lo + 1};
}

// out (rows ro x cols co of the coarse level) = decimated blur of in (rows ri x cols ci
// of the finer level of size nh x nw), indices clamped to the finer map.
__device__ void reduce_lds(const float* in, int ldi, Range ri, Range ci, float* tmp, int ldt,
                           float* out, int ldo, Range ro, Range co, int nh, int nw) {
  for (int i = threadIdx.x; i < ri.n * co.n; i += SP_BLOCK) {
    const int r = i / co.n, j = i - r * co.n;
    const int X = co.lo + j;
    float acc = 0.f;
#pragma unroll
    for (int t = -2; t <= 2; ++t) acc += binom(t) * in[r * ldi + clampi(2 * X + t, 0, nw - 1) - ci.lo];
    tmp[r * ldt + j] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ro.n * co.n; i += SP_BLOCK) {
    const int r = i / co.n, j = i - r * co.n;
    const int Y = ro.lo + r;
    float acc = 0.f;
#pragma unroll
    for (int t = -2; t <= 2; ++t) acc += binom(t) * tmp[(clampi(2 * Y + t, 0, nh - 1) - ri.lo) * ldt + j];
    out[r * ldo + j] = acc;
  }
  __syncthreads();
}

__global__ __launch_bounds__(SP_BLOCK) void k_csapply(const Job* __restrict__ jobs,
                                                      const StreamDesc* __restrict__ sds,
                                                      const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float R0[CA_R2 * CA_R2];
  __shared__ float Tm[CA_R2 * CA_R1];
  __shared__ float R1b[CA_R1 * CA_R1];
  __shared__ float fb[CA_T * CA_T];
  __shared__ float sh4[4];
  __shared__ double sh256[SP_BLOCK];
  __shared__ NParams np[SP_MAXP];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* ckpt = IOF(ckpt);
  const int k = J.a, cm = sd.c_max;
  const int Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  for (int p = 0; p < sd.n_pairs; ++p) {
    const int c = sd.pc[p];
    const int nt = sd.ntiles_lvl[c];
    const float* parts = sd.cs_part + 3 * ((size_t)sd.cs_off[p] + (size_t)k * nt);
    const NParams q = nparams_from_parts(parts, nt, nblocks8(sd.Hl[c], sd.Wl[c]), sd.flat_tol, sh4, sh256);
    if (threadIdx.x == 0) np[p] = q;
  }
  for (int i = threadIdx.x; i < CA_T * CA_T; i += SP_BLOCK) fb[i] = 0.f;
  __syncthreads();
  const Range tr{J.y0, J.th}, tc{J.x0, J.tw};
  for (int p = 0; p < sd.n_pairs; ++p) {
    const NParams q = np[p];
    if (q.flat) continue;
    const int c = sd.pc[p], s = sd.ps[p], d = s - c, r = cm - c;
    const int Hc = sd.Hl[c], Wc = sd.Wl[c], Hs = sd.Hl[s], Ws = sd.Wl[s];
    const float* Xc = chan_ptr(sd, ckpt, k, c);
    const float* Xs = chan_ptr(sd, ckpt, k, s);
    if (r == 0) {
      for (int i = threadIdx.x; i < J.th * J.tw; i += SP_BLOCK) {
        const int yy = i / J.tw, xx = i - yy * J.tw;
        const int y = J.y0 + yy, x = J.x0 + xx;
        if (y < Hm && x < Wm) {
          const Tap ty = bilinear_tap(y, d, Hs), tx = bilinear_tap(x, d, Ws);
          const float F = fabsf(Xc[(size_t)y * Wc + x] - bilinear(Xs, Ws, ty, tx));
          fb[yy * CA_T + xx] += napply(q, F);
        }
      }
      __syncthreads();
      continue;
    }
    // region ranges, finest first
    Range rr1 = finer_range(tr, sd.Hl[cm - 1]), cr1 = finer_range(tc, sd.Wl[cm - 1]);
    Range rr0 = rr1, cr0 = cr1;
    if (r == 2) {
      rr0 = finer_range(rr1, sd.Hl[cm - 2]);
      cr0 = finer_range(cr1, sd.Wl[cm - 2]);
    }
    const int ld0 = cr0.n;
    for (int i = threadIdx.x; i < rr0.n * cr0.n; i += SP_BLOCK) {
      const int yy = i / cr0.n, xx = i - yy * cr0.n;
      const int y = rr0.lo + yy, x = cr0.lo + xx;
      const Tap ty = bilinear_tap(y, d, Hs), tx = bilinear_tap(x, d, Ws);
      const float F = fabsf(Xc[(size_t)y * Wc + x] - bilinear(Xs, Ws, ty, tx));
      R0[yy * ld0 + xx] = napply(q, F);
    }
    __syncthreads();
    if (r == 1) {
      reduce_lds(R0, ld0, rr0, cr0, Tm, tc.n, R1b, CA_T, tr, tc, sd.Hl[cm - 1], sd.Wl[cm - 1]);
    } else {
      reduce_lds(R0, ld0, rr0, cr0, Tm, cr1.n, R1b, cr1.n, rr1, cr1, sd.Hl[cm - 2], sd.Wl[cm - 2]);
      reduce_lds(R1b, cr1.n, rr1, cr1, Tm, tc.n, R0, CA_T, tr, tc, sd.Hl[cm - 1], sd.Wl[cm - 1]);
    }
    const float* res = (r == 1) ? R1b : R0;
    for (int i = threadIdx.x; i < J.th * J.tw; i += SP_BLOCK) {
      const int yy = i / J.tw, xx = i - yy * J.tw;
      fb[yy * CA_T + xx] += res[yy * CA_T + xx];
    }
    __syncthreads();
  }
  // store F-bar and its partial statistics (8x8 blocks per wavefront)
  const int lane = lane_id(), w = wave_id();
  const int nbx = (J.tw + 7) >> 3, nby = (J.th + 7) >> 3, nbk = nbx * nby;
  float wmn = INFINITY, wmx = -INFINITY, wsum = 0.f;
  for (int bk = w; bk < nbk; bk += 4) {
    const int by = bk / nbx, bx = bk - by * nbx;
    const int yy = 8 * by + (lane >> 3), xx = 8 * bx + (lane & 7);
    const int y = J.y0 + yy, x = J.x0 + xx;
    const bool exists = (J.y0 + 8 * by < Hm) && (J.x0 + 8 * bx < Wm);
    const bool valid = y < Hm && x < Wm && yy < J.th && xx < J.tw;
    const float v = valid ? fb[yy * CA_T + xx] : 0.f;
    if (valid) sd.fbar[(size_t)k * Hm * Wm + (size_t)y * Wm + x] = v;
    const float bmn = wave_reduce<OpMin>(valid ? v : INFINITY);
    const float bmx = wave_reduce<OpMax>(valid ? v : -INFINITY);
    if (exists) {
      wmn = fminf(wmn, bmn);
      wmx = fmaxf(wmx, bmx);
      wsum += bmx;
    }
  }
  __shared__ float wacc[4][3];
  if (lane == 0) {
    wacc[w][0] = wmn;
    wacc[w][1] = wmx;
    wacc[w][2] = wsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float* out = sd.fbar_part + 3 * ((size_t)k * sd.n_cmax_tiles + J.tid);
    out[0] = fminf(fminf(wacc[0][0], wacc[1][0]), fminf(wacc[2][0], wacc[3][0]));
    out[1] = fmaxf(fmaxf(wacc[0][1], wacc[1][1]), fmaxf(wacc[2][1], wacc[3][1]));
    out[2] = (wacc[0][2] + wacc[1][2]) + (wacc[2][2] + wacc[3][2]);
  }
}

// ---------------------------------------------------------------- conspicuity and saliency
__device__ void consp_nparams(const StreamDesc& sd, NParams* np, float* sh4, double* sh256) {
  const int cm = sd.c_max;
  const int nb = nblocks8(sd.Hl[cm], sd.Wl[cm]);
  for (int k = 0; k < SP_NCH; ++k) {
    const NParams q = nparams_from_parts(sd.fbar_part + 3 * (size_t)k * sd.n_cmax_tiles, sd.n_cmax_tiles, nb,
                                         sd.flat_tol, sh4, sh256);
    if (threadIdx.x == 0) np[k] = q;
  }
  __syncthreads();
}

// Block max of S over the tile with the first row-major argmax -> partial slot.
__device__ void smax_partial(float v, int idx, bool valid, float* out, float* sh4, int* shi4) {
  const float m = block_reduce<OpMax>(valid ? v : -INFINITY, sh4);
  int cand = (valid && v == m) ? idx : 0x7fffffff;
  cand = wave_min_i(cand);
  if (lane_id() == 0) shi4[wave_id()] = cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = m;
    out[1] = __int_as_float(min(min(shi4[0], shi4[1]), min(shi4[2], shi4[3])));
  }
}

__global__ __launch_bounds__(SP_BLOCK) void k_consp(const Job* __restrict__ jobs,
                                                    const StreamDesc* __restrict__ sds,
                                                    const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float sh4[4];
  __shared__ int shi4[4];
  __shared__ double sh256[SP_BLOCK];
  __shared__ NParams np[SP_NCH];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  float* S_out = IOF(S_out);
  float* C_out = IOF(C_out);
  float* S_tape = IOF(S_tape);
  consp_nparams(sd, np, sh4, sh256);
  const int cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const size_t plane = (size_t)Hm * Wm;
  const int yy = threadIdx.x / CA_T, xx = threadIdx.x % CA_T;
  const int y = J.y0 + yy, x = J.x0 + xx;
  const bool valid = yy < J.th && xx < J.tw && y < Hm && x < Wm;
  float S = 0.f;
  const size_t o = (size_t)min(y, Hm - 1) * Wm + min(x, Wm - 1);
  for (int k = 0; k < SP_NCH; ++k) {
    const float Ck = napply(np[k], sd.fbar[k * plane + o]);
    if (valid && C_out) C_out[k * plane + o] = Ck;
    S += sd.w[k] * Ck;
  }
  if (valid) {
    S_out[o] = S;
    if (S_tape) S_tape[o] = S;
  }
  smax_partial(S, (int)o, valid, sd.s_part + 2 * (size_t)J.tid, sh4, shi4);
}

__global__ __launch_bounds__(SP_BLOCK) void k_smax(const Job* __restrict__ jobs,
                                                   const StreamDesc* __restrict__ sds,
                                                   const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float sh4[4];
  __shared__ int shi4[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* S_in = IOF(S_in);
  const int cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const int yy = threadIdx.x / CA_T, xx = threadIdx.x % CA_T;
  const int y = J.y0 + yy, x = J.x0 + xx;
  const bool valid = yy < J.th && xx < J.tw && y < Hm && x < Wm;
  const size_t o = (size_t)min(y, Hm - 1) * Wm + min(x, Wm - 1);
  smax_partial(S_in[o], (int)o, valid, sd.s_part + 2 * (size_t)J.tid, sh4, shi4);
}

// ---------------------------------------------------------------- Kalman prior update
// q = clamp(up(S / max S), eps, 1 - eps) (0.5 if S is flat), eps on the border ring;
// f = G * pi_{t-1} (or G * seg_{t-1}); pi_t = f + K_t (q - f); eps on the border ring.
constexpr int KT = 16;
__global__ __launch_bounds__(SP_BLOCK) void k_kalman(const Job* __restrict__ jobs,
                                                     const StreamDesc* __restrict__ sds,
                                                     const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float reg[KT + 4][KT + 4];
  __shared__ float hb[KT + 4][KT];
  __shared__ float sh4[4];
  __shared__ int shi4[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* S = IOF(S_in);
  const uint8_t* seg = IOF(seg_prev);
  const float* pprev = IOF(pi_prev);
  float* pnext = IOF(pi_next);
  float* pout = IOF(prior_out);
  float* ftape = IOF(f_tape);
  float* mstape = IOF(ms_tape);
  const float K = IOF(K);
  const int t = IOF(t);
  const int H = sd.H, W = sd.W, cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  float m;
  int xs;
  smax_from_parts(sd.s_part, sd.n_cmax_tiles, &m, &xs, sh4, shi4);
  const bool flat = !(m > sd.flat_tol);
  if (t > 0) {
    for (int i = threadIdx.x; i < (KT + 4) * (KT + 4); i += SP_BLOCK) {
      const int ry = i / (KT + 4), rx = i - ry * (KT + 4);
      const int y = clampi(J.y0 - 2 + ry, 0, H - 1), x = clampi(J.x0 - 2 + rx, 0, W - 1);
      const size_t o = (size_t)y * W + x;
      reg[ry][rx] = seg ? (float)seg[o] : pprev[o];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (KT + 4) * KT; i += SP_BLOCK) {
      const int r = i / KT, j = i - r * KT;
      hb[r][j] = kB0 * reg[r][j] + kB1 * reg[r][j + 1] + kB2 * reg[r][j + 2] + kB1 * reg[r][j + 3] + kB0 * reg[r][j + 4];
    }
    __syncthreads();
  }
  const int yy = threadIdx.x / KT, xx = threadIdx.x % KT;
  const int y = J.y0 + yy, x = J.x0 + xx;
  if (yy < J.th && xx < J.tw && y < H && x < W) {
    const bool ring = on_border(y, x, H, W, sd.border);
    float q = 0.5f;
    if (!flat) {
      const float u = observe_u(S, Hm, Wm, cm, m, y, x);
      q = fminf(fmaxf(u, sd.eps), 1.f - sd.eps);
    }
    if (ring) q = sd.eps;
    float pi = q;
    const size_t o = (size_t)y * W + x;
    if (t > 0) {
      const float f = kB0 * hb[yy][xx] + kB1 * hb[yy + 1][xx] + kB2 * hb[yy + 2][xx] + kB1 * hb[yy + 3][xx] +
                      kB0 * hb[yy + 4][xx];
      pi = f + K * (q - f);
      if (ftape) ftape[o] = f;
    }
    if (ring) pi = sd.eps;
    pnext[o] = pi;
    if (pout) pout[o] = pi;
  }
  if (mstape && J.tid == 0 && threadIdx.x == 0) {
    mstape[0] = m;
    mstape[1] = __int_as_float(xs);
  }
}

// ---------------------------------------------------------------- MRF capacities
__global__ __launch_bounds__(SP_BLOCK) void k_mrf(const Job* __restrict__ jobs,
                                                  const StreamDesc* __restrict__ sds,
                                                  const StepIO* __restrict__ ios, StepIO io0,
                                                  const float* __restrict__ prior) {
  __shared__ unsigned long long sh[SP_BLOCK];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const uint8_t* rgb = IOF(rgb);
  float* unary = IOF(unary);
  float* pairw = IOF(pairwise);
  float* beta_out = IOF(beta_out);
  const int H = sd.H, W = sd.W;
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < sd.n_rgb; i += SP_BLOCK) s += sd.rgb_d2_part[i];
  s = block_sum_u64(s, sh);
  const unsigned long long cnt = (unsigned long long)H * (W - 1) + (unsigned long long)(H - 1) * W +
                                 2ull * (unsigned long long)(H - 1) * (W - 1);
  const double mean = cnt ? (double)s / (double)cnt : 0.0;
  const float beta = (mean > 0.0) ? (float)(1.0 / (2.0 * mean)) : 0.f;
  const int yy = threadIdx.x / 16, xx = threadIdx.x % 16;
  const int y = J.y0 + yy, x = J.x0 + xx;
  if (yy < J.th && xx < J.tw && y < H && x < W) {
    const size_t o = (size_t)y * W + x, plane = (size_t)H * W;
    const float pi = prior[o];
    unary[o] = -log1pf(-fminf(pi, 1.f - sd.eps));
    unary[plane + o] = -logf(fmaxf(pi, sd.eps));
    const uint8_t* p = rgb + o * 3;
    const int r = p[0], g = p[1], b = p[2];
    const int dys[4] = {0, 1, 1, 1}, dxs[4] = {1, 0, 1, -1};
    const float dist[4] = {1.f, 1.f, 1.41421356237f, 1.41421356237f};
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
      const int y2 = y + dys[dd], x2 = x + dxs[dd];
      float wv = 0.f;
      if (y2 < H && x2 >= 0 && x2 < W) {
        const uint8_t* q = rgb + ((size_t)y2 * W + x2) * 3;
        const int dr = r - q[0], dg = g - q[1], db = b - q[2];
        const float d2 = (float)(dr * dr + dg * dg + db * db);
        wv = sd.potts + sd.lam * expf(-beta * d2) / dist[dd];
      }
      pairw[dd * plane + o] = wv;
    }
  }
  if (beta_out && J.tid == 0 && threadIdx.x == 0) beta_out[0] = beta;
}

// ---------------------------------------------------------------- adjoint
// 1-D weight of forward tap source yp on output y for the clamp-to-edge binomial:
// sum_i k_i [clamp(yp + i) == y].
__device__ __forceinline__ float tap_weight_T(int yp, int y, int n) {
  float w = 0.f;
#pragma unroll
  for (int i = -2; i <= 2; ++i) w += (clampi(yp + i, 0, n - 1) == y) ? binom(i) : 0.f;
  return w;
}

__global__ __launch_bounds__(SP_BLOCK) void k_bwd_nu(const Job* __restrict__ jobs,
                                                     const StreamDesc* __restrict__ sds,
                                                     const BwdIO* __restrict__ bios, BwdIO b0) {
  __shared__ float reg[KT + 4][KT + 4];
  __shared__ float hb[KT + 4][KT];
  __shared__ float sh4[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const BwdIO& B = bios ? bios[J.stream] : b0;
  const int H = sd.H, W = sd.W, cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const bool carry = (B.nu_next != nullptr) && (B.carry != 0.f);
  if (carry) {
    for (int i = threadIdx.x; i < (KT + 4) * (KT + 4); i += SP_BLOCK) {
      const int ry = i / (KT + 4), rx = i - ry * (KT + 4);
      const int y = J.y0 - 2 + ry, x = J.x0 - 2 + rx;
      reg[ry][rx] = (y >= 0 && y < H && x >= 0 && x < W) ? B.nu_next[(size_t)y * W + x] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (KT + 4) * KT; i += SP_BLOCK) {
      const int r = i / KT, j = i - r * KT;
      const int x = J.x0 + j;
      float acc = 0.f;
      if (x < W) {
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
          const int xp = x + dx;
          if (xp >= 0 && xp < W) acc += reg[r][j + 2 + dx] * tap_weight_T(xp, x, W);
        }
      }
      hb[r][j] = acc;
    }
    __syncthreads();
  }
  const float m = B.ms[0];
  const bool flat = !(m > sd.flat_tol);
  const int yy = threadIdx.x / KT, xx = threadIdx.x % KT;
  const int y = J.y0 + yy, x = J.x0 + xx;
  float contrib = 0.f;
  if (yy < J.th && xx < J.tw && y < H && x < W) {
    const size_t o = (size_t)y * W + x;
    float nu = B.grad[o];
    if (carry) {
      float acc = 0.f;
#pragma unroll
      for (int dy = -2; dy <= 2; ++dy) {
        const int yp = y + dy;
        if (yp >= 0 && yp < H) acc += hb[yy + 2 + dy][xx] * tap_weight_T(yp, y, H);
      }
      nu += B.carry * acc;
    }
    const bool ring = on_border(y, x, H, W, sd.border);
    const float nut = ring ? 0.f : nu;
    float q = 0.5f, gu = 0.f;
    if (!flat) {
      const float u = observe_u(B.S, Hm, Wm, cm, m, y, x);
      q = fminf(fmaxf(u, sd.eps), 1.f - sd.eps);
      if (u > sd.eps && u < 1.f - sd.eps && !ring) gu = B.K * nut;
    }
    if (ring) q = sd.eps;
    if (B.f) contrib = nut * (q - B.f[o]);
    B.nu_out[o] = nut;
    B.gu[o] = gu;
  }
  const float tot = block_reduce<OpSum>(contrib, sh4);
  if (threadIdx.x == 0) B.gk_part[J.tid] = tot;
}

// Transpose of the bilinear up-sample from c_max to level 0 (gather form).
__global__ __launch_bounds__(SP_BLOCK) void k_bwd_gs(const Job* __restrict__ jobs,
                                                     const StreamDesc* __restrict__ sds,
                                                     const BwdIO* __restrict__ bios, BwdIO b0) {
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const BwdIO& B = bios ? bios[J.stream] : b0;
  const int H = sd.H, W = sd.W, cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const int yy = threadIdx.x / CA_T, xx = threadIdx.x % CA_T;
  const int Y = J.y0 + yy, X = J.x0 + xx;
  if (!(yy < J.th && xx < J.tw && Y < Hm && X < Wm)) return;
  const int sc = 1 << cm;
  const int ylo = max(0, sc * (Y - 1) + 1), yhi = min(H - 1, sc * (Y + 1) - 1);
  const int xlo = max(0, sc * (X - 1) + 1), xhi = min(W - 1, sc * (X + 1) - 1);
  float acc = 0.f;
  for (int y = ylo; y <= yhi; ++y) {
    const Tap ty = bilinear_tap(y, cm, Hm);
    const float wy = (ty.i0 == Y ? 1.f - ty.w : 0.f) + (ty.i1 == Y ? ty.w : 0.f);
    if (wy == 0.f) continue;
    float row = 0.f;
    for (int x = xlo; x <= xhi; ++x) {
      const Tap tx = bilinear_tap(x, cm, Wm);
      const float wx = (tx.i0 == X ? 1.f - tx.w : 0.f) + (tx.i1 == X ? tx.w : 0.f);
      row += wx * B.gu[(size_t)y * W + x];
    }
    acc += wy * row;
  }
  B.gs[(size_t)Y * Wm + X] = acc;
}

// Recomputed conspicuity maps dotted with the adjoint g_s of each frame:
// partial sums of g_s * C_k per tile, and C_k at the frame's argmax.
__global__ __launch_bounds__(SP_BLOCK) void k_consp_dot(const Job* __restrict__ jobs,
                                                        const StreamDesc* __restrict__ sds,
                                                        const StepIO* __restrict__ ios, StepIO io0,
                                                        const float* __restrict__ gs_all,
                                                        const float* __restrict__ ms_all,
                                                        const int* __restrict__ frame_of,
                                                        float* __restrict__ dot_part, float* __restrict__ cx_out) {
  __shared__ float sh4[4];
  __shared__ double sh256[SP_BLOCK];
  __shared__ NParams np[SP_NCH];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  consp_nparams(sd, np, sh4, sh256);
  const int f = frame_of[J.stream];
  const int cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const size_t plane = (size_t)Hm * Wm;
  const int yy = threadIdx.x / CA_T, xx = threadIdx.x % CA_T;
  const int y = J.y0 + yy, x = J.x0 + xx;
  const bool valid = yy < J.th && xx < J.tw && y < Hm && x < Wm;
  const size_t o = (size_t)min(y, Hm - 1) * Wm + min(x, Wm - 1);
  const float g = valid ? gs_all[(size_t)f * plane + o] : 0.f;
  const int xs = __float_as_int(ms_all[2 * (size_t)f + 1]);
  for (int k = 0; k < SP_NCH; ++k) {
    const float Ck = napply(np[k], sd.fbar[k * plane + o]);
    const float tot = block_reduce<OpSum>(valid ? g * Ck : 0.f, sh4);
    if (threadIdx.x == 0) dot_part[((size_t)f * sd.n_cmax_tiles + J.tid) * SP_NCH + k] = tot;
    if (valid && (int)o == xs) cx_out[(size_t)f * SP_NCH + k] = Ck;
  }
}

// Reduction of the per-frame partials and the scalar FP64 sweep over the gains.
__global__ __launch_bounds__(SP_BLOCK) void k_bwd_final(int T, int n_lvl0_tiles, int n_cmax_tiles,
                                                        const float* __restrict__ gk_part,
                                                        const float* __restrict__ dot_part,
                                                        const float* __restrict__ cx,
                                                        const float* __restrict__ ms_all,
                                                        const double* __restrict__ Kd,
                                                        const double* __restrict__ Pd, double Q, double R,
                                                        const float* __restrict__ w, float flat_tol,
                                                        double* __restrict__ gK_scratch,
                                                        float* grad_w, float* grad_q, float* grad_r) {
  __shared__ double sh256[SP_BLOCK];
  __shared__ double gw[SP_NCH];
  if (threadIdx.x < SP_NCH) gw[threadIdx.x] = 0.0;
  __syncthreads();
  for (int t = 0; t < T; ++t) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n_lvl0_tiles; i += SP_BLOCK) s += (double)gk_part[(size_t)t * n_lvl0_tiles + i];
    s = block_sum_d(s, sh256);
    if (threadIdx.x == 0) gK_scratch[t] = s;
    double A[SP_NCH];
    for (int k = 0; k < SP_NCH; ++k) {
      double a = 0.0;
      for (int i = threadIdx.x; i < n_cmax_tiles; i += SP_BLOCK)
        a += (double)dot_part[((size_t)t * n_cmax_tiles + i) * SP_NCH + k];
      A[k] = block_sum_d(a, sh256);
    }
    const double m = (double)ms_all[2 * t];
    if (threadIdx.x == 0 && m > (double)flat_tol) {
      double Bs = 0.0;
      for (int k = 0; k < SP_NCH; ++k) Bs += (double)w[k] * A[k];
      for (int k = 0; k < SP_NCH; ++k) gw[k] += A[k] / m - (double)cx[(size_t)t * SP_NCH + k] * Bs / (m * m);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double gQ = 0.0, gR = 0.0, gP = 0.0;
    for (int t = T - 1; t >= 1; --t) {
      const double g = gK_scratch[t] + R * gP;
      gR += Kd[t] * gP;
      const double a = Pd[t - 1] + Q;
      const double den = (a + R) * (a + R);
      const double ga = g * R / den;
      gR -= g * a / den;
      gQ += ga;
      gP = ga;
    }
    gR += gP;
    *grad_q = (float)gQ;
    *grad_r = (float)gR;
    for (int k = 0; k < SP_NCH; ++k) grad_w[k] = (float)gw[k];
  }
}

// ---------------------------------------------------------------- masked MSE loss helper
__global__ __launch_bounds__(SP_BLOCK) void k_loss(const float* __restrict__ prior, const uint8_t* __restrict__ mask,
                                                   size_t n, float inv_n, float* __restrict__ grad,
                                                   float* __restrict__ part) {
  __shared__ float sh4[4];
  float acc = 0.f;
  const size_t stride = (size_t)gridDim.x * SP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += stride) {
    const float d = prior[i] - (float)mask[i];
    acc += d * d;
    if (grad) grad[i] = 2.f * d * inv_n;
  }
  acc = block_reduce<OpSum>(acc, sh4);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(SP_BLOCK) void k_loss_final(const float* __restrict__ part, int n, float inv_n,
                                                         float* loss) {
  __shared__ double sh256[SP_BLOCK];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) s += (double)part[i];
  s = block_sum_d(s, sh256);
  if (threadIdx.x == 0) *loss = (float)(s * (double)inv_n);
}

// ---------------------------------------------------------------- batched step bookkeeping
// Start of a step: every stream's inputs, Kalman gain (FP64) and prior buffers.
__global__ void k_batch_begin(int n, BatchState* __restrict__ st, const uint8_t* const* __restrict__ in_ptrs,
                              StepIO* __restrict__ ios, double Q, double R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  BatchState s = st[i];
  double K, P;
  if (s.t == 0) {
    K = 1.0;
    P = R;
  } else {
    const double a = s.P + Q;
    K = a / (a + R);
    P = R * K;
  }
  StepIO io;
  memset(&io, 0, sizeof io);
  io.rgb = in_ptrs[i];
  io.rgb_prev = (s.t == 0) ? nullptr : s.last_rgb;
  io.S_out = s.S;
  io.S_in = s.S;
  io.pi_prev = s.pi[s.cur];
  io.pi_next = s.pi[s.cur ^ 1];
  io.K = (float)K;
  io.t = (int32_t)(s.t < 0x7fffffff ? s.t : 0x7fffffff);
  ios[i] = io;
  s.t += 1;
  s.P = P;
  s.cur ^= 1;
  s.last_rgb = io.rgb;
  st[i] = s;
}

__global__ void k_batch_reset(int n, BatchState* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  st[i].t = 0;
  st[i].P = 0.0;
  st[i].cur = 0;
  st[i].last_rgb = nullptr;
}

// Copies each stream's current prior to the caller's buffers (blockIdx.y = stream).
__global__ void k_batch_copy_out(const BatchState* __restrict__ st, const StreamDesc* __restrict__ sds,
                                 float* const* __restrict__ out) {
  const int s = blockIdx.y;
  const size_t n = (size_t)sds[s].H * sds[s].W;
  const float* src = st[s].pi[st[s].cur];
  float* dst = out[s];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------- launchers
static inline hipError_t chk() { return hipGetLastError(); }

hipError_t sp_launch(int kind, const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios,
                     const StepIO* io0, int flag, const float* aux, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 g(n), b(SP_BLOCK);
  StepIO z{};
  const StepIO& io = io0 ? *io0 : z;
  switch (kind) {
    case JOB_RGB: hipLaunchKernelGGL(k_rgb, g, b, 0, st, jobs, sds, ios, io, flag); break;
    case JOB_FEAT: hipLaunchKernelGGL((k_feat<16, 16>), g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_DOWN: hipLaunchKernelGGL((k_down<16, 16>), g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_GABOR: hipLaunchKernelGGL(k_gabor, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_CSSTATS: hipLaunchKernelGGL(k_csstats, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_CSAPPLY: hipLaunchKernelGGL(k_csapply, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_CONSP: hipLaunchKernelGGL(k_consp, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_SMAX: hipLaunchKernelGGL(k_smax, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_KALMAN: hipLaunchKernelGGL(k_kalman, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_MRF: hipLaunchKernelGGL(k_mrf, g, b, 0, st, jobs, sds, ios, io, aux); break;
    default: return hipErrorInvalidValue;
  }
  return chk();
}

hipError_t sp_launch_bwd(int kind, const Job* jobs, int n, const StreamDesc* sds, const BwdIO* bios,
                         const BwdIO* b0, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  BwdIO z{};
  const BwdIO& b = b0 ? *b0 : z;
  switch (kind) {
    case JOB_BWD_NU: hipLaunchKernelGGL(k_bwd_nu, dim3(n), dim3(SP_BLOCK), 0, st, jobs, sds, bios, b); break;
    case JOB_BWD_GS: hipLaunchKernelGGL(k_bwd_gs, dim3(n), dim3(SP_BLOCK), 0, st, jobs, sds, bios, b); break;
    default: return hipErrorInvalidValue;
  }
  return chk();
}

hipError_t sp_launch_consp_dot(const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios,
                               const float* gs_all, const float* ms_all, const int* frame_of,
                               float* dot_part, float* cx_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  StepIO z{};
  hipLaunchKernelGGL(k_consp_dot, dim3(n), dim3(SP_BLOCK), 0, st, jobs, sds, ios, z, gs_all, ms_all, frame_of,
                     dot_part, cx_out);
  return chk();
}

hipError_t sp_launch_bwd_final(int T, int n_lvl0_tiles, int n_cmax_tiles, const float* gk_part,
                               const float* dot_part, const float* cx, const float* ms_all, const double* Kd,
                               const double* Pd, double Q, double R, const float* w, float flat_tol,
                               double* gK_scratch, float* grad_w, float* grad_q, float* grad_r, hipStream_t st) {
  hipLaunchKernelGGL(k_bwd_final, dim3(1), dim3(SP_BLOCK), 0, st, T, n_lvl0_tiles, n_cmax_tiles, gk_part, dot_part,
                     cx, ms_all, Kd, Pd, Q, R, w, flat_tol, gK_scratch, grad_w, grad_q, grad_r);
  return chk();
}

hipError_t sp_launch_loss(const float* prior, const uint8_t* mask, size_t n, float* grad, float* part, int nblk,
                          float* loss, hipStream_t st) {
  const float inv_n = (float)(1.0 / (double)n);
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(SP_BLOCK), 0, st, prior, mask, n, inv_n, grad, part);
  hipError_t e = chk();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(SP_BLOCK), 0, st, part, nblk, inv_n, loss);
  return chk();
}

hipError_t sp_launch_batch_begin(int n, BatchState* st, const uint8_t* const* in_ptrs, StepIO* ios, double Q,
                                 double R, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_begin, dim3((n + 63) / 64), dim3(64), 0, stream, n, st, in_ptrs, ios, Q, R);
  return chk();
}

hipError_t sp_launch_batch_reset(int n, BatchState* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_reset, dim3((n + 63) / 64), dim3(64), 0, stream, n, st);
  return chk();
}

hipError_t sp_launch_batch_copy_out(int n, const BatchState* st, const StreamDesc* sds, float* const* out,
                                    hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_copy_out, dim3(64, n), dim3(SP_BLOCK), 0, stream, st, sds, out);
  return chk();
}
