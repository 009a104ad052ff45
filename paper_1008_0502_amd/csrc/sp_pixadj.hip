// Pixel-level adjoint of the saliency model (Section 3 / Section 7.2): dL/d frame_t from
// dL/dS_t, through the weighted sum, N(.), the across-scale sum, centre-surround, the Gabor
// maps, the pyramid and the level-0 features (the motion feature also reaches frame t-1).
// The forward maps of the frame are recomputed by the forward kernels first.  Every pass
// here gathers: one thread per output element, each output a fixed-order sum over the
// inputs that depend on it, so results do not depend on scheduling.  Non-differentiable
// points follow one convention: the global minimum and maximum and each 8x8 block maximum
// of an N(.) input take the gradient at the first position in row-major order whose
// normalised value lies within 2^-20 of the extreme (maps with a vanishing difference
// over whole regions hold exact ties there, which rounding must not decide), a map at
// or below flat_tol passes none, |.| has sign(0) = 0, max(0, .) passes nothing at 0 and
// min(r', g') passes to r' on ties; the chromatic mask and colour maximum are constants.
// The branches of the features are decided from the frame's bytes, where they are exact
// (2R - G - B > 0 for the red opponent, and so on), not from the rounded ratios R / I.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "sp_internal.h"
#include "sp_kernels.h"
#include "sp_device.h"

namespace {


__device__ __forceinline__ float kb(int i) {   // i in -2..2
  return i == 0 ? 0.375f : ((i == 1 || i == -1) ? 0.25f : 0.0625f);
}

// dL/dS = gs / m - [x = x*] sum(gs S) / m^2 (zero when S was flat), in two launches.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_gs(const float* __restrict__ gs, const float* __restrict__ S,
                                                    const float* __restrict__ ms, int n, float flat_tol,
                                                    float* __restrict__ gS, double* __restrict__ part) {
  // every workgroup: SP_BLOCK elements of gs / m and its FP64 partial of sum gs S; the
  // element at the argmax is left to k_pa_gs_fix
  __shared__ double sh[SP_BLOCK];
  const float m = ms[0];
  const int xs = __float_as_int(ms[1]);
  const bool flat = !(m > flat_tol);
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  const float g = i < n ? gs[i] : 0.f;
  const double dot = block_sum_d(i < n ? (double)g * (double)S[i] : 0.0, sh);
  if (i < n && i != xs) gS[i] = flat ? 0.f : g * (1.f / m);
  if (threadIdx.x == 0) part[blockIdx.x] = dot;
}

// The argmax element of gS: gs / m - (sum gs S) / m^2, the sum from the workgroups' partials
// in a fixed order.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_gs_fix(const float* __restrict__ gs, const float* __restrict__ ms,
                                                        int n, int nparts, float flat_tol, float* __restrict__ gS,
                                                        const double* __restrict__ part) {
  __shared__ double sh[SP_BLOCK];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nparts; k += SP_BLOCK) acc += part[k];
  const double dot = block_sum_d(acc, sh);
  const int xs = __float_as_int(ms[1]);
  if (threadIdx.x == 0 && xs >= 0 && xs < n) {   // an index outside the map was written by k_pa_gs
    const float m = ms[0];
    const float corr = (float)(dot / ((double)m * (double)m));
    gS[xs] = !(m > flat_tol) ? 0.f : gs[xs] * (1.f / m) - corr;
  }
}

// Tolerance (on the normalised map) within which values count as tied with an extreme.
constexpr float kTie = 0x1p-20f;

// Statistics of the N(.) adjoint, in three launches over all maps: (1) the (min, max) of
// tiles of SP_PA_MMT pixels; (2) per 8-row strip, with the map's range reduced from (1):
// each 8x8 block's maximum of Y = (X - mn) / range and its first position (row-major)
// within kTie of it, the strip's sums of the block maxima, g Y and g (FP64), and the first
// positions within kTie of the minimum and the maximum; (3) per map, the scalars below.

__device__ __forceinline__ int block_min_i(int v, int* sh4) {
  v = wave_min_i(v);
  __syncthreads();
  if (lane_id() == 0) sh4[wave_id()] = v;
  __syncthreads();
  return min(min(sh4[0], sh4[1]), min(sh4[2], sh4[3]));
}

// The map's (min, max) from its tile partials (every thread gets them).
__device__ __forceinline__ void map_range(const PaMap& M, float* sh4, float& mn, float& mx) {
  const int nt = (M.h * M.w + SP_PA_MMT - 1) / SP_PA_MMT;
  float a = INFINITY, b = -INFINITY;
  for (int k = threadIdx.x; k < nt; k += SP_BLOCK) {
    const float2 v = M.mm[k];
    a = fminf(a, v.x);
    b = fmaxf(b, v.y);
  }
  mn = block_reduce<OpMin>(a, sh4);
  mx = block_reduce<OpMax>(b, sh4);
}

__global__ __launch_bounds__(SP_BLOCK) void k_pa_nmm(const PaMap* __restrict__ maps) {
  __shared__ float sh4[4];
  const PaMap M = maps[blockIdx.y];
  const int n = M.h * M.w, base = blockIdx.x * SP_PA_MMT;
  if (base >= n) return;   // uniform
  float mn = INFINITY, mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < SP_PA_MMT / SP_BLOCK; ++k) {
    const int i = base + k * SP_BLOCK + threadIdx.x;
    const float v = M.X[min(i, n - 1)];
    mn = i < n ? fminf(mn, v) : mn;
    mx = i < n ? fmaxf(mx, v) : mx;
  }
  mn = block_reduce<OpMin>(mn, sh4);
  mx = block_reduce<OpMax>(mx, sh4);
  if (threadIdx.x == 0) M.mm[blockIdx.x] = make_float2(mn, mx);
}

__global__ __launch_bounds__(SP_BLOCK) void k_pa_nstrip(const PaMap* __restrict__ maps, float flat_tol) {
  __shared__ float sh4[4];
  __shared__ int shi[4];
  __shared__ double sh[SP_BLOCK];
  const PaMap M = maps[blockIdx.y];
  if ((int)blockIdx.x >= (M.h + 7) >> 3) return;   // uniform
  float mn, mx;
  map_range(M, sh4, mn, mx);
  const float rng = mx - mn;
  if (!(rng > flat_tol)) return;   // uniform: a flat map passes no gradient
  const float rr = 1.f / rng;
  const int y0 = blockIdx.x * 8, nrow = min(8, M.h - y0), nbx = (M.w + 7) >> 3;
  double sb = 0.0, sgy = 0.0, sg = 0.0;
  int jn = 0x7fffffff, jx = 0x7fffffff;
  // a thread takes column x of the strip; the eight columns of a block are eight
  // consecutive lanes (the chunks of SP_BLOCK columns start at multiples of 8)
  for (int x0 = 0; x0 < M.w; x0 += SP_BLOCK) {
    const int x = x0 + threadIdx.x;
    const bool cv = x < M.w;
    float Y[8], cb = -INFINITY;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const bool ok = cv && r < nrow;
      const int i = (y0 + min(r, nrow - 1)) * M.w + min(x, M.w - 1);
      const float v = (M.X[i] - mn) * rr;
      Y[r] = ok ? v : -INFINITY;
      cb = fmaxf(cb, Y[r]);
      if (ok) {
        const double g = (double)M.g[i] * (double)M.gs;
        sgy += g * (double)v;
        sg += g;
        if (v <= kTie) jn = min(jn, i);
        if (v >= 1.f - kTie) jx = min(jx, i);
      }
    }
    // the block's maximum and its first position within kTie (row-major: smallest index)
    float best = cb;
    best = fmaxf(best, __shfl_xor(best, 1));
    best = fmaxf(best, __shfl_xor(best, 2));
    best = fmaxf(best, __shfl_xor(best, 4));
    int cand = 0x7fffffff;
#pragma unroll
    for (int r = 7; r >= 0; --r)
      if (Y[r] >= best - kTie) cand = (y0 + r) * M.w + x;
    cand = min(cand, __shfl_xor(cand, 1));
    cand = min(cand, __shfl_xor(cand, 2));
    cand = min(cand, __shfl_xor(cand, 4));
    if ((threadIdx.x & 7) == 0 && cv) {
      M.bpos[(y0 >> 3) * nbx + (x >> 3)] = cand;
      sb += (double)best;
    }
  }
  sb = block_sum_d(sb, sh);
  sgy = block_sum_d(sgy, sh);
  sg = block_sum_d(sg, sh);
  jn = block_min_i(jn, shi);
  jx = block_min_i(jx, shi);
  if (threadIdx.x == 0) M.strip[blockIdx.x] = PaStrip{sb, sgy, sg, jn, jx};
}

__global__ __launch_bounds__(SP_BLOCK) void k_pa_nfin(const PaMap* __restrict__ maps, float flat_tol) {
  __shared__ float sh4[4];
  __shared__ int shi[4];
  __shared__ double sh[SP_BLOCK];
  const PaMap M = maps[blockIdx.x];
  float mn, mx;
  map_range(M, sh4, mn, mx);
  const float rng = mx - mn;
  if (!(rng > flat_tol)) {
    if (threadIdx.x == 0) {
      for (int k = 0; k < SP_PA_SC; ++k) M.sc[k] = 0.f;
      M.sc[6] = 1.f;
    }
    return;
  }
  const int ns = (M.h + 7) >> 3;
  double sb = 0.0, sgy = 0.0, sg = 0.0;
  int jn = 0x7fffffff, jx = 0x7fffffff;
  for (int k = threadIdx.x; k < ns; k += SP_BLOCK) {
    const PaStrip p = M.strip[k];
    sb += p.sb;
    sgy += p.sgy;
    sg += p.sg;
    jn = min(jn, p.jn);
    jx = min(jx, p.jx);
  }
  const double Sb = block_sum_d(sb, sh);
  const double Sgy = block_sum_d(sgy, sh);
  const double Sg = block_sum_d(sg, sh);
  const int gimn = block_min_i(jn, shi), gimx = block_min_i(jx, shi);
  const int nb = ((M.w + 7) >> 3) * ns;
  if (threadIdx.x == 0) {
    const double mbar = nb > 1 ? (Sb - 1.0) / (nb - 1) : 0.0;
    const double A = (1.0 - mbar) * (1.0 - mbar);
    const double gb = nb > 1 ? -2.0 * (1.0 - mbar) * Sgy / (nb - 1) : 0.0;
    const double sgyy = A * Sgy + gb * Sb;   // sum gY Y
    const double sgyt = A * Sg + gb * nb;    // sum gY
    M.sc[0] = (float)(A / rng);
    M.sc[1] = (float)(gb / rng);
    M.sc[2] = (float)((sgyy - sgyt) / rng);
    M.sc[3] = (float)(-sgyy / rng);
    M.sc[4] = __int_as_float(gimn);
    M.sc[5] = __int_as_float(gimx);
    M.sc[6] = 0.f;
    M.sc[7] = (float)nb;
  }
}

// dL/dX = gN A / range + [block maximum] gb / range + [argmin] g(min) + [argmax] g(max).
__global__ __launch_bounds__(SP_BLOCK) void k_pa_napply(const PaMap* __restrict__ maps) {
  const PaMap M = maps[blockIdx.y];
  const int n = M.h * M.w;
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (i >= n) return;
  if (M.sc[6] != 0.f) {
    M.out[i] = 0.f;
    return;
  }
  const int y = i / M.w, x = i - y * M.w;
  const int nbx = (M.w + 7) >> 3;
  float v = M.g[i] * M.gs * M.sc[0];
  if (M.bpos[(y >> 3) * nbx + (x >> 3)] == i) v += M.sc[1];
  if (i == __float_as_int(M.sc[4])) v += M.sc[2];
  if (i == __float_as_int(M.sc[5])) v += M.sc[3];
  M.out[i] = v;
}

// Weight of output position yo (of a clamped 5-tap blur over n positions) in the blur at yp.
__device__ __forceinline__ float blur_w(int yo, int yp, int n) {
  float a = 0.f;
#pragma unroll
  for (int i = -2; i <= 2; ++i) a += clampi(yp + i, 0, n - 1) == yo ? kb(i) : 0.f;
  return a;
}

// Transpose of one pyramid step: out (ha x wa, the finer level) +=/= sum over the coarser
// level b of g(y2, x2) a(y, 2 y2) a(x, 2 x2).  Plane table entry: a = coarse input, out.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_reduce_t(const PaPlane* __restrict__ tab, int accumulate) {
  const PaPlane P = tab[blockIdx.y];
  const int n = P.ha * P.wa;
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int y = i / P.wa, x = i - y * P.wa;
  float acc = 0.f;
  for (int y2 = max(0, (y - 1) >> 1); y2 <= min(P.hb - 1, (y + 2) >> 1); ++y2) {
    const float wy = blur_w(y, 2 * y2, P.ha);
    if (wy == 0.f) continue;
    float r = 0.f;
    for (int x2 = max(0, (x - 1) >> 1); x2 <= min(P.wb - 1, (x + 2) >> 1); ++x2)
      r += P.a[y2 * P.wb + x2] * blur_w(x, 2 * x2, P.wa);
    acc += wy * r;
  }
  P.out[i] = accumulate ? P.out[i] + acc : acc;
}

// Bilinear sample-aligned tap of target position y at level offset d on n source samples.
__device__ __forceinline__ void tap(int y, int d, int n, int& i0, int& i1, float& w) {
  const float fy = fminf((float)y * __int_as_float((127 - d) << 23), (float)(n - 1));   // y * 2^-d, exact
  i0 = (int)fy;
  i1 = min(i0 + 1, n - 1);
  w = fy - (float)i0;
}

__device__ __forceinline__ float cs_diff(const PaPlane& P, int y, int x) {
  int y0, y1, x0, x1;
  float wy, wx;
  tap(y, P.d, P.hb, y0, y1, wy);
  tap(x, P.d, P.wb, x0, x1, wx);
  const float* s = P.b;
  const float top = (1.f - wx) * s[y0 * P.wb + x0] + wx * s[y0 * P.wb + x1];
  const float bot = (1.f - wx) * s[y1 * P.wb + x0] + wx * s[y1 * P.wb + x1];
  return P.a[y * P.wa + x] - ((1.f - wy) * top + wy * bot);
}

// F = |X(c) - up X(s)| for one pair and channel per plane entry (a = X(c), b = X(s)), and
// the pair's scale max(max |X(c)|, max |X(s)|) by an atomic maximum on the float's bits
// (order-preserving for non-negative floats; the slot starts at zero).
__global__ __launch_bounds__(SP_BLOCK) void k_pa_csmap(const PaPlane* __restrict__ tab) {
  __shared__ float red[SP_BLOCK / 64];
  const PaPlane P = tab[blockIdx.y];
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  float m = 0.f;
  if (i < P.ha * P.wa) {
    const int y = i / P.wa, x = i - y * P.wa;
    P.out[i] = fabsf(cs_diff(P, y, x));
    m = fabsf(P.a[i]);
    if (i < P.hb * P.wb) m = fmaxf(m, fabsf(P.b[i]));
  }
  // the workgroup's maximum, then one atomic per workgroup
  m = wave_reduce<OpMax>(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = red[0];
    for (int k = 1; k < SP_BLOCK / 64; ++k) t = fmaxf(t, red[k]);
    atomicMax(P.amax + (blockIdx.x & (SP_PA_AMAX - 1)), __float_as_uint(t));
  }
}

// Derivative of |D| taken as 0 within this fraction of the pair's scale: there the sign of
// D is below what FP32 maps resolve (D vanishes identically on flat regions of both levels).
constexpr float kSignBand = 0x1p-16f;

// gD = sign(D) dL/dF outside the band (0 inside), in place in the plane of F (out), added
// to dL/dX(c) (gc).
__global__ __launch_bounds__(SP_BLOCK) void k_pa_csadj(const PaPlane* __restrict__ tab, float* const* __restrict__ gc) {
  const PaPlane P = tab[blockIdx.y];
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (i >= P.ha * P.wa) return;
  const int y = i / P.wa, x = i - y * P.wa;
  const float D = cs_diff(P, y, x);
  uint32_t am = 0;   // the pair's scale: the largest of its slots (all >= 0, compared as bits)
#pragma unroll
  for (int k = 0; k < SP_PA_AMAX; ++k) am = max(am, P.amax[k]);
  const float band = kSignBand * __uint_as_float(am);
  const float gd = D > band ? P.out[i] : (D < -band ? -P.out[i] : 0.f);
  P.out[i] = gd;
  gc[blockIdx.y][i] += gd;
}

// dL/dX(s) += up^T(-gD): the level-s element gathers every level-c element whose bilinear
// taps read it, a window of at most 2^(d+1) + 1 rows and columns.  Plane entry: a = gD
// (level c, ha x wa), out = dL/dX(s) (hb x wb).  Sixteen lanes (one DPP row) per level-s
// element: lane j takes the window's rows j, j + 16, ..., each as the tap-weighted sum of
// its columns, and the row adds the lanes' sums in a fixed order.
constexpr int UPT_L = 16;   // lanes per level-s element
__global__ __launch_bounds__(SP_BLOCK) void k_pa_up_t(const PaPlane* __restrict__ tab) {
  const PaPlane P = tab[blockIdx.y];
  const int e = blockIdx.x * (SP_BLOCK / UPT_L) + (int)(threadIdx.x / UPT_L);
  const int j = threadIdx.x & (UPT_L - 1);
  const bool valid = e < P.hb * P.wb;   // every lane stays for the row's sum
  const int i = valid ? e : 0;
  const int ys = i / P.wb, xs = i - ys * P.wb;
  const int st = 1 << P.d;
  const int x_lo = max(0, (xs - 1) * st), x_hi = min(P.wa - 1, (xs + 1) * st);
  float acc = 0.f;
  if (valid)
    for (int y = max(0, (ys - 1) * st) + j; y <= min(P.ha - 1, (ys + 1) * st); y += UPT_L) {
      int y0, y1;
      float wy;
      tap(y, P.d, P.hb, y0, y1, wy);
      const float ay = (y0 == ys ? 1.f - wy : 0.f) + (y1 == ys ? wy : 0.f);
      if (ay == 0.f) continue;
      float r = 0.f;
      for (int x = x_lo; x <= x_hi; ++x) {
        int x0, x1;
        float wx;
        tap(x, P.d, P.wb, x0, x1, wx);
        const float ax = (x0 == xs ? 1.f - wx : 0.f) + (x1 == xs ? wx : 0.f);
        r += ax * P.a[y * P.wa + x];
      }
      acc += ay * r;
    }
  // the sixteen lanes' sums: pairs, quads, halves, the row (every lane ends with the total)
  acc += dpp_f<0xB1>(acc);
  acc += dpp_f<0x4E>(acc);
  acc += dpp_f<0x141>(acc);
  acc += dpp_f<0x140>(acc);
  if (valid && j == 0) P.out[e] -= acc;
}

// dL/dI(l) += sum over the four orientations of the clamped Gabor correlation's transpose.
// With E(q) = sum_{v,u} h(v, u) gO(q - (v, u)) on the plane extended by the radius (gO zero
// outside the level), the transpose at p is the sum of E(q) over the q that clamp to p: q = p
// inside the level, the outside strip folded onto its border row or column.  One 16x16 tile
// of p per workgroup: the four orientation gradients of the tile plus twice the radius are
// staged in LDS (orientations interleaved), with the taps; E is computed once for each q the
// tile's outputs need (the tile, plus the outside strips of a tile on the border), then each
// output sums its fold set.  a: the four orientation gradients at a plane stride of ha * wa;
// out: dL/dI(l); taps [4][2 SP_PA_R + 1]^2, tap (v, u) of radius R = d at row v + R and
// column u + R of each.  RC: the radius when known at compile time (0: read from d).
constexpr int GT = 16;
constexpr int GN = GT + 4 * SP_PA_R;
constexpr int GQ = GT + 2 * SP_PA_R;
template <int RC>
__global__ __launch_bounds__(SP_BLOCK) void k_pa_gabor_t(PaGabLevels L, const float* __restrict__ taps) {
  __shared__ float4 go[GN * GN];
  __shared__ float4 tp[(2 * SP_PA_R + 1) * (2 * SP_PA_R + 1)];
  __shared__ float eq[GQ * GQ];
  const PaPlane P = *L.tab[blockIdx.y];   // the level of this workgroup (one launch for every level)
  const int h = P.ha, w = P.wa, R = RC ? RC : P.d, K = 2 * R + 1;
  const size_t n = (size_t)h * w;
  const int ntx = (w + GT - 1) / GT;
  if ((int)blockIdx.x >= ntx * ((h + GT - 1) / GT)) return;   // the level has fewer tiles
  const int ty0 = (blockIdx.x / ntx) * GT, tx0 = (blockIdx.x % ntx) * GT;
  const int E = GT + 4 * R, oy = ty0 - 2 * R, ox = tx0 - 2 * R;
  for (int i = threadIdx.x; i < E * E; i += SP_BLOCK) {
    const int r = i / E, c = i - r * E, y = oy + r, x = ox + c;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (y >= 0 && y < h && x >= 0 && x < w) {
      const size_t o = (size_t)y * w + x;
      v = make_float4(P.a[o], P.a[n + o], P.a[2 * n + o], P.a[3 * n + o]);
    }
    go[r * GN + c] = v;
  }
  constexpr int KT = 2 * SP_PA_R + 1;   // row stride of the global tap table
  for (int i = threadIdx.x; i < K * K; i += SP_BLOCK) {
    const int v = i / K, u = i - v * K;
    const int o = v * KT + u;
    tp[i] = make_float4(taps[o], taps[KT * KT + o], taps[2 * KT * KT + o], taps[3 * KT * KT + o]);
  }
  __syncthreads();
  // the q the tile needs: its own positions, and the outside strips on the level's borders
  const int th = min(GT, h - ty0), tw = min(GT, w - tx0);
  const int qy0 = ty0 == 0 ? -R : ty0, qy1 = ty0 + th - 1 + (ty0 + th == h ? R : 0);
  const int qx0 = tx0 == 0 ? -R : tx0, qx1 = tx0 + tw - 1 + (tx0 + tw == w ? R : 0);
  const int nqx = qx1 - qx0 + 1, nq = (qy1 - qy0 + 1) * nqx;
  for (int i = threadIdx.x; i < nq; i += SP_BLOCK) {
    const int qy = qy0 + i / nqx, qx = qx0 + i % nqx;
    const float4* g0 = go + (qy + R - oy) * GN + (qx + R - ox);   // q - (v - R, u - R) at g0 - v GN - u
    float e = 0.f;
#pragma unroll
    for (int v = 0; v < (RC ? 2 * RC + 1 : 1); ++v) {
      if (!RC) break;
      const float4* gr = g0 - v * GN;
      const float4* tr = tp + v * K;
#pragma unroll
      for (int u = 0; u < 2 * RC + 1; ++u) {
        const float4 g = gr[-u], t = tr[u];
        e = fmaf(t.x, g.x, fmaf(t.y, g.y, fmaf(t.z, g.z, fmaf(t.w, g.w, e))));
      }
    }
    if (!RC) {
      for (int v = 0; v < K; ++v) {
        const float4* gr = g0 - v * GN;
        const float4* tr = tp + v * K;
        for (int u = 0; u < K; ++u) {
          const float4 g = gr[-u], t = tr[u];
          e = fmaf(t.x, g.x, fmaf(t.y, g.y, fmaf(t.z, g.z, fmaf(t.w, g.w, e))));
        }
      }
    }
    eq[(qy - qy0) * GQ + (qx - qx0)] = e;
  }
  __syncthreads();
  const int py = ty0 + (int)(threadIdx.x >> 4), px = tx0 + (int)(threadIdx.x & 15);
  if (py >= h || px >= w) return;
  const int fy0 = py == 0 ? -R : py, fy1 = py == h - 1 ? h - 1 + R : py;
  const int fx0 = px == 0 ? -R : px, fx1 = px == w - 1 ? w - 1 + R : px;
  float acc = 0.f;
  for (int qy = fy0; qy <= fy1; ++qy)
    for (int qx = fx0; qx <= fx1; ++qx) acc += eq[(qy - qy0) * GQ + (qx - qx0)];
  P.out[(size_t)py * w + px] += acc;
}

// Level-0 features back to the frame: g_frame[t] = own part; g_frame[t-1] += motion part.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_feat(const uint8_t* __restrict__ rgb, const uint8_t* __restrict__ prev,
                                                      const uint32_t* __restrict__ maxp, int nmax,
                                                      const float* __restrict__ g0, int n,
                                                      float* __restrict__ gout, float* __restrict__ gprev) {
  __shared__ float sh4[4];
  // the frame's colour maximum from the partials (integers below 2^24: exact as floats)
  uint32_t m = 0;
  for (int k = threadIdx.x; k < nmax; k += SP_BLOCK) m = max(m, maxp[k]);
  const uint32_t smax = (uint32_t)block_reduce<OpMax>((float)m, sh4);
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (i >= n) return;
  // channels of the level-0 block: I, RG, BY at planes 0-2, M at plane 7
  const float gI = g0[i], gRG = g0[(size_t)n + i], gBY = g0[2 * (size_t)n + i], gM = g0[7 * (size_t)n + i];
  const uint32_t R8 = rgb[3 * i], G8 = rgb[3 * i + 1], B8 = rgb[3 * i + 2];
  const float r = R8 * (1.f / 255.f), g = G8 * (1.f / 255.f), b = B8 * (1.f / 255.f);
  const float I = (r + g + b) / 3.f;
  const bool chrom = 10u * (R8 + G8 + B8) > smax;
  float gIt = gI;
  if (prev) {
    // the sign of I_t - I_{t-1}, exact from the byte sums
    const int dm = (int)(R8 + G8 + B8) - (int)(prev[3 * i] + prev[3 * i + 1] + prev[3 * i + 2]);
    const float sg = dm > 0 ? gM : (dm < 0 ? -gM : 0.f);
    gIt += sg;
    const float gp = -sg / 3.f / 255.f;
    gprev[3 * i] += gp;
    gprev[3 * i + 1] += gp;
    gprev[3 * i + 2] += gp;
  }
  float gr = 0.f, gg = 0.f, gb = 0.f;
  if (chrom) {
    const float ri = 1.f / I;
    // the branches of the opponent channels, exact from the bytes (r' = R / I with I > 0)
    const int r8 = (int)R8, g8 = (int)G8, b8 = (int)B8;
    const float guR = 2 * r8 - g8 - b8 > 0 ? gRG : 0.f, guG = 2 * g8 - r8 - b8 > 0 ? -gRG : 0.f;
    const float guB = 2 * b8 - r8 - g8 > 0 ? gBY : 0.f, guY = min(r8, g8) - b8 > 0 ? -gBY : 0.f;
    float grp = guR - 0.5f * guG - 0.5f * guB;
    float ggp = -0.5f * guR + guG - 0.5f * guB;
    const float gbp = -0.5f * guR - 0.5f * guG + guB - guY;
    if (r8 <= g8) grp += guY;
    else ggp += guY;
    gr = grp * ri;
    gg = ggp * ri;
    gb = gbp * ri;
    gIt -= (grp * r + ggp * g + gbp * b) * ri * ri;
  }
  gr += gIt / 3.f;
  gg += gIt / 3.f;
  gb += gIt / 3.f;
  gout[3 * i] = gr / 255.f;
  gout[3 * i + 1] = gg / 255.f;
  gout[3 * i + 2] = gb / 255.f;
}

__global__ void k_pa_zero(float* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * SP_BLOCK) p[i] = 0.f;
}

inline int blocks(long long n) { return (int)((n + SP_BLOCK - 1) / SP_BLOCK); }

}  // namespace

hipError_t sp_pa_gs(const float* gs, const float* S, const float* ms, int n, float flat_tol, float* gS,
                    double* part, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pa_gs, dim3(blocks(n)), dim3(SP_BLOCK), 0, st, gs, S, ms, n, flat_tol, gS, part);
  hipLaunchKernelGGL(k_pa_gs_fix, dim3(1), dim3(SP_BLOCK), 0, st, gs, ms, n, blocks(n), flat_tol, gS, part);
  return hipGetLastError();
}
hipError_t sp_pa_nadjoint(const PaMap* maps, int nmaps, int maxn, int maxh, float flat_tol, hipStream_t st) {
  if (nmaps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pa_nmm, dim3((maxn + SP_PA_MMT - 1) / SP_PA_MMT, nmaps), dim3(SP_BLOCK), 0, st, maps);
  hipLaunchKernelGGL(k_pa_nstrip, dim3((maxh + 7) / 8, nmaps), dim3(SP_BLOCK), 0, st, maps, flat_tol);
  hipLaunchKernelGGL(k_pa_nfin, dim3(nmaps), dim3(SP_BLOCK), 0, st, maps, flat_tol);
  hipLaunchKernelGGL(k_pa_napply, dim3(blocks(maxn), nmaps), dim3(SP_BLOCK), 0, st, maps);
  return hipGetLastError();
}
hipError_t sp_pa_plane(int kind, const PaPlane* tab, int nplanes, int maxn, int flag, float* const* gc,
                       const float* taps, hipStream_t st, int gabor_r) {
  if (nplanes <= 0 || maxn <= 0) return hipSuccess;
  const dim3 g(blocks(maxn), nplanes);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_pa_reduce_t, g, dim3(SP_BLOCK), 0, st, tab, flag); break;
    case 1: hipLaunchKernelGGL(k_pa_csmap, g, dim3(SP_BLOCK), 0, st, tab); break;
    case 2: hipLaunchKernelGGL(k_pa_csadj, g, dim3(SP_BLOCK), 0, st, tab, gc); break;
    case 3: hipLaunchKernelGGL(k_pa_up_t, dim3(blocks(maxn * UPT_L), nplanes), dim3(SP_BLOCK), 0, st, tab); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t sp_pa_gabor(const PaGabLevels& L, int max_tiles, const float* taps, hipStream_t st, int gabor_r) {
  if (L.n <= 0 || max_tiles <= 0) return hipSuccess;
  const dim3 grid(max_tiles, L.n);
  if (gabor_r == 6)
    hipLaunchKernelGGL(k_pa_gabor_t<6>, grid, dim3(SP_BLOCK), 0, st, L, taps);
  else
    hipLaunchKernelGGL(k_pa_gabor_t<0>, grid, dim3(SP_BLOCK), 0, st, L, taps);
  return hipGetLastError();
}
hipError_t sp_pa_feat(const uint8_t* rgb, const uint8_t* prev, const uint32_t* maxp, int nmax, const float* g0, int n,
                      float* gout, float* gprev, hipStream_t st) {
  hipLaunchKernelGGL(k_pa_feat, dim3(blocks(n)), dim3(SP_BLOCK), 0, st, rgb, prev, maxp, nmax, g0, n, gout, gprev);
  return hipGetLastError();
}
hipError_t sp_pa_zero(float* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pa_zero, dim3((int)std::min<size_t>((n + SP_BLOCK - 1) / SP_BLOCK, 4096)), dim3(SP_BLOCK), 0, st, p, n);
  return hipGetLastError();
}
