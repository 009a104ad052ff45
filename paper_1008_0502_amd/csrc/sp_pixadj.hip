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

// dL/dS = gs / m - [x = x*] sum(gs S) / m^2 (one workgroup; zero when S was flat).
__global__ __launch_bounds__(SP_BLOCK) void k_pa_gs(const float* __restrict__ gs, const float* __restrict__ S,
                                                    const float* __restrict__ ms, int n, float flat_tol,
                                                    float* __restrict__ gS) {
  __shared__ double sh[SP_BLOCK];
  const float m = ms[0];
  const int xs = __float_as_int(ms[1]);
  const bool flat = !(m > flat_tol);
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) acc += (double)gs[i] * (double)S[i];
  const double dot = block_sum_d(acc, sh);
  const float corr = (float)(dot / ((double)m * (double)m));
  const float rm = 1.f / m;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK)
    gS[i] = flat ? 0.f : gs[i] * rm - (i == xs ? corr : 0.f);
}

// Tolerance (on the normalised map) within which values count as tied with an extreme.
constexpr float kTie = 0x1p-20f;

// Statistics of the N(.) adjoint of one map per workgroup.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_nstats(const PaMap* __restrict__ maps, float flat_tol) {
  __shared__ float smn[SP_BLOCK], smx[SP_BLOCK];
  __shared__ int imn[SP_BLOCK], imx[SP_BLOCK];
  __shared__ double sh[SP_BLOCK];
  const PaMap M = maps[blockIdx.x];
  const int n = M.h * M.w;
  float mn = INFINITY, mx = -INFINITY;
  int jn = 0x7fffffff, jx = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) {
    const float v = M.X[i];
    if (v < mn) mn = v, jn = i;
    if (v > mx) mx = v, jx = i;
  }
  smn[threadIdx.x] = mn;
  smx[threadIdx.x] = mx;
  imn[threadIdx.x] = jn;
  imx[threadIdx.x] = jx;
  __syncthreads();
  for (int s = SP_BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const int o = threadIdx.x + s;
      if (smn[o] < smn[threadIdx.x] || (smn[o] == smn[threadIdx.x] && imn[o] < imn[threadIdx.x]))
        smn[threadIdx.x] = smn[o], imn[threadIdx.x] = imn[o];
      if (smx[o] > smx[threadIdx.x] || (smx[o] == smx[threadIdx.x] && imx[o] < imx[threadIdx.x]))
        smx[threadIdx.x] = smx[o], imx[threadIdx.x] = imx[o];
    }
    __syncthreads();
  }
  mn = smn[0];
  mx = smx[0];
  const float rng = mx - mn;
  if (!(rng > flat_tol)) {
    if (threadIdx.x == 0) {
      for (int k = 0; k < SP_PA_SC; ++k) M.sc[k] = 0.f;
      M.sc[6] = 1.f;
    }
    return;
  }
  const float rr = 1.f / rng;
  // the extremes take their gradient at the first position within kTie of them (on
  // Y = (X - mn) / range): exact ties then resolve the same way whatever the rounding
  int jn2 = 0x7fffffff, jx2 = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) {
    const float y = (M.X[i] - mn) * rr;
    if (y <= kTie) jn2 = min(jn2, i);
    if (y >= 1.f - kTie) jx2 = min(jx2, i);
  }
  __syncthreads();
  imn[threadIdx.x] = jn2;
  imx[threadIdx.x] = jx2;
  __syncthreads();
  for (int s = SP_BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      imn[threadIdx.x] = min(imn[threadIdx.x], imn[threadIdx.x + s]);
      imx[threadIdx.x] = min(imx[threadIdx.x], imx[threadIdx.x + s]);
    }
    __syncthreads();
  }
  const int gimn = imn[0], gimx = imx[0];
  // block maxima of Y, each at the first position within kTie of it
  const int nbx = (M.w + 7) >> 3, nby = (M.h + 7) >> 3, nb = nbx * nby;
  double sb = 0.0;
  for (int j = threadIdx.x; j < nb; j += SP_BLOCK) {
    const int by = (j / nbx) * 8, bx = (j % nbx) * 8;
    float best = -INFINITY;
    for (int y = by; y < min(by + 8, M.h); ++y)
      for (int x = bx; x < min(bx + 8, M.w); ++x) best = fmaxf(best, (M.X[y * M.w + x] - mn) * rr);
    int bi = -1;
    for (int y = by; y < min(by + 8, M.h) && bi < 0; ++y)
      for (int x = bx; x < min(bx + 8, M.w); ++x)
        if ((M.X[y * M.w + x] - mn) * rr >= best - kTie) {
          bi = y * M.w + x;
          break;
        }
    M.bpos[j] = bi;
    sb += (double)best;
  }
  const double Sb = block_sum_d(sb, sh);
  double sgy = 0.0, sg = 0.0;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) {
    const double g = (double)M.g[i] * (double)M.gs;
    sgy += g * (double)((M.X[i] - mn) * rr);
    sg += g;
  }
  const double Sgy = block_sum_d(sgy, sh);
  const double Sg = block_sum_d(sg, sh);
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
  const float fy = fminf((float)y / (float)(1 << d), (float)(n - 1));
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
  const PaPlane P = tab[blockIdx.y];
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  float m = 0.f;
  if (i < P.ha * P.wa) {
    const int y = i / P.wa, x = i - y * P.wa;
    P.out[i] = fabsf(cs_diff(P, y, x));
    m = fabsf(P.a[i]);
    if (i < P.hb * P.wb) m = fmaxf(m, fabsf(P.b[i]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(P.amax, __float_as_uint(m));
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
  const float band = kSignBand * __uint_as_float(*P.amax);
  const float gd = D > band ? P.out[i] : (D < -band ? -P.out[i] : 0.f);
  P.out[i] = gd;
  gc[blockIdx.y][i] += gd;
}

// dL/dX(s) += up^T(-gD): the level-s element gathers every level-c element whose bilinear
// taps read it.  Plane entry: a = gD (level c, ha x wa), out = dL/dX(s) (hb x wb).
__global__ __launch_bounds__(SP_BLOCK) void k_pa_up_t(const PaPlane* __restrict__ tab) {
  const PaPlane P = tab[blockIdx.y];
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (i >= P.hb * P.wb) return;
  const int ys = i / P.wb, xs = i - ys * P.wb;
  const int st = 1 << P.d;
  float acc = 0.f;
  for (int y = max(0, (ys - 1) * st); y <= min(P.ha - 1, (ys + 1) * st); ++y) {
    int y0, y1;
    float wy;
    tap(y, P.d, P.hb, y0, y1, wy);
    const float ay = (y0 == ys ? 1.f - wy : 0.f) + (y1 == ys ? wy : 0.f);
    if (ay == 0.f) continue;
    float r = 0.f;
    for (int x = max(0, (xs - 1) * st); x <= min(P.wa - 1, (xs + 1) * st); ++x) {
      int x0, x1;
      float wx;
      tap(x, P.d, P.wb, x0, x1, wx);
      const float ax = (x0 == xs ? 1.f - wx : 0.f) + (x1 == xs ? wx : 0.f);
      r += ax * P.a[y * P.wa + x];
    }
    acc += ay * r;
  }
  P.out[i] -= acc;
}

// dL/dI(l) += sum over the four orientations of the clamped Gabor correlation's transpose:
// output (y, x) collects every tap (v, u) of every position (y', x') with
// clamp(y' + v) = y and clamp(x' + u) = x.  a: the four orientation gradients of the level
// at a plane stride of ha * wa; out: dL/dI(l); taps [4][2 SP_PA_R + 1][2 SP_PA_R + 1], the
// radius R = d centred in each.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_gabor_t(const PaPlane* __restrict__ tab, const float* __restrict__ taps) {
  const PaPlane P = tab[blockIdx.y];
  const int n = P.ha * P.wa;
  const int i = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int y = i / P.wa, x = i - y * P.wa;
  const int R = P.d;
  constexpr int K = 2 * SP_PA_R + 1;   // row stride of the tap table (radius up to SP_PA_R)
  float acc = 0.f;
  for (int v = -R; v <= R; ++v) {
    // rows y' with clamp(y' + v) = y
    const int ylo = y == 0 ? 0 : max(0, y - v), yhi = y == P.ha - 1 ? P.ha - 1 : min(P.ha - 1, y - v);
    if (ylo > yhi) continue;
    for (int u = -R; u <= R; ++u) {
      const int xlo = x == 0 ? 0 : max(0, x - u), xhi = x == P.wa - 1 ? P.wa - 1 : min(P.wa - 1, x - u);
      if (xlo > xhi) continue;
      float s4[4] = {0.f, 0.f, 0.f, 0.f};
      for (int yy = ylo; yy <= yhi; ++yy)
        for (int xx = xlo; xx <= xhi; ++xx) {
          const int o = yy * P.wa + xx;
#pragma unroll
          for (int th = 0; th < 4; ++th) s4[th] += P.a[(size_t)th * n + o];
        }
#pragma unroll
      for (int th = 0; th < 4; ++th) acc += taps[(th * K + (v + R)) * K + (u + R)] * s4[th];
    }
  }
  P.out[i] += acc;
}

// Level-0 features back to the frame: g_frame[t] = own part; g_frame[t-1] += motion part.
__global__ __launch_bounds__(SP_BLOCK) void k_pa_feat(const uint8_t* __restrict__ rgb, const uint8_t* __restrict__ prev,
                                                      const uint32_t* __restrict__ maxp, int nmax,
                                                      const float* __restrict__ g0, int n,
                                                      float* __restrict__ gout, float* __restrict__ gprev) {
  __shared__ uint32_t smax_sh;
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int k = 0; k < nmax; ++k) m = max(m, maxp[k]);
    smax_sh = m;
  }
  __syncthreads();
  const uint32_t smax = smax_sh;
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
                    hipStream_t st) {
  hipLaunchKernelGGL(k_pa_gs, dim3(1), dim3(SP_BLOCK), 0, st, gs, S, ms, n, flat_tol, gS);
  return hipGetLastError();
}
hipError_t sp_pa_nadjoint(const PaMap* maps, int nmaps, int maxn, float flat_tol, hipStream_t st) {
  if (nmaps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pa_nstats, dim3(nmaps), dim3(SP_BLOCK), 0, st, maps, flat_tol);
  hipLaunchKernelGGL(k_pa_napply, dim3(blocks(maxn), nmaps), dim3(SP_BLOCK), 0, st, maps);
  return hipGetLastError();
}
hipError_t sp_pa_plane(int kind, const PaPlane* tab, int nplanes, int maxn, int flag, float* const* gc,
                       const float* taps, hipStream_t st) {
  if (nplanes <= 0 || maxn <= 0) return hipSuccess;
  const dim3 g(blocks(maxn), nplanes);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_pa_reduce_t, g, dim3(SP_BLOCK), 0, st, tab, flag); break;
    case 1: hipLaunchKernelGGL(k_pa_csmap, g, dim3(SP_BLOCK), 0, st, tab); break;
    case 2: hipLaunchKernelGGL(k_pa_csadj, g, dim3(SP_BLOCK), 0, st, tab, gc); break;
    case 3: hipLaunchKernelGGL(k_pa_up_t, g, dim3(SP_BLOCK), 0, st, tab); break;
    case 4: hipLaunchKernelGGL(k_pa_gabor_t, g, dim3(SP_BLOCK), 0, st, tab, taps); break;
    default: return hipErrorInvalidValue;
  }
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
