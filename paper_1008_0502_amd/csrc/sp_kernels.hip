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

#include <mutex>

#include "sp_internal.h"
#include "sp_kernels.h"
#include "sp_device.h"

namespace {

// ---------------------------------------------------------------- stream helpers
__device__ __forceinline__ const float* base_ptr(const StreamDesc& sd, const float* ckpt, int l) {
  return (l == sd.c_min && ckpt) ? ckpt : sd.base[l];
}

// Channel k (I, RG, BY, O0, O45, O90, O135, M) of level l.
__device__ __forceinline__ const float* chan_ptr(const StreamDesc& sd, const float* ckpt, int k, int l) {
  // selects rather than branches: every operand is a uniform scalar load
  const size_t plane = (size_t)sd.Hl[l] * sd.Wl[l];
  const float* b = sd.base[l];
  const float* g = sd.gab[l];
  b = (l == sd.c_min && ckpt) ? ckpt : b;
  const bool gabor = (unsigned)(k - 3) < 4u;
  const int idx = k < 3 ? k : (k == 7 ? 3 : k - 3);
  return (gabor ? g : b) + idx * plane;
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

template <class Ptr>
__device__ __forceinline__ float bilinear(Ptr X, int Ws, const Tap& ty, const Tap& tx) {
  const float a = X[(size_t)ty.i0 * Ws + tx.i0], b = X[(size_t)ty.i0 * Ws + tx.i1];
  const float c = X[(size_t)ty.i1 * Ws + tx.i0], e = X[(size_t)ty.i1 * Ws + tx.i1];
  const float top = (1.f - tx.w) * a + tx.w * b;
  const float bot = (1.f - tx.w) * c + tx.w * e;
  return (1.f - ty.w) * top + ty.w * bot;
}

// N(.) parameters of one map from its partial triples (min, max, sum of block maxima):
// N(X) = (X - mn) / (mx - mn) * (1 - mbar)^2 with mbar the mean block maximum of the
// rescaled map after removing one instance of the global maximum.
struct NParams { float mn, inv, scale; int flat; };

__device__ NParams make_nparams(float mn, float mx, double sb, int nb, float flat_tol) {
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

// One wavefront reduces the partials of two maps with the same partial count (no
// workgroup barrier); both maps' loads are in flight together.  Each lane visits its
// partials in increasing order and the wavefront reductions are fixed, so every result
// is reproducible bit for bit.
__device__ void nparams_wave2(const float* pa_, const float* pb_, int n, int nb, float flat_tol, NParams* qa,
                              NParams* qb) {
  const gp<const float> pa = G(pa_), pb = G(pb_);
  float mna = INFINITY, mxa = -INFINITY, mnb = INFINITY, mxb = -INFINITY;
  double sa = 0.0, sb = 0.0;
  int i = lane_id();
  for (; i + 64 < n; i += 128) {   // two partials per lane and map in flight
    float a[2][3], b[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        a[u][f] = pa[3 * (i + 64 * u) + f];
        b[u][f] = pb[3 * (i + 64 * u) + f];
      }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      mna = fminf(mna, a[u][0]);
      mxa = fmaxf(mxa, a[u][1]);
      sa += (double)a[u][2];
      mnb = fminf(mnb, b[u][0]);
      mxb = fmaxf(mxb, b[u][1]);
      sb += (double)b[u][2];
    }
  }
  if (i < n) {
    mna = fminf(mna, pa[3 * i]);
    mxa = fmaxf(mxa, pa[3 * i + 1]);
    sa += (double)pa[3 * i + 2];
    mnb = fminf(mnb, pb[3 * i]);
    mxb = fmaxf(mxb, pb[3 * i + 1]);
    sb += (double)pb[3 * i + 2];
  }
  mna = wave_reduce<OpMin>(mna);
  mnb = wave_reduce<OpMin>(mnb);
  mxa = wave_reduce<OpMax>(mxa);
  mxb = wave_reduce<OpMax>(mxb);
  sa = wave_sum_d(sa);
  sb = wave_sum_d(sb);
  *qa = make_nparams(mna, mxa, sa, nb, flat_tol);
  *qb = make_nparams(mnb, mxb, sb, nb, flat_tol);
}

__device__ __forceinline__ void store_np(gp<float> dst, const NParams& p) {
  dst[0] = p.mn;
  dst[1] = p.inv;
  dst[2] = p.scale;
  dst[3] = p.flat ? 1.f : 0.f;
}

__device__ __forceinline__ NParams load_np(gp<const float> src) {
  NParams p;
  p.mn = src[0];
  p.inv = src[1];
  p.scale = src[2];
  p.flat = src[3] != 0.f;
  return p;
}

__device__ __forceinline__ float napply(const NParams& p, float v) {
  return p.flat ? 0.f : ((v - p.mn) * p.inv) * p.scale;
}

__device__ __forceinline__ int nblocks8(int h, int w) { return ((h + 7) >> 3) * ((w + 7) >> 3); }

// Max of S with its first row-major index, from (max, index) partials.
__device__ void smax_from_parts(const float* parts_, int n, float* m_out, int* idx_out, float* sh4, int* shi4) {
  // one pass over the partials: each thread keeps its largest value and the smallest
  // index among its partials holding that value; the block's first argmax is then the
  // smallest index among the threads whose largest value is the block maximum
  const gp<const float> parts = G(parts_);
  float ml = -INFINITY;
  int il = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += SP_BLOCK) {
    const float v = parts[2 * i];
    const int id = __float_as_int(parts[2 * i + 1]);
    if (v > ml) {
      ml = v;
      il = id;
    } else if (v == ml) {
      il = min(il, id);
    }
  }
  const float m = block_reduce<OpMax>(ml, sh4);
  int idx = wave_min_i(ml == m ? il : 0x7fffffff);
  __syncthreads();
  if (lane_id() == 0) shi4[wave_id()] = idx;
  __syncthreads();
  *m_out = m;
  *idx_out = min(min(shi4[0], shi4[1]), min(shi4[2], shi4[3]));
}

// Observation before clamping: bilinear up-sample of S times 1 / m at level-0 pixel
// (y, x), rounded as the prior update rounds it.
__device__ __forceinline__ float observe_u(const float* S, int Hc, int Wc, int c, float m, int y, int x) {
  const Tap ty = bilinear_tap(y, c, Hc), tx = bilinear_tap(x, c, Wc);
  return bilinear(S, Wc, ty, tx) * (1.f / m);
}

__device__ __forceinline__ bool on_border(int y, int x, int H, int W, int b) {
  return y < b || y >= H - b || x < b || x >= W - b;
}

#define IOF(field) (ios ? ios[J.stream].field : io0.field)

// ---------------------------------------------------------------- colour statistics
// Colours packed as R | G << 8 | B << 16 are byte vectors with a zero fourth byte, so
// the byte dot product (v_dot4_u32_u8) gives sums and squared distances exactly in
// 32-bit integers: R + G + B = a . (1,1,1,0) and |a - b|^2 = a.a + b.b - 2 a.b.
__device__ __forceinline__ uint32_t rgb_sum(uint32_t a) { return __builtin_amdgcn_udot4(a, 0x010101u, 0u, false); }
__device__ __forceinline__ uint32_t rgb_d2i(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_udot4(a, a, 0u, false) + __builtin_amdgcn_udot4(b, b, 0u, false) -
         2u * __builtin_amdgcn_udot4(a, b, 0u, false);
}

// Largest R+G+B over a tile of th x tw pixels; with want_d2 also the sum of squared
// colour differences over the 8-neighbour pairs (E, S, SE, SW) whose first pixel is in
// the tile, so that every unordered pair of the frame is counted once.
//
// Tiles are at most 256 columns wide (starting at multiples of 4) and are split into
// four bands of rows, one per wavefront.  Lane l owns the four pixels x .. x+3,
// x = x0 + 4 l, and holds its band's rows and the row below in registers.  When rows
// start on 4-byte boundaries (width a multiple of 4, aligned frame), five aligned
// dwords of a row hold pixels x-1 .. x+4, so each row is read once with no LDS; other
// frames take a per-pixel byte path.

// Pixels x-1 .. x+4 of a row from five aligned dwords: d[1..3] hold the owned pixels
// x .. x+3 (pixel x starts dword d[1]), d[0] the dword before (pixel x-1 in its top three
// bytes), d[4] the dword after (pixel x+4 in its low three bytes).  Pixels are zeroed
// where the flags say they are outside the frame or the rows in use.
__device__ __forceinline__ void rgb_unpack6(const uint32_t (&d)[5], bool left, bool row, bool right,
                                            uint32_t (&p)[6]) {
  p[0] = left ? d[0] >> 8 : 0u;
  p[1] = row ? d[1] & 0xffffffu : 0u;
  p[2] = row ? __builtin_amdgcn_alignbyte(d[2], d[1], 3) & 0xffffffu : 0u;
  p[3] = row ? __builtin_amdgcn_alignbyte(d[3], d[2], 2) & 0xffffffu : 0u;
  p[4] = row ? d[3] >> 8 : 0u;
  p[5] = right ? d[4] & 0xffffffu : 0u;
}

__device__ __forceinline__ uint32_t rgb_at(gp<const uint8_t> rgb, size_t o) {
  return (uint32_t)rgb[3 * o] | ((uint32_t)rgb[3 * o + 1] << 8) | ((uint32_t)rgb[3 * o + 2] << 16);
}

__device__ void batch_begin_stream(int i, BatchState* __restrict__ st, const StreamDesc* __restrict__ sds,
                                   const uint8_t* const* __restrict__ in_ptrs, StepIO* __restrict__ ios, double Q,
                                   double R);

__global__ __launch_bounds__(SP_BLOCK) void k_rgb(const Job* __restrict__ jobs,
                                                  const StreamDesc* __restrict__ sds,
                                                  const StepIO* __restrict__ ios, StepIO io0, int want_d2,
                                                  BatchBegin bb) {
  __shared__ unsigned long long sh[4];
  __shared__ uint32_t shm[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  // a batched step: this launch also starts the step (the other launches read the step's
  // inputs after it completes); its own frames come from the caller's table
  if (bb.in_ptrs && blockIdx.x == 0)
    for (int i = threadIdx.x; i < bb.n; i += SP_BLOCK) batch_begin_stream(i, bb.st, sds, bb.in_ptrs, bb.ios, bb.Q, bb.R);
  const uint8_t* frame = bb.in_ptrs ? bb.in_ptrs[J.stream] : IOF(rgb);
  const gp<const uint8_t> rgb = G(frame);
  const int W = sd.W, H = sd.H;
  const int lane = lane_id(), w = wave_id();
  const int rows = (J.th + 3) >> 2;   // rows of each wavefront's band
  const int ya = J.y0 + w * rows, yb = min(ya + rows, J.y0 + J.th);
  uint32_t mx = 0, d2 = 0;
  const bool fast = (W & 3) == 0 && (reinterpret_cast<uintptr_t>(frame) & 3) == 0;
  if (fast) {
    const int x = J.x0 + 4 * lane;
    if (x < J.x0 + J.tw && ya < yb) {
      const bool left = x > 0, right = x + 4 < W;
      const gp<const uint32_t> fw = (gp<const uint32_t>)(rgb);
      const uint32_t wrow = 3u * (uint32_t)W / 4u;   // dwords per row
      // the band (at most SP_RGB_TR / 4 rows) and, for the pairs, the row below it: all
      // rows are loaded before any is used, so the band costs one memory round trip
      constexpr int RB = SP_RGB_TR / 4;
      const int nrow = yb - ya + ((want_d2 && yb < H) ? 1 : 0);
      uint32_t p[RB + 1][6];
      {
        // unconditional loads at clamped addresses (rows past the last one used read the
        // frame's last row, edge dwords read an owned dword), zeroed afterwards
        uint32_t d[RB + 1][5];
#pragma unroll
        for (int r = 0; r <= RB; ++r) {
          const uint32_t o = ((uint32_t)min(ya + r, H - 1) * wrow + 3u * (uint32_t)(x >> 2)) * 4u;
          const gp<const uint32_t> wr = at_bytes(fw, o);
          d[r][0] = *at_bytes(fw, left ? o - 4u : o);
          d[r][1] = wr[0];
          d[r][2] = wr[1];
          d[r][3] = wr[2];
          d[r][4] = *at_bytes(fw, right ? o + 12u : o + 8u);
        }
        // every loaded dword is used here, so no load is sunk into a later branch
#pragma unroll
        for (int r = 0; r <= RB; ++r)
#pragma unroll
          for (int k = 0; k < 5; ++k) asm volatile("" : "+v"(d[r][k]));
#pragma unroll
        for (int r = 0; r <= RB; ++r) rgb_unpack6(d[r], left && r < nrow, r < nrow, right && r < nrow, p[r]);
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (ya + r >= yb) break;   // uniform over the wavefront
        const uint32_t* a = p[r];
        const uint32_t* b = p[r + 1];   // zero when row ya + r + 1 is not used
        const bool s = want_d2 && ya + r + 1 < H;
#pragma unroll
        for (int k = 1; k <= 4; ++k) mx = max(mx, rgb_sum(a[k]));
        if (want_d2) {
          // squared distances of the owned pairs: E (a_k, a_k+1), S (a_k, b_k),
          // SE (a_k, b_k+1), SW (a_k, b_k-1) for k = 1..4; pairs leaving the frame are
          // dropped (their partner is a zero vector and masked out of the norm sum)
          uint32_t na[6], nb[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            na[k] = __builtin_amdgcn_udot4(a[k], a[k], 0u, false);
            nb[k] = __builtin_amdgcn_udot4(b[k], b[k], 0u, false);
          }
          uint32_t cross = 0u, nsum = 0u;
#pragma unroll
          for (int k = 1; k <= 4; ++k) {
            const bool e = k < 4 || right, sw = k > 1 || left;
            cross = __builtin_amdgcn_udot4(a[k], a[k + 1], cross, false);
            nsum += e ? na[k] + na[k + 1] : 0u;
            if (s) {
              cross = __builtin_amdgcn_udot4(a[k], b[k], cross, false);
              cross = __builtin_amdgcn_udot4(a[k], b[k + 1], cross, false);
              cross = __builtin_amdgcn_udot4(a[k], b[k - 1], cross, false);
              nsum += na[k] + nb[k];
              nsum += e ? na[k] + nb[k + 1] : 0u;
              nsum += sw ? na[k] + nb[k - 1] : 0u;
            }
          }
          d2 += nsum - 2u * cross;
        }
      }
    }
  } else {
    Walk2 wk(threadIdx.x, J.tw);
    for (int i = threadIdx.x; i < J.th * J.tw; i += SP_BLOCK, wk.next()) {
      const int y = J.y0 + wk.r, x = J.x0 + wk.c;
      const size_t o = (size_t)y * W + x;
      const uint32_t a = rgb_at(rgb, o);
      mx = max(mx, rgb_sum(a));
      if (want_d2) {
        if (x + 1 < W) d2 += rgb_d2i(a, rgb_at(rgb, o + 1));
        if (y + 1 < H) {
          d2 += rgb_d2i(a, rgb_at(rgb, o + W));
          if (x + 1 < W) d2 += rgb_d2i(a, rgb_at(rgb, o + W + 1));
          if (x > 0) d2 += rgb_d2i(a, rgb_at(rgb, o + W - 1));
        }
      }
    }
  }
  mx = wave_max_u(mx);
  if (lane_id() == 0) shm[wave_id()] = mx;
  const unsigned long long tot = want_d2 ? block_sum_u64((unsigned long long)d2, sh) : 0ull;
  __syncthreads();
  if (threadIdx.x == 0) {
    G(sd.rgb_max_part)[J.a] = max(max(shm[0], shm[1]), max(shm[2], shm[3]));
    if (want_d2) G(sd.rgb_d2_part)[J.a] = tot;
  }
}

// ---------------------------------------------------------------- pyramid
// Row pass of the blur + decimation of NCH channels of a RH x (2*TW+3) LDS region:
// Hb[c][r][j] = 5-tap binomial of F[c][r][2j-2+2 .. 2j+2+2].  A thread keeps one (r, j)
// and runs over the channels, whose offsets are compile-time constants.
template <int TW, int RH, int RW, int NCH>
__device__ __forceinline__ void down_rows(float (*F)[RH][RW], float (*Hb)[RH][TW]) {
  for (int i = threadIdx.x; i < RH * TW; i += SP_BLOCK) {
    const int r = i / TW, j = i - r * TW;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const float* row = &F[c][r][2 * j];
      Hb[c][r][j] = kB0 * row[0] + kB1 * row[1] + kB2 * row[2] + kB1 * row[3] + kB0 * row[4];
    }
  }
}

// beta from this thread's share of the squared-distance partials (the block sums them;
// integers, so the result does not depend on the order)
__device__ __forceinline__ float beta_from_share(const StreamDesc& sd, unsigned long long share,
                                                 unsigned long long* sh) {
  const unsigned long long s = block_sum_u64(share, sh);
  const int H = sd.H, W = sd.W;
  const unsigned long long cnt = (unsigned long long)H * (W - 1) + (unsigned long long)(H - 1) * W +
                                 2ull * (unsigned long long)(H - 1) * (W - 1);
  const double mean = cnt ? (double)s / (double)cnt : 0.0;
  return (mean > 0.0) ? (float)(1.0 / (2.0 * mean)) : 0.f;
}
__device__ __forceinline__ unsigned long long d2_share(const StreamDesc& sd) {
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < sd.n_rgb; i += SP_BLOCK) s += G((const unsigned long long*)sd.rgb_d2_part)[i];
  return s;
}
__device__ __forceinline__ float beta_from_parts(const StreamDesc& sd, unsigned long long* sh) {
  return beta_from_share(sd, d2_share(sd), sh);
}

// One contrast-sensitive capacity: Potts constant plus the colour term over the
// neighbour's distance (1 or sqrt 2).  lambda * exp(-beta d2) is the hardware base-2
// exponential of nb2 * d2 + log2(lambda), nb2 = -beta * log2(e) (lambda = 0 gives
// log2 = -inf and a zero term).  Shared by every kernel that writes capacities so the
// fused and the separate MRF calls agree bit for bit.
struct CapK {
  float nb2, l2lam, potts;
};
__device__ __forceinline__ CapK cap_consts(float beta, float lam, float potts) {
  return CapK{-beta * 1.44269504088896341f, __builtin_amdgcn_logf(lam), potts};
}
__device__ __forceinline__ float pair_cap(const CapK& k, float d2, bool diag) {
  const float w = __builtin_amdgcn_exp2f(fmaf(k.nb2, d2, k.l2lam));
  return diag ? fmaf(w, 0.70710678118654752f, k.potts) : k.potts + w;
}

// Unary capacities of a prior value pi (eps <= pi <= 1 - eps after the clamps):
// U0 = -ln(1 - pi) and U1 = -ln(pi), from the hardware base-2 logarithm.  For U0,
// u = 1 - pi is rounded; ln(u) * pi / (1 - u) corrects that rounding (Goldberg's
// log1p method), and U0 = pi exactly when u rounds to 1.
__device__ __forceinline__ float unary0(float pi) {
  const float u = 1.f - pi;
  const float v = -__builtin_amdgcn_logf(u) * 0.693147180559945309f * (pi * __builtin_amdgcn_rcpf(1.f - u));
  return u == 1.f ? pi : v;   // a select: v is NaN there and discarded
}
__device__ __forceinline__ float unary1(float pi) { return -__builtin_amdgcn_logf(pi) * 0.693147180559945309f; }

// Contrast-sensitive capacities of pixel (y, x) towards its E, S, SE, SW neighbours.
__device__ __forceinline__ void pairwise_at(const uint8_t* rgb, int H, int W, int y, int x, const CapK& ck,
                                            float* pairw, size_t plane) {
  const size_t o = (size_t)y * W + x;
  const uint8_t* p = rgb + o * 3;
  const int r = p[0], g = p[1], b = p[2];
  const int dys[4] = {0, 1, 1, 1}, dxs[4] = {1, 0, 1, -1};
#pragma unroll
  for (int dd = 0; dd < 4; ++dd) {
    const int y2 = y + dys[dd], x2 = x + dxs[dd];
    float wv = 0.f;
    if (y2 < H && x2 >= 0 && x2 < W) {
      const uint8_t* q = rgb + ((size_t)y2 * W + x2) * 3;
      const int dr = r - q[0], dg = g - q[1], db = b - q[2];
      const float d2 = (float)(dr * dr + dg * dg + db * db);
      wv = pair_cap(ck, d2, dd >= 2);
    }
    pairw[dd * plane + o] = wv;
  }
}

// Squared colour distance of two packed pixels as a float.
__device__ __forceinline__ float rgb_d2(uint32_t a, uint32_t b) { return (float)rgb_d2i(a, b); }

// The same from the pixels' squared norms (each computed once): na + nb - 2 a.b, exact in
// integers.
__device__ __forceinline__ uint32_t sqnorm(uint32_t a) { return __builtin_amdgcn_udot4(a, a, 0u, false); }
__device__ __forceinline__ float masked(float v, uint32_t m) { return __uint_as_float(__float_as_uint(v) & m); }
__device__ __forceinline__ float d2_norms(uint32_t a, uint32_t na, uint32_t b, uint32_t nb) {
  return (float)(na + nb - 2u * __builtin_amdgcn_udot4(a, b, 0u, false));
}

// Level-0 features of the region a level-1 tile needs, then one blur + decimation.
// With io.pairwise set it also writes the pairwise capacities of the tile's level-0
// pixels (rows 2*y0 .. 2*(y0+th)-1) from the same staged region: every E, S, SE, SW
// neighbour of those pixels lies inside it.  All region bytes are loaded into
// registers at once (no branch between the loads); the features then go through LDS
// in two halves of the tile (TH/2 output rows, TH+3 region rows each), which keeps the
// launch at 8 workgroups per CU.
template <int TH, int TW>
__global__ __launch_bounds__(SP_BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_feat(const Job* __restrict__ jobs,
                                                   const StreamDesc* __restrict__ sds,
                                                   const StepIO* __restrict__ ios, StepIO io0) {
  constexpr int RH = 2 * TH + 3, RW = 2 * TW + 3;   // region of the whole tile
  constexpr int HR = TH + 3;                        // region rows of one half
  constexpr int NP = (RH * RW + SP_BLOCK - 1) / SP_BLOCK;
  __shared__ float F[4][HR][RW];
  __shared__ float Hb[4][HR][TW];
  __shared__ uint32_t shm[4];
  __shared__ unsigned long long sh[4];
  static_assert(4 * HR * TW >= HR * RW, "packed colours fit in the row-blur buffer");
  uint32_t* Pk = reinterpret_cast<uint32_t*>(&Hb[0][0][0]);  // packed colours until the blur
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const uint8_t* __restrict__ rgb = IOF(rgb);
  const uint8_t* __restrict__ prev = IOF(rgb_prev);
  float* ckpt = IOF(ckpt);
  const gp<float> pairw = G(IOF(pairwise));
  const int H = sd.H, W = sd.W;
  const int Y0 = 2 * J.y0 - 2, X0 = 2 * J.x0 - 2;
  typedef const __attribute__((address_space(1))) uint8_t* gbytes;
  const gbytes grgb = (gbytes)rgb;
  const gbytes gprev = (gbytes)prev;
  uint32_t cv[NP], pv[NP];
  {
    // A pixel's three bytes come from one 4-byte load (global loads need no alignment):
    // at the pixel's own offset, or for the frame's last pixel at the offset one byte
    // lower, shifted down, so no load reads past the frame.  One-pixel frames take the
    // bytes one at a time.
    typedef const __attribute__((address_space(1))) uint32_t __attribute__((aligned(1))) * gu32u;
    const bool words = H * W >= 2;   // uniform
    const uint32_t last = 3u * (uint32_t)(H * W) - 4u;
    uint32_t o[NP];   // byte offsets: frames hold at most 2^28 pixels
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int i = min((int)threadIdx.x + u * SP_BLOCK, RH * RW - 1);
      const int ry = i / RW, rx = i - ry * RW;
      const int y = clampi(Y0 + ry, 0, H - 1), x = clampi(X0 + rx, 0, W - 1);
      o[u] = ((uint32_t)y * (uint32_t)W + (uint32_t)x) * 3u;
    }
    if (words) {
      uint32_t lo[NP];
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        lo[u] = min(o[u], last);
        cv[u] = *(gu32u)at_bytes(grgb, lo[u]);
      }
      if (prev) {
#pragma unroll
        for (int u = 0; u < NP; ++u) pv[u] = *(gu32u)at_bytes(gprev, lo[u]);
#pragma unroll
        for (int u = 0; u < NP; ++u) pv[u] = rgb_sum(pv[u] >> ((o[u] - lo[u]) * 8u));   // the sum ignores the top byte
      }
#pragma unroll
      for (int u = 0; u < NP; ++u) cv[u] = (cv[u] >> ((o[u] - lo[u]) * 8u)) & 0xffffffu;
    } else {
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const gbytes c = at_bytes(grgb, o[u]);
        cv[u] = (uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16);
        if (prev) {
          const gbytes q = at_bytes(gprev, o[u]);
          pv[u] = (uint32_t)q[0] + (uint32_t)q[1] + (uint32_t)q[2];
        }
      }
    }
  }
  // largest R+G+B of the frame, from the colour-statistics partials; the squared-distance
  // partials for beta are read in the same round trip
  uint32_t smax = 0;
  for (int i = threadIdx.x; i < sd.n_rgb; i += SP_BLOCK) smax = max(smax, G((const uint32_t*)sd.rgb_max_part)[i]);
  const unsigned long long d2s = pairw ? d2_share(sd) : 0ull;
  smax = wave_max_u(smax);
  if (lane_id() == 0) shm[wave_id()] = smax;
  __syncthreads();
  smax = max(max(shm[0], shm[1]), max(shm[2], shm[3]));
  float fI[NP], fRG[NP], fBY[NP], fM[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int R8 = (int)(cv[u] & 0xff), G8 = (int)((cv[u] >> 8) & 0xff), B8 = (int)(cv[u] >> 16);
    const int S8 = (int)rgb_sum(cv[u]);
    const float I = (float)S8 * (1.f / 765.f);
    float rg = 0.f, by = 0.f;
    if (__umul24((uint32_t)S8, 10u) > smax) {   // S8 <= 765: a 24-bit multiply is exact
      const float inv = 3.f * __builtin_amdgcn_rcpf((float)S8);
      const float rp = (float)R8 * inv, gp = (float)G8 * inv, bp = (float)B8 * inv;
      const float Rc = fmaxf(0.f, rp - (gp + bp) * 0.5f);
      const float Gc = fmaxf(0.f, gp - (rp + bp) * 0.5f);
      const float Bc = fmaxf(0.f, bp - (rp + gp) * 0.5f);
      const float Yc = fmaxf(0.f, fminf(rp, gp) - bp);
      rg = Rc - Gc;
      by = Bc - Yc;
    }
    fI[u] = I;
    fRG[u] = rg;
    fBY[u] = by;
    // |I_t - I_{t-1}| from the byte sums: exactly zero where they agree (an FMA-contracted
    // difference of the two rounded intensities would leave the rounding error of I)
    fM[u] = prev ? (float)abs(S8 - (int)pv[u]) * (1.f / 765.f) : 0.f;
  }
  float beta = 0.f;
  const int H1 = sd.Hl[1], W1 = sd.Wl[1];
  const gp<float> dst = G((sd.c_min == 1 && ckpt) ? ckpt : sd.base[1]);
  const size_t plane1 = (size_t)H1 * W1;
  for (int h = 0; h < 2; ++h) {
    if (h == 1 && J.th <= TH / 2) break;
    const int r0 = h * TH;   // first region row of this half
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int i = threadIdx.x + u * SP_BLOCK;
      const int ry = i / RW, rx = i - ry * RW;
      if (i < RH * RW && ry >= r0 && ry < r0 + HR) {
        const int r = ry - r0;
        F[0][r][rx] = fI[u];
        F[1][r][rx] = fRG[u];
        F[2][r][rx] = fBY[u];
        F[3][r][rx] = fM[u];
        if (pairw) Pk[r * RW + rx] = cv[u];
      }
    }
    if (pairw) {
      if (h == 0)
        beta = beta_from_share(sd, d2s, sh);   // synchronises the block before and after its reduction
      else
        __syncthreads();
      // level-0 rows of this half: 2*y0 + r0 .. +TH-1 (rows 2 .. TH+1 of the staged half),
      // columns 2*x0 .. +2*TW-1 (region columns 2 .. 2*TW+1).  A thread takes one column and
      // two consecutive rows: the pixel below its first is its second, and the first's south
      // neighbours are the second's west, own and east pixels, so eight packed colours and
      // their norms serve both.  The staged region holds every neighbour (clamped at the
      // frame edge), so all capacities are computed and the ones that leave the frame zeroed.
      static_assert(2 * TW == 32 && TH == 2 * (SP_BLOCK / 32), "one column and two rows per thread");
      const int ylo = 2 * J.y0 + r0, nrow = min(min(H, 2 * (J.y0 + J.th)), ylo + TH) - ylo;
      const int xlo = 2 * J.x0, cw = min(W, 2 * (J.x0 + J.tw)) - xlo;
      const int c = threadIdx.x & 31, rr = 2 * (threadIdx.x >> 5);
      if (c < cw && rr < nrow) {
        const uint32_t p4 = (uint32_t)H * (uint32_t)W * 4u;   // bytes of a plane: four fit in 2^32
        const CapK ck = cap_consts(beta, sd.lam, sd.potts);
        const int x = xlo + c, y = ylo + rr;
        const uint32_t* q = Pk + (rr + 2) * RW + c + 2;
        const uint32_t a0 = q[0], a1 = q[1];                         // row y: x, x+1
        const uint32_t b7 = q[RW - 1], b0 = q[RW], b1 = q[RW + 1];   // row y+1: x-1, x, x+1
        const uint32_t c7 = q[2 * RW - 1], c0 = q[2 * RW], c1 = q[2 * RW + 1];
        const uint32_t na0 = sqnorm(a0), nb0 = sqnorm(b0);
        // capacities that leave the frame are zeroed by masks (selects would become branches)
        const uint32_t me = x + 1 < W ? ~0u : 0u, mw = x > 0 ? ~0u : 0u;
        const uint32_t ms0 = y + 1 < H ? ~0u : 0u, ms1 = y + 2 < H ? ~0u : 0u;
        float v[8];
        v[0] = masked(pair_cap(ck, d2_norms(a0, na0, a1, sqnorm(a1)), false), me);
        v[1] = masked(pair_cap(ck, d2_norms(a0, na0, b0, nb0), false), ms0);
        v[2] = masked(pair_cap(ck, d2_norms(a0, na0, b1, sqnorm(b1)), true), ms0 & me);
        v[3] = masked(pair_cap(ck, d2_norms(a0, na0, b7, sqnorm(b7)), true), ms0 & mw);
        v[4] = masked(pair_cap(ck, d2_norms(b0, nb0, b1, sqnorm(b1)), false), me);
        v[5] = masked(pair_cap(ck, d2_norms(b0, nb0, c0, sqnorm(c0)), false), ms1);
        v[6] = masked(pair_cap(ck, d2_norms(b0, nb0, c1, sqnorm(c1)), true), ms1 & me);
        v[7] = masked(pair_cap(ck, d2_norms(b0, nb0, c7, sqnorm(c7)), true), ms1 & mw);
        const uint32_t ob = ((uint32_t)y * (uint32_t)W + (uint32_t)x) * 4u;
#pragma unroll
        for (int k = 0; k < 4; ++k) st_stream(at_bytes(pairw, ob + (uint32_t)k * p4), v[k]);
        if (rr + 1 < nrow) {
#pragma unroll
          for (int k = 0; k < 4; ++k) st_stream(at_bytes(pairw, ob + (uint32_t)W * 4u + (uint32_t)k * p4), v[4 + k]);
        }
      }
      if (h == 0 && J.tid == 0 && threadIdx.x == 0 && IOF(beta_out)) G(IOF(beta_out))[0] = beta;
    }
    __syncthreads();
    down_rows<TW, HR, RW, 4>(F, Hb);
    __syncthreads();
    for (int i = threadIdx.x; i < (TH / 2) * TW; i += SP_BLOCK) {
      const int yr = i / TW, xx = i - yr * TW;
      const int yy = h * (TH / 2) + yr;
      const int y = J.y0 + yy, x = J.x0 + xx;
      if (yy < J.th && xx < J.tw && y < H1 && x < W1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float v = kB0 * Hb[c][2 * yr][xx] + kB1 * Hb[c][2 * yr + 1][xx] + kB2 * Hb[c][2 * yr + 2][xx] +
                          kB1 * Hb[c][2 * yr + 3][xx] + kB0 * Hb[c][2 * yr + 4][xx];
          dst[c * plane1 + (size_t)y * W1 + x] = v;
        }
      }
    }
    __syncthreads();
  }
}

// ---- jobs of the pyramid kernel (one of DOWN, GABOR, TAIL per workgroup)
constexpr int DT = 16, DR = 2 * DT + 3;                         // down tile and its source region
constexpr int DOWN_LDS = 4 * DR * DR;                           // floats (the row pass reuses it)
constexpr int GT = 16, GW = 32;                                 // Gabor tile: rows x columns
constexpr int GRM = GT + 2 * SP_MAXR, GCM = GW + 2 * SP_MAXR;    // its largest region
constexpr int GAB_LDS = GRM * GCM + 4 * GT * (GCM + 1) + 4 * (2 * SP_MAXR + 1);
constexpr int TAIL_LDS = SP_TAIL_SRC + SP_TAIL_ALT + SP_TAIL_HB + 4 * (2 * SP_MAXR + 1);
static_assert(DOWN_LDS >= GAB_LDS, "LDS of the small pyramid kernel");

__device__ __forceinline__ gp<float> level_dst(const StreamDesc& sd, float* ckpt, int l) {
  return G((l == sd.c_min && ckpt) ? ckpt : sd.base[l]);
}

// The four 1-D Gabor factors in LDS as [4][2*SP_MAXR+1], zero beyond the n = 2R+1
// taps: the tap loops below run over the full length, unrolled and without branches, so
// all their LDS reads issue together; a zero tap adds exactly nothing.
__device__ __forceinline__ void load_taps(const StreamDesc& sd, int n, float* taps) {
  constexpr int NT = 2 * SP_MAXR + 1;
  if ((int)threadIdx.x < 4 * NT) {
    const int f = threadIdx.x / NT, v = threadIdx.x - f * NT;
    taps[threadIdx.x] = (v < n) ? sd.gf[f][v] : 0.f;
  }
}

// level a -> a+1 of the 4 base channels for one 16x16 tile of level a+1
__device__ void down_job(const Job& J, const StreamDesc& sd, float* ckpt, float* smem) {
  float* F = smem;                 // [4][DR][DR]; then the row pass [4][DR][DT] in its place
  const int l = J.a;
  const int Hs = sd.Hl[l], Ws = sd.Wl[l];
  const float* src = base_ptr(sd, ckpt, l);
  const size_t splane = (size_t)Hs * Ws;
  const int Y0 = 2 * J.y0 - 2, X0 = 2 * J.x0 - 2;
  const int wf = wave_first();
  for (int i0 = 0; i0 + (int)threadIdx.x < DR * DR; i0 += SP_BLOCK) {
    const int i = i0 + threadIdx.x, ry = i / DR, rx = i - ry * DR;
    const uint32_t ob = ((uint32_t)clampi(Y0 + ry, 0, Hs - 1) * (uint32_t)Ws + (uint32_t)clampi(X0 + rx, 0, Ws - 1)) * 4u;
#pragma unroll
    for (int c = 0; c < 4; ++c) lds_load_u(F + c * DR * DR + i0 + wf, G(src + c * splane), ob);
  }
  lds_wait();
  __syncthreads();
  // row pass of every channel into registers, then (after one barrier) into the start of
  // that channel's own staged region, no longer read: the launch keeps 8 workgroups per CU
  constexpr int NH = (DR * DT + SP_BLOCK - 1) / SP_BLOCK;
  float hv[4][NH];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int i = threadIdx.x + k * SP_BLOCK;
      const int r = min(i / DT, DR - 1), j = i % DT;
      const float* row = F + (c * DR + r) * DR + 2 * j;
      hv[c][k] = kB0 * row[0] + kB1 * row[1] + kB2 * row[2] + kB1 * row[3] + kB0 * row[4];
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int i = threadIdx.x + k * SP_BLOCK;
      if (i < DR * DT) F[c * DR * DR + i] = hv[c][k];
    }
  __syncthreads();
  const float* Hb = F;   // channel c's row pass at c * DR * DR, [DR][DT]
  const int Hd = sd.Hl[l + 1], Wd = sd.Wl[l + 1];
  const gp<float> dst = level_dst(sd, ckpt, l + 1);
  const size_t plane = (size_t)Hd * Wd;
  const int yy = threadIdx.x / DT, xx = threadIdx.x % DT;
  const int y = J.y0 + yy, x = J.x0 + xx;
  if (yy < J.th && xx < J.tw && y < Hd && x < Wd) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float* col = Hb + c * DR * DR + 2 * yy * DT + xx;
      const float v = kB0 * col[0] + kB1 * col[DT] + kB2 * col[2 * DT] + kB1 * col[3 * DT] + kB0 * col[4 * DT];
      *at_bytes(dst + c * plane, ((uint32_t)y * (uint32_t)Wd + (uint32_t)x) * 4u) = v;
    }
  }
}

// 13x13 (radius R) zero-DC even Gabor kernels applied as separable rank-1 terms:
//   O0 = H[gm] V[g], O90 = H[g] V[gm],
//   O45 = H[gc] V[gc] - H[gs] V[gs] - c45 H[g] V[g], O135 = same with + H[gs] V[gs].
// RC > 0: built for radius RC (every extent and offset a compile-time constant); RC = 0:
// any radius, loops unrolled over the zero-padded maximum of taps.
template <int RC>
__device__ void gabor_job(const Job& J, const StreamDesc& sd, const float* ckpt, float* smem) {
  constexpr int NT = RC > 0 ? 2 * RC + 1 : 2 * SP_MAXR + 1;
  float* Ir = smem;                            // [RRr][RRc] (flat)
  float* V = Ir + GRM * GCM;                   // [4][GT][GCM+1]
  float* taps = V + 4 * GT * (GCM + 1);        // [4][2*SP_MAXR+1]
  const int l = J.a, R = RC > 0 ? RC : sd.gr, n = 2 * R + 1, RRr = GT + 2 * R, RRc = GW + 2 * R;
  const int Hs = sd.Hl[l], Ws = sd.Wl[l];
  const float* I = base_ptr(sd, ckpt, l);
  load_taps(sd, n, taps);
  const gp<const float> gI = G(I);
  const int wf = wave_first();
  Walk2 wk(threadIdx.x, RRc);
  for (int i0 = 0; i0 + (int)threadIdx.x < RRr * RRc; i0 += SP_BLOCK, wk.next()) {
    const int y = clampi(J.y0 - R + wk.r, 0, Hs - 1), x = clampi(J.x0 - R + wk.c, 0, Ws - 1);
    lds_load_u(Ir + i0 + wf, gI, ((uint32_t)y * (uint32_t)Ws + (uint32_t)x) * 4u);
  }
  lds_wait();
  __syncthreads();
  // tap v of factor f: for a compile-time radius a uniform value of the stream description
  // (scalar loads, hoisted out of the loops, used directly as multiply-add operands);
  // otherwise the zero-padded LDS table
  auto tap = [&](int f, int v) -> float {
    if constexpr (RC > 0)
      return sd.gf[f][v];
    else
      return taps[f * (2 * SP_MAXR + 1) + v];
  };
  // vertical pass: the four factors of one (row, column) from one read of its column
  Walk2 wk2(threadIdx.x, RRc);
#pragma unroll 1
  for (int i = threadIdx.x; i < GT * RRc; i += SP_BLOCK, wk2.next()) {
    const int yy = wk2.r, xr = wk2.c;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int v = 0; v < NT; ++v) {
      const float iv = Ir[(yy + (RC > 0 ? v : min(v, n - 1))) * RRc + xr];
      a0 += tap(0, v) * iv;
      a1 += tap(1, v) * iv;
      a2 += tap(2, v) * iv;
      a3 += tap(3, v) * iv;
    }
    V[(0 * GT + yy) * (GCM + 1) + xr] = a0;
    V[(1 * GT + yy) * (GCM + 1) + xr] = a1;
    V[(2 * GT + yy) * (GCM + 1) + xr] = a2;
    V[(3 * GT + yy) * (GCM + 1) + xr] = a3;
  }
  __syncthreads();
  const size_t plane = (size_t)Hs * Ws;
  const gp<float> Go = G(sd.gab[l]);
#pragma unroll 1
  for (int i = threadIdx.x; i < GT * GW; i += SP_BLOCK) {
    const int yy = i / GW, xx = i % GW;
    const int y = J.y0 + yy, x = J.x0 + xx;
    const float* V0 = V + (0 * GT + yy) * (GCM + 1) + xx;
    const float* V1 = V + (1 * GT + yy) * (GCM + 1) + xx;
    const float* V2 = V + (2 * GT + yy) * (GCM + 1) + xx;
    const float* V3 = V + (3 * GT + yy) * (GCM + 1) + xx;
    float A = 0.f, B = 0.f, C = 0.f, D = 0.f, E = 0.f;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int uc = RC > 0 ? u : min(u, n - 1);
      const float vg = V0[uc];
      A += tap(1, u) * vg;
      B += tap(0, u) * vg;
      C += tap(0, u) * V1[uc];
      D += tap(2, u) * V2[uc];
      E += tap(3, u) * V3[uc];
    }
    if (yy < J.th && xx < J.tw && y < Hs && x < Ws) {
      const uint32_t ob = ((uint32_t)y * (uint32_t)Ws + (uint32_t)x) * 4u;
      *at_bytes(Go, ob) = A;
      *at_bytes(Go + plane, ob) = D - E - sd.c45 * B;
      *at_bytes(Go + 2 * plane, ob) = C;
      *at_bytes(Go + 3 * plane, ob) = D + E - sd.c45 * B;
    }
  }
}

// Gabor maps of a whole (small) level held in LDS.
// Rows [y0, y0 + nr) only: the vertical pass of an output row reads the whole level (in
// LDS), so a band needs no halo of its own.
// SC: the taps are the NT = 2R + 1 leading values of the stream's factor table gf, read as
// uniform scalars; otherwise the zero-padded LDS table taps.
template <int NT, bool SC>
__device__ void gabor_lds(const float* I, int h, int w, int y0, int nr, float* V, const float* taps,
                          const float (*gf)[2 * SP_MAXR + 1], int R, float c45, gp<float> out) {
  auto tap = [&](int f, int v) -> float {
    if constexpr (SC)
      return gf[f][v];
    else
      return taps[f * (2 * SP_MAXR + 1) + v];
  };
  const int n = nr * w, plane = h * w;
  {
    Walk2 wk(threadIdx.x, w);
    for (int pix = threadIdx.x; pix < n; pix += SP_BLOCK, wk.next()) {
      const int y = y0 + wk.r, x = wk.c;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int v = 0; v < NT; ++v) {
        const float iv = I[clampi(y + v - R, 0, h - 1) * w + x];
        a0 += tap(0, v) * iv;
        a1 += tap(1, v) * iv;
        a2 += tap(2, v) * iv;
        a3 += tap(3, v) * iv;
      }
      V[pix] = a0;
      V[n + pix] = a1;
      V[2 * n + pix] = a2;
      V[3 * n + pix] = a3;
    }
  }
  __syncthreads();
  Walk2 wk(threadIdx.x, w);
  for (int pix = threadIdx.x; pix < n; pix += SP_BLOCK, wk.next()) {
    const int y = wk.r, x = wk.c;   // y relative to the band
    float A = 0.f, B = 0.f, C = 0.f, D = 0.f, E = 0.f;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int o = y * w + clampi(x + u - R, 0, w - 1);
      const float vg = V[o];
      A += tap(1, u) * vg;
      B += tap(0, u) * vg;
      C += tap(0, u) * V[n + o];
      D += tap(2, u) * V[2 * n + o];
      E += tap(3, u) * V[3 * n + o];
    }
    const int go = y0 * w + pix;
    out[go] = A;
    out[plane + go] = D - E - c45 * B;
    out[2 * plane + go] = C;
    out[3 * plane + go] = D + E - c45 * B;
  }
  __syncthreads();
}

// Levels above source level a of one base channel, computed in LDS.  TAIL jobs
// (channel tid) compute and store every level up to the top; TAILGAB jobs rebuild the
// intensity chain up to level tid and store that level's Gabor maps for the row band
// y0 .. y0+th-1, so the Gabor work of the small levels runs in parallel workgroups.
template <int RC>
__device__ void tail_job(const Job& J, const StreamDesc& sd, float* ckpt, float* smem) {
  float* SA = smem;
  float* SB = SA + SP_TAIL_SRC;
  float* HB = SB + SP_TAIL_ALT;
  float* taps = HB + SP_TAIL_HB;
  const bool gab = J.kind == JOB_TAILGAB;
  const int ch = gab ? 0 : J.tid, L0 = J.a, R = sd.gr, nt = 2 * R + 1;
  const int last = gab ? J.tid : sd.top;
  if (gab) load_taps(sd, nt, taps);
  int cH = sd.Hl[L0], cW = sd.Wl[L0];
  {
    const float* src = base_ptr(sd, ckpt, L0) + (size_t)ch * cH * cW;
    const int wf = wave_first();
    for (int i0 = 0; i0 + (int)threadIdx.x < cH * cW; i0 += SP_BLOCK)
      lds_load_u(SA + i0 + wf, G(src), (uint32_t)(i0 + threadIdx.x) * 4u);
    lds_wait();
  }
  float* cur = SA;
  float* nxt = SB;
  for (int l = L0; l < last; ++l) {
    const int nH = sd.Hl[l + 1], nW = sd.Wl[l + 1];
    __syncthreads();
    Walk2 wk(threadIdx.x, nW);
    for (int i = threadIdx.x; i < cH * nW; i += SP_BLOCK, wk.next()) {
      const int r = wk.r, j = wk.c;
      const float* row = cur + r * cW;
      float acc = 0.f;
#pragma unroll
      for (int t = -2; t <= 2; ++t) acc += binom(t) * row[clampi(2 * j + t, 0, cW - 1)];
      HB[i] = acc;
    }
    __syncthreads();
    const gp<float> dst = gab ? nullptr : level_dst(sd, ckpt, l + 1) + (size_t)ch * nH * nW;
    Walk2 wk2(threadIdx.x, nW);
    for (int i = threadIdx.x; i < nH * nW; i += SP_BLOCK, wk2.next()) {
      const int r = wk2.r, j = wk2.c;
      float acc = 0.f;
#pragma unroll
      for (int t = -2; t <= 2; ++t) acc += binom(t) * HB[clampi(2 * r + t, 0, cH - 1) * nW + j];
      nxt[i] = acc;
      if (dst) dst[i] = acc;
    }
    __syncthreads();
    if (gab && l + 1 == last)   // its vertical passes go to the buffer of level l, now free
      gabor_lds<(RC > 0 ? 2 * RC + 1 : 2 * SP_MAXR + 1), (RC > 0)>(nxt, nH, nW, J.y0, J.th, cur, taps, sd.gf, R,
                                                               sd.c45, G(sd.gab[l + 1]));
    float* tmp = cur;
    cur = nxt;
    nxt = tmp;
    cH = nH;
    cW = nW;
  }
}

// RC: the Gabor radius the launch is built for (every stream of a launch shares it), or
// 0 for any radius.  The default radius keeps 8 workgroups per CU.
template <bool BIG, int RC>
__global__ __launch_bounds__(SP_BLOCK) void k_pyr(
    const Job* __restrict__ jobs, const StreamDesc* __restrict__ sds, const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float smem[BIG ? TAIL_LDS : DOWN_LDS];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  float* ckpt = IOF(ckpt);
  if (J.kind == JOB_DOWN) {
    down_job(J, sd, ckpt, smem);
  } else if (J.kind == JOB_GABOR) {
    gabor_job<RC>(J, sd, ckpt, smem);
  } else if (BIG && (J.kind == JOB_TAIL || J.kind == JOB_TAILGAB)) {
    tail_job<RC>(J, sd, ckpt, smem);
  }
}

// ---------------------------------------------------------------- centre-surround statistics
// A 16x16 tile of the centre level c: the 8 centre maps and, per pair (c, s), the
// footprint of the tile on level s are staged in LDS; each wavefront then takes two
// channels, reduces every map's four 8x8 blocks (a 2x2 quad per lane, DPP within each
// 16-lane row) and writes the tile's (min, max, sum of block maxima).
constexpr int CS_T = 16;
constexpr int CS_F = CS_T / 2 + 2;      // footprint edge on a coarser level (offset >= 1)

struct Foot { int y0, x0, h, w; };      // footprint of rows/cols on the surround level

__device__ __forceinline__ Foot footprint(int y0, int ny, int x0, int nx, int d, int Hs, int Ws) {
  Foot f;
  f.y0 = min(y0 >> d, Hs - 1);
  f.x0 = min(x0 >> d, Ws - 1);
  f.h = min(((y0 + ny - 1) >> d) + 1, Hs - 1) - f.y0 + 1;
  f.w = min(((x0 + nx - 1) >> d) + 1, Ws - 1) - f.x0 + 1;
  return f;
}

// Bilinear sample of a staged footprint, with explicit FMAs: every kernel that forms a
// centre-surround map from LDS gives the same bits whatever the compiler contracts.
__device__ __forceinline__ float bilinear_lds(const float* X, int ld, const Tap& ty, const Tap& tx, int fy0, int fx0) {
  const float* r0 = X + (ty.i0 - fy0) * ld - fx0;
  const float* r1 = X + (ty.i1 - fy0) * ld - fx0;
  const float top = fmaf(tx.w, r0[tx.i1], (1.f - tx.w) * r0[tx.i0]);
  const float bot = fmaf(tx.w, r1[tx.i1], (1.f - tx.w) * r1[tx.i0]);
  return fmaf(ty.w, bot, (1.f - ty.w) * top);
}

__global__ __launch_bounds__(SP_BLOCK) void k_csstats(const Job* __restrict__ jobs,
                                                      const StreamDesc* __restrict__ sds,
                                                      const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float cen[SP_NCH][CS_T * CS_T];
  __shared__ float sur[4][SP_NCH][CS_F * CS_F];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* ckpt = IOF(ckpt);
  const int c = J.a, Hc = sd.Hl[c], Wc = sd.Wl[c];
  const int lane = lane_id(), w = wave_id();
  // stage the centre tile of all channels
  const float* cptr[SP_NCH];
#pragma unroll
  for (int k = 0; k < SP_NCH; ++k) cptr[k] = chan_ptr(sd, ckpt, k, c);
  for (int i = threadIdx.x; i < CS_T * CS_T; i += SP_BLOCK) {
    const int yy = i / CS_T, xx = i - yy * CS_T;
    const size_t o = (size_t)min(J.y0 + yy, Hc - 1) * Wc + min(J.x0 + xx, Wc - 1);
#pragma unroll
    for (int k = 0; k < SP_NCH; ++k) lds_load(&cen[k][i], cptr[k] + o);
  }
  // stage the surround footprints of the pairs of centre c (slot q in pair order; the
  // footprint geometry is scalar work, recomputed below instead of kept in LDS)
  int npc = 0;
  for (int p = 0; p < sd.n_pairs && npc < 4; ++p) {
    if (sd.pc[p] != c) continue;
    const int s = sd.ps[p], Ws = sd.Wl[s], q = npc++;
    const Foot f = footprint(J.y0, J.th, J.x0, J.tw, s - c, sd.Hl[s], Ws);
    // [k][CS_F][CS_F]: the destination follows the loop index; lanes outside the
    // footprint stay idle
    for (int i = threadIdx.x; i < SP_NCH * CS_F * CS_F; i += SP_BLOCK) {
      const int k = i / (CS_F * CS_F), r = i - k * (CS_F * CS_F), fy = r / CS_F, fx = r - fy * CS_F;
      if (fy < f.h && fx < f.w)
        lds_load(&sur[q][0][0] + i, chan_ptr(sd, ckpt, k, s) + (size_t)(f.y0 + fy) * Ws + f.x0 + fx);
    }
  }
  lds_wait();
  __syncthreads();
  // Wavefront w takes channels 2w and 2w+1 of every pair; its 64 lanes cover the tile as
  // four 16-lane rows, one 8x8 block per row and a 2x2 pixel quad per lane.  Pixels
  // beyond a ragged edge repeat the last valid row/column of their block (no effect on
  // min and max); blocks with no valid pixel are left out.
  const int blk = lane >> 4, by = blk >> 1, bx = blk & 1;
  const int qy = 8 * by + 2 * ((lane >> 2) & 3), qx = 8 * bx + 2 * (lane & 3);
  int yc[2], xc[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    yc[u] = J.y0 + min(qy + u, J.th - 1);
    xc[u] = J.x0 + min(qx + u, J.tw - 1);
  }
  bool bval[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) bval[i] = 8 * (i >> 1) < J.th && 8 * (i & 1) < J.tw;
  int q = -1;
  for (int p = 0; p < sd.n_pairs && q + 1 < npc; ++p) {
    if (sd.pc[p] != c) continue;
    ++q;
    const int s = sd.ps[p], d = s - c;
    const Foot f = footprint(J.y0, J.th, J.x0, J.tw, d, sd.Hl[s], sd.Wl[s]);
    Tap ty[2], tx[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ty[u] = bilinear_tap(yc[u], d, sd.Hl[s]);
      tx[u] = bilinear_tap(xc[u], d, sd.Wl[s]);
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int k = 2 * w + kk;
      float mn = INFINITY, mx = 0.f;   // F >= 0
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const float up = bilinear_lds(sur[q][k], CS_F, ty[u], tx[v], f.y0, f.x0);
          const float F = fabsf(cen[k][(yc[u] - J.y0) * CS_T + (xc[v] - J.x0)] - up);
          mn = fmin_nn(mn, F);
          mx = fmax_nn(mx, F);
        }
      // 8x8 block minimum and maximum: DPP within each 16-lane row
      row16_minmax_nn(mn, mx);
      float bmn[4], bmx[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // read unconditionally, then select: a readlane under the condition becomes a branch
        const float rmn = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mn), 16 * i));
        const float rmx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mx), 16 * i));
        bmn[i] = bval[i] ? rmn : INFINITY;
        bmx[i] = bval[i] ? rmx : -INFINITY;
      }
      if (lane == 0) {
        const gp<float> out = G(sd.cs_part) + 3 * ((size_t)sd.cs_off[p] + (size_t)k * sd.ntiles_lvl[c] + J.tid);
        out[0] = fminf(fminf(bmn[0], bmn[1]), fminf(bmn[2], bmn[3]));
        out[1] = fmaxf(fmaxf(bmx[0], bmx[1]), fmaxf(bmx[2], bmx[3]));
        out[2] = ((bval[0] ? bmx[0] : 0.f) + (bval[1] ? bmx[1] : 0.f)) + ((bval[2] ? bmx[2] : 0.f) + (bval[3] ? bmx[3] : 0.f));
      }
    }
  }
}

// N(.) parameters of the 8 maps of one pair (job a = pair), two maps per wavefront.
__global__ __launch_bounds__(SP_BLOCK) void k_csfinal(const Job* __restrict__ jobs,
                                                      const StreamDesc* __restrict__ sds,
                                                      const StepIO* __restrict__ ios, StepIO io0) {
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const int p = J.a, c = sd.pc[p], nt = sd.cs_nt[p], nb = nblocks8(sd.Hl[c], sd.Wl[c]);
  static_assert(SP_NCH == 8, "two maps per wavefront");
  const int k = wave_id();
  NParams qa, qb;
  nparams_wave2(sd.cs_part + 3 * ((size_t)sd.cs_off[p] + (size_t)k * nt),
                sd.cs_part + 3 * ((size_t)sd.cs_off[p] + (size_t)(k + 4) * nt), nt, nb, sd.flat_tol, &qa, &qb);
  if (lane_id() == 0) {
    store_np(G(sd.cs_np) + 4 * ((size_t)p * SP_NCH + k), qa);
    store_np(G(sd.cs_np) + 4 * ((size_t)p * SP_NCH + k + 4), qb);
  }
}

// ---------------------------------------------------------------- across-scale sum
// F-bar_k on a 16x16 tile of c_max = sum over pairs of REDUCE^(c_max - c)(N(F(c, s))).
// Every input is staged in (dynamically sized) LDS in one round trip; N(F) of all pairs
// that share a centre level are summed before that level is reduced (REDUCE is
// linear), and the sum from two levels down is folded into the level above it.
constexpr int CA_T = SP_CA_T;           // c_max tile edge

struct Range { int lo, n; };            // contiguous valid rows (or columns)

__device__ __forceinline__ Range finer_range(Range r, int n_finer) {
  const int lo = clampi(2 * r.lo - 2, 0, n_finer - 1);
  const int hi = clampi(2 * (r.lo + r.n - 1) + 2, 0, n_finer - 1);
  return Range{lo, hi - lo + 1};
}

// One pair of a centre level as the per-pixel loop needs it.  Its footprint sits at the
// same offset in the LDS block of every channel of the workgroup.
struct CaPair {
  int off, fy0, fx0, fw;   // staged footprint: LDS offset in a channel block, origin on level s, row length
  int d, Hs, Ws, fh;       // s - c and the size of level s; footprint rows
};

// NC consecutive channels (from job a) of one c_max tile per workgroup: the sampling
// geometry (bilinear taps, LDS offsets) is computed once per pixel and pair and applied
// to every channel.  Each channel owns a block of L.total floats of dynamic LDS with the
// layout of csapply_layout.  A flat map has zero N parameters (inv = scale = 0), which
// adds exactly 0.
template <int NC>
__global__ __launch_bounds__(SP_BLOCK) void k_csapply(const Job* __restrict__ jobs,
                                                      const StreamDesc* __restrict__ sds,
                                                      const StepIO* __restrict__ ios, StepIO io0) {
  extern __shared__ float dyn[];
  __shared__ CaPair cpt[3][4];
  __shared__ float cnp[3][4][NC][3];   // N parameters (mn, inv, scale) per level, pair and channel
  __shared__ int ncp[3];
  __shared__ float fb[NC][CA_T * CA_T];
  __shared__ float wacc[4][NC][3];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* ckpt = IOF(ckpt);
  const int k0 = J.a, cm = sd.c_max;
  const int Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const CaLayout L = csapply_layout(sd.pc, sd.ps, sd.n_pairs, cm);
  const int CS = L.total;   // floats per channel block
  unsigned hm = 0;
  for (int p = 0; p < sd.n_pairs; ++p) hm |= 1u << (cm - sd.pc[p]);
  const bool has0 = (hm & 1u) != 0, has1 = (hm & 2u) != 0, has2 = (hm & 4u) != 0;
  // regions of the tile on the centre levels (r = c_max - c)
  const Range rg0{J.y0, J.th}, cg0{J.x0, J.tw};
  Range rg1 = rg0, cg1 = cg0, rg2 = rg0, cg2 = cg0;
  if (has1 || has2) {
    rg1 = finer_range(rg0, sd.Hl[cm - 1]);
    cg1 = finer_range(cg0, sd.Wl[cm - 1]);
  }
  if (has2) {
    rg2 = finer_range(rg1, sd.Hl[cm - 2]);
    cg2 = finer_range(cg1, sd.Wl[cm - 2]);
  }
  // ---- one round trip: centre regions and every pair's footprint for each channel of
  // the group (the geometry is scalar work), then the pair table, whose N-parameter
  // loads queue behind the staging loads
  auto stage = [&](Range rr, Range cc, int c, int xoff) {
    const int Wc = sd.Wl[c];
    const int n = rr.n * cc.n;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const float* Xc = chan_ptr(sd, ckpt, k0 + j, c);
      float* X = dyn + j * CS + xoff;
      Walk2 wk(threadIdx.x, cc.n);
      for (int i = threadIdx.x; i < n; i += SP_BLOCK, wk.next())
        lds_load(X + i, Xc + (size_t)(rr.lo + wk.r) * Wc + cc.lo + wk.c);
    }
  };
  if (has0) stage(rg0, cg0, cm, L.x0);
  if (has1) stage(rg1, cg1, cm - 1, L.x1);
  if (has2) stage(rg2, cg2, cm - 2, L.x2);
  if (!has1 && has2)
    for (int j = 0; j < NC; ++j)
      for (int i = threadIdx.x; i < rg1.n * cg1.n; i += SP_BLOCK) dyn[j * CS + L.x1 + i] = 0.f;
  {
    int off = L.foot0;
    for (int p = 0; p < sd.n_pairs; ++p) {
      const int c = sd.pc[p], r = cm - c, s = sd.ps[p], Ws = sd.Wl[s];
      const Range rr = (r == 0) ? rg0 : ((r == 1) ? rg1 : rg2);
      const Range cc = (r == 0) ? cg0 : ((r == 1) ? cg1 : cg2);
      const Foot f = footprint(rr.lo, rr.n, cc.lo, cc.n, s - c, sd.Hl[s], Ws);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const float* Xs = chan_ptr(sd, ckpt, k0 + j, s);
        float* dst = dyn + j * CS + off;
        Walk2 wk(threadIdx.x, f.w);
        for (int i = threadIdx.x; i < f.h * f.w; i += SP_BLOCK, wk.next())
          lds_load(dst + i, Xs + (size_t)(f.y0 + wk.r) * Ws + f.x0 + wk.c);
      }
      off += csapply_foot_cap(r, s - c);
    }
  }
  // pair table: thread p fills pair p (its slot and LDS offset follow from the pairs
  // before it)
  if ((int)threadIdx.x < sd.n_pairs) {
    const int p = threadIdx.x;
    const int c = sd.pc[p], r = cm - c, s = sd.ps[p];
    int q = 0, off = L.foot0;
    for (int pp = 0; pp < p; ++pp) {
      q += (sd.pc[pp] == c) ? 1 : 0;
      off += csapply_foot_cap(cm - sd.pc[pp], sd.ps[pp] - sd.pc[pp]);
    }
    if (q < 4) {
      const Range rr = (r == 0) ? rg0 : ((r == 1) ? rg1 : rg2);
      const Range cc = (r == 0) ? cg0 : ((r == 1) ? cg1 : cg2);
      const Foot f = footprint(rr.lo, rr.n, cc.lo, cc.n, s - c, sd.Hl[s], sd.Wl[s]);
      CaPair& P = cpt[r][q];
      P.off = off;
      P.fy0 = f.y0;
      P.fx0 = f.x0;
      P.fw = f.w;
      P.fh = f.h;
      P.d = s - c;
      P.Hs = sd.Hl[s];
      P.Ws = sd.Wl[s];
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const NParams np = load_np(G((const float*)sd.cs_np) + 4 * ((size_t)p * SP_NCH + k0 + j));
        cnp[r][q][j][0] = np.mn;
        cnp[r][q][j][1] = np.flat ? 0.f : np.inv;
        cnp[r][q][j][2] = np.flat ? 0.f : np.scale;
      }
    }
  }
  if (threadIdx.x < 3) {
    int n = 0;
    for (int p = 0; p < sd.n_pairs; ++p) n += (cm - sd.pc[p] == (int)threadIdx.x) ? 1 : 0;
    ncp[threadIdx.x] = min(n, 4);
  }
  for (int i = threadIdx.x; i < NC * CA_T * CA_T; i += SP_BLOCK) (&fb[0][0])[i] = 0.f;
  lds_wait();
  __syncthreads();
  // ---- N(F) summed over the pairs of each centre level, in place of the centre values
  auto nsum = [&](int r, Range rr, Range cc, int xoff) {
    const int n = rr.n * cc.n, nq = ncp[r];
    Walk2 wk(threadIdx.x, cc.n);
    for (int i = threadIdx.x; i < n; i += SP_BLOCK, wk.next()) {
      const int y = rr.lo + wk.r, x = cc.lo + wk.c;
      float xc[NC], acc[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        xc[j] = dyn[j * CS + xoff + i];
        acc[j] = 0.f;
      }
      for (int q = 0; q < nq; ++q) {
        const CaPair& P = cpt[r][q];
        const Tap ty = bilinear_tap(y, P.d, P.Hs), tx = bilinear_tap(x, P.d, P.Ws);
        const int o0 = P.off + (ty.i0 - P.fy0) * P.fw - P.fx0, o1 = P.off + (ty.i1 - P.fy0) * P.fw - P.fx0;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const float* B = dyn + j * CS;
          // explicit fused multiply-adds: the result must not depend on NC through the
          // compiler's contraction choices
          const float top = fmaf(tx.w, B[o0 + tx.i1], (1.f - tx.w) * B[o0 + tx.i0]);
          const float bot = fmaf(tx.w, B[o1 + tx.i1], (1.f - tx.w) * B[o1 + tx.i0]);
          const float up = fmaf(ty.w, bot, (1.f - ty.w) * top);
          const float v = fabsf(xc[j] - up);
          acc[j] = fmaf((v - cnp[r][q][j][0]) * cnp[r][q][j][1], cnp[r][q][j][2], acc[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) dyn[j * CS + xoff + i] = acc[j];
    }
  };
  if (has0) nsum(0, rg0, cg0, L.x0);
  if (has1) nsum(1, rg1, cg1, L.x1);
  if (has2) nsum(2, rg2, cg2, L.x2);
  __syncthreads();
  // ---- reduce: two levels down -> one level down (added), one level down -> tile
  auto reduce = [&](int xin, int ldi, Range ri, Range ci, int xout_dyn, float* fbo, int ldo, Range ro, Range co,
                    int nh, int nw) {
    const int ldt = co.n;
    Walk2 wk(threadIdx.x, co.n);
    for (int i = threadIdx.x; i < ri.n * co.n; i += SP_BLOCK, wk.next()) {
      const int r = wk.r, X = co.lo + wk.c;
      int ix[5];
#pragma unroll
      for (int t = -2; t <= 2; ++t) ix[t + 2] = xin + r * ldi + clampi(2 * X + t, 0, nw - 1) - ci.lo;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const float* in = dyn + j * CS;
        float acc = 0.f;
#pragma unroll
        for (int t = -2; t <= 2; ++t) acc = fmaf(binom(t), in[ix[t + 2]], acc);
        dyn[j * CS + L.tm + r * ldt + wk.c] = acc;
      }
    }
    __syncthreads();
    Walk2 wk2(threadIdx.x, co.n);
    for (int i = threadIdx.x; i < ro.n * co.n; i += SP_BLOCK, wk2.next()) {
      const int r = wk2.r, c = wk2.c, Y = ro.lo + r;
      int iy[5];
#pragma unroll
      for (int t = -2; t <= 2; ++t) iy[t + 2] = L.tm + (clampi(2 * Y + t, 0, nh - 1) - ri.lo) * ldt + c;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const float* tm = dyn + j * CS;
        float acc = 0.f;
#pragma unroll
        for (int t = -2; t <= 2; ++t) acc = fmaf(binom(t), tm[iy[t + 2]], acc);
        float* out = fbo ? fbo + j * (CA_T * CA_T) : dyn + j * CS + xout_dyn;
        out[r * ldo + c] += acc;
      }
    }
    __syncthreads();
  };
  if (has2)
    reduce(L.x2, cg2.n, rg2, cg2, L.x1, nullptr, cg1.n, rg1, cg1, sd.Hl[cm - 2], sd.Wl[cm - 2]);
  if (has1 || has2)
    reduce(L.x1, cg1.n, rg1, cg1, 0, &fb[0][0], CA_T, rg0, cg0, sd.Hl[cm - 1], sd.Wl[cm - 1]);
  if (has0) {
    Walk2 wk(threadIdx.x, J.tw);
    for (int i = threadIdx.x; i < J.th * J.tw; i += SP_BLOCK, wk.next())
#pragma unroll
      for (int j = 0; j < NC; ++j) fb[j][wk.r * CA_T + wk.c] += dyn[j * CS + L.x0 + i];
    __syncthreads();
  }
  // ---- store F-bar and its partial statistics (one 8x8 block per wavefront)
  const int lane = lane_id(), w = wave_id();
  const int nbx = (J.tw + 7) >> 3, nby = (J.th + 7) >> 3;
  const bool act = w < nbx * nby;
  const int by = act ? w / nbx : 0, bx = act ? w - by * nbx : 0;
  const int yy = 8 * by + (lane >> 3), xx = 8 * bx + (lane & 7);
  const bool valid = act && yy < J.th && xx < J.tw;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    float wmn = INFINITY, wmx = -INFINITY;
    if (act) {
      const float v = valid ? fb[j][yy * CA_T + xx] : 0.f;
      if (valid) G(sd.fbar)[(size_t)(k0 + j) * Hm * Wm + (size_t)(J.y0 + yy) * Wm + J.x0 + xx] = v;
      wmn = wave_reduce<OpMin>(valid ? v : INFINITY);
      wmx = wave_reduce<OpMax>(valid ? v : -INFINITY);
    }
    if (lane == 0) {
      wacc[w][j][0] = wmn;
      wacc[w][j][1] = wmx;
      wacc[w][j][2] = act ? wmx : 0.f;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < NC) {
    const int j = threadIdx.x;
    const gp<float> out = G(sd.fbar_part) + 3 * ((size_t)(k0 + j) * sd.n_cmax_tiles + J.tid);
    out[0] = fminf(fminf(wacc[0][j][0], wacc[1][j][0]), fminf(wacc[2][j][0], wacc[3][j][0]));
    out[1] = fmaxf(fmaxf(wacc[0][j][1], wacc[1][j][1]), fmaxf(wacc[2][j][1], wacc[3][j][1]));
    out[2] = (wacc[0][j][2] + wacc[1][j][2]) + (wacc[2][j][2] + wacc[3][j][2]);
  }
}

// ---------------------------------------------------------------- reduced-map path
// N(.) is affine in F on every map and REDUCE is linear with weights summing to one, so
// REDUCE(N(F)) = N(REDUCE(F)).  When every pair has c_max - c <= 1 the
// centre-surround maps are computed once per c_max tile: their partial statistics are
// taken on the pixels the tile owns (the tile's footprint on level c), and their
// reduction to c_max (REDUCE once for c = c_max - 1, the map itself for c = c_max) is
// stored.  k_csmix then forms F-bar at c_max as the sum of N(reduced map) over pairs.
//
// One workgroup per c_max tile and group of NC channels (from job a).  Its dynamic LDS
// holds one staging block per channel and, after them, the channel-interleaved map and
// table of CgLayout: the compute loops read every channel of an element with one
// vector access.

// NC consecutive floats of LDS (one element of an interleaved buffer) in one access.
template <int NC>
__device__ __forceinline__ void lds_getv(const float* p, float (&v)[NC]) {
  if constexpr (NC == 1) {
    v[0] = p[0];
  } else if constexpr (NC == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
#pragma unroll
    for (int k = 0; k < NC; k += 4) {
      const float4 t = *reinterpret_cast<const float4*>(p + k);
      v[k] = t.x;
      v[k + 1] = t.y;
      v[k + 2] = t.z;
      v[k + 3] = t.w;
    }
  }
}
template <int NC>
__device__ __forceinline__ void lds_putv(float* p, const float (&v)[NC]) {
  if constexpr (NC == 1) {
    p[0] = v[0];
  } else if constexpr (NC == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  } else {
#pragma unroll
    for (int k = 0; k < NC; k += 4) *reinterpret_cast<float4*>(p + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
  }
}

// The pair loops carry an unroll request that only the compile-time pair set can meet.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
template <int NC, int SET>
__global__ __launch_bounds__(SP_BLOCK) void k_csg(const Job* __restrict__ jobs,
                                                  const StreamDesc* __restrict__ sds,
                                                  const StepIO* __restrict__ ios, StepIO io0) {
  extern __shared__ __align__(16) float dyn[];   // 16-byte transfers and vector reads land in it
  __shared__ float wred[4][NC][3];
  __shared__ float4 rtap[2 * SP_CA_T + 3];       // per region row: two table offsets and a weight
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* ckpt = IOF(ckpt);
  const int k0 = J.a, cm = sd.c_max;
  const int Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  // the pairs as (r, d) = (c_max - c, s - c): compile-time constants for a known set
  // (its pair loops unroll), else read from the stream description
  const int np = SET ? CG_SET1_N : sd.n_pairs;
  auto pr = [&](int p) { return SET ? cg_set1_r(p) : cm - sd.pc[p]; };
  auto pd = [&](int p) { return SET ? cg_set1_d(p) : sd.ps[p] - sd.pc[p]; };
  CgLayout L;
  if constexpr (SET != 0) {
    constexpr int R[CG_SET1_N] = {cg_set1_r(0), cg_set1_r(1), cg_set1_r(2), cg_set1_r(3)};
    constexpr int D[CG_SET1_N] = {cg_set1_d(0), cg_set1_d(1), cg_set1_d(2), cg_set1_d(3)};
    L = csg_layout_rd(R, D, CG_SET1_N);
  } else {
    L = csg_layout(sd.pc, sd.ps, sd.n_pairs, cm);
  }
  float* const X1 = dyn;                    // [NC][CG_X1N]
  float* const X0 = X1 + NC * L.x1n;        // [NC][SP_CA_T * SP_CA_T]
  float* const FT = X0 + NC * L.x0n;        // per pair: [NC][cap]
  float* const FQ = FT + NC * L.footn;      // [region pixel][NC]
  float* const TT = FQ + NC * L.fqn;        // [footprint row][region column][NC], then [region row][tile column][NC]
  bool has0 = false, has1 = false;
#pragma unroll
  for (int p = 0; p < np; ++p) {
    has0 |= pr(p) == 0;
    has1 |= pr(p) == 1;
  }
  const Range rg0{J.y0, J.th}, cg0{J.x0, J.tw};
  Range rg1 = rg0, cg1 = cg0;
  if (has1) {
    rg1 = finer_range(rg0, sd.Hl[cm - 1]);
    cg1 = finer_range(cg0, sd.Wl[cm - 1]);
  }
  const gp<float> gmap = G(sd.gmap);
  const size_t plane = (size_t)Hm * Wm;
  // ---- one round trip: the c_max tile, the region of the level below and every pair's
  // footprint, for each channel of the group.  The tile and the region are staged in
  // whole rows of 16-byte quads: row stride pw in LDS, first staged column
  // xa = (first column) & ~3, so column x sits at x - xa.  Rows are 16-byte aligned in
  // memory when the level width is a multiple of 4 and the plane is 16-byte aligned;
  // otherwise 4-byte transfers fill the same layout.
  const int xa0 = cg0.lo & ~3, pw0 = ((cg0.lo + cg0.n + 3) & ~3) - xa0;
  const int xa1 = cg1.lo & ~3, pw1 = ((cg1.lo + cg1.n + 3) & ~3) - xa1;
  // One index walk per region drives the transfers of every channel of the group (the
  // channels differ only in their plane and LDS block).
  const int wf = wave_first();
  auto stage = [&](Range rr, int xa, int pw, int c, float* xbase, int xstride) {
    const uint32_t Wc = sd.Wl[c];
    gp<const float> Xc[NC];
    bool vec = (Wc & 3) == 0;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      Xc[j] = G(chan_ptr(sd, ckpt, k0 + j, c));
      vec = vec && (reinterpret_cast<uintptr_t>(Xc[j]) & 15) == 0;
    }
    if (vec) {
      const int nq = pw >> 2, n = rr.n * nq;
      Walk2 wk(threadIdx.x, nq);
      for (int q0 = 0; q0 + (int)threadIdx.x < n; q0 += SP_BLOCK, wk.next()) {
        const uint32_t ob = ((uint32_t)(rr.lo + wk.r) * Wc + (uint32_t)(xa + 4 * wk.c)) * 4u;
#pragma unroll
        for (int j = 0; j < NC; ++j) lds_load4_u(xbase + j * xstride + 4 * (q0 + wf), Xc[j], ob);
      }
    } else {
      const int n = rr.n * pw;
      Walk2 wk(threadIdx.x, pw);
      for (int i0 = 0; i0 + (int)threadIdx.x < n; i0 += SP_BLOCK, wk.next()) {
        const uint32_t ob = ((uint32_t)(rr.lo + wk.r) * Wc + (uint32_t)min(xa + wk.c, (int)Wc - 1)) * 4u;
#pragma unroll
        for (int j = 0; j < NC; ++j) lds_load_u(xbase + j * xstride + i0 + wf, Xc[j], ob);
      }
    }
  };
  if (has0) stage(rg0, xa0, pw0, cm, X0, SP_CA_T * SP_CA_T);
  if (has1) stage(rg1, xa1, pw1, cm - 1, X1, CG_X1N);
  {
    float* fb = FT;
#pragma unroll
    for (int p = 0; p < np; ++p) {
      const int r = pr(p), d = pd(p), s = cm - r + d, Ws = sd.Wl[s];
      const Range rr = (r == 0) ? rg0 : rg1, cc = (r == 0) ? cg0 : cg1;
      const Foot f = footprint(rr.lo, rr.n, cc.lo, cc.n, d, sd.Hl[s], Ws);
      const int cap = csapply_foot_cap(r, d);
      gp<const float> Xs[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) Xs[j] = G(chan_ptr(sd, ckpt, k0 + j, s));
      Walk2 wk(threadIdx.x, f.w);
      for (int i0 = 0; i0 + (int)threadIdx.x < f.h * f.w; i0 += SP_BLOCK, wk.next()) {
        const uint32_t ob = ((uint32_t)(f.y0 + wk.r) * (uint32_t)Ws + (uint32_t)(f.x0 + wk.c)) * 4u;
#pragma unroll
        for (int j = 0; j < NC; ++j) lds_load_u(fb + j * cap + i0 + wf, Xs[j], ob);
      }
      fb += NC * cap;
    }
  }
  lds_wait();
  __syncthreads();
  const int lane = lane_id(), w = wave_id();
  const int sy = (lane >> 2) & 3, sx = lane & 3;
  // ---- pairs with c = c_max: one wavefront per map covers the tile's four 8x8 blocks
  // (a 2x2 quad per lane, DPP inside each 16-lane row); the map is its own reduction
  if (has0) {
    const int blk = lane >> 4, by = blk >> 1, bx = blk & 1;
    const int qy = 8 * by + 2 * sy, qx = 8 * bx + 2 * sx;
    bool bval[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bval[i] = 8 * (i >> 1) < J.th && 8 * (i & 1) < J.tw;
    int m = 0;
    const float* fb = FT;
#pragma unroll
    for (int p = 0; p < np; ++p) {
      const int r = pr(p), d = pd(p), s = cm - r + d;
      const int cap = csapply_foot_cap(r, d);
      if (r == 0) {
        const Foot f = footprint(J.y0, J.th, J.x0, J.tw, d, sd.Hl[s], sd.Wl[s]);
        int yl[2], xl[2];
        Tap ty[2], tx[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          yl[u] = min(qy + u, J.th - 1);
          xl[u] = min(qx + u, J.tw - 1);
          ty[u] = bilinear_tap(J.y0 + yl[u], d, sd.Hl[s]);
          tx[u] = bilinear_tap(J.x0 + xl[u], d, sd.Wl[s]);
        }
#pragma unroll
        for (int j = 0; j < NC; ++j, ++m) {
          if ((m & 3) != w) continue;   // wave-uniform
          const float* B = X0 + j * (SP_CA_T * SP_CA_T) + cg0.lo - xa0;
          float mn = INFINITY, mx = 0.f;   // F >= 0
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) {
              const float up = bilinear_lds(fb + j * cap, f.w, ty[u], tx[v], f.y0, f.x0);
              const float F = fabsf(B[yl[u] * pw0 + xl[v]] - up);
              mn = fmin_nn(mn, F);
              mx = fmax_nn(mx, F);
              if (qy + u < J.th && qx + v < J.tw)
                gmap[((size_t)p * SP_NCH + k0 + j) * plane + (size_t)(J.y0 + qy + u) * Wm + J.x0 + qx + v] = F;
            }
          row16_minmax_nn(mn, mx);
          float bmn[4], bmx[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            // read unconditionally, then select: a readlane under the condition becomes a branch
            const float rmn = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mn), 16 * i));
            const float rmx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mx), 16 * i));
            bmn[i] = bval[i] ? rmn : INFINITY;
            bmx[i] = bval[i] ? rmx : -INFINITY;
          }
          if (lane == 0) {
            const gp<float> out = G(sd.cs_part) + 3 * ((size_t)sd.cs_off[p] + (size_t)(k0 + j) * sd.cs_nt[p] + J.tid);
            out[0] = fminf(fminf(bmn[0], bmn[1]), fminf(bmn[2], bmn[3]));
            out[1] = fmaxf(fmaxf(bmx[0], bmx[1]), fmaxf(bmx[2], bmx[3]));
            out[2] = ((bval[0] ? bmx[0] : 0.f) + (bval[1] ? bmx[1] : 0.f)) +
                     ((bval[2] ? bmx[2] : 0.f) + (bval[3] ? bmx[3] : 0.f));
          }
        }
      }
      fb += NC * cap;
    }
  }
  // ---- pairs with c = c_max - 1, one at a time: the footprint's rows interpolated at the
  // region's columns (the separable first half of the bilinear up-sample), the map on
  // the whole region, its statistics on the 2*th x 2*tw pixels the tile owns (wavefront
  // w: block row w, a 2x2 quad per lane), then REDUCE to the tile
  if (has1) {
    const int c1 = cm - 1, H1 = sd.Hl[c1], W1 = sd.Wl[c1];
    const int n1r = rg1.n, n1c = cg1.n;
    const int oh = min(2 * J.th, H1 - 2 * J.y0), ow = min(2 * J.tw, W1 - 2 * J.x0);
    const int oy0 = 2 * J.y0 - rg1.lo, ox0 = 2 * J.x0 - cg1.lo;   // region offset of the owned pixels
    const int bx = lane >> 4, qy = 8 * w + 2 * sy, qx = 8 * bx + 2 * sx;
    int ro[2], co[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ro[u] = oy0 + min(qy + u, oh - 1);
      co[u] = ox0 + min(qx + u, ow - 1);
    }
    const bool rowval = 8 * w < oh;
    bool bval[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bval[i] = rowval && 8 * i < ow;
    // reduction taps: a row-pass thread keeps one tile column (the tile width divides the
    // block), a column-pass thread one output
    const int rc = threadIdx.x % SP_CA_T, rr0 = threadIdx.x / SP_CA_T;
    int ix[5], iy[5];
#pragma unroll
    for (int t = -2; t <= 2; ++t) {
      ix[t + 2] = clampi(2 * (cg0.lo + rc) + t, 0, W1 - 1) - cg1.lo;
      iy[t + 2] = clampi(2 * (rg0.lo + rr0) + t, 0, H1 - 1) - rg1.lo;
    }
    // the table and map passes: a thread keeps region column rcol and steps over the rows
    // (G1 rows at a time; threads beyond G1 * n1c sit these passes out)
    const int G1 = SP_BLOCK / n1c, g1 = threadIdx.x / n1c, rcol = threadIdx.x - g1 * n1c;
    const float* const x1c = X1 + (cg1.lo - xa1) + rcol;   // row r of channel j at x1c + j * CG_X1N + r * pw1
    const float* fb = FT;
#pragma unroll
    for (int p = 0; p < np; ++p) {
      const int r = pr(p), d = pd(p), s = cm - r + d;
      const int cap = csapply_foot_cap(r, d);
      if (r == 1) {
        const int Hs = sd.Hl[s], Ws = sd.Wl[s];
        const Foot f = footprint(rg1.lo, n1r, cg1.lo, n1c, d, Hs, Ws);
        if (g1 < G1) {
          const Tap tx = bilinear_tap(cg1.lo + rcol, d, Ws);
          const float* f0 = fb + tx.i0 - f.x0;
          const float* f1 = fb + tx.i1 - f.x0;
          for (int rr = g1; rr < f.h; rr += G1) {
            float v[NC];
#pragma unroll
            for (int j = 0; j < NC; ++j)
              v[j] = fmaf(tx.w, f1[j * cap + rr * f.w], (1.f - tx.w) * f0[j * cap + rr * f.w]);
            lds_putv<NC>(TT + (rr * n1c + rcol) * NC, v);
          }
        }
        {
          if ((int)threadIdx.x < n1r) {
            const Tap ty = bilinear_tap(rg1.lo + threadIdx.x, d, Hs);
            rtap[threadIdx.x] = make_float4(__int_as_float((ty.i0 - f.y0) * n1c * NC),
                                            __int_as_float((ty.i1 - f.y0) * n1c * NC), ty.w, 1.f - ty.w);
          }
        }
        __syncthreads();
        // the map on the region
        if (g1 < G1) {
          for (int rr = g1; rr < n1r; rr += G1) {
            const float4 rt = rtap[rr];
            float t0[NC], t1[NC], F[NC];
            lds_getv<NC>(TT + __float_as_int(rt.x) + rcol * NC, t0);
            lds_getv<NC>(TT + __float_as_int(rt.y) + rcol * NC, t1);
            const float* xr = x1c + rr * pw1;
#pragma unroll
            for (int j = 0; j < NC; ++j) F[j] = fabsf(xr[j * CG_X1N] - fmaf(rt.z, t1[j], rt.w * t0[j]));
            lds_putv<NC>(FQ + (rr * n1c + rcol) * NC, F);
          }
        }
        __syncthreads();
        // statistics of the owned pixels
        {
          float q[4][NC];
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) lds_getv<NC>(FQ + (ro[u] * n1c + co[v]) * NC, q[2 * u + v]);
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            float mn = fmin_nn(fmin_nn(q[0][j], q[1][j]), fmin_nn(q[2][j], q[3][j]));   // F >= 0
            float mx = fmax_nn(fmax_nn(q[0][j], q[1][j]), fmax_nn(q[2][j], q[3][j]));
            row16_minmax_nn(mn, mx);
            float bmn[4], bmx[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              // read unconditionally, then select: a readlane under the condition becomes a branch
              const float rmn = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mn), 16 * i));
              const float rmx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mx), 16 * i));
              bmn[i] = bval[i] ? rmn : INFINITY;
              bmx[i] = bval[i] ? rmx : -INFINITY;
            }
            if (lane == 0) {
              wred[w][j][0] = fminf(fminf(bmn[0], bmn[1]), fminf(bmn[2], bmn[3]));
              wred[w][j][1] = fmaxf(fmaxf(bmx[0], bmx[1]), fmaxf(bmx[2], bmx[3]));
              wred[w][j][2] = ((bval[0] ? bmx[0] : 0.f) + (bval[1] ? bmx[1] : 0.f)) +
                              ((bval[2] ? bmx[2] : 0.f) + (bval[3] ? bmx[3] : 0.f));
            }
          }
        }
        // REDUCE to the tile: row pass (region rows x tile columns) into the table, then
        // column pass
        if (rc < cg0.n) {
          for (int rr = rr0; rr < n1r; rr += SP_BLOCK / SP_CA_T) {
            float acc[NC];
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[j] = 0.f;
#pragma unroll
            for (int t = 0; t < 5; ++t) {
              float v[NC];
              lds_getv<NC>(FQ + (rr * n1c + ix[t]) * NC, v);
#pragma unroll
              for (int j = 0; j < NC; ++j) acc[j] = fmaf(binom(t - 2), v[j], acc[j]);
            }
            lds_putv<NC>(TT + (rr * SP_CA_T + rc) * NC, acc);
          }
        }
        __syncthreads();
        if (rr0 < rg0.n && rc < cg0.n) {
          float acc[NC];
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[j] = 0.f;
#pragma unroll
          for (int t = 0; t < 5; ++t) {
            float v[NC];
            lds_getv<NC>(TT + (iy[t] * SP_CA_T + rc) * NC, v);
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[j] = fmaf(binom(t - 2), v[j], acc[j]);
          }
          const size_t o = (size_t)(rg0.lo + rr0) * Wm + cg0.lo + rc;
#pragma unroll
          for (int j = 0; j < NC; ++j) gmap[((size_t)p * SP_NCH + k0 + j) * plane + o] = acc[j];
        }
        if ((int)threadIdx.x < NC) {
          const int j = threadIdx.x;
          const gp<float> out = G(sd.cs_part) + 3 * ((size_t)sd.cs_off[p] + (size_t)(k0 + j) * sd.cs_nt[p] + J.tid);
          out[0] = fminf(fminf(wred[0][j][0], wred[1][j][0]), fminf(wred[2][j][0], wred[3][j][0]));
          out[1] = fmaxf(fmaxf(wred[0][j][1], wred[1][j][1]), fmaxf(wred[2][j][1], wred[3][j][1]));
          out[2] = (wred[0][j][2] + wred[1][j][2]) + (wred[2][j][2] + wred[3][j][2]);
        }
        __syncthreads();   // the map, the table, the row taps and wred are reused by the next pair
      }
      fb += NC * cap;
    }
  }
}

// The reduced-map job for pair set 1 ((r, d) = (1,2), (1,3), (0,2), (0,3) in the stream's
// pair order; the default pairs), with a fixed geometry.  The region one level below c_max
// is always the 35x35 block at (2 y0 - 2, 2 x0 - 2) and each footprint the block at the
// region's (or the tile's) origin shifted down by d levels, staged from coordinates clamped
// into their level: a replicated row or column holds exactly the value that clamp-to-edge
// sampling reads there, and the up-sample taps of the region's rows and columns are taken
// at the clamped coordinate (a per-workgroup table).  Every loop bound, reduction offset
// and staging index is then a compile-time constant, for edge tiles too.  The arithmetic
// and the order of every sum are those of k_csg, so the maps and statistics are the same.
namespace cg1 {
constexpr int T = SP_CA_T;             // c_max tile edge
constexpr int N1 = 2 * T + 3;          // region edge one level below c_max
constexpr int PW = CG_PW1;             // LDS row stride of the region: whole quads, region column cc at cc + 2
constexpr int X1N = N1 * PW;
constexpr int FN = 11 * 11 + 7 * 7 + 5 * 5 + 3 * 3;   // footprints of pairs 0..3, back to back
constexpr int FQN = N1 * N1;
constexpr int TTN = N1 * T;            // >= 11 * N1, the widest footprint table
constexpr int PER_CH = X1N + T * T + FN + FQN + TTN;
__host__ __device__ constexpr int fe(int p) { return p == 0 ? 11 : (p == 1 ? 7 : (p == 2 ? 5 : 3)); }
__host__ __device__ constexpr int fo(int p) { return p == 0 ? 0 : (p == 1 ? 121 : (p == 2 ? 170 : 195)); }
}  // namespace cg1

template <int NC>
__global__ __launch_bounds__(SP_BLOCK) void k_csg1(const Job* __restrict__ jobs,
                                                   const StreamDesc* __restrict__ sds,
                                                   const StepIO* __restrict__ ios, StepIO io0) {
  using namespace cg1;
  static_assert(PW == 40 && N1 == 35 && T == 16, "layout of the fixed-geometry job");
  extern __shared__ __align__(16) float dyn[];
  __shared__ float4 rtab[2][N1], ctab[2][N1];   // pairs 0, 1: taps (i0, i1 as offsets, w, 1 - w)
  __shared__ float wred[4][NC][3];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const float* ckpt = IOF(ckpt);
  const int k0 = J.a, cm = sd.c_max, c1 = cm - 1;
  const int Hm = sd.Hl[cm], Wm = sd.Wl[cm], H1 = sd.Hl[c1], W1 = sd.Wl[c1];
  const int y0 = J.y0, x0 = J.x0, ry0 = 2 * y0 - 2, rx0 = 2 * x0 - 2;
  float* const X1 = dyn;                 // [NC][N1][PW]
  float* const X0 = X1 + NC * X1N;       // [NC][T][T]
  float* const FP = X0 + NC * T * T;     // [NC][FN]
  float* const FQ = FP + NC * FN;        // [N1][N1][NC]
  float* const TT = FQ + NC * FQN;       // [..][NC]
  const int tid = threadIdx.x, wf = wave_first();
  // ---- staging, one round trip
  {
    gp<const float> Xc[NC];
    bool vec = (W1 & 3) == 0 && rx0 >= 2 && rx0 + PW - 2 <= W1;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      Xc[j] = G(chan_ptr(sd, ckpt, k0 + j, c1));
      vec = vec && (reinterpret_cast<uintptr_t>(Xc[j]) & 15) == 0;
    }
    if (vec) {
      constexpr int NQ = N1 * (PW / 4);
#pragma unroll
      for (int q0 = 0; q0 < NQ; q0 += SP_BLOCK) {
        const int q = q0 + tid;
        if (q < NQ) {
          const int r = q / (PW / 4), cq = q - r * (PW / 4);
          const uint32_t ob = ((uint32_t)clampi(ry0 + r, 0, H1 - 1) * (uint32_t)W1 + (uint32_t)(rx0 - 2 + 4 * cq)) * 4u;
#pragma unroll
          for (int j = 0; j < NC; ++j) lds_load4_u(X1 + j * X1N + 4 * (q0 + wf), Xc[j], ob);
        }
      }
    } else {
#pragma unroll
      for (int i0 = 0; i0 < X1N; i0 += SP_BLOCK) {
        const int i = i0 + tid;
        if (i < X1N) {
          const int r = i / PW, cc = i - r * PW;
          const uint32_t ob = ((uint32_t)clampi(ry0 + r, 0, H1 - 1) * (uint32_t)W1 +
                               (uint32_t)clampi(rx0 - 2 + cc, 0, W1 - 1)) * 4u;
#pragma unroll
          for (int j = 0; j < NC; ++j) lds_load_u(X1 + j * X1N + i0 + wf, Xc[j], ob);
        }
      }
    }
  }
  {
    gp<const float> Xc[NC];
    bool vec = (Wm & 3) == 0 && x0 + T <= Wm;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      Xc[j] = G(chan_ptr(sd, ckpt, k0 + j, cm));
      vec = vec && (reinterpret_cast<uintptr_t>(Xc[j]) & 15) == 0;
    }
    if (vec) {
      if (tid < T * T / 4) {
        const uint32_t ob = ((uint32_t)min(y0 + (tid >> 2), Hm - 1) * (uint32_t)Wm + (uint32_t)(x0 + 4 * (tid & 3))) * 4u;
#pragma unroll
        for (int j = 0; j < NC; ++j) lds_load4_u(X0 + j * T * T + 4 * wf, Xc[j], ob);
      }
    } else {
      const uint32_t ob = ((uint32_t)min(y0 + (tid >> 4), Hm - 1) * (uint32_t)Wm + (uint32_t)min(x0 + (tid & 15), Wm - 1)) * 4u;
#pragma unroll
      for (int j = 0; j < NC; ++j) lds_load_u(X0 + j * T * T + wf, Xc[j], ob);
    }
  }
  // footprints, one pair at a time (uniform level and base; lane = element)
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int d = 2 + (p & 1), s = (p < 2 ? c1 : cm) + d;
    const int oy = (p < 2 ? ry0 : y0) >> d, ox = (p < 2 ? rx0 : x0) >> d;
    const int Hs = sd.Hl[s], Ws = sd.Wl[s];
    if (tid < fe(p) * fe(p)) {
      const int i = tid / fe(p), e = tid - i * fe(p);
      const uint32_t ob = ((uint32_t)clampi(oy + i, 0, Hs - 1) * (uint32_t)Ws + (uint32_t)clampi(ox + e, 0, Ws - 1)) * 4u;
#pragma unroll
      for (int j = 0; j < NC; ++j) lds_load_u(FP + j * FN + fo(p) + wf, G(chan_ptr(sd, ckpt, k0 + j, s)), ob);
    }
  }
  if (tid < 4 * N1) {
    // taps of the region's rows (which = 0, 2) and columns (1, 3) for pairs 0 and 1, at the
    // clamped coordinate, relative to the footprint's first (unclamped) row or column
    const int which = tid / N1, k = tid - which * N1;
    const int p = which >> 1, d = 2 + p, s = c1 + d;
    const bool col = which & 1;
    const int o = col ? rx0 : ry0;
    const Tap t = bilinear_tap(clampi(o + k, 0, (col ? W1 : H1) - 1), d, col ? sd.Wl[s] : sd.Hl[s]);
    // rows: offsets of the table rows (footprint row * N1 * NC); columns: footprint columns
    const int sc = col ? 1 : N1 * NC;
    const float4 v = make_float4(__int_as_float((t.i0 - (o >> d)) * sc), __int_as_float((t.i1 - (o >> d)) * sc), t.w,
                                 1.f - t.w);
    if (col)
      ctab[p][k] = v;
    else
      rtab[p][k] = v;
  }
  lds_wait();
  __syncthreads();
  const gp<float> gmap = G(sd.gmap);
  const size_t plane = (size_t)Hm * Wm;
  const int lane = lane_id(), w = wave_id();
  const int sy = (lane >> 2) & 3, sx = lane & 3;
  // ---- pairs 2 and 3 (c = c_max): one wavefront per map covers the tile's four 8x8
  // blocks (a 2x2 quad per lane, DPP inside each 16-lane row)
  {
    const int blk = lane >> 4, by = blk >> 1, bx = blk & 1;
    const int qy = 8 * by + 2 * sy, qx = 8 * bx + 2 * sx;
    const bool bvalid = 8 * by < J.th && 8 * bx < J.tw;   // the lane's 8x8 block lies in the tile
    int m = 0;
#pragma unroll
    for (int p = 2; p < 4; ++p) {
      const int d = 2 + (p & 1), s = cm + d;
      int yl[2], xl[2];
      Tap ty[2], tx[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        yl[u] = min(qy + u, J.th - 1);
        xl[u] = min(qx + u, J.tw - 1);
        ty[u] = bilinear_tap(y0 + yl[u], d, sd.Hl[s]);
        tx[u] = bilinear_tap(x0 + xl[u], d, sd.Wl[s]);
      }
#pragma unroll
      for (int j = 0; j < NC; ++j, ++m) {
        if ((m & 3) != w) continue;   // wave-uniform
        const float* B = X0 + j * T * T;
        float mn = INFINITY, mx = 0.f;   // F >= 0
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const float up = bilinear_lds(FP + j * FN + fo(p), fe(p), ty[u], tx[v], y0 >> d, x0 >> d);
            const float F = fabsf(B[yl[u] * T + xl[v]] - up);
            mn = fmin_nn(mn, F);
            mx = fmax_nn(mx, F);
            if (qy + u < J.th && qx + v < J.tw)
              *at_bytes(gmap + ((size_t)p * SP_NCH + k0 + j) * plane,
                        ((uint32_t)(y0 + qy + u) * (uint32_t)Wm + (uint32_t)(x0 + qx + v)) * 4u) = F;
          }
        row16_minmax_nn(mn, mx);
        float tmn, tmx, tsum;
        rows4_combine_nn(mn, mx, bvalid, tmn, tmx, tsum);
        if (lane == 63) {
          const gp<float> out = G(sd.cs_part) + 3 * ((size_t)sd.cs_off[p] + (size_t)(k0 + j) * sd.cs_nt[p] + J.tid);
          out[0] = tmn;
          out[1] = tmx;
          out[2] = tsum;
        }
      }
    }
  }
  // ---- pairs 0 and 1 (c = c_max - 1), one at a time: the footprint's rows interpolated at
  // the region's columns, the map on the region, its statistics on the pixels the tile owns
  // (region rows and columns 2 .. 33; wavefront w: block row w, a 2x2 quad per lane), then
  // REDUCE to the tile
  {
    const int oh = min(2 * T, H1 - 2 * y0), ow = min(2 * T, W1 - 2 * x0);
    const int bxl = lane >> 4, qy = 8 * w + 2 * sy, qx = 8 * bxl + 2 * sx;
    int ro[2], co[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ro[u] = 2 + min(qy + u, oh - 1);
      co[u] = 2 + min(qx + u, ow - 1);
    }
    const bool bvalid = 8 * w < oh && 8 * bxl < ow;   // the lane's 8x8 block of owned pixels
    const int g1 = tid / N1, cc1 = tid - g1 * N1;   // map pass: region column cc1, rows g1 + 7 i
    const int rc = tid & (T - 1), rq = tid >> 4;     // reduction: tile column rc, row group rq
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      constexpr int NTAB[2] = {fe(0) * N1, fe(1) * N1};
#pragma unroll
      for (int e0 = 0; e0 < NTAB[p]; e0 += SP_BLOCK) {
        const int e = e0 + tid;
        if (e < NTAB[p]) {
          const int fr = e / N1, cc = e - fr * N1;
          const float4 ct = ctab[p][cc];
          const float* f0 = FP + fo(p) + fr * fe(p) + __float_as_int(ct.x);
          const float* f1 = FP + fo(p) + fr * fe(p) + __float_as_int(ct.y);
          float v[NC];
#pragma unroll
          for (int j = 0; j < NC; ++j) v[j] = fmaf(ct.z, f1[j * FN], ct.w * f0[j * FN]);
          lds_putv<NC>(TT + e * NC, v);
        }
      }
      __syncthreads();
      // the map on the region
      if (g1 < 7) {
        const float* xr = X1 + g1 * PW + cc1 + 2;
        float* fq = FQ + (g1 * N1 + cc1) * NC;
#pragma unroll
        for (int i = 0; i < N1 / 7; ++i) {
          const float4 rt = rtab[p][g1 + 7 * i];
          float t0[NC], t1[NC], F[NC];
          lds_getv<NC>(TT + __float_as_int(rt.x) + cc1 * NC, t0);
          lds_getv<NC>(TT + __float_as_int(rt.y) + cc1 * NC, t1);
#pragma unroll
          for (int j = 0; j < NC; ++j) F[j] = fabsf(xr[j * X1N + 7 * i * PW] - fmaf(rt.z, t1[j], rt.w * t0[j]));
          lds_putv<NC>(fq + 7 * i * N1 * NC, F);
        }
      }
      __syncthreads();
      // statistics of the owned pixels
      {
        float q[4][NC];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) lds_getv<NC>(FQ + (ro[u] * N1 + co[v]) * NC, q[2 * u + v]);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          float mn = fmin_nn(fmin_nn(q[0][j], q[1][j]), fmin_nn(q[2][j], q[3][j]));   // F >= 0
          float mx = fmax_nn(fmax_nn(q[0][j], q[1][j]), fmax_nn(q[2][j], q[3][j]));
          row16_minmax_nn(mn, mx);
          float tmn, tmx, tsum;
          rows4_combine_nn(mn, mx, bvalid, tmn, tmx, tsum);
          if (lane == 63) {
            wred[w][j][0] = tmn;
            wred[w][j][1] = tmx;
            wred[w][j][2] = tsum;
          }
        }
      }
      // REDUCE to the tile: row pass (region rows x tile columns) into the table, then
      // column pass; taps 2 rc .. 2 rc + 4 of the region (a replicated edge is the clamp)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int rr = rq + 16 * i;
        if (rr < N1) {
          float acc[NC];
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[j] = 0.f;
#pragma unroll
          for (int t = 0; t < 5; ++t) {
            float v[NC];
            lds_getv<NC>(FQ + (rr * N1 + 2 * rc + t) * NC, v);
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[j] = fmaf(binom(t - 2), v[j], acc[j]);
          }
          lds_putv<NC>(TT + (rr * T + rc) * NC, acc);
        }
      }
      __syncthreads();
      {
        float acc[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[j] = 0.f;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          float v[NC];
          lds_getv<NC>(TT + ((2 * rq + t) * T + rc) * NC, v);
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[j] = fmaf(binom(t - 2), v[j], acc[j]);
        }
        if (rq < J.th && rc < J.tw) {
          const uint32_t ob = ((uint32_t)(y0 + rq) * (uint32_t)Wm + (uint32_t)(x0 + rc)) * 4u;
#pragma unroll
          for (int j = 0; j < NC; ++j) *at_bytes(gmap + ((size_t)p * SP_NCH + k0 + j) * plane, ob) = acc[j];
        }
      }
      if (tid < NC) {
        const int j = tid;
        const gp<float> out = G(sd.cs_part) + 3 * ((size_t)sd.cs_off[p] + (size_t)(k0 + j) * sd.cs_nt[p] + J.tid);
        out[0] = fminf(fminf(wred[0][j][0], wred[1][j][0]), fminf(wred[2][j][0], wred[3][j][0]));
        out[1] = fmaxf(fmaxf(wred[0][j][1], wred[1][j][1]), fmaxf(wred[2][j][1], wred[3][j][1]));
        out[2] = (wred[0][j][2] + wred[1][j][2]) + (wred[2][j][2] + wred[3][j][2]);
      }
      __syncthreads();   // the map, the table and wred are reused by the next pair
    }
  }
}
#pragma clang diagnostic pop

// N(.) parameters of the eight maps of a pair from their per-tile partials, one wavefront:
// lanes 8k..8k+7 take map k, lane 8k+j its tiles j, j+8, j+16, ...  The first 80 tiles are
// requested at once by load(); finish() takes any further tiles one at a time, then the
// eight lanes of each map combine by DPP in a fixed order, so the parameters are
// reproducible bit for bit.  Other loads can be issued between the two calls.
struct Part3 { float mn, mx, sb; };   // one tile's (min, max, sum of block maxima), 12 bytes

struct PairNp {
  static constexpr int C = 10;   // tiles per lane requested by load()
  Part3 v[C];

  __device__ void load(const StreamDesc& sd, int p) {
    const int nt = sd.cs_nt[p], j = lane_id() & 7;
    const gp<const float> part = G((const float*)sd.cs_part) + 3 * (size_t)sd.cs_off[p];   // uniform base
    const uint32_t ko = (uint32_t)(lane_id() >> 3) * (uint32_t)nt;
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const uint32_t t = (uint32_t)min(j + 8 * u, nt - 1);
      const gp<const Part3> q = (gp<const Part3>)at_bytes(part, 12u * (ko + t));
      v[u].mn = q->mn;
      v[u].mx = q->mx;
      v[u].sb = q->sb;
    }
  }
  // dst[k] = (mn, inv, scale) of map k, inv = scale = 0 for a flat map
  __device__ void finish(const StreamDesc& sd, int p, float (*dst)[3]) {
    const int nt = sd.cs_nt[p], c = sd.pc[p], nb = nblocks8(sd.Hl[c], sd.Wl[c]);
    const int k = lane_id() >> 3, j = lane_id() & 7;
    float mn = INFINITY, mx = -INFINITY;
    double s = 0.0;
    // a position past the last tile read the last tile again: harmless to the minimum and
    // maximum, masked to +0 in the sum (sums of F >= 0 start at +0, so adding +0 is exact)
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int keep = -(int)(j + 8 * u < nt);
      mn = fminf(mn, v[u].mn);
      mx = fmaxf(mx, v[u].mx);
      s += (double)__int_as_float(__float_as_int(v[u].sb) & keep);
    }
    if (nt > 8 * C) {   // large frames
      const gp<const float> part = G((const float*)sd.cs_part) + 3 * (size_t)sd.cs_off[p];
      const uint32_t ko = (uint32_t)k * (uint32_t)nt;
      for (int t = 8 * C + j; t < nt; t += 8) {
        const gp<const Part3> q = (gp<const Part3>)at_bytes(part, 12u * (ko + (uint32_t)t));
        mn = fminf(mn, q->mn);
        mx = fmaxf(mx, q->mx);
        s += (double)q->sb;
      }
    }
    // quad_perm [1,0,3,2], quad_perm [2,3,0,1], then row_half_mirror (lane i with lane
    // 7 - i of its eight)
    mn = fminf(mn, dpp_f<0xB1>(mn));
    mx = fmaxf(mx, dpp_f<0xB1>(mx));
    s += dpp_d<0xB1>(s);
    mn = fminf(mn, dpp_f<0x4E>(mn));
    mx = fmaxf(mx, dpp_f<0x4E>(mx));
    s += dpp_d<0x4E>(s);
    mn = fminf(mn, dpp_f<0x141>(mn));
    mx = fmaxf(mx, dpp_f<0x141>(mx));
    s += dpp_d<0x141>(s);
    const NParams q = make_nparams(mn, mx, s, nb, sd.flat_tol);
    if (j == 0) {
      dst[k][0] = q.mn;
      dst[k][1] = q.flat ? 0.f : q.inv;
      dst[k][2] = q.flat ? 0.f : q.scale;
    }
  }
};

// F-bar_k on a 16x16 c_max tile = sum over pairs of N(reduced map), all 8 channels; then
// its partial statistics (one 8x8 block per wavefront).
__global__ __launch_bounds__(SP_BLOCK) void k_csmix(const Job* __restrict__ jobs,
                                                    const StreamDesc* __restrict__ sds,
                                                    const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float nps[SP_MAXP][SP_NCH][3];
  __shared__ float wacc[4][SP_NCH][3];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const int cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const size_t plane = (size_t)Hm * Wm;
  const int lane = lane_id(), w = wave_id();
  const int by = w >> 1, bx = w & 1;
  const int yy = 8 * by + (lane >> 3), xx = 8 * bx + (lane & 7);
  const bool bvalid = 8 * by < J.th && 8 * bx < J.tw;
  const bool valid = yy < J.th && xx < J.tw;
  const uint32_t ob = ((uint32_t)(J.y0 + min(yy, J.th - 1)) * (uint32_t)Wm + (uint32_t)(J.x0 + min(xx, J.tw - 1))) * 4u;
  const size_t o = ob / 4u;
  // the maps of PG pairs are loaded together, the first group before the N parameters
  // are staged; pairs are added in increasing order
  constexpr int PG = 4;
  const int np = sd.n_pairs;
  float g[PG][SP_NCH];
  auto load_group = [&](int p0) {
#pragma unroll
    for (int u = 0; u < PG; ++u) {
      const int p = max(min(p0 + u, np - 1), 0);   // past the last pair: loaded again, not added
#pragma unroll
      for (int k = 0; k < SP_NCH; ++k) g[u][k] = *at_bytes(G(sd.gmap + ((size_t)p * SP_NCH + k) * plane), ob);
    }
  };
  // the N parameters of every map, from the partials of the across-scale launch, one
  // wavefront per pair: the first pair's partials are requested before the first group of
  // maps and reduced while those are in flight
  const int w0 = __builtin_amdgcn_readfirstlane(w);
  {
    PairNp q;
    q.load(sd, min(w0, np - 1));   // a wavefront without a pair loads the last one's, unused
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the maps'
    load_group(0);
    if (w0 < np) q.finish(sd, w0, nps[w0]);
  }
  for (int p = w0 + SP_BLOCK / 64; p < np; p += SP_BLOCK / 64) {
    PairNp q;
    q.load(sd, p);
    q.finish(sd, p, nps[p]);
  }
  __syncthreads();
  float acc[SP_NCH];
#pragma unroll
  for (int k = 0; k < SP_NCH; ++k) acc[k] = 0.f;
  for (int p0 = 0; p0 < np; p0 += PG) {
    if (p0 > 0) load_group(p0);
#pragma unroll
    for (int u = 0; u < PG; ++u) {
      const int p = p0 + u;
      if (p < np) {
#pragma unroll
        for (int k = 0; k < SP_NCH; ++k)
          acc[k] = fmaf((g[u][k] - nps[p][k][0]) * nps[p][k][1], nps[p][k][2], acc[k]);
      }
    }
  }
  const gp<float> fbar = G(sd.fbar);
#pragma unroll
  for (int k = 0; k < SP_NCH; ++k) {
    if (valid) fbar[(size_t)k * plane + o] = acc[k];
    const float wmn = wave_reduce<OpMin>(valid ? acc[k] : INFINITY);
    const float wmx = wave_reduce<OpMax>(valid ? acc[k] : -INFINITY);
    if (lane == 0) {
      wacc[w][k][0] = wmn;
      wacc[w][k][1] = wmx;
      wacc[w][k][2] = bvalid ? wmx : 0.f;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < SP_NCH) {
    const int k = threadIdx.x;
    const gp<float> out = G(sd.fbar_part) + 3 * ((size_t)k * sd.n_cmax_tiles + J.tid);
    out[0] = fminf(fminf(wacc[0][k][0], wacc[1][k][0]), fminf(wacc[2][k][0], wacc[3][k][0]));
    out[1] = fmaxf(fmaxf(wacc[0][k][1], wacc[1][k][1]), fmaxf(wacc[2][k][1], wacc[3][k][1]));
    out[2] = (wacc[0][k][2] + wacc[1][k][2]) + (wacc[2][k][2] + wacc[3][k][2]);
  }
}

// ---------------------------------------------------------------- conspicuity and saliency
__device__ void consp_nparams(const StreamDesc& sd, NParams* np) {
  const int cm = sd.c_max;
  const int nb = nblocks8(sd.Hl[cm], sd.Wl[cm]);
  const int k = wave_id(), nt = sd.n_cmax_tiles;
  NParams qa, qb;
  nparams_wave2(sd.fbar_part + 3 * (size_t)k * nt, sd.fbar_part + 3 * (size_t)(k + 4) * nt, nt, nb, sd.flat_tol,
                &qa, &qb);
  if (lane_id() == 0) {
    np[k] = qa;
    np[k + 4] = qb;
  }
  __syncthreads();
}

// Block max of S over the tile with the first row-major argmax -> partial slot.  Each
// wavefront finds its maximum and the first index holding it; the block's first index of
// its maximum is the least of those of the wavefronts whose maximum it is (one barrier).
__device__ void smax_partial(float v, int idx, bool valid, gp<float> out, float* sh4, int* shi4) {
  const float wm = wave_reduce<OpMax>(valid ? v : -INFINITY);
  const int cand = wave_min_i((valid && v == wm) ? idx : 0x7fffffff);
  if (lane_id() == 0) {
    sh4[wave_id()] = wm;
    shi4[wave_id()] = cand;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(sh4[0], sh4[1]), fmaxf(sh4[2], sh4[3]));
    int first = 0x7fffffff;
#pragma unroll
    for (int w = 0; w < 4; ++w) first = sh4[w] == m ? min(first, shi4[w]) : first;
    out[0] = m;
    out[1] = __int_as_float(first);
  }
}

__global__ __launch_bounds__(SP_BLOCK) void k_consp(const Job* __restrict__ jobs,
                                                    const StreamDesc* __restrict__ sds,
                                                    const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ float sh4[4];
  __shared__ int shi4[4];
  __shared__ NParams np[SP_NCH];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const gp<float> S_out = G(IOF(S_out));
  const gp<float> C_out = G(IOF(C_out));
  const gp<float> S_tape = G(IOF(S_tape));
  const int cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const size_t plane = (size_t)Hm * Wm;
  const int yy = threadIdx.x / CA_T, xx = threadIdx.x % CA_T;
  const int y = J.y0 + yy, x = J.x0 + xx;
  const bool valid = yy < J.th && xx < J.tw;
  const size_t o = (size_t)min(y, Hm - 1) * Wm + min(x, Wm - 1);
  const uint32_t ob = (uint32_t)o * 4u;
  float fv[SP_NCH];
#pragma unroll
  for (int k = 0; k < SP_NCH; ++k) fv[k] = *at_bytes(G((const float*)sd.fbar) + k * plane, ob);
  consp_nparams(sd, np);
  float S = 0.f;
#pragma unroll
  for (int k = 0; k < SP_NCH; ++k) {
    const float Ck = napply(np[k], fv[k]);
    if (valid && C_out) *at_bytes(C_out + k * plane, ob) = Ck;
    S += sd.w[k] * Ck;
  }
  if (valid) {
    S_out[o] = S;
    if (S_tape) S_tape[o] = S;
  }
  smax_partial(S, (int)o, valid, G(sd.s_part) + 2 * (size_t)J.tid, sh4, shi4);
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
  const bool valid = yy < J.th && xx < J.tw;
  const size_t o = (size_t)min(y, Hm - 1) * Wm + min(x, Wm - 1);
  float v = S_in[o];
  float* sn = IOF(ssm_next);
  if (sn) {
    // stochastic saliency map: mu_t = mu_{t-1} + K_s (S_t - mu_{t-1}), mu_0 = S_0
    const float* sp = IOF(ssm_prev);
    if (sp) v = fmaf(IOF(Ks), v - sp[o], sp[o]);
    if (valid) sn[o] = v;
  }
  smax_partial(v, (int)o, valid, G(sd.s_part) + 2 * (size_t)J.tid, sh4, shi4);
}

// ---------------------------------------------------------------- Kalman prior update
// q = clamp(up(S / max S), eps, 1 - eps) (0.5 if S is flat), eps on the border ring;
// f = G * pi_{t-1} (or G * seg_{t-1}); pi_t = f + K_t (q - f); eps on the border ring.
// With io.unary set it also writes the unary capacities of pi_t.
constexpr int KT = 16;        // tile edge of the level-0 adjoint sweep
constexpr int KTR = SP_KAL_ROWS;   // tile rows of the level-0 update
constexpr int KTW_MAX = 64;   // widest tile (the width is chosen per stream by the host)
__global__ __launch_bounds__(SP_BLOCK) void k_kalman(const Job* __restrict__ jobs,
                                                     const StreamDesc* __restrict__ sds,
                                                     const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ __align__(16) float reg[(KTR + 4) * (KTW_MAX + 8)];   // flat, row stride rs
  __shared__ float Sl[(KTR / 2 + 2) * (KTW_MAX / 2 + 2)];   // footprint of the tile on level c_max >= 1
  __shared__ int4 rtab[KTR];   // per tile row: offsets in Sl of its two footprint rows, weight bits
  __shared__ float sh4[4];
  __shared__ int shi4[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const gp<const uint8_t> seg = G(IOF(seg_prev));
  const float* pprev = IOF(pi_prev);
  const gp<float> pnext = G(IOF(pi_next));
  const gp<float> pout = G(IOF(prior_out));
  const gp<float> ftape = G(IOF(f_tape));
  const gp<float> mstape = G(IOF(ms_tape));
  const gp<float> unary = G(IOF(unary));
  const float K = IOF(K);
  const int t = IOF(t);
  const int H = sd.H, W = sd.W, cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  // the prior region: rows y0-2 .. y0+KTR+1, columns from x0-4 in whole 16-byte quads
  // (row stride rs; column x at x - x0 + 4), clamped to the frame.  Interior tiles of a
  // float prior whose rows are 16-byte aligned are staged by 16-byte transfers.
  const int tw = J.tw, rs = (tw + 11) & ~3;
  const gp<const float> fmap = G((const float*)IOF(f_map));
  if (t > 0 && !fmap) {
    const bool quads = !seg && (W & 3) == 0 && (tw & 3) == 0 && J.x0 >= 4 && J.x0 + tw + 4 <= W &&
                       (reinterpret_cast<uintptr_t>(pprev) & 15) == 0;
    const gp<const float> gprev = G(pprev);
    const int wf = wave_first();
    if (quads) {
      const int nq = rs >> 2;
      Walk2 wk(threadIdx.x, nq);
      for (int q0 = 0; q0 + (int)threadIdx.x < (KTR + 4) * nq; q0 += SP_BLOCK, wk.next())
        lds_load4_u(reg + 4 * (q0 + wf), gprev,
                    ((uint32_t)clampi(J.y0 - 2 + wk.r, 0, H - 1) * (uint32_t)W + (uint32_t)(J.x0 - 4 + 4 * wk.c)) * 4u);
    } else {
      Walk2 wk(threadIdx.x, rs);
      for (int i0 = 0; i0 + (int)threadIdx.x < (KTR + 4) * rs; i0 += SP_BLOCK, wk.next()) {
        const int y = clampi(J.y0 - 2 + wk.r, 0, H - 1), x = clampi(J.x0 - 4 + wk.c, 0, W - 1);
        const uint32_t o = (uint32_t)y * (uint32_t)W + (uint32_t)x;
        if (seg)
          reg[i0 + threadIdx.x] = (float)seg[o];
        else
          lds_load_u(reg + i0 + wf, gprev, o * 4u);
      }
    }
  }
  // the saliency samples of the tile: its footprint on level c_max, flat with row
  // stride f.w
  const Foot sf = footprint(J.y0, J.th, J.x0, tw, cm, Hm, Wm);
  {
    const gp<const float> Sg = G(IOF(S_in));
    const int wf = wave_first();
    Walk2 wk(threadIdx.x, sf.w);
    for (int i0 = 0; i0 + (int)threadIdx.x < sf.h * sf.w; i0 += SP_BLOCK, wk.next())
      lds_load_u(Sl + i0 + wf, Sg, ((uint32_t)(sf.y0 + wk.r) * (uint32_t)Wm + (uint32_t)(sf.x0 + wk.c)) * 4u);
    if ((int)threadIdx.x < J.th) {
      const Tap ty = bilinear_tap(J.y0 + threadIdx.x, cm, Hm);
      rtab[threadIdx.x] = make_int4((ty.i0 - sf.y0) * sf.w - sf.x0, (ty.i1 - sf.y0) * sf.w - sf.x0, __float_as_int(ty.w), 0);
    }
  }
  // the partial maxima are read while the staging loads are still in flight
  float m;
  int xs;
  smax_from_parts(sd.s_part, sd.n_cmax_tiles, &m, &xs, sh4, shi4);
  lds_wait();
  __syncthreads();
  const bool flat = !(m > sd.flat_tol);
  // threads map to columns modulo cw, the power of two >= tw (it divides the block), and
  // take nr consecutive tile rows from ya: the horizontal pass of the blur for those rows
  // and the four below stays in registers, so the vertical pass needs no LDS round trip
  const int cw = tw <= 1 ? 1 : 1 << (32 - __clz(tw - 1));
  const int xx = threadIdx.x & (cw - 1);
  constexpr int RPMAX = KTR / (SP_BLOCK / KTW_MAX);   // rows per thread at the widest tile
  const int ng = SP_BLOCK / cw, rp = (J.th + ng - 1) / ng;   // rp <= RPMAX: cw <= KTW_MAX
  const int ya = (int)(threadIdx.x / cw) * rp, nr = min(rp, J.th - ya);
  float hv[RPMAX + 4];
  if (t > 0 && !fmap && xx < tw) {
#pragma unroll
    for (int k = 0; k < RPMAX + 4; ++k)
      if (k < nr + 4) {   // region rows ya .. ya + nr + 3 <= th + 3, all staged
        const float* g = reg + (ya + k) * rs + xx + 2;
        hv[k] = kB0 * g[0] + kB1 * g[1] + kB2 * g[2] + kB1 * g[3] + kB0 * g[4];
      }
  }
  // consecutive lanes take consecutive pixels of a row, so every store of a wavefront
  // covers a contiguous run.  Each thread keeps its column (horizontal tap and border
  // test) and steps down its rows.
  const float eps = sd.eps, rm = flat ? 0.f : 1.f / m;
  const int x = J.x0 + xx;
  const bool xring = x < sd.border || x >= W - sd.border;
  const Tap tx = bilinear_tap(x, cm, Wm);
  const gp<float> unary1p = unary + (size_t)H * W;
#pragma unroll
  for (int k = 0; k < RPMAX; ++k) {
    const int yy = ya + k;
    const int y = J.y0 + yy;
    if (k >= nr || y >= H || xx >= tw || x >= W) continue;
    const bool ring = xring || y < sd.border || y >= H - sd.border;
    float q = 0.5f;
    if (!flat) {
      // the bilinear up-sample of bilinear_lds, with the row offsets from the table
      const int4 rt = rtab[yy];
      const float wy = __int_as_float(rt.z);
      const float* r0 = Sl + rt.x;
      const float* r1 = Sl + rt.y;
      const float top = (1.f - tx.w) * r0[tx.i0] + tx.w * r0[tx.i1];
      const float bot = (1.f - tx.w) * r1[tx.i0] + tx.w * r1[tx.i1];
      const float u = ((1.f - wy) * top + wy * bot) * rm;
      q = fminf(fmaxf(u, eps), 1.f - eps);
    }
    if (ring) q = eps;
    float pi = q;
    const uint32_t ob = ((uint32_t)y * (uint32_t)W + (uint32_t)x) * 4u;
    if (t > 0) {
      const float f = fmap ? *at_bytes(fmap, ob)
                           : kB0 * hv[k] + kB1 * hv[k + 1] + kB2 * hv[k + 2] + kB1 * hv[k + 3] + kB0 * hv[k + 4];
      pi = f + K * (q - f);
      if (ftape) *at_bytes(ftape, ob) = f;
    }
    if (ring) pi = eps;
    st_stream(at_bytes(pnext, ob), pi);
    if (pout) *at_bytes(pout, ob) = pi;
    if (unary) {
      st_stream(at_bytes(unary, ob), unary0(fminf(pi, 1.f - eps)));
      st_stream(at_bytes(unary1p, ob), unary1(fmaxf(pi, eps)));
    }
  }
  if (mstape && J.tid == 0 && threadIdx.x == 0) {
    mstape[0] = m;
    mstape[1] = __int_as_float(xs);
  }
}

// ---------------------------------------------------------------- distance-transform prediction
// f(A, x) = exp(-d(x)^2 / (2 sigma^2)), d the Euclidean distance from x to the nearest
// object pixel of the previous segmentation (or of prior > 1/2 without one).  The search
// radius R has exp(-R^2 / (2 sigma^2)) below FP32's normal range, so a pixel with no object
// within R gets 0 and every other pixel its exact squared distance: a column pass gives the
// distance to the nearest object in the pixel's column within R, a row pass the minimum of
// v(x')^2 + (x - x')^2 over |x - x'| <= R.
constexpr int DT_N = SP_DT_T + 2 * SP_DT_RMAX;
constexpr int DT_W = (DT_N + 31) / 32;   // 32-bit words of a region column or row mask
constexpr int DT_INF = 1 << 30;
__global__ __launch_bounds__(SP_BLOCK) void k_dt(const Job* __restrict__ jobs, const StreamDesc* __restrict__ sds,
                                                 const StepIO* __restrict__ ios, StepIO io0) {
  __shared__ uint32_t cmask[DT_N][DT_W];       // per region column: bit r = object at region row r
  __shared__ uint32_t rmask[SP_DT_T][DT_W];    // per tile row: bit c = an object within R in column c
  __shared__ int vd[SP_DT_T * DT_N];           // squared column distance (or DT_INF) per tile row and region column
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const gp<const uint8_t> seg = G(IOF(seg_prev));
  const gp<const float> pprev = G(IOF(pi_prev));
  const gp<float> fout = G(IOF(f_map));
  const int H = sd.H, W = sd.W, R = sd.dt_r;
  const int nr = J.th + 2 * R, nc = J.tw + 2 * R;
  const int ry0 = J.y0 - R, rx0 = J.x0 - R;
  const int tid = threadIdx.x;
  for (int i = tid; i < DT_N * DT_W; i += SP_BLOCK) (&cmask[0][0])[i] = 0u;
  for (int i = tid; i < SP_DT_T * DT_W; i += SP_BLOCK) (&rmask[0][0])[i] = 0u;
  __syncthreads();
  // the object pixels of the region (outside the frame: none), eight loads in flight per
  // thread (unconditional, from clamped addresses, then selected); the source (segmentation
  // bytes or the previous prior) is chosen outside the loop, so no branch splits a batch
  auto stage = [&](auto is_obj) {
    const int n = nr * nc;
    Walk2 wk(tid, nc);
    for (int i0 = 0; i0 < n; i0 += 8 * SP_BLOCK) {
      int r[8], c[8], in[8], ob[8];
      uint32_t a[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        r[k] = wk.r;
        c[k] = wk.c;
        wk.next();
        const int y = ry0 + r[k], x = rx0 + c[k];
        a[k] = (uint32_t)clampi(y, 0, H - 1) * (uint32_t)W + (uint32_t)clampi(x, 0, W - 1);
        // in the region and in the frame, as an integer (no short-circuit branch)
        in[k] = (int)(i0 + k * SP_BLOCK + tid < n) & (int)((unsigned)y < (unsigned)H) & (int)((unsigned)x < (unsigned)W);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) ob[k] = is_obj(a[k]);   // all eight loads issued before any use
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (in[k] & ob[k]) atomicOr(&cmask[c[k]][r[k] >> 5], 1u << (r[k] & 31));
    }
  };
  if (seg)
    stage([&](uint32_t a) { return (int)(seg[a] != 0); });
  else
    stage([&](uint32_t a) { return (int)(pprev[a] > 0.5f); });
  __syncthreads();
  // column pass: the nearest object row at or above / at or below each tile row, from the
  // column's mask (clz / ctz on the word holding the row, then the words before / after)
  const int R2 = R * R;
  for (int q = tid; q < J.th * nc; q += SP_BLOCK) {
    const int t = q / nc, c = q - t * nc, rr = t + R;
    const int w = rr >> 5, b = rr & 31;
    uint32_t cm[DT_W];
#pragma unroll
    for (int k = 0; k < DT_W; ++k) cm[k] = cmask[c][k];   // all words read together
    const uint32_t lo = b == 31 ? 0xffffffffu : ((2u << b) - 1u), hi = ~((1u << b) - 1u);
    // the highest object row at or above rr (the last nonzero word upward wins) and the
    // lowest at or below (the last nonzero word downward wins), without data-dependent loops
    int up = -DT_INF, dn = DT_INF;
#pragma unroll
    for (int k = 0; k < DT_W; ++k) {
      const uint32_t m = k < w ? cm[k] : (k == w ? cm[k] & lo : 0u);
      up = m ? 32 * k + 31 - __clz(m) : up;
    }
#pragma unroll
    for (int k = DT_W - 1; k >= 0; --k) {
      const uint32_t m = k > w ? cm[k] : (k == w ? cm[k] & hi : 0u);
      dn = m ? 32 * k + __ffs(m) - 1 : dn;
    }
    const int d = min(rr - up, dn - rr);
    const bool near = d <= R;
    vd[t * nc + c] = near ? d * d : DT_INF;
    if (near) atomicOr(&rmask[t][c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  // row pass: min over |k| <= R of vd(x + k) + k^2 (exact squared distance within R), the
  // search skipped when no column within R holds an object
  const float k2 = sd.dt_k;
  Walk2 wk(tid, J.tw);
  for (int i0 = 0; i0 + tid < J.th * J.tw; i0 += SP_BLOCK, wk.next()) {
    const int* row = vd + wk.r * nc + wk.c + R;
    // columns wk.c .. wk.c + 2R of the region (the window around the pixel)
    const int lo = wk.c, hi = wk.c + 2 * R;
    bool any = false;
    for (int k = lo >> 5; k <= hi >> 5; ++k) {
      uint32_t m = rmask[wk.r][k];
      if (k == lo >> 5) m &= ~((1u << (lo & 31)) - 1u);
      if (k == hi >> 5 && (hi & 31) != 31) m &= (2u << (hi & 31)) - 1u;
      any |= m != 0;
    }
    int best = DT_INF;
    if (any) {
      best = row[0];
      for (int k = 1; k <= R && k * k < best; ++k) best = min(best, min(row[-k], row[k]) + k * k);
    }
    const float f = best <= R2 ? __builtin_amdgcn_exp2f((float)best * k2) : 0.f;
    fout[(uint32_t)(J.y0 + wk.r) * (uint32_t)W + (uint32_t)(J.x0 + wk.c)] = f;
  }
}

// Prior of the first frame from manual labels: 1 -> 1, 0 -> eps, anything else -> 0.5.
__global__ __launch_bounds__(SP_BLOCK) void k_manual(const uint8_t* __restrict__ lab, float* __restrict__ pnext,
                                                     float* __restrict__ pout, uint32_t n, float eps) {
  for (uint32_t i = blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += gridDim.x * SP_BLOCK) {
    const uint8_t l = lab[i];
    const float v = l == 1 ? 1.f : (l == 0 ? eps : 0.5f);
    pnext[i] = v;
    if (pout) pout[i] = v;
  }
}

// ---------------------------------------------------------------- MRF capacities
__global__ __launch_bounds__(SP_BLOCK) void k_mrf(const Job* __restrict__ jobs,
                                                  const StreamDesc* __restrict__ sds,
                                                  const StepIO* __restrict__ ios, StepIO io0,
                                                  const float* __restrict__ prior) {
  __shared__ unsigned long long sh[4];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const uint8_t* rgb = IOF(rgb);
  float* unary = IOF(unary);
  float* pairw = IOF(pairwise);
  float* beta_out = IOF(beta_out);
  const int H = sd.H, W = sd.W;
  const float beta = beta_from_parts(sd, sh);
  const int yy = threadIdx.x / 16, xx = threadIdx.x % 16;
  const int y = J.y0 + yy, x = J.x0 + xx;
  if (yy < J.th && xx < J.tw && y < H && x < W) {
    const size_t o = (size_t)y * W + x, plane = (size_t)H * W;
    const float pi = prior[o];
    unary[o] = unary0(fminf(pi, 1.f - sd.eps));
    unary[plane + o] = unary1(fmaxf(pi, sd.eps));
    pairwise_at(rgb, H, W, y, x, cap_consts(beta, sd.lam, sd.potts), pairw, plane);
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

// Recomputed conspicuity maps dotted with the adjoint g_s of each frame (one recorded
// frame per stream of the launch, its buffers named by the stream's StepIO): partial
// sums of g_s * C_k per tile, and C_k at the frame's argmax.
__global__ __launch_bounds__(SP_BLOCK) void k_consp_dot(const Job* __restrict__ jobs,
                                                        const StreamDesc* __restrict__ sds,
                                                        const StepIO* __restrict__ ios) {
  __shared__ float sh4[4];
  __shared__ NParams np[SP_NCH];
  const Job J = jobs[blockIdx.x];
  const StreamDesc& sd = sds[J.stream];
  const StepIO& io = ios[J.stream];
  consp_nparams(sd, np);
  const int cm = sd.c_max, Hm = sd.Hl[cm], Wm = sd.Wl[cm];
  const size_t plane = (size_t)Hm * Wm;
  const int yy = threadIdx.x / CA_T, xx = threadIdx.x % CA_T;
  const int y = J.y0 + yy, x = J.x0 + xx;
  const bool valid = yy < J.th && xx < J.tw && y < Hm && x < Wm;
  const size_t o = (size_t)min(y, Hm - 1) * Wm + min(x, Wm - 1);
  const float g = valid ? io.gs[o] : 0.f;
  const int xs = __float_as_int(io.ms_tape[1]);
  for (int k = 0; k < SP_NCH; ++k) {
    const float Ck = napply(np[k], sd.fbar[k * plane + o]);
    const float tot = block_reduce<OpSum>(valid ? g * Ck : 0.f, sh4);
    if (threadIdx.x == 0) io.dot[(size_t)J.tid * SP_NCH + k] = tot;
    if (valid && (int)o == xs) io.cx[k] = Ck;
  }
}

// Reduction of the per-frame partials and the scalar FP64 sweep over the gains; one
// workgroup per stream (tab[blockIdx.x]; tab null: the single stream `one`).  Every
// stream of a launch ran the same T steps with the same Q and R, so the gains Kd and
// variances Pd are shared.
// One step t (blockIdx.x) of stream blockIdx.y: dL/dK_t from its tile partials, and the
// step's share of dL/dw (zero-weight steps, where max S is flat, have none), each sum in a
// fixed order.  The steps are independent, so they run side by side.
__global__ __launch_bounds__(SP_BLOCK) void k_bwd_step(const BwdFin* __restrict__ tab, BwdFin one, int T,
                                                       float flat_tol) {
  __shared__ double sh256[SP_BLOCK];
  const BwdFin F = tab ? tab[blockIdx.y] : one;
  const int t = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < F.n_lvl0_tiles; i += SP_BLOCK) s += (double)F.gk_part[(size_t)t * F.n_lvl0_tiles + i];
  s = block_sum_d(s, sh256);
  if (threadIdx.x == 0) F.gK[t] = s;
  double A[SP_NCH];
  for (int k = 0; k < SP_NCH; ++k) {
    double a = 0.0;
    for (int i = threadIdx.x; i < F.n_cmax_tiles; i += SP_BLOCK)
      a += (double)F.dot_part[((size_t)t * F.n_cmax_tiles + i) * SP_NCH + k];
    A[k] = block_sum_d(a, sh256);
  }
  const double m = (double)F.ms[2 * t];
  if (threadIdx.x == 0 && m > (double)flat_tol) {
    double Bs = 0.0;
    for (int k = 0; k < SP_NCH; ++k) Bs += (double)F.w[k] * A[k];
    double* gw = F.gK + T + (size_t)t * SP_NCH;
    for (int k = 0; k < SP_NCH; ++k) gw[k] = A[k] / m - (double)F.cx[(size_t)t * SP_NCH + k] * Bs / (m * m);
  }
}

// Per stream (blockIdx.x): dL/dw as the sum of the steps' shares in step order (a thread
// per weight), and the reverse sweep of the scalar gain recursion for dL/dQ and dL/dR
// (FP64, one thread).
__global__ void k_bwd_final(const BwdFin* __restrict__ tab, BwdFin one, int T, const double* __restrict__ Kd,
                            const double* __restrict__ Pd, double Q, double R, float flat_tol) {
  const BwdFin F = tab ? tab[blockIdx.x] : one;
  if ((int)threadIdx.x < SP_NCH) {   // thread k: dL/dw_k over the steps in order
    const int k = threadIdx.x;
    double gw = 0.0;
    for (int t = 0; t < T; ++t)
      if ((double)F.ms[2 * t] > (double)flat_tol) gw += F.gK[T + (size_t)t * SP_NCH + k];
    F.grad_w[k] = (float)gw;
  }
  if (threadIdx.x == 0) {
    double gQ = 0.0, gR = 0.0, gP = 0.0;
    for (int t = T - 1; t >= 1; --t) {
      const double g = F.gK[t] + R * gP;
      gR += Kd[t] * gP;
      const double a = Pd[t - 1] + Q;
      const double den = (a + R) * (a + R);
      const double ga = g * R / den;
      gR -= g * a / den;
      gQ += ga;
      gP = ga;
    }
    gR += gP;
    *F.grad_q = (float)gQ;
    *F.grad_r = (float)gR;
  }
}

// ---------------------------------------------------------------- masked MSE loss helper
// L = mean (prior - mask)^2 over one stream's clip, and dL/dprior; blockIdx.y (or
// blockIdx.x of the final pass) picks the stream's LossIO (tab null: `one`).
__global__ __launch_bounds__(SP_BLOCK) void k_loss(const LossIO* __restrict__ tab, LossIO one) {
  __shared__ float sh4[4];
  const LossIO L = tab ? tab[blockIdx.y] : one;
  const size_t n = (size_t)L.n;
  const float inv_n = (float)(1.0 / (double)n);
  float acc = 0.f;
  const size_t stride = (size_t)gridDim.x * SP_BLOCK;
  const bool quads = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(L.prior) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(L.mask) & 3) == 0 && (reinterpret_cast<uintptr_t>(L.grad) & 15) == 0;
  if (quads) {
    // four consecutive elements per thread: one 16-byte prior load, one 4-byte mask load,
    // one 16-byte gradient store
    typedef float v4f __attribute__((ext_vector_type(4)));
    const gp<const v4f> P4 = G(reinterpret_cast<const v4f*>(L.prior));
    const gp<const uint32_t> M4 = G(reinterpret_cast<const uint32_t*>(L.mask));
    const gp<v4f> G4 = G(reinterpret_cast<v4f*>(L.grad));
    for (size_t q = (size_t)blockIdx.x * SP_BLOCK + threadIdx.x; q < (n >> 2); q += stride) {
      const v4f p = P4[q];
      const uint32_t m = M4[q];
      const float d0 = p.x - (float)(m & 0xffu), d1 = p.y - (float)((m >> 8) & 0xffu);
      const float d2 = p.z - (float)((m >> 16) & 0xffu), d3 = p.w - (float)(m >> 24);
      acc += d0 * d0;
      acc += d1 * d1;
      acc += d2 * d2;
      acc += d3 * d3;
      if (L.grad) {
        v4f g;
        g.x = 2.f * d0 * inv_n;
        g.y = 2.f * d1 * inv_n;
        g.z = 2.f * d2 * inv_n;
        g.w = 2.f * d3 * inv_n;
        G4[q] = g;
      }
    }
  } else {
    for (size_t i = (size_t)blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += stride) {
      const float d = L.prior[i] - (float)L.mask[i];
      acc += d * d;
      if (L.grad) L.grad[i] = 2.f * d * inv_n;
    }
  }
  acc = block_reduce<OpSum>(acc, sh4);
  if (threadIdx.x == 0) L.part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(SP_BLOCK) void k_loss_final(const LossIO* __restrict__ tab, LossIO one, int nblk) {
  __shared__ double sh256[SP_BLOCK];
  const LossIO L = tab ? tab[blockIdx.x] : one;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += SP_BLOCK) s += (double)L.part[i];
  s = block_sum_d(s, sh256);
  if (threadIdx.x == 0) *L.loss = (float)(s / (double)L.n);
}

// ---------------------------------------------------------------- batched step bookkeeping
// Start of a step for stream i: its inputs, Kalman gain (FP64) and prior buffers.
__device__ void batch_begin_stream(int i, BatchState* __restrict__ st, const StreamDesc* __restrict__ sds,
                                   const uint8_t* const* __restrict__ in_ptrs, StepIO* __restrict__ ios, double Q,
                                   double R) {
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
  StepIO* io = ios + i;
  const uint8_t* cur = in_ptrs[i];
  io->rgb = cur;
  io->rgb_prev = (s.t == 0) ? nullptr : s.last_rgb;
  io->S_out = s.S;
  io->C_out = s.C;
  io->S_in = s.S;
  io->seg_prev = nullptr;
  io->pi_prev = s.cur ? s.pi[1] : s.pi[0];
  io->pi_next = s.cur ? s.pi[0] : s.pi[1];
  if (s.t < s.tape_cap) {
    // recorded step: level c_min goes straight to its checkpoint slot; S, f, (max S,
    // argmax) and the prior are kept for the adjoint
    const StreamDesc& sd = sds[i];
    const size_t k = (size_t)s.t, hw = (size_t)sd.H * sd.W;
    io->ckpt = s.tape_ckpt + k * 4 * (size_t)sd.Hl[sd.c_min] * sd.Wl[sd.c_min];
    io->S_tape = s.tape_S + k * (size_t)sd.Hl[sd.c_max] * sd.Wl[sd.c_max];
    io->f_tape = s.tape_f + k * hw;
    io->ms_tape = s.tape_ms + 2 * k;
    io->prior_out = s.tape_pi + k * hw;
  } else {
    io->ckpt = nullptr;
    io->S_tape = nullptr;
    io->f_tape = nullptr;
    io->ms_tape = nullptr;
    io->prior_out = nullptr;
  }
  io->unary = s.unary;
  io->pairwise = s.pairwise;
  io->beta_out = s.beta;
  io->f_map = nullptr;
  io->ssm_prev = nullptr;
  io->ssm_next = nullptr;
  io->Ks = 0.f;
  io->K = (float)K;
  io->t = (int32_t)(s.t < 0x7fffffff ? s.t : 0x7fffffff);
  s.t += 1;
  s.P = P;
  s.cur ^= 1;
  s.last_rgb = cur;
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
  const float* src = st[s].cur ? st[s].pi[1] : st[s].pi[0];
  float* dst = out[s];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------- counter calibration
// Copies n16 16-byte units from src to dst in one of the access forms the kernels use, so
// that the HBM byte counters can be read against a known number of bytes: 0 = a 4-byte
// load and store per lane, 1 = a 16-byte load and store per lane, 2 = 4-byte direct
// global->LDS loads of a 1 KB slice per wavefront, then 4-byte stores from LDS.
__global__ __launch_bounds__(SP_BLOCK) void k_calib(const float* __restrict__ src, float* __restrict__ dst,
                                                    size_t n16, int mode) {
  __shared__ float buf[SP_BLOCK * 4];
  const size_t nf = n16 * 4;
  const gp<const float> gs = G(src);
  const gp<float> gd = G(dst);
  if (mode == 1) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const gp<const v4f> s4 = (gp<const v4f>)gs;
    const gp<v4f> d4 = (gp<v4f>)gd;
    for (size_t i = (size_t)blockIdx.x * SP_BLOCK + threadIdx.x; i < n16; i += (size_t)gridDim.x * SP_BLOCK)
      d4[i] = s4[i];
  } else if (mode == 0) {
    for (size_t i = (size_t)blockIdx.x * SP_BLOCK + threadIdx.x; i < nf; i += (size_t)gridDim.x * SP_BLOCK)
      gd[i] = gs[i];
  } else {
    // each wavefront stages 4 x 64 floats (4 loads of 256 bytes) per round
    const int wf = wave_first(), lane = lane_id();
    const size_t chunk = (size_t)SP_BLOCK * 4;
    for (size_t b0 = (size_t)blockIdx.x * chunk; b0 < nf; b0 += (size_t)gridDim.x * chunk) {
      const size_t w0 = b0 + (size_t)wf * 4;
      if (w0 + 4 * 64 <= nf) {
#pragma unroll
        for (int k = 0; k < 4; ++k) lds_load_u(buf + wf * 4 + k * 64, gs, (uint32_t)((w0 + k * 64 + lane) * 4u));
        lds_wait();
#pragma unroll
        for (int k = 0; k < 4; ++k) gd[w0 + k * 64 + lane] = buf[wf * 4 + k * 64 + lane];
      } else {
        for (size_t i = w0 + lane; i < nf && i < w0 + 4 * 64; i += 64) gd[i] = gs[i];
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
static inline hipError_t chk() { return hipGetLastError(); }

hipError_t sp_launch(int kind, const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios,
                     const StepIO* io0, int flag, const float* aux, hipStream_t st, size_t lds) {
  if (n <= 0) return hipSuccess;
  const dim3 g(n), b(SP_BLOCK);
  StepIO z{};
  const StepIO& io = io0 ? *io0 : z;
  switch (kind) {
    case JOB_RGB: hipLaunchKernelGGL(k_rgb, g, b, 0, st, jobs, sds, ios, io, flag, BatchBegin{}); break;
    case JOB_FEAT: hipLaunchKernelGGL((k_feat<16, 16>), g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_DOWN:   // pyramid launch without tail jobs (DOWN and GABOR jobs)
    case JOB_GABOR:   // flag: the Gabor radius of the launch
      if (flag == 6)
        hipLaunchKernelGGL((k_pyr<false, 6>), g, b, 0, st, jobs, sds, ios, io);
      else
        hipLaunchKernelGGL((k_pyr<false, 0>), g, b, 0, st, jobs, sds, ios, io);
      break;
    case JOB_TAIL:
      if (flag == 6)
        hipLaunchKernelGGL((k_pyr<true, 6>), g, b, 0, st, jobs, sds, ios, io);
      else
        hipLaunchKernelGGL((k_pyr<true, 0>), g, b, 0, st, jobs, sds, ios, io);
      break;
    case JOB_CSSTATS: hipLaunchKernelGGL(k_csstats, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_CSFINAL: hipLaunchKernelGGL(k_csfinal, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_CSG: {   // flag: channels per workgroup | pair set << 8
      const int nc = flag & 0xff, set = flag >> 8;
      if (set == 1) {
        if (nc == 8)
          hipLaunchKernelGGL((k_csg1<8>), g, b, lds, st, jobs, sds, ios, io);
        else if (nc == 4)
          hipLaunchKernelGGL((k_csg1<4>), g, b, lds, st, jobs, sds, ios, io);
        else if (nc == 2)
          hipLaunchKernelGGL((k_csg1<2>), g, b, lds, st, jobs, sds, ios, io);
        else
          hipLaunchKernelGGL((k_csg1<1>), g, b, lds, st, jobs, sds, ios, io);
      } else {
        if (nc == 8)
          hipLaunchKernelGGL((k_csg<8, 0>), g, b, lds, st, jobs, sds, ios, io);
        else if (nc == 4)
          hipLaunchKernelGGL((k_csg<4, 0>), g, b, lds, st, jobs, sds, ios, io);
        else if (nc == 2)
          hipLaunchKernelGGL((k_csg<2, 0>), g, b, lds, st, jobs, sds, ios, io);
        else
          hipLaunchKernelGGL((k_csg<1, 0>), g, b, lds, st, jobs, sds, ios, io);
      }
      break;
    }
    case JOB_CSMIX: hipLaunchKernelGGL(k_csmix, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_CSAPPLY:   // flag: channels per workgroup
      if (flag == 8)
        hipLaunchKernelGGL(k_csapply<8>, g, b, lds, st, jobs, sds, ios, io);
      else if (flag == 4)
        hipLaunchKernelGGL(k_csapply<4>, g, b, lds, st, jobs, sds, ios, io);
      else if (flag == 2)
        hipLaunchKernelGGL(k_csapply<2>, g, b, lds, st, jobs, sds, ios, io);
      else
        hipLaunchKernelGGL(k_csapply<1>, g, b, lds, st, jobs, sds, ios, io);
      break;
    case JOB_CONSP: hipLaunchKernelGGL(k_consp, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_SMAX: hipLaunchKernelGGL(k_smax, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_KALMAN: hipLaunchKernelGGL(k_kalman, g, b, 0, st, jobs, sds, ios, io); break;
    case JOB_MRF: hipLaunchKernelGGL(k_mrf, g, b, 0, st, jobs, sds, ios, io, aux); break;
    case JOB_DT: hipLaunchKernelGGL(k_dt, g, b, 0, st, jobs, sds, ios, io); break;
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

hipError_t sp_launch_consp_dot(const Job* jobs, int n, const StreamDesc* sds, const StepIO* ios, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_consp_dot, dim3(n), dim3(SP_BLOCK), 0, st, jobs, sds, ios);
  return chk();
}

hipError_t sp_launch_bwd_final(const BwdFin* tab, const BwdFin* one, int n_streams, int T, const double* Kd,
                               const double* Pd, double Q, double R, float flat_tol, hipStream_t st) {
  if (n_streams <= 0) return hipSuccess;
  if (T <= 0) return hipErrorInvalidValue;
  BwdFin z{};
  const BwdFin& o = one ? *one : z;
  hipLaunchKernelGGL(k_bwd_step, dim3(T, n_streams), dim3(SP_BLOCK), 0, st, tab, o, T, flat_tol);
  hipError_t e = chk();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bwd_final, dim3(n_streams), dim3(64), 0, st, tab, o, T, Kd, Pd, Q, R, flat_tol);
  return chk();
}

hipError_t sp_launch_loss(const LossIO* tab, const LossIO* one, int n_streams, int nblk, hipStream_t st) {
  if (n_streams <= 0) return hipSuccess;
  LossIO z{};
  const LossIO& o = one ? *one : z;
  hipLaunchKernelGGL(k_loss, dim3(nblk, n_streams), dim3(SP_BLOCK), 0, st, tab, o);
  hipError_t e = chk();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(n_streams), dim3(SP_BLOCK), 0, st, tab, o, nblk);
  return chk();
}

hipError_t sp_launch_batch_rgb(const Job* jobs, int n_jobs, const StreamDesc* sds, StepIO* ios, int want_d2,
                               const BatchBegin& bb, hipStream_t stream) {
  hipLaunchKernelGGL(k_rgb, dim3(n_jobs), dim3(SP_BLOCK), 0, stream, jobs, sds, ios, StepIO{}, want_d2, bb);
  return chk();
}

void sp_batch_rgb_node_params(RgbNodeArgs* a, int n_jobs, hipKernelNodeParams* p) {
  a->argv[0] = &a->jobs;
  a->argv[1] = &a->sds;
  a->argv[2] = &a->ios;
  a->argv[3] = &a->io0;
  a->argv[4] = &a->want_d2;
  a->argv[5] = &a->bb;
  *p = hipKernelNodeParams{};
  p->func = reinterpret_cast<void*>(&k_rgb);
  p->gridDim = dim3(n_jobs);
  p->blockDim = dim3(SP_BLOCK);
  p->sharedMemBytes = 0;
  p->kernelParams = a->argv;
  p->extra = nullptr;
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

hipError_t sp_csapply_reserve_lds(size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  const void* fns[12] = {reinterpret_cast<const void*>(&k_csapply<1>), reinterpret_cast<const void*>(&k_csapply<2>),
                         reinterpret_cast<const void*>(&k_csapply<4>), reinterpret_cast<const void*>(&k_csapply<8>),
                         reinterpret_cast<const void*>(&k_csg<1, 0>),  reinterpret_cast<const void*>(&k_csg<2, 0>),
                         reinterpret_cast<const void*>(&k_csg<4, 0>),  reinterpret_cast<const void*>(&k_csg<8, 0>),
                         reinterpret_cast<const void*>(&k_csg1<1>),    reinterpret_cast<const void*>(&k_csg1<2>),
                         reinterpret_cast<const void*>(&k_csg1<4>),    reinterpret_cast<const void*>(&k_csg1<8>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t sp_launch_manual(const uint8_t* labels, float* pnext, float* pout, size_t n, float eps, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + SP_BLOCK - 1) / SP_BLOCK, 4096);
  hipLaunchKernelGGL(k_manual, dim3(blocks), dim3(SP_BLOCK), 0, st, labels, pnext, pout, (uint32_t)n, eps);
  return chk();
}

hipError_t sp_launch_calib(const float* src, float* dst, size_t n16, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_calib, dim3(2048), dim3(SP_BLOCK), 0, st, src, dst, n16, mode);
  return chk();
}


// ---------------------------------------------------------------- allocation-free scratch
// Device memory of the allocation-free saliency entry point: a file-scope array that every
// GPU the library runs on holds from the library's load until the process ends.  Its name
// in host code is only a host-side stand-in, never a device address: host code uses the
// address hipGetSymbolAddress returns, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SP_NOALLOC_BYTES];

hipError_t sp_noalloc_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[SP_NOALLOC_DEVICES] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SP_NOALLOC_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!a) return hipErrorInvalidSymbol;
    addr[dev] = a;
  }
  *ptr = addr[dev];
  return hipSuccess;
}
