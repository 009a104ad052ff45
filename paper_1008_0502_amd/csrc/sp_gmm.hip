// Colour likelihood of the t-links (Section 4: psi_1 = -log p(C | A) with p(C | A) a
// Gaussian mixture over RGB fitted by EM; Section 5: every pixel is a sample, weighted by
// the prior p(A = 1) for the object and by 1 - p for the background; Section 8.1: M = 3).
//
// Per label and iteration: one pass over tiles of SP_GMM_TILE pixels takes the E-step under
// the current mixtures (read as scalars) and accumulates, for every component, the
// responsibility-weighted count and the first and second moments about the component's
// mean (FP32 per thread, FP64 from the workgroup sum on, one partial per workgroup); one
// workgroup then reduces the partials in a fixed order and fits the new weights, means and
// covariances, their inverses and log-normalisers in FP64, one thread per label and
// component.  The start is the weighted mean and covariance of each label's samples with
// the means spread along the covariance's leading eigenvector.  A final pass adds psi_1 of
// both labels to the unary costs.
// The pixel passes read 7 bytes per pixel.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <algorithm>

#include "sp_internal.h"
#include "sp_kernels.h"
#include "sp_device.h"

namespace {

constexpr int GPX = SP_GMM_TILE / SP_BLOCK;   // pixels per thread of an accumulation tile
constexpr float kInv255 = 1.f / 255.f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr double kLog2Pi = 1.8378770664093453;

__device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

// Squared Mahalanobis distance d' P d with P stored as (xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ float quad(const float* P, float dx, float dy, float dz) {
  const float a = P[0] * dx * dx + P[3] * dy * dy + P[5] * dz * dz;
  const float b = P[1] * dx * dy + P[2] * dx * dz + P[4] * dy * dz;
  return fmaf(2.f, b, a);
}

// Moments of one sample with weight wr about the centre: count, first (3) and second (6).
__device__ __forceinline__ void add_moments(float* a, float wr, float dx, float dy, float dz) {
  a[0] += wr;
  const float ux = wr * dx, uy = wr * dy, uz = wr * dz;
  a[1] += ux;
  a[2] += uy;
  a[3] += uz;
  a[4] = fmaf(ux, dx, a[4]);
  a[5] = fmaf(ux, dy, a[5]);
  a[6] = fmaf(ux, dz, a[6]);
  a[7] = fmaf(uy, dy, a[7]);
  a[8] = fmaf(uy, dz, a[8]);
  a[9] = fmaf(uz, dz, a[9]);
}

// The mixtures as the pixel loops use them, in scalar registers (read from LDS once).
__device__ __forceinline__ float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
template <int NC>
struct Mix {
  float mu[2][NC][3], P[2][NC][6], ln[2][NC];
  bool on[2][NC], lab[2];
  __device__ __forceinline__ void load(const GmmState& S) {
#pragma unroll
    for (int L = 0; L < 2; ++L) {
      lab[L] = __builtin_amdgcn_readfirstlane(S.label_on[L]) != 0;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const GmmComp& g = S.comp[L][m];
        on[L][m] = __builtin_amdgcn_readfirstlane(g.on) != 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) mu[L][m][i] = uni(g.mu[i]);
#pragma unroll
        for (int i = 0; i < 6; ++i) P[L][m][i] = uni(g.P[i]);
        ln[L][m] = uni(g.lnorm);
      }
    }
  }
  // log(alpha_m N(c; mu_m, Sigma_m)) of label L's components, -inf for a dropped one
  __device__ __forceinline__ void logp(int L, float cx, float cy, float cz, float (&lp)[NC], float& mx) const {
    mx = -INFINITY;
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      lp[m] = on[L][m] ? ln[L][m] - 0.5f * quad(P[L][m], cx - mu[L][m][0], cy - mu[L][m][1], cz - mu[L][m][2])
                       : -INFINITY;
      mx = fmaxf(mx, lp[m]);
    }
  }
};

// The workgroup's tile of pixels, held in registers: colours in [0, 1] and the prior.
struct Tile {
  float c[GPX][3];
  float pi[GPX];
};

__device__ __forceinline__ void load_tile(const GmmIO& io, Tile& T) {
  const gp<const uint8_t> rgb = G(io.rgb);
  const gp<const float> prior = G(io.prior);
  const uint32_t base = blockIdx.x * SP_GMM_TILE;
#pragma unroll
  for (int k = 0; k < GPX; ++k) {
    const uint32_t i = min(base + k * SP_BLOCK + threadIdx.x, (uint32_t)io.n - 1u);   // past the end: not used
    T.c[k][0] = (float)rgb[3 * i] * kInv255;
    T.c[k][1] = (float)rgb[3 * i + 1] * kInv255;
    T.c[k][2] = (float)rgb[3 * i + 2] * kInv255;
    T.pi[k] = prior[i];
  }
}

// Moments of the tile into the partial slot of the workgroup.  EM = false: the start's
// moments of both labels about (0.5, 0.5, 0.5); EM = true: the E-step under the mixtures S
// and the moments of every component about its mean.  Each thread accumulates its pixels in
// FP32; the workgroup sum goes through LDS transposed: value v's 256 thread sums are split
// into SEG interleaved segments, each summed in FP64 by one thread with four accumulators
// in a fixed order, and the segments are added in order.
template <int M, bool EM>
__device__ __forceinline__ void tile_moments(const GmmIO& io, const Tile& T, const GmmState& S) {
  constexpr int NC = EM ? M : 1;
  constexpr int NV = 2 * NC * 10;
  constexpr int SEG = SP_BLOCK / NV >= 8 ? 8 : (SP_BLOCK / NV >= 4 ? 4 : 2);
  constexpr int PER = SP_BLOCK / SEG;
  __shared__ float tr[NV][SP_BLOCK + 1];
  __shared__ double segs[NV][SEG];
  float acc[2][NC][10];
#pragma unroll
  for (int L = 0; L < 2; ++L)
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int v = 0; v < 10; ++v) acc[L][m][v] = 0.f;
  Mix<NC> X;
  if (EM) X.load(S);
  const uint32_t base = blockIdx.x * SP_GMM_TILE;
#pragma unroll
  for (int k = 0; k < GPX; ++k) {
    if (base + k * SP_BLOCK + threadIdx.x >= (uint32_t)io.n) continue;
    const float cx = T.c[k][0], cy = T.c[k][1], cz = T.c[k][2];
    const float w[2] = {1.f - T.pi[k], T.pi[k]};
#pragma unroll
    for (int L = 0; L < 2; ++L) {
      if (!EM) {
        add_moments(acc[L][0], w[L], cx - 0.5f, cy - 0.5f, cz - 0.5f);
        continue;
      }
      if (!X.lab[L]) continue;
      float lp[NC], mx;
      X.logp(L, cx, cy, cz, lp, mx);
      float r[NC], sum = 0.f;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        r[m] = X.on[L][m] ? ex(lp[m] - mx) : 0.f;
        sum += r[m];
      }
      const float ws = w[L] / sum;
#pragma unroll
      for (int m = 0; m < NC; ++m)
        if (X.on[L][m])
          add_moments(acc[L][m], ws * r[m], cx - X.mu[L][m][0], cy - X.mu[L][m][1], cz - X.mu[L][m][2]);
    }
  }
#pragma unroll
  for (int L = 0; L < 2; ++L)
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int v = 0; v < 10; ++v) tr[(L * NC + m) * 10 + v][threadIdx.x] = acc[L][m][v];
  __syncthreads();
  if ((int)threadIdx.x < NV * SEG) {
    const int v = threadIdx.x / SEG, sg = threadIdx.x % SEG;
    const float* row = tr[v] + sg;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < PER; ++j) a[j & 3] += (double)row[j * SEG];
    segs[v][sg] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double t = 0.0;
#pragma unroll
    for (int sg = 0; sg < SEG; ++sg) t += segs[threadIdx.x][sg];
    io.part_out[(size_t)threadIdx.x * io.ntiles + blockIdx.x] = t;
  }
}

// Symmetric 3x3 (xx, xy, xz, yy, yz, zz): determinant and inverse by cofactors.
__device__ __forceinline__ double sym_inverse(const double* A, double* I) {
  const double c00 = A[3] * A[5] - A[4] * A[4], c01 = A[2] * A[4] - A[1] * A[5], c02 = A[1] * A[4] - A[2] * A[3];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double id = 1.0 / det;
  I[0] = c00 * id;
  I[1] = c01 * id;
  I[2] = c02 * id;
  I[3] = (A[0] * A[5] - A[2] * A[2]) * id;
  I[4] = (A[1] * A[2] - A[0] * A[4]) * id;
  I[5] = (A[0] * A[3] - A[1] * A[1]) * id;
  return det;
}

// Positive definite by its leading principal minors.
__device__ __forceinline__ bool sym_pd(const double* A) {
  const double m2 = A[0] * A[3] - A[1] * A[1];
  const double det = A[0] * (A[3] * A[5] - A[4] * A[4]) - A[1] * (A[1] * A[5] - A[4] * A[2]) +
                     A[2] * (A[1] * A[4] - A[3] * A[2]);
  return A[0] > 0.0 && m2 > 0.0 && det > 0.0 && isfinite(det);
}

__device__ __forceinline__ void set_comp(GmmState& st, int L, int m, double alpha) {
  GmmComp& g = st.comp[L][m];
  double P[6];
  const double det = sym_inverse(st.cov[L][m], P);
  for (int i = 0; i < 3; ++i) g.mu[i] = (float)st.mu[L][m][i];
  for (int i = 0; i < 6; ++i) g.P[i] = (float)P[i];
  g.lnorm = (float)(log(alpha) - 0.5 * log(det) - 1.5 * kLog2Pi);
  g.on = 1;
}

// The partial moments of every tile reduced in a fixed order: wavefront v % 4 takes value
// v, lane t sums tiles t, t+64, ... in increasing order, then the wavefront sum.  The
// loads of all the wavefront's values and of five tiles per lane are in flight together.
template <int NV>
__device__ __forceinline__ void reduce_parts(const double* __restrict__ part, int ntiles, double* sums) {
  constexpr int VPW = (NV + 3) / 4, TB = 5;
  const int lane = lane_id(), wv = wave_id();
  const gp<const double> pp = G(part);
  double acc[VPW];
#pragma unroll
  for (int b = 0; b < VPW; ++b) acc[b] = 0.0;
  for (int t0 = 0; t0 < ntiles; t0 += 64 * TB) {
    double x[VPW][TB];
#pragma unroll
    for (int b = 0; b < VPW; ++b)
#pragma unroll
      for (int k = 0; k < TB; ++k) {
        const int v = wv + 4 * b, t = t0 + 64 * k + lane;
        x[b][k] = (v < NV && t < ntiles) ? pp[(size_t)v * ntiles + t] : 0.0;
      }
#pragma unroll
    for (int b = 0; b < VPW; ++b)
#pragma unroll
      for (int k = 0; k < TB; ++k) acc[b] += x[b][k];
  }
#pragma unroll
  for (int b = 0; b < VPW; ++b) {
    const double t = wave_sum_d(acc[b]);
    if (lane == 0 && wv + 4 * b < NV) sums[wv + 4 * b] = t;
  }
}

// The mixtures of both labels from the reduced moments, into S (LDS), by threads
// q = L * M + m.  FIRST: the start (per label the weighted mean and covariance, the
// leading eigenvector by 64 power steps from (1, 1, 1) / sqrt 3, means spread along it);
// else the M-step from the previous mixtures P (moments taken about P's means).
template <int M, bool FIRST>
__device__ __forceinline__ void fit(const double* sums, const GmmState& P, GmmState& S, float reg, int n) {
  constexpr int NC = FIRST ? 1 : M;
  __shared__ double ax[2][12];   // FIRST: per label d (3), S (6), v (3) after the power steps
  __shared__ double lam_s[2];
  __shared__ double nm[2][SP_GMM_MAXM];
  const int q = threadIdx.x;
  if (FIRST) {
    if (q < 2) {
      const int L = q;
      const double* a = sums + L * 10;
      const double W0 = a[0];
      S.label_on[L] = W0 > 1e-12 * (double)n ? 1 : 0;
      if (S.label_on[L]) {
        const double d[3] = {a[1] / W0, a[2] / W0, a[3] / W0};
        const double C[6] = {a[4] / W0 - d[0] * d[0], a[5] / W0 - d[0] * d[1], a[6] / W0 - d[0] * d[2],
                             a[7] / W0 - d[1] * d[1], a[8] / W0 - d[1] * d[2], a[9] / W0 - d[2] * d[2]};
        // 64 normalised power steps from v0 = (1, 1, 1) / sqrt 3 give C^64 v0 / |C^64 v0|: C^64
        // by six squarings (each scaled by its largest entry), then one product.  For a
        // symmetric C, C v0 = 0 is the only way the steps stop early, and then v stays v0.
        double A[6] = {C[0], C[1], C[2], C[3], C[4], C[5]};
        for (int it = 0; it < 6; ++it) {
          const double B[6] = {A[0] * A[0] + A[1] * A[1] + A[2] * A[2], A[0] * A[1] + A[1] * A[3] + A[2] * A[4],
                               A[0] * A[2] + A[1] * A[4] + A[2] * A[5], A[1] * A[1] + A[3] * A[3] + A[4] * A[4],
                               A[1] * A[2] + A[3] * A[4] + A[4] * A[5], A[2] * A[2] + A[4] * A[4] + A[5] * A[5]};
          double big = 0.0;
          for (int i = 0; i < 6; ++i) big = fmax(big, fabs(B[i]));
          const double sc = big > 0.0 ? 1.0 / big : 0.0;
          for (int i = 0; i < 6; ++i) A[i] = B[i] * sc;
        }
        double v[3] = {0.5773502691896258, 0.5773502691896258, 0.5773502691896258};
        {
          const double u0 = (A[0] * v[0] + A[1] * v[1] + A[2] * v[2]);
          const double u1 = (A[1] * v[0] + A[3] * v[1] + A[4] * v[2]);
          const double u2 = (A[2] * v[0] + A[4] * v[1] + A[5] * v[2]);
          const double nn = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
          const bool moves = (C[0] * v[0] + C[1] * v[1] + C[2] * v[2]) != 0.0 || (C[1] * v[0] + C[3] * v[1] + C[4] * v[2]) != 0.0 ||
                             (C[2] * v[0] + C[4] * v[1] + C[5] * v[2]) != 0.0;
          if (moves && nn > 0.0) {
            v[0] = u0 / nn;
            v[1] = u1 / nn;
            v[2] = u2 / nn;
          }
        }
        int k = 0;
        for (int i = 1; i < 3; ++i)
          if (fabs(v[i]) > fabs(v[k])) k = i;
        if (v[k] < 0) v[0] = -v[0], v[1] = -v[1], v[2] = -v[2];
        const double Sv0 = C[0] * v[0] + C[1] * v[1] + C[2] * v[2];
        const double Sv1 = C[1] * v[0] + C[3] * v[1] + C[4] * v[2];
        const double Sv2 = C[2] * v[0] + C[4] * v[1] + C[5] * v[2];
        lam_s[L] = v[0] * Sv0 + v[1] * Sv1 + v[2] * Sv2;
        for (int i = 0; i < 3; ++i) ax[L][i] = d[i];
        for (int i = 0; i < 6; ++i) ax[L][3 + i] = C[i];
        for (int i = 0; i < 3; ++i) ax[L][9 + i] = v[i];
      }
    }
    __syncthreads();
    if (q < 2 * M) {
      const int L = q / M, m = q % M;
      S.alpha[L][m] = 0.0;
      S.comp[L][m].on = 0;
      if (S.label_on[L]) {
        const double sl = sqrt(fmax(lam_s[L], 0.0));
        const double z = M == 1 ? 0.0 : (m == M - 1 ? 1.0 : m * (2.0 / (M - 1)) - 1.0);
        for (int i = 0; i < 3; ++i) S.mu[L][m][i] = 0.5 + ax[L][i] + z * sl * ax[L][9 + i];
        for (int i = 0; i < 6; ++i) S.cov[L][m][i] = ax[L][3 + i] + ((i == 0 || i == 3 || i == 5) ? (double)reg : 0.0);
        S.alpha[L][m] = 1.0 / M;
        if (sym_pd(S.cov[L][m]))
          set_comp(S, L, m, S.alpha[L][m]);
        else
          S.alpha[L][m] = 0.0;
      }
    }
  } else {
    if (q < 2 * M) {
      const int L = q / M, m = q % M;
      // a component that drops out keeps its mean and covariance
      for (int i = 0; i < 3; ++i) S.mu[L][m][i] = P.mu[L][m][i];
      for (int i = 0; i < 6; ++i) S.cov[L][m][i] = P.cov[L][m][i];
      S.alpha[L][m] = P.alpha[L][m];
      S.comp[L][m] = P.comp[L][m];
      if (m == 0) S.label_on[L] = P.label_on[L];
      nm[L][m] = 0.0;
      if (P.label_on[L]) {
        double W0 = 0.0;
        for (int j = 0; j < M; ++j) W0 += sums[(L * NC + j) * 10];
        const double* a = sums + (L * NC + m) * 10;
        const double N = a[0];
        const GmmComp& g = P.comp[L][m];
        if (g.on && N > 1e-12 * W0) {
          const double d[3] = {a[1] / N, a[2] / N, a[3] / N};
          double C[6] = {a[4] / N - d[0] * d[0], a[5] / N - d[0] * d[1], a[6] / N - d[0] * d[2],
                         a[7] / N - d[1] * d[1], a[8] / N - d[1] * d[2], a[9] / N - d[2] * d[2]};
          C[0] += reg;
          C[3] += reg;
          C[5] += reg;
          if (sym_pd(C)) {
            for (int i = 0; i < 3; ++i) S.mu[L][m][i] = (double)g.mu[i] + d[i];
            for (int i = 0; i < 6; ++i) S.cov[L][m][i] = C[i];
            nm[L][m] = N;
          }
        }
      }
    }
    __syncthreads();
    if (q < 2 * M) {
      const int L = q / M, m = q % M;
      if (P.label_on[L]) {
        double tot = 0.0;
        for (int j = 0; j < M; ++j) tot += nm[L][j];
        S.alpha[L][m] = tot > 0 ? nm[L][m] / tot : 0.0;
        if (S.alpha[L][m] > 0.0)
          set_comp(S, L, m, S.alpha[L][m]);
        else
          S.comp[L][m].on = 0;
      }
    }
  }
  __syncthreads();
}

// Workgroup 0 publishes the mixtures (the next launch's P, and the caller's copy).
template <int M>
__device__ __forceinline__ void publish(const GmmState& S, GmmState* out_st, float* out) {
  if (blockIdx.x != 0) return;
  const int* src = reinterpret_cast<const int*>(&S);
  int* dst = reinterpret_cast<int*>(out_st);
  for (int i = threadIdx.x; i < (int)(sizeof(GmmState) / sizeof(int)); i += SP_BLOCK) dst[i] = src[i];
  const int q = threadIdx.x;
  if (out && q < 2 * M) {
    const int L = q / M, m = q % M;
    float* o = out + ((size_t)L * M + m) * 10;
    const bool live = S.label_on[L] && S.alpha[L][m] > 0.0;
    o[0] = live ? (float)S.alpha[L][m] : 0.f;
    for (int i = 0; i < 3; ++i) o[1 + i] = live ? (float)S.mu[L][m][i] : 0.f;
    for (int i = 0; i < 6; ++i) o[4 + i] = live ? (float)S.cov[L][m][i] : 0.f;
  }
}

// The moments of every tile: the start's (EM = false) or the E-step's under the mixtures
// fitted by the previous launch (read from global memory into scalar registers).
template <int M, bool EM>
__global__ __launch_bounds__(SP_BLOCK) void k_gmm_acc(GmmIO io) {
  Tile T;
  load_tile(io, T);
  tile_moments<M, EM>(io, T, *io.st_prev);
}

// The previous mixtures copied into LDS (loads issued ahead of the reduction).
__device__ __forceinline__ void load_prev(const GmmState* src, GmmState& P) {
  const gp<const int> s = G(reinterpret_cast<const int*>(src));
  int* d = reinterpret_cast<int*>(&P);
  for (int i = threadIdx.x; i < (int)(sizeof(GmmState) / sizeof(int)); i += SP_BLOCK) d[i] = s[i];
}

// One workgroup: the tiles' moments reduced in a fixed order, then the start (FIRST) or the
// M-step, stored for the next launch (and the caller's copy).
template <int M, bool FIRST>
__global__ __launch_bounds__(SP_BLOCK) void k_gmm_fit(GmmIO io) {
  constexpr int NVI = 2 * (FIRST ? 1 : M) * 10;
  __shared__ double sums[NVI];
  __shared__ GmmState S, P;
  if (!FIRST) load_prev(io.st_prev, P);
  reduce_parts<NVI>(io.part_in, io.ntiles, sums);
  __syncthreads();
  fit<M, FIRST>(sums, P, S, io.reg, io.n);
  publish<M>(S, io.st_next, io.out);
}

// psi_1 = -log sum_m alpha_m N(c; mu_m, Sigma_m) added to the unary cost of its label.
template <int M>
__global__ __launch_bounds__(SP_BLOCK) void k_gmm_psi(GmmIO io) {
  Tile T;
  load_tile(io, T);
  Mix<M> X;
  X.load(*io.st_prev);
  const gp<float> un = G(io.unary);
  const uint32_t base = blockIdx.x * SP_GMM_TILE;
#pragma unroll
  for (int k = 0; k < GPX; ++k) {
    const uint32_t i = base + k * SP_BLOCK + threadIdx.x;
    if (i >= (uint32_t)io.n) continue;
    const float cx = T.c[k][0], cy = T.c[k][1], cz = T.c[k][2];
#pragma unroll
    for (int L = 0; L < 2; ++L) {
      if (!X.lab[L]) continue;
      float lp[M], mx;
      X.logp(L, cx, cy, cz, lp, mx);
      if (!(mx > -INFINITY)) continue;
      float sum = 0.f;
#pragma unroll
      for (int m = 0; m < M; ++m) sum += X.on[L][m] ? ex(lp[m] - mx) : 0.f;
      const uint32_t o = (uint32_t)L * (uint32_t)io.n + i;
      un[o] = un[o] - (mx + lg(sum));
    }
  }
}

template <int M>
hipError_t launch_m(int phase, const GmmIO& io, hipStream_t st) {
  const dim3 grid(io.ntiles), block(SP_BLOCK);
  switch (phase) {
    case 0: hipLaunchKernelGGL((k_gmm_acc<M, false>), grid, block, 0, st, io); break;
    case 1: hipLaunchKernelGGL((k_gmm_fit<M, true>), dim3(1), block, 0, st, io); break;
    case 2: hipLaunchKernelGGL((k_gmm_acc<M, true>), grid, block, 0, st, io); break;
    case 3: hipLaunchKernelGGL((k_gmm_fit<M, false>), dim3(1), block, 0, st, io); break;
    default: hipLaunchKernelGGL((k_gmm_psi<M>), grid, block, 0, st, io); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t sp_launch_gmm(int phase, int M, const GmmIO& io, hipStream_t st) {
  if (io.n <= 0) return hipSuccess;
  switch (M) {
    case 1: return launch_m<1>(phase, io, st);
    case 2: return launch_m<2>(phase, io, st);
    case 3: return launch_m<3>(phase, io, st);
    case 4: return launch_m<4>(phase, io, st);
    default: return hipErrorInvalidValue;
  }
}
